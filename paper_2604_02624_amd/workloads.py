"""Seeded synthetic workloads for multi-wavelength diffractive propagation.

This module only draws inputs: design geometry, height maps and target images.
It holds none of the propagation, loss or gradient arithmetic, so both the
GPU path and the FP64 oracle can consume its arrays without sharing code.

Geometry follows the paper's problem statement (Section 2, Fig. 1/2 and
Section 4 "Optical forward model"): K layers of N x N features at a pitch of
half a wavelength, a list of wavelengths each paired with one target image,
refractive index n(lambda) of the layer material, and free-space gaps between
layers.  The paper's datasets (CIFAR100 and MNIST targets, Section 4 "Data
preparation") are not available; smooth grayscale noise stands in for the
natural images and p = 0.5 binary patterns stand in for the handwritten
digits.

Every random stream is drawn from
``numpy.random.default_rng(SeedSequence([260402624, cfg, stream, ...]))`` with
streams 0 = heights, 1 = targets, 2 = design draws, 3 = finite-difference
pixel sample, 4 = finite-difference directions.

A design is a plain dict:

    n, layers, n_wl, fov, bin, pad : int
    dx, n_medium                    : float  (metres, refractive index)
    wl, n_mat, kappa                : float64 [n_wl]   (kappa may be None)
    z                               : float64 [layers] (z[k] = gap after layer k)
    z_in (optional)                 : float (input plane -> first layer)

A workload is a dict with ``designs`` (list), ``h`` (list of float32
[layers, n, n] arrays, metres), ``targets`` (list of float32 [n_wl, T, T]) and
``u_in`` (list of None = unit plane wave).
"""
from __future__ import annotations

import math

import numpy as np

ROOT_SEED = 260402624

STREAM_HEIGHTS = 0
STREAM_TARGETS = 1
STREAM_DESIGNS = 2
STREAM_FD_PIXELS = 3
STREAM_FD_DIRS = 4


def rng(cfg: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, cfg, stream, *extra]))


def cauchy_index(wl_m: np.ndarray, a: float = 1.50, b_um2: float = 0.0045) -> np.ndarray:
    """Cauchy dispersion n = a + b / lambda^2 with lambda in micrometres."""
    wl_um = np.asarray(wl_m, dtype=np.float64) * 1e6
    return a + b_um2 / (wl_um * wl_um)


# N-BK7 (Schott) Sellmeier coefficients, lambda in micrometres: n^2 - 1 = sum B_i l^2 / (l^2 - C_i)
NBK7_B = (1.03961212, 0.231792344, 1.01046945)
NBK7_C = (0.00600069867, 0.0200179144, 103.560653)


def nbk7_index(wl_m: np.ndarray) -> np.ndarray:
    """Refractive index of N-BK7 glass, the layer material of the paper's designs (Section 4,
    ref. 54), from the glass maker's Sellmeier formula; no absorption in the visible."""
    l2 = (np.asarray(wl_m, dtype=np.float64) * 1e6) ** 2
    n2 = 1.0 + sum(b * l2 / (l2 - c) for b, c in zip(NBK7_B, NBK7_C))
    return np.sqrt(n2)


def make_design(n, layers, wl, n_mat, dx, z, fov, bin_=1, pad=2, n_medium=1.0, kappa=None):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    n_mat = np.ascontiguousarray(np.broadcast_to(np.asarray(n_mat, dtype=np.float64), wl.shape))
    z = np.ascontiguousarray(np.broadcast_to(np.asarray(z, dtype=np.float64), (layers,)))
    if kappa is not None:
        kappa = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, dtype=np.float64), wl.shape))
    return dict(n=int(n), layers=int(layers), n_wl=int(wl.size), fov=int(fov), bin=int(bin_),
                pad=int(pad), dx=float(dx), n_medium=float(n_medium), wl=wl, n_mat=n_mat,
                kappa=kappa, z=z)


def uniform_heights(g: np.random.Generator, layers: int, n: int, h_max: float) -> np.ndarray:
    """Heights drawn in float64 and rounded once to float32 (both sides use the float32 values)."""
    return (g.random((layers, n, n)) * h_max).astype(np.float32)


def binary_targets(g: np.random.Generator, n_wl: int, t: int) -> np.ndarray:
    return (g.random((n_wl, t, t)) < 0.5).astype(np.float32)


def grayscale_targets(g: np.random.Generator, n_wl: int, t: int, sigma: float = 2.0) -> np.ndarray:
    """Smoothed Gaussian noise: N(0,1) -> periodic Gaussian blur (sigma px) -> standardise
    per image -> 0.5 + 0.25 z -> clip to [0, 1]."""
    from scipy.ndimage import gaussian_filter

    z = g.standard_normal((n_wl, t, t))
    z = gaussian_filter(z, sigma=(0.0, sigma, sigma), mode="wrap")
    mu = z.mean(axis=(1, 2), keepdims=True)
    sd = z.std(axis=(1, 2), keepdims=True)
    z = (z - mu) / np.where(sd > 0, sd, 1.0)
    return np.clip(0.5 + 0.25 * z, 0.0, 1.0).astype(np.float32)


# --------------------------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------------------------

def _experiment_pair(cfg: int):
    """Two 64x64 layers, the six experimental wavelengths 500..740 nm (Section 2 "Experimental
    validation"), n = 1.5, pitch 0.5 lambda_m with lambda_m = 620 nm, gaps of 40 lambda_m."""
    lam_m = 620e-9
    wl = np.arange(500, 741, 48, dtype=np.float64) * 1e-9
    n_const = 1.5
    d = make_design(n=64, layers=2, wl=wl, n_mat=n_const, dx=0.5 * lam_m, z=40 * lam_m, fov=32)
    d["h_max"] = lam_m / (n_const - 1.0)
    h = uniform_heights(rng(cfg, STREAM_HEIGHTS), 2, 64, d["h_max"])
    tau = binary_targets(rng(cfg, STREAM_TARGETS), d["n_wl"], 32)
    return d, h, tau


def _visible_band(cfg: int, n: int, layers: int, n_wl: int, t: int, gray: bool, extra=()):
    """lambda in [450, 750] nm, lambda_m = 600 nm, pitch 300 nm, gaps 50 lambda_m = 30 um,
    Cauchy n(lambda), heights U[0, lambda_m / (n(lambda_m) - 1)]."""
    lam_m = 600e-9
    wl = np.linspace(450e-9, 750e-9, n_wl, dtype=np.float64)
    n_mat = cauchy_index(wl)
    h_max = lam_m / (float(cauchy_index(np.array([lam_m]))[0]) - 1.0)
    d = make_design(n=n, layers=layers, wl=wl, n_mat=n_mat, dx=0.5 * lam_m, z=50 * lam_m, fov=t)
    d["h_max"] = h_max
    h = uniform_heights(rng(cfg, STREAM_HEIGHTS, *extra), layers, n, h_max)
    g = rng(cfg, STREAM_TARGETS, *extra)
    tau = grayscale_targets(g, n_wl, t) if gray else binary_targets(g, n_wl, t)
    return d, h, tau


def paper_geometry(n_wl: int = 4096, layers: int = 8, n: int = 800, cfg: int = 6):
    """The Fig. 2 design (Section 2 and Section 4 "Optical forward model"): 800 x 800 N-BK7
    features per layer at a pitch of half the shortest wavelength (200 nm), K = 8, wavelengths
    from 750 nm down to 400 nm (longest first), an input aperture and an output field of view
    of about 69.56 lambda_m (200 samples), 25 x 25 output pixels of 8 x 8 samples, and an axial
    span of about 1260 lambda_m from the aperture to the output plane, split here into equal
    gaps (input plane, K layers, output plane: K + 1 gaps).  Smaller n_wl / layers / n keep the
    same optics for tests."""
    lam_short, lam_long = 400e-9, 750e-9
    lam_m = 0.5 * (lam_short + lam_long)
    dx = 0.5 * lam_short
    wl = np.linspace(lam_long, lam_short, n_wl, dtype=np.float64)
    gap = 1260.0 * lam_m / (layers + 1)
    side = 200 if n >= 400 else n // 4          # aperture / field-of-view side in samples
    side -= side % 8
    d = make_design(n=n, layers=layers, wl=wl, n_mat=nbk7_index(wl), dx=dx, z=gap, fov=side,
                    bin_=8, pad=2)
    d["z_in"] = gap
    d["h_max"] = lam_m / (float(nbk7_index(np.array([lam_m]))[0]) - 1.0)
    a = (n - side) // 2
    u_in = np.zeros((n, n), np.complex64)
    u_in[a:a + side, a:a + side] = 1.0
    h = uniform_heights(rng(cfg, STREAM_HEIGHTS), layers, n, d["h_max"])
    tau = grayscale_targets(rng(cfg, STREAM_TARGETS), n_wl, side // 8)
    return d, h, tau, u_in


def make_workload(cfg: int) -> dict:
    """cfg 1..6: the workloads (small forward, small fwd+adjoint, batched, large, uneven, and
    the paper's own Fig. 2 geometry)."""
    if cfg in (1, 2):
        d, h, tau = _experiment_pair(cfg)
        designs, hs, taus = [d], [h], [tau]
    elif cfg == 3:
        d, h, tau = _visible_band(3, n=256, layers=5, n_wl=256, t=64, gray=True)
        designs, hs, taus = [d], [h], [tau]
    elif cfg == 4:
        d, h, tau = _visible_band(4, n=512, layers=4, n_wl=4096, t=64, gray=True)
        designs, hs, taus = [d], [h], [tau]
    elif cfg == 5:
        g = rng(5, STREAM_DESIGNS)
        designs, hs, taus = [], [], []
        for i in range(64):
            n = int(g.choice([96, 128, 192, 256]))
            layers = int(g.integers(2, 6))
            n_wl = int(round(math.exp(g.uniform(math.log(6.0), math.log(512.0)))))
            d, h, tau = _visible_band(5, n=n, layers=layers, n_wl=n_wl, t=n // 4, gray=False,
                                      extra=(i,))
            designs.append(d)
            hs.append(h)
            taus.append(tau)
    elif cfg == 6:
        d, h, tau, u_in = paper_geometry()
        return dict(cfg=cfg, designs=[d], h=[h], targets=[tau], u_in=[u_in])
    else:
        raise ValueError(f"unknown workload {cfg}")
    return dict(cfg=cfg, designs=designs, h=hs, targets=taus, u_in=[None] * len(designs))


def subset_wavelengths(design: dict, idx) -> dict:
    """A copy of ``design`` restricted to the wavelengths ``idx`` (same order)."""
    idx = np.asarray(idx, dtype=np.int64)
    d = dict(design)
    d["wl"] = np.ascontiguousarray(design["wl"][idx])
    d["n_mat"] = np.ascontiguousarray(design["n_mat"][idx])
    if design.get("kappa") is not None:
        d["kappa"] = np.ascontiguousarray(design["kappa"][idx])
    d["n_wl"] = int(idx.size)
    return d


def target_side(design: dict) -> int:
    return design["fov"] // design["bin"]


def describe(cfg: int) -> str:
    w = make_workload(cfg)
    parts = []
    for d in w["designs"][:4]:
        parts.append(f"N={d['n']} M={d['pad'] * d['n']} K={d['layers']} W={d['n_wl']} F={d['fov']}")
    more = "" if len(w["designs"]) <= 4 else f" ... ({len(w['designs'])} designs)"
    return "; ".join(parts) + more
