"""Pins of the oracle's misalignment terms (lateral translation per gap, axial jitter, layer
offsets -> gap translations) against the Fourier shift theorem on a periodic grid, closed-form
plane waves, the centroid of a Gaussian beam, a physically displaced periodic stack and finite
differences of the loss; CPU only."""
import cmath
import math

import numpy as np
import pytest

from oracle import dpx_oracle as o
from paper_2604_02624_amd import workloads as wk


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def crand(g, shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


@pytest.mark.parametrize("kx,ky", [(3, -2), (-5, 0), (0, 7)])
def test_integer_shift_on_periodic_grid_is_a_roll(kx, ky):
    """pad = 1: translating by whole pixels is exactly a circular roll of the propagated field
    (+x is the last axis, +y the first)."""
    N, wl, dx, z = 32, 0.5e-6, 0.3e-6, 7.7e-6
    u = crand(np.random.default_rng(1), (N, N))
    ref = o.propagate(u, 1, dx, wl, 1.0, z, "fft")
    got = o.propagate(u, 1, dx, wl, 1.0, z, "fft", shift=(kx * dx, ky * dx))
    assert rel(got, np.roll(ref, (ky, kx), axis=(0, 1))) < 1e-12


def test_subpixel_shift_moves_the_gaussian_centroid_by_the_shift():
    """pad = 2, a Gaussian beam far from the window edge and well inside the band: the
    intensity centroid moves by exactly (sx, sy); sampling errors of a Gaussian this wide are
    exponentially small."""
    N, wl, dx, z, w0 = 64, 0.5e-6, 0.25e-6, 5e-6, 2e-6
    c = (np.arange(N) - N / 2 + 0.5) * dx
    u = np.exp(-(c[None, :] ** 2 + c[:, None] ** 2) / w0 ** 2).astype(complex)

    def centroid(f):
        I = np.abs(f) ** 2
        return (I.sum(0) @ c) / I.sum(), (I.sum(1) @ c) / I.sum()

    s = (0.37e-6, -0.61e-6)
    x0, y0 = centroid(o.propagate(u, 2, dx, wl, 1.0, z, "fft"))
    x1, y1 = centroid(o.propagate(u, 2, dx, wl, 1.0, z, "fft", shift=s))
    assert abs((x1 - x0) - s[0]) < 1e-6 * dx
    assert abs((y1 - y0) - s[1]) < 1e-6 * dx


@pytest.mark.parametrize("ax,ay", [(0, 0), (3, -4)])
def test_axial_jitter_adds_to_the_gap(ax, ay):
    """A transparent layer (h = 0) over a periodic window: a grid plane wave gains
    exp(j kz (z + dz)) with kz = sqrt(k^2 - kx^2 - ky^2)."""
    N, wl, dx, z, dz = 16, 0.5e-6, 0.25e-6, 9e-6, 0.2e-6
    d = wk.make_design(n=N, layers=1, wl=np.array([wl]), n_mat=1.5, dx=dx, z=[z], fov=N, pad=1)
    d["dz"] = np.array([dz])
    yy, xx = np.mgrid[0:N, 0:N]
    u = np.exp(2j * math.pi * (ax * xx + ay * yy) / N)
    _, _, out = o.forward(d, np.zeros((1, N, N)), u, "fft", keep=True)
    k = 2 * math.pi / wl
    kx, ky = 2 * math.pi * ax / (N * dx), 2 * math.pi * ay / (N * dx)
    kz = math.sqrt(k * k - kx * kx - ky * ky)
    assert rel(out[0], u * cmath.exp(1j * kz * (z + dz))) < 1e-12


def test_layer_offsets_match_a_physically_displaced_stack():
    """pad = 1, uniform input: displacing layer l by whole pixels D[l] (rolling its heights) and
    observing on the fixed output plane gives the same intensity as the undisplaced heights
    with the gap translations D[l] - D[l+1] (D[K] = 0)."""
    N, K = 32, 3
    wl = np.array([0.5e-6, 0.62e-6])
    d = wk.make_design(n=N, layers=K, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6,
                       z=[6e-6, 5e-6, 8e-6], fov=N, pad=1)
    g = np.random.default_rng(3)
    h = g.random((K, N, N)) * 1.2e-6
    D = np.array([[2, -1], [-3, 4], [1, 1]])   # (x, y) pixels per layer
    moved = np.stack([np.roll(h[l], (D[l, 1], D[l, 0]), axis=(0, 1)) for l in range(K)])
    ref = o.forward(d, moved, None, "fft")
    s = o.gap_shifts_from_layer_offsets(D * d["dx"])
    ds = dict(d, shift_x=s[:, 0], shift_y=s[:, 1])
    assert rel(o.forward(ds, h, None, "fft"), ref) < 1e-12


def test_gradient_with_misalignment_matches_central_differences():
    """The adjoint of a translated, jittered gap is the same chain with conj(H ramp)."""
    wl = np.array([0.48e-6, 0.55e-6, 0.71e-6])
    d = wk.make_design(n=16, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.24e-6,
                       z=[4e-6, 6e-6], fov=8, pad=2)
    d.update(shift_x=np.array([0.07e-6, -0.11e-6]), shift_y=np.array([-0.05e-6, 0.13e-6]),
             dz=np.array([0.09e-6, -0.04e-6]))
    g = np.random.default_rng(11)
    h = g.random((2, 16, 16)) * 1.1e-6
    tau = g.random((3, 8, 8))
    _, dI, _ = o.loss(o.forward(d, h, None, "naive"), tau)
    dh = o.grad(d, h, None, dI, "naive")
    delta = 1e-4 * 0.6e-6
    pix = [(int(g.integers(2)), int(g.integers(16)), int(g.integers(16))) for _ in range(8)]
    fd = o.fd_pixels(d, h, None, tau, pix, delta, "naive")
    assert rel(np.array([dh[p] for p in pix]), fd) < 1e-6
    v = g.standard_normal(h.shape)
    assert abs((dh * v).sum() - o.fd_direction(d, h, None, tau, v, delta, "naive")) \
        < 1e-6 * abs((dh * v).sum())


def test_axial_layer_offsets_match_moved_plane_positions():
    """Gap lengths recomputed from the displaced plane positions (layer l at Z_l + Dz_l, output
    plane fixed) equal z_l plus the jitter the conversion gives."""
    z = np.array([6e-6, 5e-6, 8e-6])
    Dz = np.array([0.3e-6, -0.2e-6, 0.45e-6])
    Z = np.concatenate([[0.0], np.cumsum(z)])          # layer planes, then the output plane
    moved = Z + np.append(Dz, 0.0)
    assert np.allclose(np.diff(moved), z + o.gap_jitter_from_layer_offsets(Dz), rtol=0, atol=1e-20)
    # every layer moved by the same amount: only the last gap changes, by minus that amount
    assert np.allclose(o.gap_jitter_from_layer_offsets(np.full(3, 0.1e-6)), [0, 0, -0.1e-6], atol=1e-22)
