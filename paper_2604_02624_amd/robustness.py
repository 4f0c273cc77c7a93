"""Robustness tools on top of the fused path (paper Section 2, robustness of the multiplexed
storage to misalignment and to wavelength detuning).

* Misalignment: layer l displaced laterally by (Dx_l, Dy_l) and axially by Dz_l, the output
  plane fixed.  The library takes per-gap values (dpx_plan_set_misalignment): gap l runs from
  layer l to layer l+1 (the last one to the output plane).  Seen from a displaced element the
  incoming field is translated by minus its displacement, and propagation commutes with
  translations, so gap l translates the field by D_l - D_(l+1) and its length changes by
  Dz_(l+1) - Dz_l (D_K = Dz_K = 0).  The input field moves with the first layer.
* Vaccination: training draws a fresh misalignment, uniform in +-d_xy laterally and +-d_z
  axially for every layer, at every step.
* Detuning: every wavelength moved by the same offset, material index evaluated at the moved
  wavelength by the caller's dispersion function, PSNR of the output against the channel's
  target; one plan serves every probe (dpx_plan_set_wavelengths).
"""
from __future__ import annotations

import numpy as np


def gap_offsets(lateral: np.ndarray, axial: np.ndarray | None = None):
    """Layer displacements -> per-gap (dz, shift_x, shift_y), each of length K.

    lateral: [K, 2] (Dx, Dy) per layer in metres; axial: [K] Dz per layer or None."""
    lateral = np.asarray(lateral, np.float64).reshape(-1, 2)
    K = lateral.shape[0]
    nxt = np.zeros_like(lateral)
    nxt[:-1] = lateral[1:]
    shift = lateral - nxt
    dz = np.zeros(K)
    if axial is not None:
        axial = np.asarray(axial, np.float64).reshape(K)
        dz[:-1] = axial[1:] - axial[:-1]
        dz[-1] = -axial[-1]
    return dz, shift[:, 0].copy(), shift[:, 1].copy()


def draw_layer_offsets(rng: np.random.Generator, layers: int, d_xy: float, d_z: float):
    """Uniform layer displacements: lateral [K, 2] in +-d_xy, axial [K] in +-d_z (metres)."""
    lateral = rng.uniform(-d_xy, d_xy, (layers, 2))
    axial = rng.uniform(-d_z, d_z, layers)
    return lateral, axial


def detuning_psnr(plan, h, targets, offsets, n_of_wl, u_in=None, kappa_of_wl=None) -> np.ndarray:
    """PSNR (dB) [len(offsets), W] of a one-design plan with every wavelength moved by
    offsets[i] metres; n_of_wl(wl) (and kappa_of_wl, else the design's kappa) give the material
    at the moved wavelengths.  The plan's own wavelengths are restored afterwards."""
    if len(plan.designs) != 1:
        raise ValueError("detuning_psnr takes a plan of one design")
    d = plan.designs[0]
    wl0 = np.asarray(d["wl"], np.float64)
    n0 = np.asarray(d["n_mat"], np.float64)
    k0 = d.get("kappa")
    out = []
    try:
        for off in offsets:
            wl = wl0 + float(off)
            kap = k0 if kappa_of_wl is None else np.asarray(kappa_of_wl(wl), np.float64)
            plan.set_wavelengths(0, wl, np.asarray(n_of_wl(wl), np.float64), kap)
            out.append(plan.psnr(plan.forward(h, u_in), targets).cpu().numpy())
    finally:
        plan.set_wavelengths(0, wl0, n0, k0)
    return np.stack(out)
