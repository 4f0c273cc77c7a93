"""Pins of the oracle's input gap (the input aperture plane z_in before layer 1): equivalence
with a leading transparent layer, a closed-form plane wave and the gradient by finite
differences; CPU only."""
import cmath
import math

import numpy as np

from oracle import dpx_oracle as o
from paper_2604_02624_amd import workloads as wk


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_input_gap_equals_a_leading_transparent_layer():
    """Propagating the aperture over z_in and then running K layers is the (K+1)-layer cascade
    whose first layer has zero thickness and whose first gap is z_in."""
    wl = np.array([0.45e-6, 0.6e-6, 0.72e-6])
    N = 32
    g = np.random.default_rng(4)
    h = g.random((2, N, N)) * 1.2e-6
    ap = np.zeros((N, N), complex)
    ap[8:24, 8:24] = 1.0
    d = wk.make_design(n=N, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6, z=[9e-6, 7e-6],
                       fov=16, bin_=2, pad=2)
    d["z_in"] = 11e-6
    ref = wk.make_design(n=N, layers=3, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6,
                         z=[11e-6, 9e-6, 7e-6], fov=16, bin_=2, pad=2)
    h3 = np.concatenate([np.zeros((1, N, N)), h])
    assert rel(o.forward(d, h, ap, "fft"), o.forward(ref, h3, ap, "fft")) < 1e-12
    # and it matters
    assert rel(o.forward(dict(d, z_in=0.0), h, ap, "fft"), o.forward(d, h, ap, "fft")) > 1e-2


def test_input_gap_plane_wave_phase():
    """Periodic window, uniform input, transparent layer: the output field is
    exp(j 2 pi n (z_in + z) / lambda)."""
    N, wl = 16, 0.5e-6
    d = wk.make_design(n=N, layers=1, wl=np.array([wl]), n_mat=1.5, dx=0.25e-6, z=[6e-6], fov=N, pad=1)
    d["z_in"] = 4.3e-6
    _, _, out = o.forward(d, np.zeros((1, N, N)), None, "fft", keep=True)
    assert rel(out[0], np.full((N, N), cmath.exp(2j * math.pi * (4.3e-6 + 6e-6) / wl))) < 1e-12


def test_gradient_with_input_gap_matches_central_differences():
    wl = np.array([0.48e-6, 0.55e-6, 0.71e-6])
    N = 16
    d = wk.make_design(n=N, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.24e-6,
                       z=[4e-6, 6e-6], fov=8, pad=2)
    d["z_in"] = 5e-6
    g = np.random.default_rng(11)
    ap = np.zeros((N, N), complex)
    ap[4:12, 4:12] = 1.0
    h = g.random((2, N, N)) * 1.1e-6
    tau = g.random((3, 8, 8))
    _, dI, _ = o.loss(o.forward(d, h, ap, "naive"), tau)
    dh = o.grad(d, h, ap, dI, "naive")
    delta = 1e-4 * 0.6e-6
    v = g.standard_normal(h.shape)
    fd = o.fd_direction(d, h, ap, tau, v, delta, "naive")
    assert abs((dh * v).sum() - fd) < 1e-6 * abs(fd)
