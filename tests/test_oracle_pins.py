"""Pins of the FP64 oracle against things other than itself: brute-force sums, a library FFT,
closed forms of wave optics, the direct Rayleigh-Sommerfeld integral of Eq. 4/5, exact
invariances of the model, and central finite differences.

Each test is chosen so that a plausible slip in the oracle (a dropped factor, a flipped sign,
a transposed frequency axis, a wrong crop offset, a missing term of the gradient) fails it.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest

from oracle import dpx_oracle as o
from paper_2604_02624_amd import workloads as wk

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def crand(g, shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


# ------------------------------------------------------------------------------------------
# DFT
# ------------------------------------------------------------------------------------------

def test_dft_brute_force_tiny():
    """Quadruple loop over the textbook definition, M = 6 (includes a radix-3 factor)."""
    g = np.random.default_rng(1)
    M = 6
    U = crand(g, (M, M))
    ref = np.zeros((M, M), complex)
    for ky in range(M):
        for kx in range(M):
            s = 0j
            for y in range(M):
                for x in range(M):
                    s += U[y, x] * cmath.exp(-2j * math.pi * (ky * y + kx * x) / M)
            ref[ky, kx] = s
    assert rel(o.dft2(U, "naive"), ref) < 1e-13
    assert rel(o.idft2(ref, "naive"), U) < 1e-13


@pytest.mark.parametrize("M", [8, 12, 64, 96, 128])
def test_dft_naive_matches_pocketfft(M):
    g = np.random.default_rng(M)
    U = crand(g, (3, M, M))
    assert rel(o.dft2(U, "naive"), np.fft.fft2(U)) < 1e-12
    assert rel(o.idft2(U, "naive"), np.fft.ifft2(U)) < 1e-12
    assert rel(o.idft2(o.dft2(U, "naive"), "naive"), U) < 1e-13


def test_signed_index_is_fftfreq():
    for M in (7, 8, 128, 192):
        assert np.array_equal(o.signed_index(M), np.rint(np.fft.fftfreq(M) * M).astype(int))


# ------------------------------------------------------------------------------------------
# Single gap: closed forms
# ------------------------------------------------------------------------------------------

def test_normal_plane_wave_picks_up_exp_jkz():
    """pad = 1 (periodic window): a uniform field is a plane wave along z and gains
    exp(j 2 pi n z / lambda) exactly."""
    N, wl, n_m, z = 32, 0.55e-6, 1.33, 17.3e-6
    u = np.full((N, N), 0.7 - 0.2j)
    out = o.propagate(u, 1, wl / 2, wl, n_m, z, "naive")
    assert rel(out, u * cmath.exp(2j * math.pi * n_m * z / wl)) < 1e-13


@pytest.mark.parametrize("ax,ay", [(3, 0), (0, 5), (4, -7), (-9, 2), (15, 15)])
def test_tilted_plane_wave(ax, ay):
    """A plane wave with transverse wavenumbers (kx, ky) travels with
    kz = sqrt(k^2 - kx^2 - ky^2); with k^2 < kx^2 + ky^2 the cut removes it."""
    N, wl, n_m, z = 32, 0.5e-6, 1.0, 9.1e-6
    dx = wl / 2
    yy, xx = np.mgrid[0:N, 0:N]
    u = np.exp(2j * math.pi * (ax * xx + ay * yy) / N)
    out = o.propagate(u, 1, dx, wl, n_m, z, "fft")
    kx, ky = 2 * math.pi * ax / (N * dx), 2 * math.pi * ay / (N * dx)
    k = 2 * math.pi * n_m / wl
    if kx * kx + ky * ky < k * k:
        kz = math.sqrt(k * k - kx * kx - ky * ky)
        assert rel(out, u * cmath.exp(1j * kz * z)) < 1e-12
    else:
        assert np.abs(out).max() < 1e-13


def test_evanescent_wave_is_cut_even_at_short_range():
    """Evanescent components are dropped (H = 0), not attenuated: even over 50 nm, where an
    exponentially decaying wave would keep a large part of its amplitude, nothing is left."""
    N, wl, dx = 32, 0.5e-6, 0.25e-6
    yy, xx = np.mgrid[0:N, 0:N]
    u = np.exp(2j * math.pi * (15 * xx + 15 * yy) / N)
    out = o.propagate(u, 1, dx, wl, 1.0, 50e-9, "fft")
    assert np.abs(out).max() < 1e-13


def _gaussian_error(w0, wl, N, dx, z_over_zr):
    x = (np.arange(N) - N / 2) * dx
    X, Y = np.meshgrid(x, x)
    r2 = X * X + Y * Y
    u = np.exp(-r2 / w0 ** 2)
    zr = math.pi * w0 ** 2 / wl
    z = z_over_zr * zr
    out = o.propagate(u, 2, dx, wl, 1.0, z, "fft")
    k = 2 * math.pi / wl
    wz = w0 * math.sqrt(1 + (z / zr) ** 2)
    Rz = z * (1 + (zr / z) ** 2)
    gouy = math.atan(z / zr)
    ref = (w0 / wz) * np.exp(-r2 / wz ** 2) * np.exp(1j * (k * z + k * r2 / (2 * Rz) - gouy))
    mask = r2 < (2.5 * wz) ** 2
    return rel(out[mask], ref[mask]), out, ref, wz, x


def test_gaussian_beam_paraxial_limit():
    """Gaussian beam: width w0 sqrt(1 + (z/zR)^2), curvature, Gouy phase.  The paraxial
    form is exact only to O((lambda / (pi w0))^2), so the error must be of that size and
    must shrink by about 4x when w0 doubles."""
    wl = 0.5e-6
    e1, out, ref, wz, x = _gaussian_error(4 * wl, wl, 256, wl / 2, 1.0)
    e2, *_ = _gaussian_error(8 * wl, wl, 512, wl / 2, 1.0)
    theta2 = (wl / (math.pi * 4 * wl)) ** 2
    assert e1 < 3 * theta2
    assert 2.5 < e1 / e2 < 6.0
    # second-moment width of |u|^2 equals w(z)/2 per axis
    I = np.abs(out) ** 2
    X = x[None, :]
    var = float((I * X * X).sum() / I.sum())
    assert abs(math.sqrt(var) - wz / 2) / (wz / 2) < 3 * theta2


def test_parseval_band_limited():
    """|H| = 1 on propagating frequencies: a field whose spectrum lies there keeps its
    energy (periodic window); an evanescent component loses exactly its own energy."""
    g = np.random.default_rng(3)
    N, wl = 64, 0.5e-6
    dx = 0.4e-6
    f = o.spatial_frequencies(N, dx)
    inside = (f[None, :] ** 2 + f[:, None] ** 2) < (0.95 / wl) ** 2
    spec = crand(g, (N, N)) * inside
    u = np.fft.ifft2(spec)
    out = o.propagate(u, 1, dx, wl, 1.0, 33e-6, "naive")
    assert abs(np.linalg.norm(out) / np.linalg.norm(u) - 1) < 1e-13
    ev = crand(g, (N, N)) * (~inside & ((f[None, :] ** 2 + f[:, None] ** 2) > (1.01 / wl) ** 2))
    u2 = u + np.fft.ifft2(ev)
    out2 = o.propagate(u2, 1, dx, wl, 1.0, 33e-6, "naive")
    assert abs(np.linalg.norm(out2) / np.linalg.norm(u) - 1) < 1e-13


def test_semigroup_z1_plus_z2():
    g = np.random.default_rng(4)
    N, wl, dx = 48, 0.6e-6, 0.3e-6
    u = crand(g, (N, N))
    a = o.propagate(o.propagate(u, 1, dx, wl, 1.0, 7e-6, "naive"), 1, dx, wl, 1.0, 11e-6, "naive")
    b = o.propagate(u, 1, dx, wl, 1.0, 18e-6, "naive")
    assert rel(a, b) < 1e-12


def test_adjoint_dot_product():
    """<P x, y> = <x, P^H y> for the padded, cropped gap operator."""
    g = np.random.default_rng(5)
    N, wl, dx = 40, 0.5e-6, 0.25e-6
    x, y = crand(g, (N, N)), crand(g, (N, N))
    Px = o.propagate(x, 2, dx, wl, 1.0, 12e-6, "naive")
    PHy = o.propagate(y, 2, dx, wl, 1.0, 12e-6, "naive", adjoint=True)
    lhs = np.vdot(y, Px)
    rhs = np.vdot(PHy, x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


@pytest.mark.parametrize("w0,z,pad,tol", [(1.5e-6, 10e-6, 2, 1e-12), (1.0e-6, 40e-6, 4, 1e-10),
                                          (1.0e-6, 40e-6, 2, 1e-4)])
def test_angular_spectrum_matches_direct_rayleigh_sommerfeld(w0, z, pad, tol):
    """Eq. 4/5 summed directly (with dx^2) versus the angular spectrum.  For a smooth input
    whose spectrum has no evanescent part the two agree to rounding, as long as the window
    (pad * N) holds the spreading output; with pad = 2 at the larger distance the periodic
    window wraps and the difference is of the order of the wrapped energy."""
    wl, dx = 0.5e-6, 0.25e-6
    N = 64
    x = (np.arange(N) - (N - 1) / 2) * dx
    u = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / w0 ** 2).astype(complex)
    ref = o.rs_direct(u, dx, wl, 1.0, z)
    a = o.propagate(u, pad, dx, wl, 1.0, z, "fft")
    err = rel(a, ref)
    assert err < tol
    if pad == 2 and tol > 1e-6:
        assert err > 1e-7           # the wrap is real, not hidden by the comparison


def test_mirror_symmetry_and_linearity():
    g = np.random.default_rng(6)
    N, wl, dx = 30, 0.5e-6, 0.25e-6
    a, b = crand(g, (N, N)), crand(g, (N, N))
    P = lambda u: o.propagate(u, 2, dx, wl, 1.0, 8e-6, "naive")
    assert rel(P(a[::-1, ::-1]), P(a)[::-1, ::-1]) < 1e-12
    assert rel(P(a.T), P(a).T) < 1e-12
    c1, c2 = 0.3 - 1.1j, -2.0 + 0.5j
    assert rel(P(c1 * a + c2 * b), c1 * P(a) + c2 * P(b)) < 1e-12


# ------------------------------------------------------------------------------------------
# Transmission and cascade
# ------------------------------------------------------------------------------------------

def _one_layer_design(N, wl, n_mat, z, pad=2, fov=None, kappa=None, layers=1, dx=None):
    wl = np.atleast_1d(np.asarray(wl, float))
    return wk.make_design(n=N, layers=layers, wl=wl, n_mat=n_mat, dx=dx or wl.min() / 2, z=z,
                          fov=fov or N, pad=pad, kappa=kappa)


def test_prism_deflects_toward_thicker_side():
    """Sign of the Eq. 1 phase (read as +j, the convention of Eq. 4's exp(+jkr)): a linear
    thickness ramp is a prism, which tilts the beam toward its thick side by
    sin(theta) = (n - 1) dh/dx; the centroid moves by z tan(theta)."""
    N, wl, n = 256, 0.5e-6, 1.5
    dx = wl / 2
    x = (np.arange(N) - N / 2) * dx
    X, Y = np.meshgrid(x, x)
    w0 = 6e-6
    u_in = np.exp(-(X * X + Y * Y) / w0 ** 2)
    slope = 0.1
    h = (slope * (X - x.min()))[None].astype(np.float32)
    z = 20e-6
    d = _one_layer_design(N, wl, n, z, pad=2, dx=dx)
    I = o.forward(d, h, u_in, "fft")[0]
    cx = float((I * X).sum() / I.sum())
    theta = math.asin((n - 1) * slope)
    assert cx > 0
    assert abs(cx - z * math.tan(theta)) < 0.02 * z * math.tan(theta)


@pytest.mark.parametrize("N,F,b", [(16, 8, 1), (18, 8, 2), (20, 12, 4)])
def test_field_of_view_is_the_central_window(N, F, b):
    """Placement of the F x F field of view (Section 4, the output window in the middle of the
    output plane): on a periodic grid (pad 1) a uniform wave plus a tilted one interferes into
    the closed form I(x, y) = 2 + 2 cos(2 pi (p x + q y) / N + kz_t z - k z), so the binned
    image of the window starting at ((N - F) / 2, (N - F) / 2) is known sample by sample.
    p != q, so a window displaced along either axis (or with its axes swapped) fails; the
    sizes are chosen so that no tested displacement is a whole period of the pattern."""
    wl, n_m, z, p, q = 0.5e-6, 1.0, 7.3e-6, 1, 2
    dx = wl / 2
    yy, xx = np.mgrid[0:N, 0:N]
    u_in = 1.0 + np.exp(2j * math.pi * (p * xx + q * yy) / N)
    d = _one_layer_design(N, [wl], 1.5, z, pad=1, fov=F, dx=dx)
    d["bin"] = b
    I = o.forward(d, np.zeros((1, N, N), np.float32), u_in, "fft")[0]
    k = 2 * math.pi * n_m / wl
    kt = 2 * math.pi / (N * dx)
    dphi = math.sqrt(k * k - (p * kt) ** 2 - (q * kt) ** 2) * z - k * z
    a = (N - F) // 2
    ys, xs = np.mgrid[a:a + F, a:a + F]
    full = 2.0 + 2.0 * np.cos(2 * math.pi * (p * xs + q * ys) / N + dphi)
    T = F // b
    ref = full.reshape(T, b, T, b).sum(axis=(1, 3))
    assert I.shape == (T, T)
    assert rel(I, ref) < 1e-12


def test_field_of_view_of_a_symmetric_design_is_flip_symmetric():
    """A design that is mirror symmetric about the centre of its N x N aperture (uniform input,
    heights symmetric under x -> N-1-x and y -> N-1-y, zero padding around the aperture) has a
    mirror-symmetric output field, and the central window maps onto itself under the same
    mirror; so the binned image is symmetric under both flips.  A window shifted off the centre
    (a = 0, a = N - F, or one sample off) sees a different part of the field and fails."""
    g = np.random.default_rng(11)
    N, F = 24, 10
    wl = np.array([0.5e-6, 0.62e-6])
    half = g.uniform(0, 1e-6, (2, N // 2, N // 2))
    h = np.concatenate([half, half[:, :, ::-1]], axis=2)
    h = np.concatenate([h, h[:, ::-1, :]], axis=1).astype(np.float32)
    d = _one_layer_design(N, wl, 1.5, [6e-6, 4e-6], pad=2, fov=F, layers=2, dx=0.25e-6)
    I = o.forward(d, h, None, "fft")
    assert rel(I, I[:, ::-1, :]) < 1e-12
    assert rel(I, I[:, :, ::-1]) < 1e-12
    # the field is not flat over the aperture, so the symmetry is not trivial
    full = o.forward(dict(d, fov=N), h, None, "fft")
    assert rel(full[:, :F, :F], full[:, :F, :F][:, ::-1, ::-1]) > 1e-3


def test_global_phase_and_two_pi_wrap_invariance():
    g = np.random.default_rng(7)
    N, K = 24, 2
    wl = np.array([0.5e-6, 0.61e-6])
    d = _one_layer_design(N, wl, [1.5, 1.48], 6e-6, layers=K, fov=12)
    h = (g.random((K, N, N)) * 1e-6)
    I0 = o.forward(d, h, None, "naive")
    I1 = o.forward(d, h + 0.37e-6, None, "naive")
    assert rel(I1, I0) < 1e-12
    d1 = wk.subset_wavelengths(d, [1])
    h2 = h.copy()
    h2[1, 3:9, 5:20] += d1["wl"][0] / (d1["n_mat"][0] - 1.0)
    assert rel(o.forward(d1, h2, None, "naive"), o.forward(d1, h, None, "naive")) < 1e-11
    assert rel(o.forward(d1, h + 1e-7 * (np.arange(N) / N)[None, None, :], None, "naive"),
               o.forward(d1, h, None, "naive")) > 1e-3


def test_flat_layers_periodic_window_keep_uniform_intensity():
    N = 16
    d = _one_layer_design(N, [0.45e-6, 0.7e-6], 1.5, 3e-6, pad=1, layers=3, fov=8)
    d["bin"] = 2
    I = o.forward(d, np.zeros((3, N, N), np.float32), None, "naive")
    assert np.allclose(I, 4.0, rtol=0, atol=1e-12)


def test_transparent_zero_gap_layer_is_identity():
    """A layer with h = 0 followed by a zero gap leaves a band-limited field unchanged."""
    g = np.random.default_rng(8)
    N, wl, dx = 32, 0.5e-6, 0.3e-6
    f = o.spatial_frequencies(N, dx)
    inside = (f[None, :] ** 2 + f[:, None] ** 2) < (0.9 / wl) ** 2
    u = np.fft.ifft2(crand(g, (N, N)) * inside)
    d2 = _one_layer_design(N, wl, 1.5, [5e-6, 0.0], pad=1, layers=2, dx=dx)
    d1 = _one_layer_design(N, wl, 1.5, 5e-6, pad=1, layers=1, dx=dx)
    h = g.random((2, N, N)) * 1e-6
    h[1] = 0
    assert rel(o.forward(d2, h, u, "naive"), o.forward(d1, h[:1], u, "naive")) < 1e-12


def test_batch_invariance():
    w = wk.make_workload(1)
    d, h = w["designs"][0], w["h"][0]
    I = o.forward(d, h, None, "fft")
    for i in (0, 3, 5):
        Ii = o.forward(wk.subset_wavelengths(d, [i]), h, None, "fft")
        assert np.array_equal(I[i], Ii[0])


def test_naive_and_fft_modes_agree_on_workload():
    w = wk.make_workload(2)
    d, h = w["designs"][0], w["h"][0]
    assert rel(o.forward(d, h, None, "naive"), o.forward(d, h, None, "fft")) < 1e-12


# ------------------------------------------------------------------------------------------
# Loss
# ------------------------------------------------------------------------------------------

def test_loss_zero_and_scale_invariance():
    g = np.random.default_rng(9)
    tau = g.random((3, 8, 8))
    assert o.loss(2.5 * tau, tau)[0] < 1e-30
    I = g.random((3, 8, 8))
    L = o.loss(I, tau)[0]
    assert abs(o.loss(7.0 * I, tau)[0] - L) < 1e-15 * max(1.0, L)
    assert abs(o.loss(I, 0.2 * tau)[0] - L) < 1e-15 * max(1.0, L)


def test_loss_gradient_finite_difference_and_euler():
    g = np.random.default_rng(10)
    I = g.random((2, 5, 5)) + 0.1
    tau = (g.random((2, 5, 5)) < 0.5).astype(float)
    L, dI, _ = o.loss(I, tau)
    # Euler: L is homogeneous of degree 0 in each wavelength's I
    assert np.abs((dI * I).sum(axis=(1, 2))).max() < 1e-15
    fd = np.zeros_like(I)
    eps = 1e-6
    for idx in np.ndindex(I.shape):
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += eps
        Im[idx] -= eps
        fd[idx] = (o.loss(Ip, tau)[0] - o.loss(Im, tau)[0]) / (2 * eps)
    assert rel(dI, fd) < 1e-7


def test_loss_by_hand_two_pixels():
    """W = 1, T^2 = 2 pixels (as 1x2): I = (1, 3) -> (1/4, 3/4); tau = (1, 1) -> (1/2, 1/2);
    L = ((1/4 - 1/2)^2 + (3/4 - 1/2)^2) / 2 = 1/16."""
    I = np.array([[[1.0, 3.0]]])
    tau = np.array([[[1.0, 1.0]]])
    L, dI, per = o.loss(I, tau)
    assert abs(L - 1.0 / 16) < 1e-16
    assert per.shape == (1,)


def test_loss_degenerate_wavelength_contributes_zero():
    tau = np.ones((2, 3, 3))
    I = np.ones((2, 3, 3))
    I[1] = 0.0
    L, dI, _ = o.loss(I, tau)
    assert np.all(dI[1] == 0)
    # first wavelength matches its target; second: every pixel (0 - 1/9)^2 = 1/81, mean 1/81;
    # the mean over the two wavelengths is 1/162
    assert abs(L - 1.0 / 162) < 1e-16


# ------------------------------------------------------------------------------------------
# Gradient
# ------------------------------------------------------------------------------------------

def _small_design(kappa=False, pad=2, b=1):
    wl = np.array([0.48e-6, 0.55e-6, 0.71e-6])
    d = wk.make_design(n=16, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.24e-6,
                       z=[4e-6, 6e-6], fov=8, bin_=b, pad=pad,
                       kappa=(np.array([0.01, 0.02, 0.005]) if kappa else None))
    g = np.random.default_rng(11)
    h = g.random((2, 16, 16)) * 1.1e-6
    tau = g.random((3, 8 // b, 8 // b))
    return d, h, tau


@pytest.mark.parametrize("kappa,b", [(False, 1), (True, 1), (False, 2)])
def test_gradient_matches_central_differences(kappa, b):
    d, h, tau = _small_design(kappa, b=b)
    L, dI, _ = o.loss(o.forward(d, h, None, "naive"), tau)
    dh = o.grad(d, h, None, dI, "naive")
    g = np.random.default_rng(12)
    pix = [(int(g.integers(2)), int(g.integers(16)), int(g.integers(16))) for _ in range(12)]
    # step 1e-4 lambda_m: truncation (c_t delta)^2 / 6 ~ 3e-8 relative
    delta = 1e-4 * 0.6e-6
    fd = o.fd_pixels(d, h, None, tau, pix, delta, "naive")
    an = np.array([dh[p] for p in pix])
    assert rel(an, fd) < 1e-6
    v = g.standard_normal(h.shape)
    assert abs((dh * v).sum() - o.fd_direction(d, h, None, tau, v, delta, "naive")) \
        < 1e-6 * abs((dh * v).sum())


def test_gradient_per_layer_sum_vanishes():
    """Adding a constant to one layer's heights multiplies every wavelength's field by a
    constant (a phase, and with kappa a real factor); the per-wavelength normalised loss
    does not change, so the gradient of each layer sums to zero."""
    d, h, tau = _small_design(kappa=True)
    _, dI, _ = o.loss(o.forward(d, h, None, "naive"), tau)
    dh = o.grad(d, h, None, dI, "naive")
    s = np.abs(dh.sum(axis=(1, 2)))
    assert s.max() < 1e-10 * np.abs(dh).sum()


def test_gradient_with_input_field_and_periodic_window():
    d, h, tau = _small_design(pad=1)
    g = np.random.default_rng(13)
    u = crand(g, (16, 16))
    _, dI, _ = o.loss(o.forward(d, h, u, "naive"), tau)
    dh = o.grad(d, h, u, dI, "naive")
    v = g.standard_normal(h.shape)
    delta = 1e-4 * 0.6e-6
    lp = o.loss_of_heights(d, h + delta * v, u, tau)
    lm = o.loss_of_heights(d, h - delta * v, u, tau)
    assert abs((dh * v).sum() - (lp - lm) / (2 * delta)) < 1e-6 * abs((dh * v).sum())


# ------------------------------------------------------------------------------------------
# Paper geometry (golden values printed in the paper)
# ------------------------------------------------------------------------------------------

def test_paper_geometry_golden():
    with open(os.path.join(HERE, "golden", "paper_geometry.json")) as f:
        gold = json.load(f)
    fig2 = gold["fig2_design"]
    lam_m = 0.5 * (fig2["lambda_long_nm"] + fig2["lambda_short_nm"])
    pitch = 0.5 * fig2["lambda_short_nm"]
    assert abs(pitch - fig2["pitch_nm"]) < 1e-9
    assert abs(fig2["features_per_side"] * pitch / lam_m - fig2["layer_side_over_lambda_m"]) < 0.5
    assert abs(fig2["fov_side_over_lambda_m"] / fig2["fov_pixels"]
               - fig2["fov_pixel_over_lambda_m"]) < 0.01
    exp = gold["experiment"]
    assert exp["wavelengths_nm"] == list(range(500, 741, 48))
    w = wk.make_workload(1)
    assert np.allclose(w["designs"][0]["wl"] * 1e9, exp["wavelengths_nm"])
