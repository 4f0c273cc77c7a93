"""Pins of the oracle's fabrication and model variants: the phase bit-depth quantiser on the
heights, the band-limited angular spectrum and the phase-only layer of Eq. 3; CPU only."""
import math

import numpy as np
import pytest

from oracle import dpx_oracle as o
from paper_2604_02624_amd import workloads as wk


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ------------------------------------------------------------------------------------------
# phase bit depth
# ------------------------------------------------------------------------------------------

def test_quantiser_one_bit_and_exact_levels():
    h_max = 1.3e-6
    h = np.array([0.0, 0.3e-6, 0.64e-6, 0.66e-6, 1.0e-6, 1.3e-6], np.float32)
    assert np.array_equal(o.quantize_heights(h, h_max, 1), np.float32([0, 0, 0, h_max, h_max, h_max]))
    for bits in (4, 6, 8, 16):
        levels = (1 << bits) - 1
        step = np.float32(h_max / levels)
        k = np.random.default_rng(bits).integers(0, levels + 1, 1000).astype(np.float32)
        lv = k * step
        assert np.array_equal(o.quantize_heights(lv, h_max, bits), lv)


def test_quantiser_ties_go_to_even_levels():
    """With h_max = 2^B - 1 the scale and the step are exactly 1: k + 1/2 goes to the even one."""
    bits = 4
    h_max = float((1 << bits) - 1)
    h = np.float32([0.5, 1.5, 2.5, 3.5, 14.5])
    assert np.array_equal(o.quantize_heights(h, h_max, bits), np.float32([0, 2, 2, 4, 14]))


@pytest.mark.parametrize("bits", [4, 6, 8, 16])
def test_quantiser_error_bound_monotone_and_clamped(bits):
    h_max = 1.1e-6
    levels = (1 << bits) - 1
    step = h_max / levels
    h = np.sort(np.random.default_rng(3).uniform(-0.1 * h_max, 1.1 * h_max, 20000)).astype(np.float32)
    q = o.quantize_heights(h, h_max, bits).astype(np.float64)
    inside = (h >= 0) & (h <= h_max)
    assert np.all(np.abs(q[inside] - h[inside]) <= 0.5 * step * (1 + 1e-5) + 1e-7 * h_max)
    assert np.all(np.diff(q) >= 0)
    assert q.min() == 0.0 and abs(q.max() - h_max) <= 1e-7 * h_max
    assert len(np.unique(q)) <= levels + 1


# ------------------------------------------------------------------------------------------
# band-limited angular spectrum
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("M,z", [(64, 20e-6), (128, 5e-6), (256, 80e-6)])
def test_band_limit_is_where_the_sampled_phase_steps_by_pi(M, z):
    """At the band limit the phase 2 pi z sqrt(k^2 - f^2) changes by pi per frequency sample
    1 / (M dx) (its derivative by central differences)."""
    wl, dx, n = 0.55e-6, 0.25e-6, 1.0
    lim = o.band_limit(M, dx, wl, n, z)
    k = n / wl
    phi = lambda f: 2 * math.pi * z * math.sqrt(k * k - f * f)
    e = 1e-6 * lim
    slope = abs(phi(lim + e) - phi(lim - e)) / (2 * e)
    assert abs(slope / (M * dx) - math.pi) < 1e-6


def test_band_limited_transfer_function_is_a_symmetric_mask():
    M, dx, wl, z = 64, 0.25e-6, 0.5e-6, 30e-6
    H = o.transfer_function(M, dx, wl, 1.0, z)
    Hb = o.transfer_function(M, dx, wl, 1.0, z, band_limited=True)
    keep = Hb != 0
    assert np.array_equal(Hb[keep], H[keep])
    assert np.array_equal(keep, keep.T)            # same limit on both axes
    f = o.spatial_frequencies(M, dx)
    lim = o.band_limit(M, dx, wl, 1.0, z)
    assert np.array_equal(keep[0], (np.abs(f) <= lim) & (H[0] != 0))


def test_band_limited_spectrum_is_closer_to_the_direct_sum_over_a_long_gap():
    """A small random source over 30 um: the plain angular spectrum's undersampled transfer
    function wraps its impulse response around the window; the band-limited one does not."""
    wl, dx, N, z = 0.5e-6, 0.25e-6, 32, 30e-6
    g = np.random.default_rng(1)
    u = np.zeros((N, N), complex)
    u[13:19, 13:19] = g.standard_normal((6, 6)) + 1j * g.standard_normal((6, 6))
    ref = o.rs_direct(u, dx, wl, 1.0, z)
    plain = rel(o.propagate(u, 2, dx, wl, 1.0, z, "fft"), ref)
    bl = rel(o.propagate(u, 2, dx, wl, 1.0, z, "fft", band_limited=True), ref)
    assert bl < 0.5 and plain > 5 * bl


def test_band_limited_gradient_matches_central_differences():
    wl = np.array([0.48e-6, 0.71e-6])
    d = wk.make_design(n=16, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.24e-6,
                       z=[20e-6, 25e-6], fov=8, pad=2)
    d["band_limited"] = True
    g = np.random.default_rng(11)
    h = g.random((2, 16, 16)) * 1.1e-6
    tau = g.random((2, 8, 8))
    _, dI, _ = o.loss(o.forward(d, h, None, "naive"), tau)
    dh = o.grad(d, h, None, dI, "naive")
    v = g.standard_normal(h.shape)
    fd = o.fd_direction(d, h, None, tau, v, 1e-4 * 0.6e-6, "naive")
    assert abs((dh * v).sum() - fd) < 1e-6 * abs(fd)
    assert rel(o.forward(d, h, None, "fft"), o.forward(dict(d, band_limited=False), h, None, "fft")) > 1e-3


# ------------------------------------------------------------------------------------------
# phase-only layer (Eq. 3)
# ------------------------------------------------------------------------------------------

def test_phase_only_layer_is_the_unit_contrast_thickness_model():
    """exp(+j phi lambda_ref / lambda) is exactly the thickness model with n - n_m = 1, no
    absorption and h = phi lambda_ref / (2 pi); at lambda_ref it is exp(+j phi)."""
    phi = np.random.default_rng(2).uniform(0, 2 * np.pi, (8, 8))
    lam_ref = 0.6e-6
    assert rel(o.phase_only_transmission(phi, lam_ref, lam_ref), np.exp(1j * phi)) < 1e-15
    for wl in (0.45e-6, 0.6e-6, 0.74e-6):
        t = o.transmission(phi * lam_ref / (2 * np.pi), wl, 1.0 + 1.0, 0.0, 1.0)
        assert rel(o.phase_only_transmission(phi, wl, lam_ref), t) < 1e-13


@pytest.mark.parametrize("wl", [0.6e-6, 0.47e-6])
def test_phase_only_grating_diffraction_orders(wl):
    """Closed form for a cascade of Eq. 3 layers: a sinusoidal phase grating
    phi(x) = a cos(2 pi p x / N) at lambda_ref transmits exp(j a' cos theta), a' = a lambda_ref /
    lambda, which by the Jacobi-Anger expansion is sum_m j^m J_m(a') exp(j m theta); on a periodic
    grid of N samples (pad 1) order m is the grid frequency s = m p mod N (signed), which
    propagates with kz = sqrt(k^2 - (2 pi s / (N dx))^2) and is cut when that is imaginary.  The
    window intensity follows sample by sample."""
    from scipy.special import jv
    N, F, p, a, lam_ref, z = 32, 16, 3, 1.7, 0.6e-6, 5.3e-6
    dx = 0.3e-6
    d = wk.make_design(n=N, layers=1, wl=np.array([wl]), n_mat=2.0, dx=dx, z=[z], fov=F, pad=1)
    x = np.arange(N)
    phi = np.broadcast_to(a * np.cos(2 * np.pi * p * x / N), (N, N))[None]
    I = o.forward_phase_only(d, phi, lam_ref, None, "fft")[0]
    k = 2 * np.pi / wl
    ap = a * lam_ref / wl
    xs = np.arange((N - F) // 2, (N + F) // 2)
    field = np.zeros(F, complex)
    for m in range(-40, 41):           # |J_m(a')| < 1e-30 beyond
        sf = (m * p) % N
        sf = sf - N if sf >= N // 2 else sf
        kx = 2 * np.pi * sf / (N * dx)
        if kx * kx >= k * k:
            continue
        kz = np.sqrt(k * k - kx * kx)
        field += (1j ** m) * jv(m, ap) * np.exp(1j * (2 * np.pi * sf * xs / N + kz * z))
    ref = np.broadcast_to(np.abs(field) ** 2, (F, F))
    assert rel(I, ref) < 1e-12


def test_phase_only_cascade_is_the_unit_contrast_thickness_cascade():
    """Eq. 3 layers are the thickness model with n - n_m = 1, no absorption and
    h = phi lambda_ref / (2 pi) (an identity of the two transmissions), so the two cascades agree
    wherever the heights carry the phases exactly."""
    g = np.random.default_rng(5)
    wl = np.array([0.45e-6, 0.6e-6, 0.74e-6])
    lam_ref = 0.6e-6
    d = wk.make_design(n=16, layers=3, wl=wl, n_mat=2.0, dx=0.25e-6, z=[4e-6, 3e-6, 5e-6], fov=8)
    h = g.uniform(0, 1.2e-6, (3, 16, 16)).astype(np.float32)
    phi = h.astype(np.float64) * (2 * np.pi / lam_ref)
    I_p = o.forward_phase_only(d, phi, lam_ref, None, "naive")
    I_t = o.forward(d, h, None, "naive")
    assert rel(I_p, I_t) < 1e-12
