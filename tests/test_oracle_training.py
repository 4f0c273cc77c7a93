"""Pins of the oracle's training helpers (Adam, the sigmoid bound on the heights, PSNR, channel
swapping) against closed forms, finite differences and invariances; CPU only."""
import numpy as np

from oracle import dpx_oracle as o
from paper_2604_02624_amd import train


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2 at every step, so each
    step is -lr g / (|g| + eps) exactly."""
    g = np.array([3e-3, -2.0, 5e-9, -7e-7])
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    for step in range(1, 6):
        d, m, v = o.adam_update(g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8)
        np.testing.assert_allclose(d, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_is_scale_invariant_without_eps():
    rng = np.random.default_rng(3)
    gs = rng.standard_normal((4, 10))
    m1 = v1 = m2 = v2 = np.zeros(10)
    for step, g in enumerate(gs, start=1):
        d1, m1, v1 = o.adam_update(g, m1, v1, step, eps=0.0)
        d2, m2, v2 = o.adam_update(1e4 * g, m2, v2, step, eps=0.0)
        np.testing.assert_allclose(d1, d2, rtol=1e-12)
    # and the second step differs from the first (moments carry the history)
    d_a, ma, va = o.adam_update(gs[0], np.zeros(10), np.zeros(10), 1)
    d_b, _, _ = o.adam_update(gs[1], ma, va, 2)
    assert not np.allclose(d_b, -1e-3 * gs[1] / (np.abs(gs[1]) + 1e-8))


def test_sigmoid_step_follows_the_chain_rule():
    """b1 = b2 = 0: the first step is -lr g / (|g| + eps) with g = dL/dtheta; recover |g| from the
    step and compare with central differences of L(theta) = sum c h(theta)."""
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(12)
    c = rng.standard_normal(12) * 1e3
    h_max = 1.2e-6
    lr, eps = 1e-3, 1e-8
    t2, h2, _, _ = o.adam_sigmoid_step(theta, c, np.zeros(12), np.zeros(12), 1, h_max, lr=lr, b1=0.0,
                                       b2=0.0, eps=eps)
    d = t2 - theta
    g_from_step = -np.sign(d) * eps * np.abs(d) / (lr - np.abs(d))
    dt = 1e-6
    L = lambda th: c * (h_max / (1 + np.exp(-th)))
    g_fd = (L(theta + dt) - L(theta - dt)) / (2 * dt)
    np.testing.assert_allclose(g_from_step, g_fd, rtol=1e-5)
    np.testing.assert_allclose(h2, h_max / (1 + np.exp(-t2)), rtol=1e-15)
    assert np.all((h2 > 0) & (h2 < h_max))


def test_psnr_of_a_known_perturbation():
    """Uniform target, image = target (1 + e s) with a zero-sum +-1 pattern s: the normalised
    difference is e s / P, so PSNR = -20 log10 e whatever the overall scale of the image."""
    P = 8
    tau = np.ones((2, P, P))
    s = np.where((np.add.outer(np.arange(P), np.arange(P)) % 2) == 0, 1.0, -1.0)
    I = np.stack([tau[0] * (1 + 1e-3 * s), 7.5 * tau[1] * (1 + 1e-2 * s)])
    np.testing.assert_allclose(o.psnr(I, tau), [60.0, 40.0], rtol=1e-10)
    assert np.isinf(o.psnr(tau.copy(), tau)).all()


def test_channel_swap_assigns_best_images_to_longest_wavelengths():
    wl = np.array([450e-9, 600e-9, 750e-9, 525e-9])
    ps = np.array([10.0, 30.0, 20.0, 40.0])
    src = o.channel_swap(ps, wl)
    assert sorted(src) == [0, 1, 2, 3]
    # PSNR of the image each wavelength now holds, wavelengths from the longest down
    by_length = np.argsort(-wl)
    assert list(ps[src][by_length]) == [40.0, 30.0, 20.0, 10.0]
    # the training module's own implementation agrees (it shares no code with the oracle)
    rng = np.random.default_rng(2)
    for _ in range(5):
        wl = rng.permutation(np.linspace(400e-9, 750e-9, 9))
        ps = rng.standard_normal(9) * 10
        np.testing.assert_array_equal(train.channel_swap_order(ps, wl), o.channel_swap(ps, wl))
