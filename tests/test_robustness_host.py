"""Host logic of the robustness tools: layer displacements to per-gap values agree with the
oracle's independent conversion, and the draws stay in their bounds."""
import numpy as np

from oracle import dpx_oracle as o
from paper_2604_02624_amd import robustness as rb


def test_gap_offsets_match_the_oracle_conversion():
    g = np.random.default_rng(2)
    for K in (1, 2, 5):
        lateral = g.uniform(-1e-7, 1e-7, (K, 2))
        axial = g.uniform(-3e-7, 3e-7, K)
        dz, sx, sy = rb.gap_offsets(lateral, axial)
        s = o.gap_shifts_from_layer_offsets(lateral)
        assert np.array_equal(sx, s[:, 0]) and np.array_equal(sy, s[:, 1])
        assert np.array_equal(dz, o.gap_jitter_from_layer_offsets(axial))
        dz0, _, _ = rb.gap_offsets(lateral)
        assert np.array_equal(dz0, np.zeros(K))


def test_draws_are_bounded_and_seeded():
    a = rb.draw_layer_offsets(np.random.default_rng(5), 4, 40e-9, 200e-9)
    b = rb.draw_layer_offsets(np.random.default_rng(5), 4, 40e-9, 200e-9)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[0].shape == (4, 2) and a[1].shape == (4,)
    assert np.abs(a[0]).max() <= 40e-9 and np.abs(a[1]).max() <= 200e-9
