"""Phase-only layers through the thickness model: the helper's design and heights give the
oracle's direct statement of Eq. 3 at every wavelength; CPU only."""
import numpy as np

from oracle import dpx_oracle as o
from paper_2604_02624_amd import layer_models as lm
from paper_2604_02624_amd import workloads as wk


def test_phase_only_design_reproduces_eq3():
    wl = np.array([0.45e-6, 0.55e-6, 0.65e-6, 0.74e-6])
    d = lm.phase_only_design(wk.make_design(n=8, layers=1, wl=wl, n_mat=wk.nbk7_index(wl), dx=0.3e-6,
                                            z=[10e-6], fov=8, kappa=np.full(4, 0.01)))
    lam_ref = 0.6e-6
    phi = np.random.default_rng(1).uniform(0, 2 * np.pi, (8, 8))
    h = lm.heights_from_phase(phi, lam_ref)
    for w in range(4):
        t = o.transmission(h, wl[w], d["n_mat"][w], 0.0 if d["kappa"] is None else d["kappa"][w], d["n_medium"])
        # the float32 heights carry the phase to about 1e-7 radians
        assert np.max(np.abs(t - o.phase_only_transmission(phi, wl[w], lam_ref))) < 1e-6
    assert np.allclose(lm.phase_from_heights(h, lam_ref), phi, atol=1e-6)
