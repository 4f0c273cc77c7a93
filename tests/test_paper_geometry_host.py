"""The paper's Fig. 2 geometry as built by the workload recipe, against the numbers the paper
prints (tests/golden/paper_geometry.json), and the N-BK7 index against the glass maker's
published line indices; CPU only."""
import json
import os

import numpy as np

from paper_2604_02624_amd import workloads as wk

HERE = os.path.dirname(os.path.abspath(__file__))


def test_nbk7_sellmeier_matches_the_published_line_indices():
    """Schott N-BK7 datasheet: n_d = 1.51680 (587.56 nm), n_F = 1.52238 (486.13 nm),
    n_C = 1.51432 (656.27 nm), Abbe number 64.17."""
    n = wk.nbk7_index(np.array([587.5618e-9, 486.1327e-9, 656.2725e-9]))
    assert np.allclose(n, [1.51680, 1.52238, 1.51432], rtol=0, atol=2e-5)
    assert abs((n[0] - 1) / (n[1] - n[2]) - 64.17) < 0.02


def test_paper_geometry_matches_the_printed_design():
    with open(os.path.join(HERE, "golden", "paper_geometry.json")) as f:
        fig2 = json.load(f)["fig2_design"]
    d, h, tau, u_in = wk.paper_geometry()
    lam_m = 0.5 * (fig2["lambda_long_nm"] + fig2["lambda_short_nm"]) * 1e-9
    assert d["n"] == fig2["features_per_side"] and d["layers"] == fig2["layers"]
    assert d["n_wl"] == fig2["wavelengths"]
    assert abs(d["dx"] - fig2["pitch_nm"] * 1e-9) < 1e-15
    # wavelengths from the longest down (lambda_1 is the longest)
    assert np.isclose(d["wl"][0], fig2["lambda_long_nm"] * 1e-9, rtol=1e-14, atol=0)
    assert np.isclose(d["wl"][-1], fig2["lambda_short_nm"] * 1e-9, rtol=1e-14, atol=0)
    assert np.all(np.diff(d["wl"]) < 0)
    # output field of view: 25 x 25 pixels of 8 x 8 samples, about 69.56 lambda_m wide
    assert d["fov"] // d["bin"] == fig2["fov_pixels"] and tau.shape[1:] == (25, 25)
    assert abs(d["fov"] * d["dx"] / lam_m - fig2["fov_side_over_lambda_m"]) < 0.1
    assert abs(d["bin"] * d["dx"] / lam_m - fig2["fov_pixel_over_lambda_m"]) < 0.01
    # input aperture the same size, centred; layer about 278 lambda_m wide
    side = int(np.abs(u_in).sum(axis=0).max())
    assert side == d["fov"] and np.abs(u_in).sum() == side * side
    assert abs(d["n"] * d["dx"] / lam_m - fig2["layer_side_over_lambda_m"]) < 0.5
    # axial span about 1260 lambda_m from the aperture to the output plane
    assert abs((d["z_in"] + d["z"].sum()) / lam_m - 1260.0) < 1e-6
    assert h.shape == (8, 800, 800) and 0 <= h.min() and h.max() <= d["h_max"]
