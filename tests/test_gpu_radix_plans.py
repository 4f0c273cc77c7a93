"""Radix plans of the transforms (the autotuner's plan choices) on the GPU against the FP64
oracle: every plan of the transform lengths that have several (512 and 1024, zero-padded and
periodic), the autotuner's choice and its cache file, and a translated gap, whose column pass
runs on plan 0 whatever the design's plan."""
import os
import sys

import numpy as np
import pytest

from oracle import dpx_oracle as o
from paper_2604_02624_amd import workloads as wk

pytestmark = pytest.mark.gpu

INT_TOL = 1e-5


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2604_02624_amd import dpx
    dpx.load_library()
    return torch


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def design(n, pad, seed, W=5, K=2, fov=48, **kw):
    g = np.random.default_rng(seed)
    wl = np.linspace(450e-9, 750e-9, W)
    d = wk.make_design(n=n, layers=K, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6, z=30e-6, fov=fov, pad=pad)
    d.update(kw)
    h = g.uniform(0, 1.1e-6, (K, n, n)).astype(np.float32)
    tau = g.uniform(0, 1, (W, fov, fov)).astype(np.float32)
    return d, h, tau


def check(torch, d, h, tau, **plan_kw):
    from paper_2604_02624_amd import dpx
    plan = dpx.Plan([d], **plan_kw)
    ht = plan.pack_heights([h])
    I = plan.forward(ht)
    _, g = plan.loss(I, plan.pack_images([tau]))
    dh = plan.backward(ht, None, g)
    torch.cuda.synchronize()
    I_ref = o.forward(d, h, None, "fft")
    _, g_ref, _ = o.loss(I_ref, tau)
    dh_ref = o.grad(d, h, None, g_ref.astype(np.float32), "fft")
    Ig = I.cpu().numpy().reshape(I_ref.shape)
    e_i = max(rel_l2(Ig[k], I_ref[k]) for k in range(I_ref.shape[0]))
    e_g = rel_l2(dh.cpu().numpy().reshape(h.shape), dh_ref)
    radix = plan.radix(0)
    plan.close()
    return e_i, e_g, radix


@pytest.mark.parametrize("n,pad", [(256, 2), (512, 1), (512, 2), (1024, 1)])
def test_every_radix_plan_matches_the_oracle(torch_dev, n, pad):
    from paper_2604_02624_amd import dpx
    M = n * pad
    names = dpx.radix_plan_names(M)
    assert len(names) == 3
    d, h, tau = design(n, pad, M + pad)
    for k, name in enumerate(names):
        e_i, e_g, radix = check(torch_dev, d, h, tau, force_plan=k)
        say(f"transform {M} (N={n}, pad {pad}) plan {k} ({name}): intensities {e_i:.2e}, dL/dh {e_g:.2e}")
        assert radix == (k, k)
        assert e_i <= INT_TOL
        assert e_g <= 1e-4


def test_radix_plans_on_every_column_variant(torch_dev):
    d, h, tau = design(512, 2, 11, W=3)
    for v in range(4):
        e_i, e_g, _ = check(torch_dev, d, h, tau, force_plan=1, force_variant=v)
        say(f"transform 1024 plan 1, column variant {v}: intensities {e_i:.2e}, dL/dh {e_g:.2e}")
        assert e_i <= INT_TOL and e_g <= 1e-4


def test_translated_gap_runs_its_column_pass_on_plan_zero(torch_dev):
    d, h, tau = design(256, 2, 5, W=4)
    K = d["layers"]
    dm = dict(d, shift_x=np.full(K, 0.37e-6), shift_y=np.full(K, -0.21e-6), dz=np.full(K, 0.1e-6))
    e_i, e_g, radix = check(torch_dev, dm, h, tau, force_plan=2)
    say(f"translated gaps with plan 2 (column pass on plan 0): intensities {e_i:.2e}, dL/dh {e_g:.2e}")
    assert radix == (2, 2)
    assert e_i <= INT_TOL and e_g <= 1e-4


def test_autotuner_picks_plans_and_keeps_them_in_its_cache_file(torch_dev, tmp_path, monkeypatch):
    from paper_2604_02624_amd import dpx
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DPX_TUNE_CACHE", str(cache))
    d, h, tau = design(512, 2, 21, W=6)
    e_i, e_g, radix = check(torch_dev, d, h, tau, autotune=True)
    lines = cache.read_text().splitlines()
    say(f"autotuned plans {radix}: {lines}; intensities {e_i:.2e}, dL/dh {e_g:.2e}")
    assert e_i <= INT_TOL and e_g <= 1e-4
    assert len(lines) == 1 and lines[0].startswith("dpx-tune 1024 2 0 6 ")  # 6 wavelengths timed
    rp, cp, cv = (int(x) for x in lines[0].split()[5:8])
    assert (rp, cp) == radix and 0 <= rp < 3 and 0 <= cp < 3
    # a second plan takes the choice from the file and times nothing
    plan = dpx.Plan([d], autotune=True)
    assert plan.radix(0) == radix and plan.variant(0) == cv
    plan.close()
    assert len(cache.read_text().splitlines()) == 1
    # a line for a built length with a plan the library does not have is ignored
    cache.write_text("dpx-tune 1024 2 0 6 7 7 0\n")
    plan = dpx.Plan([d], autotune=True)
    assert all(0 <= x < 3 for x in plan.radix(0))
    plan.close()


def test_radix_plan_rejections(torch_dev):
    from paper_2604_02624_amd import dpx
    d, h, tau = design(256, 2, 1, W=2)
    with pytest.raises(dpx.DpxError) as e:
        dpx.Plan([d], force_plan=3)
    assert e.value.status == dpx.DPX_E_UNSUPPORTED
    with pytest.raises(dpx.DpxError) as e:
        dpx.Plan([d], force_plan=1, transfer_table=2)
    assert e.value.status == dpx.DPX_E_UNSUPPORTED
    with pytest.raises(dpx.DpxError) as e:
        dpx.Plan([dict(d, band_limited=1)], force_plan=1)
    assert e.value.status == dpx.DPX_E_UNSUPPORTED
    d2, _, _ = design(64, 2, 1, W=2, fov=32)
    with pytest.raises(dpx.DpxError):
        dpx.Plan([d2], force_plan=1)          # transform 128 has one plan
