"""Fabrication and model variants on the GPU against the FP64 oracle: the phase bit-depth
quantiser (bit-exact), the band-limited angular spectrum (forward and dL/dh) and training with
quantised heights (straight-through) against an oracle-driven loop."""
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


@pytest.mark.parametrize("bits", [1, 4, 6, 8, 16, 24])
def test_quantiser_bit_exact(torch_dev, bits):
    say(f"phase bit depth {bits}: quantised heights vs the oracle, bit for bit")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    g = np.random.default_rng(bits)
    h_max = 1.1114e-6
    h = g.uniform(-0.05 * h_max, 1.05 * h_max, 100003).astype(np.float32)
    levels = (1 << bits) - 1
    # exact levels and exact midpoints in the float32 decision
    k = g.integers(0, levels + 1, 1000).astype(np.float32)
    h[:1000] = k * np.float32(h_max / levels)
    h[1000:2000] = (k + np.float32(0.5)) / np.float32(levels / h_max)
    ht = torch.as_tensor(h).cuda()
    q = dpx.quantize_heights(ht, h_max, bits).cpu().numpy()
    assert np.array_equal(q, o.quantize_heights(h, h_max, bits))
    dpx.quantize_heights(ht, h_max, bits, out=ht)          # in place
    assert np.array_equal(ht.cpu().numpy(), q)
    with pytest.raises(dpx.DpxError):
        dpx.quantize_heights(ht, h_max, 0)
    with pytest.raises(dpx.DpxError):
        dpx.quantize_heights(ht, -1.0, bits)


def band_case(name):
    if name == "64x64 pad 2 (transform 128), 60 um gaps":
        w = wk.make_workload(2)
        d = dict(w["designs"][0], z=np.array([60e-6, 45e-6]), band_limited=True)
        return d, w["h"][0], w["targets"][0], None
    if name == "256x256 pad 2 (transform 512)":
        wl = np.linspace(450e-9, 750e-9, 4)
        d = wk.make_design(n=256, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=300e-9, z=[150e-6, 120e-6],
                           fov=64, pad=2)
        d["band_limited"] = True
        g = np.random.default_rng(5)
        return d, (g.random((2, 256, 256)) * 1.3e-6).astype(np.float32), g.random((4, 64, 64)).astype(np.float32), None
    if name == "512x512 pad 2 (transform 1024), input gap":
        wl = np.linspace(450e-9, 750e-9, 2)
        d = wk.make_design(n=512, layers=1, wl=wl, n_mat=wk.cauchy_index(wl), dx=300e-9, z=[300e-6],
                           fov=64, pad=2)
        d.update(band_limited=True, z_in=200e-6)
        g = np.random.default_rng(6)
        return d, (g.random((1, 512, 512)) * 1.3e-6).astype(np.float32), g.random((2, 64, 64)).astype(np.float32), None
    d, h, tau, u_in = wk.paper_geometry(n_wl=2, layers=1)
    d["band_limited"] = True
    return d, h, tau, u_in


BAND_CASES = ["64x64 pad 2 (transform 128), 60 um gaps", "256x256 pad 2 (transform 512)",
              "512x512 pad 2 (transform 1024), input gap", "paper geometry 800x800 (transform 1600)"]


@pytest.mark.parametrize("case", BAND_CASES)
def test_band_limited_matches_oracle(torch_dev, case):
    say(f"band-limited angular spectrum: {case}")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    d, h, tau, u_in = band_case(case)
    u = None if u_in is None else torch.view_as_real(torch.as_tensor(u_in)).reshape(-1).cuda()
    outs = []
    for v in (0, 1):
        plan = dpx.Plan([d], force_variant=v)
        hh = plan.pack_heights([h])
        I = plan.forward(hh, u)
        _, g = plan.loss(I, plan.pack_images([tau]))
        dh = plan.backward(hh, u, g)
        outs.append((I.cpu().numpy(), g.cpu().numpy(), dh.cpu().numpy()))
        plan.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    I, g, dh = outs[0]
    I_ref = o.forward(d, h, u_in, "fft")
    errs = [rel_l2(I.reshape(I_ref.shape)[i], I_ref[i]) for i in range(I_ref.shape[0])]
    say(f"per-wavelength rel L2 {max(errs):.2e}")
    assert max(errs) <= INT_TOL
    assert rel_l2(o.forward(dict(d, band_limited=False), h, u_in, "fft"), I_ref) > 100 * INT_TOL
    dh_ref = o.grad(d, h, u_in, g.reshape(tau.shape).astype(np.float64), "fft")
    e = rel_l2(dh.reshape(dh_ref.shape), dh_ref)
    say(f"gradient vs oracle adjoint {e:.2e}")
    assert e <= 1e-4


def test_band_limited_rejections(torch_dev):
    say("band-limited designs: mirrored variants, tables, lateral translations rejected")
    from paper_2604_02624_amd import dpx
    d = dict(wk.make_workload(2)["designs"][0], band_limited=True)
    for kw in (dict(force_variant=2), dict(force_variant=4), dict(transfer_table=2)):
        with pytest.raises(dpx.DpxError):
            dpx.Plan([d], **kw)
    plan = dpx.Plan([d])
    assert plan.variant(0) in (0, 1)
    with pytest.raises(dpx.DpxError):
        plan.set_misalignment(0, shift_x=np.full(2, 1e-7))
    plan.set_misalignment(0, dz=np.full(2, 1e-7))
    plan.close()
    assert dpx.Plan([d, d]).schedule() == 1


def test_quantised_training_matches_oracle_loop(torch_dev):
    say("four Adam steps with 6-bit heights (straight-through) vs the oracle-driven loop")
    from paper_2604_02624_amd import train
    w = wk.make_workload(2)
    d, tau = w["designs"][0], w["targets"][0]
    h_max, bits = 1.24e-6, 6
    theta0 = (0.5 * np.random.default_rng(7).standard_normal((d["layers"], d["n"], d["n"]))).astype(np.float32)
    tr = train.Trainer(d, tau, h_max, theta0=theta0, batch=3, lr=1e-2, bits=bits)
    t_ref = theta0.astype(np.float64)
    m_ref = np.zeros_like(t_ref)
    v_ref = np.zeros_like(t_ref)
    h32 = (np.float32(h_max) / (np.float32(1) + np.exp(-theta0, dtype=np.float32)))
    for step, gi in enumerate([0, 1, 1, 0], start=1):
        L_gpu = float(tr.train_step(gi).cpu())
        hq = o.quantize_heights(h32, h_max, bits)
        sub = wk.subset_wavelengths(d, tr.groups[gi])
        I = o.forward(sub, hq, None, "fft")
        L_ref, g_ref, _ = o.loss(I, tau[tr.groups[gi]])
        dh = o.grad(sub, hq, None, g_ref, "fft")
        t_ref, h_ref, m_ref, v_ref = o.adam_sigmoid_step(t_ref, dh, m_ref, v_ref, step, h_max, lr=1e-2)
        # the oracle quantises its own heights (a height on a level midpoint may round to the
        # other level than on the GPU: one pixel by one level, far inside the loss tolerance)
        h32 = h_ref.astype(np.float32)
        say(f"step {step} batch {gi}: loss gpu {L_gpu:.6e} oracle {L_ref:.6e}")
        assert abs(L_gpu - L_ref) <= 1e-4 * L_ref
    th = tr.theta.cpu().numpy().reshape(t_ref.shape)
    rel = np.linalg.norm(th - t_ref) / np.linalg.norm(t_ref - theta0)
    say(f"theta after 4 steps: relative difference {rel:.2e} of the distance travelled")
    assert rel <= 2e-2
    ps16, ps4 = tr.evaluate(bits=16), tr.evaluate(bits=4)
    assert np.isfinite(ps16).all() and np.isfinite(ps4).all()
    tr.close()


@pytest.mark.parametrize("n,K,W", [(64, 2, 6), (512, 4, 3)])
def test_phase_only_layers_match_the_eq3_cascade(torch_dev, n, K, W):
    """Phase-only layers (Eq. 3) run on the thickness kernels through layer_models; the oracle
    multiplies by the Eq. 3 transmission directly (its own cascade).  Transforms 128 and 1024."""
    say(f"phase-only layers: N={n} (transform {2 * n}), {K} layers, {W} wavelengths vs the Eq. 3 cascade")
    from paper_2604_02624_amd import dpx, layer_models as lm
    g = np.random.default_rng(n + K)
    wl = np.linspace(450e-9, 750e-9, W)
    lam_ref = 600e-9
    F = min(n, 64)
    base = wk.make_design(n=n, layers=K, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6, z=30e-6, fov=F)
    d = lm.phase_only_design(base)
    phi = g.uniform(0.0, 2 * np.pi, (K, n, n))
    h = lm.heights_from_phase(phi, lam_ref)
    phi_h = lm.phase_from_heights(h, lam_ref)          # the phases the float32 heights carry
    I_ref = o.forward_phase_only(d, phi_h, lam_ref, None, "fft")
    plan = dpx.Plan([d])
    ht = plan.pack_heights([h])
    I = plan.forward(ht).cpu().numpy().reshape(I_ref.shape)
    errs = [rel_l2(I[i], I_ref[i]) for i in range(W)]
    say(f"rel L2 {np.max(errs):.2e}")
    assert max(errs) <= INT_TOL
    if n == 64:
        # dL/dphi = dL/dh lambda_ref / (2 pi): the thickness adjoint against the oracle's
        tau = g.uniform(0.0, 1.0, (W, F, F)).astype(np.float32)
        I_t = torch_dev.as_tensor(I.reshape(-1)).cuda()
        _, gi = plan.loss(I_t, plan.pack_images([tau]))
        dh = plan.backward(ht, None, gi).cpu().numpy().reshape(K, n, n)
        _, g_ref, _ = o.loss(I_ref, tau)
        dh_ref = o.grad(d, h, None, g_ref.astype(np.float32), "fft")
        err = rel_l2(dh, dh_ref)
        say(f"gradient rel {err:.2e}")
        assert err <= 1e-4
    plan.close()
