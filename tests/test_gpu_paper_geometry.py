"""The paper's own geometry on the GPU against the FP64 oracle: 1600-point transforms (radix 5,
transforms spanning wavefronts), the input aperture and input gap before the first layer, and
the full Fig. 2 design (8 layers of 800 x 800, 4096 wavelengths) in the benchmark's launch
configuration with sampled wavelengths."""
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


def field(torch, u):
    return None if u is None else torch.view_as_real(torch.as_tensor(np.asarray(u, np.complex64))).reshape(-1).cuda()


def run(torch, d, h, tau, u_in=None, dl_di=None, **kw):
    from paper_2604_02624_amd import dpx
    plan = dpx.Plan([d], **kw)
    hh = plan.pack_heights([h])
    u = field(torch, u_in)
    I = plan.forward(hh, u)
    L, g = plan.loss(I, plan.pack_images([tau]))
    if dl_di is not None:
        g = plan.pack_images([dl_di])
    dh = plan.backward(hh, u, g)
    torch.cuda.synchronize()
    out = (I.cpu().numpy(), g.cpu().numpy(), dh.cpu().numpy())
    plan.close()
    return out


def test_transform_1600_with_aperture_and_input_gap(torch_dev):
    say("800x800 (transform 1600), 2 layers, 3 wavelengths, aperture + input gap, 8x8 bins")
    d, h, tau, u_in = wk.paper_geometry(n_wl=3, layers=2)
    I, g, dh = run(torch_dev, d, h, tau, u_in)
    I = I.reshape(tau.shape)
    I_ref = o.forward(d, h, u_in, "fft")
    errs = [rel_l2(I[i], I_ref[i]) for i in range(3)]
    say(f"per-wavelength rel L2 {max(errs):.2e}")
    assert max(errs) <= INT_TOL
    dh_ref = o.grad(d, h, u_in, g.reshape(tau.shape).astype(np.float64), "fft")
    e = rel_l2(dh.reshape(dh_ref.shape), dh_ref)
    say(f"gradient vs oracle adjoint {e:.2e}")
    assert e <= 1e-4


def test_transform_1600_variants_and_periodic_window(torch_dev):
    say("transform 1600: column variants 0 and 1 identical; periodic window 1600x1600")
    d, h, tau, u_in = wk.paper_geometry(n_wl=2, layers=1)
    outs = [run(torch_dev, d, h, tau, u_in, force_variant=v) for v in (0, 1)]
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    # pad 1: N = M = 1600, no input gap, plane-wave input
    wl = np.array([0.45e-6, 0.7e-6])
    dp = wk.make_design(n=1600, layers=1, wl=wl, n_mat=wk.nbk7_index(wl), dx=0.2e-6, z=[20e-6],
                        fov=400, bin_=8, pad=1)
    hp = (np.random.default_rng(3).random((1, 1600, 1600)) * 1.1e-6).astype(np.float32)
    taup = np.random.default_rng(4).random((2, 50, 50)).astype(np.float32)
    I, g, dh = run(torch_dev, dp, hp, taup)
    I_ref = o.forward(dp, hp, None, "fft")
    assert max(rel_l2(I.reshape(I_ref.shape)[i], I_ref[i]) for i in range(2)) <= INT_TOL
    dh_ref = o.grad(dp, hp, None, g.reshape(taup.shape).astype(np.float64), "fft")
    assert rel_l2(dh.reshape(dh_ref.shape), dh_ref) <= 1e-4


def test_input_gap_on_the_other_lengths(torch_dev):
    say("input gap + aperture at transform 128: store, recompute and table plans vs the oracle")
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(2)
    d = dict(w["designs"][0], z_in=17e-6)
    h, tau = w["h"][0], w["targets"][0]
    ap = np.zeros((64, 64), np.complex64)
    ap[16:48, 20:44] = 1.0
    ref = run(torch_dev, d, h, tau, ap)
    I_ref = o.forward(d, h, ap, "fft")
    assert max(rel_l2(ref[0].reshape(I_ref.shape)[i], I_ref[i]) for i in range(6)) <= INT_TOL
    dh_ref = o.grad(d, h, ap, ref[1].reshape(tau.shape).astype(np.float64), "fft")
    assert rel_l2(ref[2].reshape(dh_ref.shape), dh_ref) <= 1e-4
    rec = run(torch_dev, d, h, tau, ap, checkpoint_mode=1, wl_chunk=2)
    # same forward bits; dL/dh summed over other wavelength blocks (order of the partial sums)
    assert np.array_equal(ref[0], rec[0]) and np.array_equal(ref[1], rec[1])
    assert rel_l2(rec[2], ref[2]) <= 1e-6
    tab = run(torch_dev, d, h, tau, ap, transfer_table=2)
    for a, b in zip(ref, tab):
        assert np.array_equal(a, b)
    with pytest.raises(dpx.DpxError):
        dpx.Plan([d, d], schedule=2)


def test_paper_geometry_full_scale_sampled(torch_dev):
    say("Fig. 2 design at full size: 8 layers 800x800, 4096 wavelengths, sampled wavelengths")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    w = wk.make_workload(6)
    d, h, tau, u_in = w["designs"][0], w["h"][0], w["targets"][0], w["u_in"][0]
    plan = dpx.Plan([d])
    say(f"plan holds {plan.layouts[0]['workspace_bytes'] / 1e9:.1f} GB")
    hh = plan.pack_heights([h])
    u = field(torch, u_in)
    I = plan.forward(hh, u)
    # the adjoint seeded on the sampled wavelengths only, so that dL/dh is their sum
    sample = [0, 1365, 2730, 4095]
    seed = np.zeros_like(tau)
    g = np.random.default_rng(5)
    seed[sample] = g.standard_normal((len(sample),) + tau.shape[1:]).astype(np.float32) * 1e-3
    dh = plan.backward(hh, u, plan.pack_images([seed]))
    torch.cuda.synchronize()
    I = I.cpu().numpy().reshape(tau.shape)
    dh = dh.cpu().numpy().reshape(h.shape)
    plan.close()
    I_ref = o.forward(d, h, u_in, "fft", wavelengths=sample)
    errs = [rel_l2(I[w_], I_ref[i]) for i, w_ in enumerate(sample)]
    say(f"sampled wavelengths {sample}: rel L2 {max(errs):.2e}")
    assert max(errs) <= INT_TOL
    dh_ref = o.grad(d, h, u_in, seed[sample].astype(np.float64), "fft", wavelengths=sample)
    e = rel_l2(dh, dh_ref)
    say(f"gradient of the sampled wavelengths vs oracle adjoint {e:.2e}")
    assert e <= 1e-4


def test_transform_1600_schedules_and_modes(torch_dev):
    say("transform 1600: grouped schedule of two designs, recompute mode, tables, two lanes vs the base plan")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    d, h, tau, _ = wk.paper_geometry(n_wl=4, layers=2)
    d = dict(d, z_in=0.0)                       # the grouped schedule runs designs without an input gap
    d2, h2, tau2, _ = wk.paper_geometry(n_wl=3, layers=1, cfg=7)
    d2 = dict(d2, z_in=0.0)

    def go(designs, hs, taus, **kw):
        plan = dpx.Plan(designs, **kw)
        hh = plan.pack_heights(hs)
        I = plan.forward(hh)
        _, g = plan.loss(I, plan.pack_images(taus))
        dh = plan.backward(hh, None, g)
        torch.cuda.synchronize()
        out = (I.cpu().numpy(), dh.cpu().numpy(), plan.schedule())
        plan.close()
        return out

    base = go([d], [h], [tau])
    I_ref = o.forward(d, h, None, "fft")
    assert max(rel_l2(base[0].reshape(I_ref.shape)[i], I_ref[i]) for i in range(4)) <= INT_TOL
    # two designs: one grouped launch per pass and transform length
    both = go([d, d2], [h, h2], [tau, tau2])
    assert both[2] == 2
    n1 = base[0].size
    assert np.array_equal(both[0][:n1], base[0])
    assert rel_l2(both[1][:h.size], base[1]) <= 1e-6
    I2_ref = o.forward(d2, h2, None, "fft")
    assert max(rel_l2(both[0][n1:].reshape(I2_ref.shape)[i], I2_ref[i]) for i in range(3)) <= INT_TOL
    for kw in (dict(checkpoint_mode=1, wl_chunk=2), dict(transfer_table=2), dict(streams=2, wl_chunk=2)):
        r = go([d], [h], [tau], **kw)
        say(f"  {kw}: same intensities, gradient within {rel_l2(r[1], base[1]):.1e}")
        assert np.array_equal(r[0], base[0])
        assert rel_l2(r[1], base[1]) <= 1e-6
