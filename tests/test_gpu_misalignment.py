"""Misaligned gaps on the GPU against the FP64 oracle: per-gap lateral translation and axial
jitter folded into the transfer function (forward intensities and dL/dh), bit-identical
results across column variants, return to the aligned kernels, captured graphs, and the
rejected configurations."""
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


def misaligned(d, seed, max_px=1.5, dz_frac=0.05):
    """The design with seeded per-gap translations (up to max_px pixels, sub-pixel parts
    included) and axial jitter (up to dz_frac of each gap)."""
    g = np.random.default_rng(seed)
    K = d["layers"]
    out = dict(d)
    out["shift_x"] = g.uniform(-max_px, max_px, K) * d["dx"]
    out["shift_y"] = g.uniform(-max_px, max_px, K) * d["dx"]
    out["dz"] = g.uniform(-dz_frac, dz_frac, K) * np.asarray(d["z"], np.float64)
    return out


def visible(n, layers, n_wl, fov, pad, seed):
    wl = np.linspace(450e-9, 750e-9, n_wl)
    d = wk.make_design(n=n, layers=layers, wl=wl, n_mat=wk.cauchy_index(wl), dx=300e-9,
                       z=np.full(layers, 30e-6), fov=fov, pad=pad)
    g = np.random.default_rng(seed)
    h = (g.random((layers, n, n)) * 1.3e-6).astype(np.float32)
    tau = g.random((n_wl, fov, fov)).astype(np.float32)
    return d, h, tau


def run(torch, d, h, tau, **kw):
    from paper_2604_02624_amd import dpx
    plan = dpx.Plan([d], **kw)
    hh = plan.pack_heights([h])
    I = plan.forward(hh)
    L, g = plan.loss(I, plan.pack_images([tau]))
    dh = plan.backward(hh, None, g)
    torch.cuda.synchronize()
    out = (I.cpu().numpy(), g.cpu().numpy(), dh.cpu().numpy())
    plan.close()
    return out


CASES = {
    "64x64 pad 2 (transform 128)": lambda: (wk.make_workload(2)["designs"][0], wk.make_workload(2)["h"][0],
                                            wk.make_workload(2)["targets"][0]),
    "256x256 pad 2 (transform 512)": lambda: visible(256, 3, 6, 64, 2, 5),
    "192x192 pad 2 (transform 384)": lambda: visible(192, 2, 5, 48, 2, 6),
    "96x96 pad 1 (periodic, transform 96)": lambda: visible(96, 3, 4, 96, 1, 7),
}


@pytest.mark.parametrize("case", list(CASES))
def test_misaligned_forward_and_gradient_match_oracle(torch_dev, case):
    d0, h, tau = CASES[case]()
    d = misaligned(d0, seed=len(case), max_px=3.5 if d0["pad"] == 1 else 1.5)
    say(f"{case}: {d['layers']} gaps, shifts {np.round(d['shift_x'] / d['dx'], 2)} / "
        f"{np.round(d['shift_y'] / d['dx'], 2)} px, dz {np.round(d['dz'] * 1e9, 1)} nm")
    I, g, dh = run(torch_dev, d, h, tau)
    W, T = d["n_wl"], d["fov"] // d["bin"]
    I = I.reshape(W, T, T)
    I_ref = o.forward(d, h, None, "fft")
    errs = np.array([rel_l2(I[i], I_ref[i]) for i in range(W)])
    say(f"per-wavelength rel L2 {errs.max():.2e}")
    assert errs.max() <= INT_TOL
    # the misalignment changes the result (not silently ignored)
    assert rel_l2(o.forward(d0, h, None, "fft"), I_ref) > 100 * INT_TOL
    _, g_ref, _ = o.loss(I_ref, tau)
    dh_ref = o.grad(d, h, None, g.reshape(g_ref.shape).astype(np.float64), "fft")
    e = rel_l2(dh.reshape(dh_ref.shape), dh_ref)
    say(f"gradient vs oracle adjoint {e:.2e}")
    assert e <= 1e-4


def test_misaligned_variants_are_bit_identical(torch_dev):
    say("translated gaps: column variants 0-3 give identical bits")
    w = wk.make_workload(2)
    d = misaligned(w["designs"][0], seed=3)
    outs = [run(torch_dev, d, w["h"][0], w["targets"][0], force_variant=v) for v in range(4)]
    for v in range(1, 4):
        for a, b in zip(outs[0], outs[v]):
            assert np.array_equal(a, b), f"variant {v}"


def test_misalignment_set_and_cleared(torch_dev):
    say("set_misalignment on a live plan, then back to zero, with and without graphs")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    w = wk.make_workload(2)
    d0, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    d = misaligned(d0, seed=9)
    ref_mis = run(torch, d, h, tau)
    ref_al = run(torch, d0, h, tau)
    for graph in (False, True):
        plan = dpx.Plan([d0], use_graph=graph)
        hh = plan.pack_heights([h])
        t = plan.pack_images([tau])

        def go():
            I = plan.forward(hh)
            _, g = plan.loss(I, t)
            dh = plan.backward(hh, None, g)
            return I.cpu().numpy(), g.cpu().numpy(), dh.cpu().numpy()

        for a, b in zip(go(), ref_al):
            assert np.array_equal(a, b)
        plan.set_misalignment(0, d["dz"], d["shift_x"], d["shift_y"])
        for a, b in zip(go(), ref_mis):
            assert np.array_equal(a, b)
        plan.set_misalignment(0)
        for a, b in zip(go(), ref_al):
            assert np.array_equal(a, b)
        plan.close()


def test_misalignment_rejections(torch_dev):
    say("rejected misalignments: counts, negative gaps, grouped / table plans, matrix-core variant")
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(2)
    d = w["designs"][0]
    K = d["layers"]
    plan = dpx.Plan([d])
    with pytest.raises(dpx.DpxError):   # through the C ABI: the binding checks shapes itself
        dpx._check(plan.lib, plan.lib.dpx_plan_set_misalignment(plan._h, 0, None, None, None, K + 1))
    with pytest.raises(dpx.DpxError):
        plan.set_misalignment(0, dz=-2.0 * np.asarray(d["z"]))
    with pytest.raises(dpx.DpxError):
        plan.set_misalignment(1, dz=np.zeros(K))
    plan.close()
    grouped = dpx.Plan([d, d], schedule=2)
    with pytest.raises(dpx.DpxError):
        grouped.set_misalignment(0, shift_x=np.full(K, 1e-7))
    grouped.set_misalignment(0)   # zeros are accepted everywhere
    grouped.close()
    tables = dpx.Plan([d], transfer_table=2)
    with pytest.raises(dpx.DpxError):
        tables.set_misalignment(0, dz=np.full(K, 1e-8))
    tables.close()
    gemm = dpx.Plan([d], force_variant=4)
    with pytest.raises(dpx.DpxError):
        gemm.set_misalignment(0, shift_y=np.full(K, 1e-7))
    gemm.set_misalignment(0, dz=np.full(K, 1e-7))   # axial jitter alone is fine there
    gemm.close()


def test_axial_jitter_on_matrix_core_variant_matches_oracle(torch_dev):
    say("axial jitter with the matrix-core column variant vs the oracle")
    w = wk.make_workload(2)
    d = dict(w["designs"][0], dz=np.array([0.4e-6, -0.7e-6]))
    I, _, _ = run(torch_dev, d, w["h"][0], w["targets"][0], force_variant=4)
    I_ref = o.forward(d, w["h"][0], None, "fft")
    assert rel_l2(I.reshape(I_ref.shape), I_ref) <= INT_TOL


def test_translated_gaps_at_transform_1600(torch_dev):
    say("translated and lengthened gaps at transform 1600 (800x800, input aperture and gap): "
        "variants 0 and 1 vs the oracle")
    d0, h, tau, u_in = wk.paper_geometry(n_wl=2, layers=2)
    d = misaligned(d0, seed=16)
    from paper_2604_02624_amd import dpx
    outs = []
    for v in (0, 1):
        plan = dpx.Plan([d], force_variant=v)
        hh = plan.pack_heights([h])
        u = torch_dev.view_as_real(torch_dev.as_tensor(u_in)).reshape(-1).cuda()
        I = plan.forward(hh, u)
        _, g = plan.loss(I, plan.pack_images([tau]))
        dh = plan.backward(hh, u, g)
        torch_dev.cuda.synchronize()
        outs.append((I.cpu().numpy(), g.cpu().numpy(), dh.cpu().numpy()))
        plan.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    I, g, dh = outs[0]
    I_ref = o.forward(d, h, u_in, "fft")
    errs = [rel_l2(I.reshape(I_ref.shape)[i], I_ref[i]) for i in range(2)]
    say(f"per-wavelength rel L2 {max(errs):.2e}")
    assert max(errs) <= INT_TOL
    assert rel_l2(o.forward(d0, h, u_in, "fft"), I_ref) > 100 * INT_TOL
    dh_ref = o.grad(d, h, u_in, g.reshape(tau.shape).astype(np.float64), "fft")
    e = rel_l2(dh.reshape(dh_ref.shape), dh_ref)
    say(f"gradient vs oracle adjoint {e:.2e}")
    assert e <= 1e-4


def test_misaligned_large_workload_sampled(torch_dev):
    say("large workload (4 layers 512x512, transform 1024, 4096 wavelengths) misaligned as in the "
        "benchmark: sampled wavelengths vs the oracle")
    from paper_2604_02624_amd import dpx, robustness
    torch = torch_dev
    w = wk.make_workload(4)
    d0, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    lateral, axial = robustness.draw_layer_offsets(np.random.default_rng(1), d0["layers"], 40e-9, 200e-9)
    s = o.gap_shifts_from_layer_offsets(lateral)
    d = dict(d0, shift_x=s[:, 0], shift_y=s[:, 1], dz=o.gap_jitter_from_layer_offsets(axial))
    plan = dpx.Plan([d])
    hh = plan.pack_heights([h])
    I = plan.forward(hh)
    sample = [0, 2047, 4095]
    seed = np.zeros_like(tau)
    seed[sample] = np.random.default_rng(2).standard_normal((3,) + tau.shape[1:]).astype(np.float32) * 1e-3
    dh = plan.backward(hh, None, plan.pack_images([seed]))
    torch.cuda.synchronize()
    I = I.cpu().numpy().reshape(tau.shape)
    dh = dh.cpu().numpy().reshape(h.shape)
    plan.close()
    I_ref = o.forward(d, h, None, "fft", wavelengths=sample)
    errs = [rel_l2(I[w_], I_ref[i]) for i, w_ in enumerate(sample)]
    say(f"sampled wavelengths: rel L2 {max(errs):.2e}")
    assert max(errs) <= INT_TOL
    assert rel_l2(o.forward(d0, h, None, "fft", wavelengths=sample), I_ref) > 10 * INT_TOL
    dh_ref = o.grad(d, h, None, seed[sample].astype(np.float64), "fft", wavelengths=sample)
    e = rel_l2(dh, dh_ref)
    say(f"gradient of the sampled wavelengths vs oracle adjoint {e:.2e}")
    assert e <= 1e-4
