"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Intensities: per-wavelength relative L2 <= 1e-5 against the FP64 oracle.  Gradients: relative
L2 <= 1e-3 against central finite differences of the FP64 oracle (64 pixels per layer plus
8 random directions, step 1e-3 lambda_m) and against the oracle's own adjoint.  At the large
sizes the GPU runs the whole workload in the launch configuration the benchmark uses and the
oracle recomputes sampled wavelengths one by one.
"""
import sys

import numpy as np
import pytest

from oracle import dpx_oracle as o
from tests import oracle_threads as ot
from paper_2604_02624_amd import workloads as wk

pytestmark = pytest.mark.gpu

INT_TOL = 1e-5
GRAD_TOL = 1e-3


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


def per_wl_rel(a, b):
    return np.array([rel_l2(a[i], b[i]) for i in range(a.shape[0])])


def run_gpu(torch, designs, hs, taus, u_ins=None, backward=True, dl_di=None, **plan_kw):
    from paper_2604_02624_amd import dpx
    plan = dpx.Plan(designs, **plan_kw)
    h = plan.pack_heights(hs)
    tau = plan.pack_images(taus)
    u = None
    if u_ins is not None:
        u = torch.cat([torch.view_as_real(torch.as_tensor(np.asarray(x, np.complex64))).reshape(-1)
                       for x in u_ins]).cuda()
    I = plan.forward(h, u)
    L, g = plan.loss(I, tau)
    out = dict(plan=plan, h=h, u=u, I=I, L=L, g=g)
    if backward:
        gin = g if dl_di is None else plan.pack_images(dl_di)
        out["dh"] = plan.backward(h, u, gin)
    torch.cuda.synchronize()
    return out


# ------------------------------------------------------------------------------------------
# small workloads: full comparison
# ------------------------------------------------------------------------------------------

def test_forward_small_experiment_geometry(torch_dev):
    say("forward, 2 layers 64x64 pad 128, 6 wavelengths")
    w = wk.make_workload(1)
    d, h = w["designs"][0], w["h"][0]
    r = run_gpu(torch_dev, [d], [h], w["targets"], backward=False)
    I_gpu = r["I"].cpu().numpy().reshape(6, 32, 32)
    I_ref = o.forward(d, h, None, "naive")
    errs = per_wl_rel(I_gpu, I_ref)
    say(f"per-wavelength rel L2 {errs}")
    assert errs.max() <= INT_TOL


def test_forward_adjoint_small_vs_finite_differences(torch_dev):
    say("forward + adjoint, 2 layers 64x64, 6 wavelengths, FD check")
    w = wk.make_workload(2)
    d, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    r = run_gpu(torch_dev, [d], [h], [tau])
    I_gpu = r["I"].cpu().numpy().reshape(6, 32, 32)
    I_ref = o.forward(d, h, None, "fft")
    assert per_wl_rel(I_gpu, I_ref).max() <= INT_TOL
    L_ref, g_ref, _ = o.loss(I_ref, tau)
    assert abs(float(r["L"].cpu()[0]) - L_ref) <= 1e-4 * abs(L_ref)
    assert rel_l2(r["g"].cpu().numpy().reshape(g_ref.shape), g_ref) <= 1e-4
    dh_gpu = r["dh"].cpu().numpy().reshape(h.shape)
    dh_ref = o.grad(d, h, None, g_ref, "fft")
    say(f"gradient vs oracle adjoint {rel_l2(dh_gpu, dh_ref):.3e}")
    assert rel_l2(dh_gpu, dh_ref) <= 1e-4
    # central finite differences of the FP64 oracle: 64 pixels per layer + 8 directions
    lam_m = 620e-9
    delta = 1e-3 * lam_m
    g = wk.rng(2, wk.STREAM_FD_PIXELS)
    pix = [(l, int(g.integers(64)), int(g.integers(64))) for l in range(2) for _ in range(64)]
    fd = o.fd_pixels(d, h, None, tau, pix, delta, "fft")
    an = np.array([dh_gpu[p] for p in pix])
    say(f"gradient vs FD (128 pixels) {rel_l2(an, fd):.3e}")
    assert rel_l2(an, fd) <= GRAD_TOL
    gd = wk.rng(2, wk.STREAM_FD_DIRS)
    for _ in range(8):
        v = gd.standard_normal(h.shape)
        fdv = o.fd_direction(d, h, None, tau, v, delta / np.sqrt(v.size), "fft")
        assert abs((dh_gpu * v).sum() - fdv) <= GRAD_TOL * abs(fdv)


def test_input_field_absorption_and_binning(torch_dev):
    say("u_in + kappa + bin 2, 3 layers 32x32 pad 64, 5 wavelengths")
    g = np.random.default_rng(21)
    wl = np.linspace(480e-9, 700e-9, 5)
    d = wk.make_design(n=32, layers=3, wl=wl, n_mat=wk.cauchy_index(wl), dx=240e-9,
                       z=[5e-6, 7e-6, 9e-6], fov=16, bin_=2, pad=2, kappa=np.linspace(0, 0.03, 5))
    h = (g.random((3, 32, 32)) * 1.2e-6).astype(np.float32)
    u = (g.standard_normal((32, 32)) + 1j * g.standard_normal((32, 32))).astype(np.complex64)
    tau = g.random((5, 8, 8)).astype(np.float32)
    r = run_gpu(torch_dev, [d], [h], [tau], u_ins=[u])
    I_ref = o.forward(d, h, u, "naive")
    assert per_wl_rel(r["I"].cpu().numpy().reshape(5, 8, 8), I_ref).max() <= INT_TOL
    _, g_ref, _ = o.loss(I_ref, tau)
    r2 = run_gpu(torch_dev, [d], [h], [tau], u_ins=[u], dl_di=[g_ref.astype(np.float32)])
    dh_ref = o.grad(d, h, u, g_ref.astype(np.float32), "naive")
    err = rel_l2(r2["dh"].cpu().numpy().reshape(h.shape), dh_ref)
    say(f"gradient rel {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("n", [64, 96, 128, 192, 256, 512, 1024])
def test_periodic_window_every_transform_length(torch_dev, n):
    say(f"pad 1 (periodic), N = M = {n}")
    g = np.random.default_rng(n)
    wl = np.array([450e-9, 600e-9, 750e-9])
    d = wk.make_design(n=n, layers=2, wl=wl, n_mat=1.5, dx=300e-9, z=[6e-6, 4e-6], fov=n // 2,
                       pad=1)
    h = (g.random((2, n, n)) * 1.2e-6).astype(np.float32)
    tau = g.random((3, n // 2, n // 2)).astype(np.float32)
    r = run_gpu(torch_dev, [d], [h], [tau])
    I_ref = o.forward(d, h, None, "fft")
    assert per_wl_rel(r["I"].cpu().numpy().reshape(I_ref.shape), I_ref).max() <= INT_TOL
    L_ref, g_ref, _ = o.loss(I_ref, tau)
    dh_ref = o.grad(d, h, None, g_ref, "fft")
    assert rel_l2(r["dh"].cpu().numpy().reshape(h.shape), dh_ref) <= 1e-4


@pytest.mark.parametrize("n", [32, 48, 64, 96, 128, 192, 256, 512])
def test_zero_padded_every_transform_length(torch_dev, n):
    say(f"pad 2, N = {n}, M = {2 * n}")
    g = np.random.default_rng(100 + n)
    wl = np.array([450e-9, 610e-9, 750e-9])
    d = wk.make_design(n=n, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=300e-9,
                       z=[30e-6, 30e-6], fov=n // 4 * 2, pad=2)
    h = (g.random((2, n, n)) * 1.17e-6).astype(np.float32)
    F = n // 4 * 2
    tau = g.random((3, F, F)).astype(np.float32)
    r = run_gpu(torch_dev, [d], [h], [tau])
    I_ref = o.forward(d, h, None, "fft")
    errs = per_wl_rel(r["I"].cpu().numpy().reshape(I_ref.shape), I_ref)
    say(f"rel L2 {errs}")
    assert errs.max() <= INT_TOL
    _, g_ref, _ = o.loss(I_ref, tau)
    dh_ref = o.grad(d, h, None, g_ref, "fft")
    assert rel_l2(r["dh"].cpu().numpy().reshape(h.shape), dh_ref) <= 1e-4


@pytest.mark.parametrize("n", [64, 256])
def test_mostly_evanescent_spectrum(torch_dev, n):
    """A fine pitch against long wavelengths: the propagating disc covers a few percent of the
    padded plane, so whole wavefronts of consecutive rows lie outside it (the evaluated transfer
    function skips them).  Every column variant against the FP64 oracle and against each other."""
    say(f"mostly evanescent spectrum, pad 2, N = {n}")
    from paper_2604_02624_amd import dpx
    g = np.random.default_rng(700 + n)
    wl = np.array([700e-9, 800e-9, 900e-9])
    d = wk.make_design(n=n, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=120e-9,
                       z=[6e-6, 6e-6], fov=n // 2, pad=2)
    # disc radius in frequency indices, M dx / lambda, against the half-width M / 2
    assert (2 * n * 120e-9 / wl).max() < 0.35 * n
    h = (g.random((2, n, n)) * 1.5e-6).astype(np.float32)
    tau = g.random((3, n // 2, n // 2)).astype(np.float32)
    I_ref = o.forward(d, h, None, "fft")
    _, g_ref, _ = o.loss(I_ref, tau)
    dh_ref = o.grad(d, h, None, g_ref, "fft")
    outs = []
    for v in range(4):
        r = run_gpu(torch_dev, [d], [h], [tau], force_variant=v)
        errs = per_wl_rel(r["I"].cpu().numpy().reshape(I_ref.shape), I_ref)
        eg = rel_l2(r["dh"].cpu().numpy().reshape(h.shape), dh_ref)
        say(f"{dpx.variant_names()[v]}: intensity rel L2 {errs.max():.2e}, dL/dh vs oracle adjoint {eg:.2e}")
        assert errs.max() <= INT_TOL
        assert eg <= 1e-4
        outs.append(r)
    for r in outs[1:]:
        assert torch_dev.equal(r["I"], outs[0]["I"])
        assert torch_dev.equal(r["dh"], outs[0]["dh"])


def test_degenerate_zero_field_and_zero_target(torch_dev):
    say("zero input field (zero intensity) and an all-zero target: finite loss, zero gradient")
    g = np.random.default_rng(12)
    wl = np.array([520e-9, 610e-9, 700e-9])
    for small in (0, 1):
        d = wk.make_design(n=64, layers=2, wl=wl, n_mat=1.5, dx=300e-9, z=[9e-6, 9e-6], fov=32, pad=2)
        h = (g.random((2, 64, 64)) * 1e-6).astype(np.float32)
        tau = g.random((3, 32, 32)).astype(np.float32)
        tau[1] = 0.0
        u0 = np.zeros((64, 64), np.complex64)
        r = run_gpu(torch_dev, [d], [h], [tau], u_ins=[u0], small_path=small)
        I = r["I"].cpu().numpy()
        assert not I.any()
        L_ref, g_ref, _ = o.loss(np.zeros((3, 32, 32)), tau)
        assert np.isfinite(r["L"].cpu().numpy()).all()
        assert abs(float(r["L"].cpu()[0]) - L_ref) <= 1e-6 * max(L_ref, 1e-30)
        assert not r["g"].cpu().numpy().any() and not g_ref.any()
        assert not r["dh"].cpu().numpy().any()
        # all-zero target with a live field: the target term drops out (sum rule)
        r2 = run_gpu(torch_dev, [d], [h], [tau])
        I2 = r2["I"].cpu().numpy().reshape(3, 32, 32)
        L2_ref, g2_ref, _ = o.loss(I2.astype(np.float64), tau)
        assert abs(float(r2["L"].cpu()[0]) - L2_ref) <= 1e-5 * L2_ref
        assert rel_l2(r2["g"].cpu().numpy().reshape(3, 32, 32), g2_ref) <= 1e-5


def test_single_layer_single_wavelength_edge(torch_dev):
    say("K = 1, W = 1, F = N")
    g = np.random.default_rng(5)
    d = wk.make_design(n=64, layers=1, wl=np.array([532e-9]), n_mat=1.46, dx=266e-9, z=20e-6,
                       fov=64, pad=2)
    h = (g.random((1, 64, 64)) * 1e-6).astype(np.float32)
    tau = g.random((1, 64, 64)).astype(np.float32)
    r = run_gpu(torch_dev, [d], [h], [tau])
    I_ref = o.forward(d, h, None, "naive")
    assert rel_l2(r["I"].cpu().numpy().reshape(I_ref.shape), I_ref) <= INT_TOL
    _, g_ref, _ = o.loss(I_ref, tau)
    assert rel_l2(r["dh"].cpu().numpy().reshape(h.shape), o.grad(d, h, None, g_ref, "naive")) <= 1e-4


# ------------------------------------------------------------------------------------------
# batched workloads
# ------------------------------------------------------------------------------------------

def test_batched_five_layers_256(torch_dev):
    say("batched: 5 layers 256x256 pad 512, 256 wavelengths (oracle on 6 sampled wavelengths)")
    w = wk.make_workload(3)
    d, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    sample = [0, 37, 101, 128, 200, 255]
    I_ref = o.forward(d, h, None, "fft", wavelengths=sample)
    _, g_s, _ = o.loss(I_ref, tau[sample])
    dl_di = np.zeros((256, 64, 64), np.float32)
    dl_di[sample] = g_s
    r = run_gpu(torch_dev, [d], [h], [tau], dl_di=[dl_di])
    I_gpu = r["I"].cpu().numpy().reshape(256, 64, 64)
    errs = per_wl_rel(I_gpu[sample], I_ref)
    say(f"rel L2 {errs}")
    assert errs.max() <= INT_TOL
    dh_ref = o.grad(d, h, None, g_s.astype(np.float32), "fft", wavelengths=sample)
    err = rel_l2(r["dh"].cpu().numpy().reshape(h.shape), dh_ref)
    say(f"gradient rel {err:.3e}")
    assert err <= 1e-4


def large_sample(W=4096, wpb_row=16, wpb_col=2):
    """Eight seeded wavelengths of the large workload (stream 3): the first and last wavelength
    of one row-pass block of 16, both wavelengths of one column-pass block of 2, the two ends of
    the band and two more drawn at random, in index order."""
    g = np.random.default_rng(np.random.SeedSequence([260402624, 4, 3]))
    b = int(g.integers(1, W // wpb_row - 1))
    c = int(g.integers(0, W // wpb_col))
    picks = {0, W - 1, b * wpb_row, b * wpb_row + wpb_row - 1, wpb_col * c, wpb_col * c + 1}
    while len(picks) < 8:
        picks.add(int(g.integers(0, W)))
    return sorted(picks), g


@pytest.fixture(scope="module")
def large_run(torch_dev):
    """The large workload on the GPU in the benchmark's launch configuration (all 4096
    wavelengths, one plan, store mode), with the adjoint seeded by the oracle's dL/dI of the loss
    over the sampled wavelengths, so dL/dh is the gradient of that loss alone."""
    say("large: 4 layers 512x512 pad 1024, 4096 wavelengths (oracle on 8 seeded wavelengths)")
    w = wk.make_workload(4)
    d, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    sample, g = large_sample()
    say(f"sampled wavelengths {sample}")
    I_ref = ot.forward(d, h, None, sample)
    _, g_s, _ = o.loss(I_ref, tau[sample])
    dl_di = np.zeros((4096, 64, 64), np.float32)
    dl_di[sample] = g_s
    r = run_gpu(torch_dev, [d], [h], [tau], dl_di=[dl_di])
    out = dict(d=d, h=h, tau=tau, sample=sample, rng=g, I_ref=I_ref, g_s=g_s,
               I=r["I"].cpu().numpy().reshape(4096, 64, 64),
               dh=r["dh"].cpu().numpy().reshape(h.shape).astype(np.float64))
    r["plan"].close()
    del r
    torch_dev.cuda.empty_cache()
    return out


def test_large_full_size_sampled(large_run):
    r = large_run
    sample = r["sample"]
    errs = per_wl_rel(r["I"][sample], r["I_ref"])
    say(f"rel L2 {errs}")
    assert errs.max() <= INT_TOL
    assert np.isfinite(r["I"]).all()
    dh_ref = ot.grad(r["d"], r["h"], None, r["g_s"].astype(np.float32), sample)
    err = rel_l2(r["dh"], dh_ref)
    say(f"gradient rel {err:.3e} (oracle adjoint)")
    assert err <= 1e-4
    # property at full size: each layer's gradient sums to ~0 (global-phase invariance)
    dh = r["dh"]
    assert (np.abs(dh.sum(axis=(1, 2))) <= 1e-3 * np.abs(dh).sum(axis=(1, 2))).all()


def test_large_gradient_vs_finite_differences_directions(large_run):
    """Central differences of the FP64 oracle's loss over the sampled wavelengths along 8 seeded
    random directions (stream 4), step 1e-3 lambda_m: |<g, v> - FD_v| / |FD_v| <= 1e-3."""
    r = large_run
    d, h, sample = r["d"], r["h"], r["sample"]
    tau_s = r["tau"][sample]
    lam_m = 600e-9
    delta = 1e-3 * lam_m
    gv = np.random.default_rng(np.random.SeedSequence([260402624, 4, 4]))
    h64 = h.astype(np.float64)
    errs = []
    for k in range(8):
        v = gv.standard_normal(h.shape)
        fd = (ot.loss(d, h64 + delta * v, None, tau_s, sample)
              - ot.loss(d, h64 - delta * v, None, tau_s, sample)) / (2 * delta)
        errs.append(abs(float((r["dh"] * v).sum()) - fd) / abs(fd))
        say(f"direction {k}: rel {errs[-1]:.2e}")
    assert max(errs) <= GRAD_TOL


def test_large_gradient_vs_finite_differences_pixels(large_run):
    """Central differences of the FP64 oracle's loss over the sampled wavelengths at 64 seeded
    pixels of the last layer (stream 3), step 1e-3 lambda_m: relative L2 over the pixels
    <= 1e-3.  A height of the last layer only changes the last propagation, so each loss is
    evaluated from the field arriving at that layer (the oracle's own forward of the first
    layers, kept once) through the oracle's one-layer forward: the same operations as a full
    forward, without recomputing the unchanged layers."""
    r = large_run
    d, h, sample, g = r["d"], r["h"], r["sample"], r["rng"]
    K, N = d["layers"], d["n"]
    tau_s = r["tau"][sample]
    lam_m = 600e-9
    delta = 1e-3 * lam_m
    h64 = h.astype(np.float64)
    # the field arriving at the last layer, per sampled wavelength
    def arriving(w):
        _, vs, _ = o.forward(d, h, None, "fft", keep=True, wavelengths=[w])
        t = o.transmission(h64[K - 1], float(d["wl"][w]), float(d["n_mat"][w]), 0.0, d["n_medium"])
        return vs[0, K - 1] / t
    u_arr = dict(zip(sample, ot._map(arriving, sample)))
    last = dict(d, layers=1, z=np.asarray(d["z"])[K - 1:K])

    def loss_last(hl):
        I = np.concatenate([o.forward(last, hl[None], u_arr[w], "fft", wavelengths=[w]) for w in sample])
        return o.loss(I, tau_s)[0]

    # the suffix evaluation reproduces the full forward's loss
    full = o.loss(r["I_ref"], tau_s)[0]
    assert abs(loss_last(h64[K - 1]) - full) <= 1e-12 * abs(full)
    pix = [(int(g.integers(0, N)), int(g.integers(0, N))) for _ in range(64)]

    def fd(p):
        y, x = p
        hp = h64[K - 1].copy()
        hm = h64[K - 1].copy()
        hp[y, x] += delta
        hm[y, x] -= delta
        return (loss_last(hp) - loss_last(hm)) / (2 * delta)

    fds = np.array(ot._map(fd, pix))
    gpu = np.array([r["dh"][K - 1, y, x] for y, x in pix])
    err = float(np.linalg.norm(gpu - fds) / np.linalg.norm(fds))
    say(f"64 pixels of layer {K - 1}: rel L2 {err:.2e}")
    assert err <= GRAD_TOL


def test_uneven_designs_in_one_plan(torch_dev):
    say("uneven: 64 designs, N in {96,128,192,256}, 2-5 layers, 6-512 wavelengths")
    w = wk.make_workload(5)
    ds, hs, taus = w["designs"], w["h"], w["targets"]
    r = run_gpu(torch_dev, ds, hs, taus, backward=True)
    plan = r["plan"]
    Is = plan.unpack_images(r["I"].cpu())
    gs = plan.unpack_images(r["g"].cpu())
    dhs = plan.unpack_heights(r["dh"].cpu())
    Ls = r["L"].cpu().numpy()
    worst = 0.0
    for i in range(0, 64, 7):
        d = ds[i]
        sample = sorted({0, d["n_wl"] - 1})
        I_ref = o.forward(d, hs[i], None, "fft", wavelengths=sample)
        errs = per_wl_rel(Is[i].numpy()[sample], I_ref)
        worst = max(worst, errs.max())
    say(f"worst sampled rel L2 {worst:.3e}")
    assert worst <= INT_TOL
    # loss and gradient on two small designs in full
    for i in [j for j in range(64) if ds[j]["n_wl"] <= 24][:2]:
        d = ds[i]
        I_ref = o.forward(d, hs[i], None, "fft")
        L_ref, g_ref, _ = o.loss(I_ref, taus[i])
        assert abs(Ls[i] - L_ref) <= 1e-4 * L_ref
        assert rel_l2(gs[i].numpy(), g_ref) <= 1e-4
        dh_ref = o.grad(d, hs[i], None, gs[i].numpy(), "fft")
        assert rel_l2(dhs[i].numpy(), dh_ref) <= 1e-4


# ------------------------------------------------------------------------------------------
# reproducibility, invariance, variants, error paths
# ------------------------------------------------------------------------------------------

def test_bitwise_repeatable_and_batch_invariant(torch_dev):
    say("determinism + batch invariance (batched workload)")
    w = wk.make_workload(3)
    d, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    r1 = run_gpu(torch_dev, [d], [h], [tau])
    r2 = run_gpu(torch_dev, [d], [h], [tau])
    assert torch_dev.equal(r1["I"], r2["I"])
    assert torch_dev.equal(r1["dh"], r2["dh"])
    sub = [5, 77]
    ds = wk.subset_wavelengths(d, sub)
    rs = run_gpu(torch_dev, [ds], [h], [tau[sub]], backward=False)
    I_full = r1["I"].reshape(256, 64, 64)[sub]
    assert torch_dev.equal(rs["I"].reshape(2, 64, 64), I_full)


def test_recompute_mode_and_column_variants_agree(torch_dev):
    say("store vs recompute mode; every column-pass variant; autotuned plan")
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(3)
    d, h, tau = w["designs"][0], w["h"][0], w["targets"][0]
    base = run_gpu(torch_dev, [d], [h], [tau])
    rec = run_gpu(torch_dev, [d], [h], [tau], checkpoint_mode=1, wl_chunk=48)
    assert torch_dev.equal(rec["I"], base["I"])
    assert rel_l2(rec["dh"].cpu().numpy(), base["dh"].cpu().numpy()) <= 1e-6
    for streams, chunk in ((1, 0), (2, 32), (3, 40)):
        r = run_gpu(torch_dev, [d], [h], [tau], streams=streams, wl_chunk=chunk)
        assert torch_dev.equal(r["I"], base["I"])
        assert rel_l2(r["dh"].cpu().numpy(), base["dh"].cpu().numpy()) <= 1e-6
        r2 = run_gpu(torch_dev, [d], [h], [tau], streams=streams, wl_chunk=chunk)
        assert torch_dev.equal(r2["dh"], r["dh"])         # reproducible at a fixed lane layout
    rc = run_gpu(torch_dev, [d], [h], [tau], checkpoint_mode=1, wl_chunk=32, streams=2)
    assert torch_dev.equal(rc["I"], base["I"])
    assert rel_l2(rc["dh"].cpu().numpy(), base["dh"].cpu().numpy()) <= 1e-6
    for v in range(4):
        r = run_gpu(torch_dev, [d], [h], [tau], force_variant=v)
        assert r["plan"].variant(0) == v
        assert torch_dev.equal(r["I"], base["I"]), dpx.variant_names()[v]
        assert torch_dev.equal(r["dh"], base["dh"]), dpx.variant_names()[v]
    at = run_gpu(torch_dev, [d], [h], [tau], autotune=True)
    radix = tuple(at["plan"].radix(0))
    say(f"autotuned variant {dpx.variant_names()[at['plan'].variant(0)]}, radix plans {radix}")
    if radix == (0, 0):
        # the column variants give the same bits; so does the autotuned choice among them
        assert torch_dev.equal(at["I"], base["I"])
    else:
        # another radix plan rounds differently: the same transform within the oracle tolerances
        assert rel_l2(at["I"].cpu().numpy(), base["I"].cpu().numpy()) <= INT_TOL
        assert rel_l2(at["dh"].cpu().numpy(), base["dh"].cpu().numpy()) <= 1e-4


def test_variants_agree_on_every_transform_length(torch_dev):
    """Bitwise agreement of the column-pass variants: the evaluated and mirrored transfer
    functions, 8- and 16-column tiles; at 1024 points the mirrored kernels hold stage-1
    twiddles in registers and the others read them from the table (same values, same bits)."""
    say("column-pass variants, pad 2, N in {48, 96, 192, 256, 512}")
    from paper_2604_02624_amd import dpx
    for n in (48, 96, 192, 256, 512):
        g = np.random.default_rng(300 + n)
        wl = np.array([450e-9, 600e-9, 750e-9])
        d = wk.make_design(n=n, layers=2, wl=wl, n_mat=1.5, dx=300e-9, z=[20e-6, 30e-6],
                           fov=n // 2, pad=2)
        h = (g.random((2, n, n)) * 1.2e-6).astype(np.float32)
        tau = g.random((3, n // 2, n // 2)).astype(np.float32)
        outs = [run_gpu(torch_dev, [d], [h], [tau], force_variant=v) for v in range(4)]
        for r in outs[1:]:
            assert torch_dev.equal(r["I"], outs[0]["I"])
            assert torch_dev.equal(r["dh"], outs[0]["dh"])


@pytest.mark.parametrize("n,pad", [(64, 2), (48, 2), (96, 2), (128, 2), (256, 2), (64, 1), (192, 1)])
def test_matrix_core_column_pass(torch_dev, n, pad):
    """Column pass as DFT matrix products on the FP32 matrix cores: oracle parity."""
    say(f"DFT-GEMM (MFMA) column pass, N = {n}, pad {pad}")
    g = np.random.default_rng(500 + n + pad)
    wl = np.array([450e-9, 600e-9, 750e-9])
    d = wk.make_design(n=n, layers=2, wl=wl, n_mat=wk.cauchy_index(wl), dx=300e-9,
                       z=[20e-6, 30e-6], fov=n // 2, pad=pad)
    h = (g.random((2, n, n)) * 1.17e-6).astype(np.float32)
    tau = g.random((3, n // 2, n // 2)).astype(np.float32)
    r = run_gpu(torch_dev, [d], [h], [tau], force_variant=4)
    I_ref = o.forward(d, h, None, "fft")
    errs = per_wl_rel(r["I"].cpu().numpy().reshape(I_ref.shape), I_ref)
    say(f"rel L2 {errs}")
    assert errs.max() <= INT_TOL
    _, g_ref, _ = o.loss(I_ref, tau)
    dh_ref = o.grad(d, h, None, g_ref, "fft")
    assert rel_l2(r["dh"].cpu().numpy().reshape(h.shape), dh_ref) <= 1e-4


def test_matrix_core_variant_rejected_where_not_built(torch_dev):
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(4)
    with pytest.raises(dpx.DpxError) as e:
        dpx.Plan(w["designs"], force_variant=4)
    assert e.value.status == dpx.DPX_E_UNSUPPORTED


def test_graph_replay_matches_direct_launches(torch_dev):
    say("HIP-graph replay vs direct launches, several replays with direct work between")
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(5)
    ds, hs, taus = w["designs"][:6], w["h"][:6], w["targets"][:6]
    ref = run_gpu(torch_dev, ds, hs, taus)
    plan = dpx.Plan(ds, use_graph=True)
    h = plan.pack_heights(hs)
    tau = plan.pack_images(taus)
    I = torch_dev.empty(plan.img_count, device="cuda")
    g = torch_dev.empty(plan.img_count, device="cuda")
    L = torch_dev.empty(len(ds), dtype=torch_dev.float64, device="cuda")
    dh = torch_dev.empty(plan.h_count, device="cuda")
    for rep in range(4):
        if rep == 2:
            h.mul_(1.0)          # direct work between replays
        plan.forward(h, None, I)
        plan.loss(I, tau, L, g)
        plan.backward(h, None, g, dh)
        torch_dev.cuda.synchronize()
        assert torch_dev.equal(I, ref["I"]), rep
        assert torch_dev.equal(dh, ref["dh"]), rep
    # new contents at the same pointers are picked up by the replay
    h2 = plan.pack_heights([x * 0.5 for x in hs])
    h.copy_(h2)
    plan.forward(h, None, I)
    torch_dev.cuda.synchronize()
    ref2 = run_gpu(torch_dev, ds, [x * 0.5 for x in hs], taus, backward=False)
    assert torch_dev.equal(I, ref2["I"])


def test_concurrent_designs_match_sequential(torch_dev):
    say("uneven designs: several streams and grouped launches vs one design at a time")
    w = wk.make_workload(5)
    ds, hs, taus = w["designs"][:12], w["h"][:12], w["targets"][:12]
    seq = run_gpu(torch_dev, ds, hs, taus, streams=1, schedule=1)
    par = run_gpu(torch_dev, ds, hs, taus, schedule=1)
    par2 = run_gpu(torch_dev, ds, hs, taus, schedule=1, use_graph=True)
    grp = run_gpu(torch_dev, ds, hs, taus)
    grp2 = run_gpu(torch_dev, ds, hs, taus, use_graph=True)
    assert seq["plan"].schedule() == 1 and grp["plan"].schedule() == 2
    for r in (par, par2, grp, grp2):
        assert torch_dev.equal(r["I"], seq["I"])
        assert torch_dev.equal(r["L"], seq["L"])
        assert torch_dev.equal(r["dh"], seq["dh"])


def _mixed_designs(rng):
    """Designs that exercise every key of the grouped schedule: both pads, one transform
    length reached from two N, 1-4 layers, input fields, absorption, binning."""
    specs = [  # n, layers, W, fov, bin, pad
        (64, 3, 4, 32, 2, 2), (128, 2, 3, 64, 1, 1), (64, 1, 5, 64, 1, 2), (48, 4, 2, 24, 3, 2),
        (96, 2, 3, 48, 2, 2), (64, 2, 6, 16, 1, 2), (32, 3, 7, 16, 2, 2), (128, 1, 2, 32, 4, 1),
    ]
    ds, hs, us, taus = [], [], [], []
    for i, (n, k, W, f, b, pad) in enumerate(specs):
        wl = np.linspace(470e-9, 720e-9, W)
        ds.append(wk.make_design(n=n, layers=k, wl=wl, n_mat=wk.cauchy_index(wl), dx=280e-9,
                                 z=list(np.linspace(8e-6, 14e-6, k)), fov=f, bin_=b, pad=pad,
                                 kappa=np.linspace(0.0, 0.02, W) if i % 2 else None))
        hs.append((rng.random((k, n, n)) * 1.1e-6).astype(np.float32))
        us.append((rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64))
        taus.append(rng.random((W, f // b, f // b)).astype(np.float32))
    return ds, hs, us, taus


def test_grouped_schedule_mixed_designs(torch_dev):
    say("grouped schedule vs per design: mixed pads, lengths, layers, u_in, kappa, bins")
    ds, hs, us, taus = _mixed_designs(np.random.default_rng(77))
    ref = run_gpu(torch_dev, ds, hs, taus, u_ins=us, schedule=1, streams=1)
    grp = run_gpu(torch_dev, ds, hs, taus, u_ins=us, schedule=2)
    assert grp["plan"].schedule() == 2
    assert torch_dev.equal(grp["I"], ref["I"])
    assert torch_dev.equal(grp["L"], ref["L"])
    assert torch_dev.equal(grp["g"], ref["g"])
    assert torch_dev.equal(grp["dh"], ref["dh"])
    # and one of them against the oracle (input field + absorption + bins)
    i = 3
    I_ref = o.forward(ds[i], hs[i], us[i], "fft")
    Is = grp["plan"].unpack_images(grp["I"].cpu())
    assert per_wl_rel(Is[i].numpy(), I_ref).max() <= INT_TOL


def test_transfer_tables_match_evaluation(torch_dev):
    say("transfer tables vs H evaluated in the column pass: variants, several gaps, schedules")
    ds, hs, us, taus = _mixed_designs(np.random.default_rng(91))
    ref = run_gpu(torch_dev, ds, hs, taus, u_ins=us, schedule=1, streams=1, transfer_table=1)
    for kw in (dict(schedule=1, streams=1, transfer_table=2), dict(transfer_table=2),
               dict(transfer_table=2, force_variant=0), dict(transfer_table=2, force_variant=1)):
        r = run_gpu(torch_dev, ds, hs, taus, u_ins=us, **kw)
        assert torch_dev.equal(r["I"], ref["I"]), kw
        assert torch_dev.equal(r["dh"], ref["dh"]), kw
    # one design of a single gap length
    w = wk.make_workload(3)
    d = wk.subset_wavelengths(w["designs"][0], np.arange(0, 256, 16))
    tau = w["targets"][0][::16]
    a = run_gpu(torch_dev, [d], [w["h"][0]], [tau], transfer_table=1)
    b = run_gpu(torch_dev, [d], [w["h"][0]], [tau], transfer_table=2)
    assert b["plan"].has_transfer_tables() and not a["plan"].has_transfer_tables()
    assert torch_dev.equal(a["I"], b["I"]) and torch_dev.equal(a["dh"], b["dh"])


def test_lds_resident_path_matches_multi_pass(torch_dev):
    say("LDS-resident forward / adjoint (one launch each) vs the multi-pass kernels")
    w = wk.make_workload(2)
    ref = run_gpu(torch_dev, w["designs"], w["h"], w["targets"])
    lds = run_gpu(torch_dev, w["designs"], w["h"], w["targets"], small_path=1)
    assert lds["plan"].uses_lds_path() and not ref["plan"].uses_lds_path()
    for k in ("I", "L", "g", "dh"):
        assert torch_dev.equal(lds[k], ref[k]), k
    # every supported length and pad, input field, absorption, bins, one layer, one wavelength
    rng = np.random.default_rng(8)
    for n, pad, k, W, f, b in [(32, 2, 3, 5, 16, 2), (64, 1, 2, 3, 32, 1), (48, 2, 2, 4, 24, 3),
                               (96, 1, 1, 2, 48, 2), (64, 2, 1, 1, 64, 1)]:
        wl = np.linspace(480e-9, 700e-9, W)
        d = wk.make_design(n=n, layers=k, wl=wl, n_mat=wk.cauchy_index(wl), dx=260e-9,
                           z=list(np.linspace(6e-6, 11e-6, k)), fov=f, bin_=b, pad=pad,
                           kappa=np.linspace(0.0, 0.02, W))
        h = (rng.random((k, n, n)) * 1.1e-6).astype(np.float32)
        u = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
        tau = rng.random((W, f // b, f // b)).astype(np.float32)
        a = run_gpu(torch_dev, [d], [h], [tau], u_ins=[u])
        r = run_gpu(torch_dev, [d], [h], [tau], u_ins=[u], small_path=1)
        assert r["plan"].uses_lds_path(), (n, pad)
        for key in ("I", "L", "dh"):
            assert torch_dev.equal(r[key], a[key]), (n, pad, key)
        I_ref = o.forward(d, h, u, "fft")
        assert per_wl_rel(r["I"].cpu().numpy().reshape(I_ref.shape), I_ref).max() <= INT_TOL


def test_grouped_schedule_splits_large_groups(torch_dev):
    say("grouped schedule: 70 designs of one transform length (two launches per pass)")
    rng = np.random.default_rng(70)
    ds, hs, taus = [], [], []
    for i in range(70):
        W = 1 + i % 4
        wl = np.linspace(500e-9, 650e-9, W)
        ds.append(wk.make_design(n=32, layers=2, wl=wl, n_mat=1.5, dx=300e-9, z=[6e-6, 9e-6],
                                 fov=16, pad=2))
        hs.append((rng.random((2, 32, 32)) * 1.2e-6).astype(np.float32))
        taus.append(rng.random((W, 16, 16)).astype(np.float32))
    ref = run_gpu(torch_dev, ds, hs, taus, schedule=1, streams=1)
    grp = run_gpu(torch_dev, ds, hs, taus)
    assert grp["plan"].schedule() == 2
    assert torch_dev.equal(grp["I"], ref["I"])
    assert torch_dev.equal(grp["L"], ref["L"])
    assert torch_dev.equal(grp["dh"], ref["dh"])


def test_error_paths(torch_dev):
    say("error paths")
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(1)
    plan = dpx.Plan(w["designs"])
    h = plan.pack_heights(w["h"])
    g = torch_dev.zeros(plan.img_count, device="cuda")
    with pytest.raises(dpx.DpxError) as e:
        plan.backward(h, None, g)
    assert e.value.status == dpx.DPX_E_STATE
    I = plan.forward(h)
    with pytest.raises(dpx.DpxError) as e:
        plan.backward(h.clone(), None, g)
    assert e.value.status == dpx.DPX_E_STATE
    plan.backward(h, None, g)
    # rebinding the wavelengths or setting a misalignment leaves the stored fields stale
    d0 = w["designs"][0]
    for change in (lambda: plan.set_wavelengths(0, d0["wl"], d0["n_mat"]),
                   lambda: plan.set_misalignment(0, dz=np.full(d0["layers"], 1e-8)),
                   lambda: plan.set_misalignment(0)):
        plan.forward(h)
        change()
        with pytest.raises(dpx.DpxError) as e:
            plan.backward(h, None, g)
        assert e.value.status == dpx.DPX_E_STATE
    plan.forward(h)
    plan.backward(h, None, g)
    with pytest.raises(ValueError):
        plan.forward(h[:-1].contiguous())
    with pytest.raises(ValueError):       # an input field of the wrong size, caught by the binding
        plan.backward(h, torch_dev.zeros(2 * plan.u_count - 2, device="cuda"), g)
    lib = plan.lib
    assert lib.dpx_forward(plan._h, None, None, dpx._ptr(I), None) == dpx.DPX_E_ARG
    with pytest.raises(dpx.DpxError) as e:
        dpx.Plan(w["designs"], max_workspace_bytes=1024)
    assert e.value.status == dpx.DPX_E_NOMEM
    with pytest.raises(dpx.DpxError) as e:
        dpx.Plan(w["designs"], schedule=2, checkpoint_mode=1)
    assert e.value.status == dpx.DPX_E_UNSUPPORTED
    assert dpx.Plan(w["designs"]).schedule() == 1        # one design: per-design launches
    torch_dev.cuda.synchronize()


def test_check_finite_option(torch_dev):
    say("opts.check_finite: same bits on finite data; NaN heights, an infinite target and NaN dL/dI reported")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    w = wk.make_workload(2)
    d, h_np, tau_np = w["designs"][0], w["h"][0], w["targets"][0]
    plain = dpx.Plan([d])
    chk = dpx.Plan([d], check_finite=True)
    out = []
    for plan in (plain, chk):
        h = plan.pack_heights([h_np])
        I = plan.forward(h)
        L, g = plan.loss(I, plan.pack_images([tau_np]))
        dh = plan.backward(h, None, g)
        out.append((I.cpu(), L.cpu(), g.cpu(), dh.cpu()))
    for a, b in zip(*out):
        assert torch.equal(a, b)
    h = chk.pack_heights([h_np])
    bad_h = h.clone()
    bad_h[5] = float("nan")
    with pytest.raises(dpx.DpxError) as e:
        chk.forward(bad_h)
    assert e.value.status == dpx.DPX_E_NONFINITE and "intensity" in str(e.value)
    I = chk.forward(h)
    bad_tau = chk.pack_images([tau_np])
    bad_tau[3] = float("inf")
    with pytest.raises(dpx.DpxError) as e:
        chk.loss(I, bad_tau)
    assert e.value.status == dpx.DPX_E_NONFINITE
    L, g = chk.loss(I, chk.pack_images([tau_np]))
    g[7] = float("nan")
    with pytest.raises(dpx.DpxError) as e:
        chk.backward(h, None, g)
    assert e.value.status == dpx.DPX_E_NONFINITE and "dl_dh" in str(e.value)
    # the plan keeps working after a reported output
    L, g = chk.loss(I, chk.pack_images([tau_np]))
    assert torch.equal(chk.backward(h, None, g).cpu(), out[0][3])
    plain.close()
    chk.close()


def test_autograd_function(torch_dev):
    say("torch.autograd.Function wrapper")
    from paper_2604_02624_amd import dpx
    w = wk.make_workload(2)
    plan = dpx.Plan(w["designs"])
    h = plan.pack_heights(w["h"]).requires_grad_(True)
    tau = plan.pack_images(w["targets"])
    I = dpx.dpx_intensity(h, plan)
    _, g = plan.loss(I.detach(), tau)
    I.backward(g)
    ref = plan.backward(h.detach(), None, g)
    assert torch_dev.equal(h.grad, ref)
