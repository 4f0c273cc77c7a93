"""Seeded random designs and plan options on the GPU against the FP64 oracle: every transform
length up to 384 with pad 1 or 2, ragged wavelength counts and fields of view, detector bins,
absorption, input fields, input gaps, band-limited spectra and misaligned gaps, combined with
column variants, recompute mode, chunks and lanes.  Forward intensities (per wavelength
relative L2 <= 1e-5) and dL/dh against the oracle's adjoint (relative L2 <= 1e-4)."""
import sys

import numpy as np
import pytest

from oracle import dpx_oracle as o
from paper_2604_02624_amd import workloads as wk

pytestmark = pytest.mark.gpu

LENGTHS = [64, 96, 128, 192, 256, 384]


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


def random_case(seed):
    g = np.random.default_rng([260402624, 99, seed])
    M = int(g.choice(LENGTHS))
    pad = int(g.choice([1, 2]))
    N = M // pad
    K = int(g.integers(1, 4))
    W = int(g.integers(1, 6))
    dx = 0.3e-6
    wl = np.sort(g.uniform(0.45e-6, 0.75e-6, W))
    bin_ = int(g.choice([1, 2, 4]))
    fov = int(g.integers(1, N // (2 * bin_) + 1)) * 2 * bin_   # even, a multiple of bin, <= N
    d = wk.make_design(n=N, layers=K, wl=wl, n_mat=wk.cauchy_index(wl), dx=dx,
                       z=g.uniform(5e-6, 40e-6, K), fov=fov, bin_=bin_, pad=pad,
                       kappa=(g.uniform(0, 0.02, W) if g.random() < 0.4 else None))
    if g.random() < 0.3:
        d["z_in"] = float(g.uniform(3e-6, 20e-6))
    band = g.random() < 0.3
    if band:
        d["band_limited"] = True
    if g.random() < 0.4:
        d["dz"] = g.uniform(-0.5e-6, 0.5e-6, K)
        if not band and M <= 1024:
            d["shift_x"] = g.uniform(-2, 2, K) * dx
            d["shift_y"] = g.uniform(-2, 2, K) * dx
    h = (g.random((K, N, N)) * 1.2e-6).astype(np.float32)
    tau = g.random((W, fov // bin_, fov // bin_)).astype(np.float32)
    u_in = None
    if g.random() < 0.4:
        u_in = (g.standard_normal((N, N)) + 1j * g.standard_normal((N, N))).astype(np.complex64)
    variants = [0, 1] if band else [0, 1, 2, 3]
    opts = dict(force_variant=int(g.choice(variants)))
    r = g.random()
    if r < 0.25:
        opts.update(checkpoint_mode=1, wl_chunk=int(g.integers(1, W + 1)))
    elif r < 0.5 and W > 1:
        opts.update(streams=2, wl_chunk=int(g.integers(1, W)))
    # short transforms may run as one LDS-resident launch per wavelength (drawn last, so the
    # earlier draws of every seed stay as they were)
    plain = not band and d.get("z_in") is None and d.get("shift_x") is None and d.get("dz") is None
    if M <= 128 and plain and g.random() < 0.6:
        opts = dict(small_path=1)
    return d, h, tau, u_in, opts


@pytest.mark.parametrize("seed", range(32))
def test_random_design_matches_oracle(torch_dev, seed):
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    d, h, tau, u_in, opts = random_case(seed)
    flags = [k for k in ("z_in", "band_limited", "dz", "shift_x", "kappa") if d.get(k) is not None]
    say(f"seed {seed}: N={d['n']} pad={d['pad']} K={d['layers']} W={d['n_wl']} F={d['fov']} b={d['bin']} "
        f"u_in={u_in is not None} {flags} {opts}")
    plan = dpx.Plan([d], **opts)
    hh = plan.pack_heights([h])
    u = None if u_in is None else torch.view_as_real(torch.as_tensor(u_in)).reshape(-1).cuda()
    I = plan.forward(hh, u)
    _, g = plan.loss(I, plan.pack_images([tau]))
    dh = plan.backward(hh, u, g)
    torch.cuda.synchronize()
    I = I.cpu().numpy().reshape(tau.shape)
    g = g.cpu().numpy().reshape(tau.shape)
    dh = dh.cpu().numpy().reshape(h.shape)
    say(f"  LDS-resident path {plan.uses_lds_path()}") if opts.get("small_path") else None
    plan.close()
    I_ref = o.forward(d, h, u_in, "fft")
    errs = [rel_l2(I[i], I_ref[i]) for i in range(d["n_wl"])]
    assert max(errs) <= 1e-5, errs
    dh_ref = o.grad(d, h, u_in, g.astype(np.float64), "fft")
    e = rel_l2(dh, dh_ref)
    say(f"  intensities {max(errs):.1e}, gradient {e:.1e}")
    assert e <= 1e-4


def test_short_last_chunk_on_its_own_lane(torch_dev):
    say("short last wavelength chunk as a lane's first chunk, in freshly reused memory")
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    wl = np.linspace(0.45e-6, 0.7e-6, 3)
    d = wk.make_design(n=96, layers=3, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6,
                       z=[8e-6, 12e-6, 10e-6], fov=16, bin_=4, pad=2)
    g = np.random.default_rng(6)
    h = (g.random((3, 96, 96)) * 1.2e-6).astype(np.float32)
    tau = g.random((3, 4, 4)).astype(np.float32)

    def grad(**kw):
        plan = dpx.Plan([d], **kw)
        hh = plan.pack_heights([h])
        I = plan.forward(hh)
        _, gi = plan.loss(I, plan.pack_images([tau]))
        dh = plan.backward(hh, None, gi)
        torch.cuda.synchronize()
        out = gi.cpu().numpy().reshape(tau.shape), dh.cpu().numpy().reshape(h.shape)
        plan.close()
        return out

    for rep in range(4):
        grad(wl_chunk=1)                     # leaves gradient partials in memory it frees
        gi, dh = grad(streams=2, wl_chunk=2)  # chunks of 2 and 1 wavelengths on two lanes
        e = rel_l2(dh, o.grad(d, h, None, gi.astype(np.float64), "fft"))
        say(f"  repetition {rep}: gradient {e:.1e}")
        assert e <= 1e-4


def random_plan(seed):
    """2-4 random designs and plan options that the library accepts for them."""
    g = np.random.default_rng([260402624, 98, seed])
    nd = int(g.integers(2, 5))
    opts = {}
    r = g.random()
    if r < 0.3:
        opts["schedule"] = 2
    elif r < 0.45:
        opts["schedule"] = 1
    if g.random() < 0.3:
        opts["transfer_table"] = 2
    if g.random() < 0.3:
        opts["small_path"] = 1
    if g.random() < 0.3:
        opts["use_graph"] = True
    grouped = opts.get("schedule") == 2
    plain = not grouped and opts.get("transfer_table") != 2 and opts.get("small_path") != 1
    designs, hs, taus, us = [], [], [], []
    for i in range(nd):
        M = int(g.choice([64, 128, 192, 256]))
        pad = 2 if grouped else int(g.choice([1, 2]))
        N = M // pad
        K = int(g.integers(1, 4))
        W = int(g.integers(1, 6))
        wl = np.sort(g.uniform(0.45e-6, 0.75e-6, W))
        bin_ = int(g.choice([1, 2]))
        fov = int(g.integers(1, N // (2 * bin_) + 1)) * 2 * bin_
        d = wk.make_design(n=N, layers=K, wl=wl, n_mat=wk.cauchy_index(wl), dx=0.3e-6,
                           z=g.uniform(5e-6, 30e-6, K), fov=fov, bin_=bin_, pad=pad,
                           kappa=(g.uniform(0, 0.02, W) if g.random() < 0.3 else None))
        if not grouped and opts.get("small_path") != 1 and g.random() < 0.3:
            d["z_in"] = float(g.uniform(3e-6, 15e-6))
        if plain and g.random() < 0.3:
            d["dz"] = g.uniform(-0.4e-6, 0.4e-6, K)
            d["shift_x"] = g.uniform(-1.5, 1.5, K) * d["dx"]
        designs.append(d)
        hs.append((g.random((K, N, N)) * 1.2e-6).astype(np.float32))
        taus.append(g.random((W, fov // bin_, fov // bin_)).astype(np.float32))
        us.append(None)
    if plain and any(d.get("shift_x") is not None for d in designs):
        opts["schedule"] = 1     # misaligned designs run the per-design schedule
    return designs, hs, taus, opts


@pytest.mark.parametrize("seed", range(16))
def test_random_multi_design_plan_matches_oracle(torch_dev, seed):
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    designs, hs, taus, opts = random_plan(seed)
    say(f"seed {seed}: {len(designs)} designs "
        f"{[(d['n'] * d['pad'], d['layers'], d['n_wl']) for d in designs]} {opts}")
    plan = dpx.Plan(designs, **opts)
    hh = plan.pack_heights(hs)
    I = plan.forward(hh)
    _, g = plan.loss(I, plan.pack_images(taus))
    dh = plan.backward(hh, None, g)
    torch.cuda.synchronize()
    Is = plan.unpack_images(I.cpu())
    gs = plan.unpack_images(g.cpu())
    dhs = plan.unpack_heights(dh.cpu())
    say(f"  schedule {plan.schedule()}, LDS path {plan.uses_lds_path()}, tables {plan.has_transfer_tables()}")
    plan.close()
    for d, h, tau, Ii, gi, dhi in zip(designs, hs, taus, Is, gs, dhs):
        I_ref = o.forward(d, h, None, "fft")
        errs = [rel_l2(Ii.numpy()[w], I_ref[w]) for w in range(d["n_wl"])]
        assert max(errs) <= 1e-5, errs
        dh_ref = o.grad(d, h, None, gi.numpy().astype(np.float64), "fft")
        assert rel_l2(dhi.numpy(), dh_ref) <= 1e-4


@pytest.mark.parametrize("seed", range(10))
def test_random_rebinding_matches_fresh_plan(torch_dev, seed):
    """dpx_plan_set_wavelengths on a random design and option set gives the bits of a plan
    created with the new wavelengths."""
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    d, h, tau, u_in, opts = random_case(100 + seed)
    if seed % 3 == 0 and not d.get("band_limited"):
        opts = dict(opts, transfer_table=2) if d.get("shift_x") is None and d.get("dz") is None \
            and not opts.get("small_path") else opts
    if seed % 2 == 1:
        opts = dict(opts, use_graph=True)
    g = np.random.default_rng(seed)
    wl2 = np.sort(g.uniform(0.45e-6, 0.75e-6, d["n_wl"]))
    d2 = dict(d, wl=wl2, n_mat=wk.cauchy_index(wl2))
    if d.get("kappa") is not None:
        d2["kappa"] = g.uniform(0, 0.02, d["n_wl"])
    say(f"seed {seed}: N={d['n']} pad={d['pad']} K={d['layers']} W={d['n_wl']} {opts}")
    u = None if u_in is None else torch.view_as_real(torch.as_tensor(u_in)).reshape(-1).cuda()

    def run(plan):
        hh = plan.pack_heights([h])
        I = plan.forward(hh, u)
        _, gi = plan.loss(I, plan.pack_images([tau]))
        dh = plan.backward(hh, u, gi)
        torch.cuda.synchronize()
        return I.cpu().numpy(), dh.cpu().numpy()

    rebound = dpx.Plan([d], **opts)
    run(rebound)
    rebound.set_wavelengths(0, d2["wl"], d2["n_mat"], d2.get("kappa"))
    a = run(rebound)
    rebound.close()
    fresh = dpx.Plan([d2], **opts)
    b = run(fresh)
    fresh.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])



def random_large_case(seed):
    """A random design on the long transforms (512, 1024, 1600) with the options they support."""
    g = np.random.default_rng([260402624, 97, seed])
    M = int(g.choice([512, 1024, 1600]))
    pad = int(g.choice([1, 2])) if M <= 1024 else 2
    N = M // pad
    K = int(g.integers(1, 3))
    W = int(g.integers(1, 4))
    wl = np.sort(g.uniform(0.4e-6, 0.75e-6, W))
    bin_ = int(g.choice([1, 2, 8]))
    fov = int(g.integers(1, min(N, 256) // (2 * bin_) + 1)) * 2 * bin_
    d = wk.make_design(n=N, layers=K, wl=wl, n_mat=wk.nbk7_index(wl), dx=0.2e-6,
                       z=g.uniform(10e-6, 80e-6, K), fov=fov, bin_=bin_, pad=pad,
                       kappa=(g.uniform(0, 0.01, W) if g.random() < 0.3 else None))
    if g.random() < 0.4:
        d["z_in"] = float(g.uniform(5e-6, 60e-6))
    band = g.random() < 0.3
    if band:
        d["band_limited"] = True
    if g.random() < 0.4:
        d["dz"] = g.uniform(-0.3e-6, 0.3e-6, K)
        if not band and M <= 1024:
            d["shift_x"] = g.uniform(-2, 2, K) * d["dx"]
            d["shift_y"] = g.uniform(-2, 2, K) * d["dx"]
    h = (g.random((K, N, N)) * 1.2e-6).astype(np.float32)
    tau = g.random((W, fov // bin_, fov // bin_)).astype(np.float32)
    u_in = None
    if g.random() < 0.3:
        u_in = (g.standard_normal((N, N)) + 1j * g.standard_normal((N, N))).astype(np.complex64)
    opts = {}
    variants = [0, 1] if (band or M > 1024) else [0, 1, 2, 3]
    if g.random() < 0.6:
        opts["force_variant"] = int(g.choice(variants))
    r = g.random()
    if r < 0.25:
        opts.update(checkpoint_mode=1, wl_chunk=int(g.integers(1, W + 1)))
    elif r < 0.5 and W > 1:
        opts.update(streams=2, wl_chunk=int(g.integers(1, W)))
    if g.random() < 0.2 and not band and d.get("dz") is None:
        opts["transfer_table"] = 2
    if g.random() < 0.3:
        opts["use_graph"] = True
    return d, h, tau, u_in, opts


@pytest.mark.parametrize("seed", range(12))
def test_random_long_transform_matches_oracle(torch_dev, seed):
    from paper_2604_02624_amd import dpx
    torch = torch_dev
    d, h, tau, u_in, opts = random_large_case(seed)
    say(f"seed {seed}: M={d['n'] * d['pad']} pad={d['pad']} K={d['layers']} W={d['n_wl']} F={d['fov']} "
        f"b={d['bin']} {[k for k in ('z_in', 'band_limited', 'dz', 'shift_x', 'kappa') if d.get(k) is not None]} "
        f"u_in={u_in is not None} {opts}")
    plan = dpx.Plan([d], **opts)
    hh = plan.pack_heights([h])
    u = None if u_in is None else torch.view_as_real(torch.as_tensor(u_in)).reshape(-1).cuda()
    I = plan.forward(hh, u)
    _, g = plan.loss(I, plan.pack_images([tau]))
    dh = plan.backward(hh, u, g)
    torch.cuda.synchronize()
    I = I.cpu().numpy().reshape(tau.shape)
    g = g.cpu().numpy().reshape(tau.shape)
    dh = dh.cpu().numpy().reshape(h.shape)
    plan.close()
    I_ref = o.forward(d, h, u_in, "fft")
    assert max(rel_l2(I[i], I_ref[i]) for i in range(d["n_wl"])) <= 1e-5
    assert rel_l2(dh, o.grad(d, h, u_in, g.astype(np.float64), "fft")) <= 1e-4
