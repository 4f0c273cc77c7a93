#!/usr/bin/env python
"""Throughput of the fused multi-wavelength forward + loss + adjoint on one MI355X.

One step = dpx_forward + dpx_loss + dpx_backward over the whole workload (every wavelength,
every layer), inputs resident in device memory.  The metric is wavelength-layer propagations
per second counted forward + adjoint: W * K / step time.

Default workload: 4 layers of 512 x 512 features zero-padded to 1024 x 1024, 4096 wavelengths
uniform in 450-750 nm, Cauchy n(lambda), 30 um gaps, 64 x 64 grayscale targets, store-mode
checkpoints.  Inputs are seeded synthetic arrays (paper_2604_02624_amd.workloads).

Printed: one JSON line with the throughput, the live roofline of the dominant kernel (HIP
events around each of its launches inside the timed region, algorithmic bytes per launch),
the FP64 CPU oracle timed on a bounded sample of the same workload, and a plain per-wavelength
torch FFT loop (rocFFT + autograd) timed on a sample of wavelengths on the same GPU.  After the
timed region: the median / p10 / p90 of single steps, a forward-only rate, and this GPU's
device-copy bandwidth (context for the HBM fractions).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "wavelength·layer propagations/s (fwd+adjoint) + % HBM roofline vs plain loop"
UNIT = "propagations/s"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFS = 157.3
# the issue ceiling of single FP32 operations (the library emits no packed FP32): 256 CUs x 4
# SIMDs x 16 lanes x 2 flops (fused multiply-add) x 2.4 GHz
FP32_NONPACKED_PEAK_TFS = 78.6
# kernel instances the per-pass timers report one by one (a pass kind of the row passes is one
# kernel; the column pass kinds split into the full-plane instance and the rest)
INSTANCE_PASSES = ("col_fwd_full", "col_adj_full", "row_fwd_first", "row_fwd_mid", "row_fwd_last",
                   "row_adj_seed", "row_adj_mid", "row_adj_last", "lds_fwd", "lds_adj")
AGGREGATE_ONLY = ("col_fwd_full", "col_adj_full")   # subsets of col_fwd / col_adj
WORKLOAD_NAMES = {
    1: "small forward: 2 layers 64x64 (pad 128), 6 wavelengths 500-740 nm",
    2: "small fwd+adjoint: 2 layers 64x64 (pad 128), 6 wavelengths 500-740 nm, binary targets",
    3: "batched fwd+adjoint: 5 layers 256x256 (pad 512), 256 wavelengths 450-750 nm",
    4: "large fwd+adjoint: 4 layers 512x512 (pad 1024), 4096 wavelengths 450-750 nm, 64x64 targets",
    5: "uneven fwd+adjoint: 64 designs, N in {96,128,192,256} (pad 2N), 2-5 layers, 6-512 wavelengths",
    6: "paper geometry fwd+adjoint: 8 layers 800x800 (pad 1600), 4096 wavelengths 750-400 nm, N-BK7, "
       "200-sample aperture and input gap, 25x25 pixels of 8x8 samples",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------------------
# plain per-wavelength loop on the same GPU: pad -> fft2 -> x H -> ifft2 -> crop, torch
# autograd for the gradient.  H is precomputed per wavelength and layer outside the timing.
# ------------------------------------------------------------------------------------------
def plain_loop_rate(torch, d, h, tau, n_sample, device, u_in=None):
    import numpy as np
    N, M, K, F = d["n"], d["pad"] * d["n"], d["layers"], d["fov"]
    b = d["bin"]
    z_in = float(d.get("z_in") or 0.0)
    W = d["n_wl"]
    idx = np.linspace(0, W - 1, n_sample).round().astype(int)
    f = torch.fft.fftfreq(M, d=d["dx"], dtype=torch.float64, device=device)
    f2 = f[None, :] ** 2 + f[:, None] ** 2
    Hs = {}
    for w in idx:
        for l in range(-1 if z_in > 0 else 0, K):
            q = (d["n_medium"] / d["wl"][w]) ** 2 - f2
            ph = 2 * np.pi * (z_in if l < 0 else d["z"][l]) * torch.sqrt(torch.clamp(q, min=0))
            Hs[(w, l)] = torch.where(q > 0, torch.polar(torch.ones_like(ph), ph),
                                     torch.zeros((), dtype=torch.complex128, device=device)
                                     ).to(torch.complex64)
    u0 = (torch.ones((N, N), dtype=torch.complex64, device=device) if u_in is None
          else torch.as_tensor(np.asarray(u_in, np.complex64), device=device))
    ht = torch.as_tensor(h, device=device).requires_grad_(True)
    taut = torch.as_tensor(tau, device=device)
    a = (N - F) // 2

    def one_pass():
        ht.grad = None
        total = 0.0
        for w in idx:
            kt = float(2 * np.pi * (d["n_mat"][w] - d["n_medium"]) / d["wl"][w])
            u = u0
            if z_in > 0:
                U = torch.zeros((M, M), dtype=torch.complex64, device=device)
                U[:N, :N] = u
                u = torch.fft.ifft2(torch.fft.fft2(U) * Hs[(w, -1)])[:N, :N]
            for l in range(K):
                u = u * torch.polar(torch.ones_like(ht[l]), kt * ht[l])
                U = torch.zeros((M, M), dtype=torch.complex64, device=device)
                U[:N, :N] = u
                u = torch.fft.ifft2(torch.fft.fft2(U) * Hs[(w, l)])[:N, :N]
            I = (u[a:a + F, a:a + F].abs() ** 2).reshape(F // b, b, F // b, b).sum(dim=(1, 3))
            t = taut[w]
            Lw = ((I / I.sum() - t / t.sum()) ** 2).mean() / W
            Lw.backward()
            total += float(0)
        return total

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return n_sample * K / dt, dt


# ------------------------------------------------------------------------------------------
# FP64 CPU oracle on a bounded sample of the workload
# ------------------------------------------------------------------------------------------
def cpu_baseline(d, h, tau, budget_s, u_in=None, pool=None, threads=1):
    """The oracle as it stands, one call per wavelength (forward, loss, adjoint), run on
    `threads` host threads at once (numpy's transforms release the interpreter lock), over
    wavelengths in a seeded random order until about budget_s seconds have passed."""
    import numpy as np
    from oracle import dpx_oracle as o
    W, K = d["n_wl"], d["layers"]
    order = np.random.default_rng(7).permutation(W)

    def one(w):
        w = int(w)
        I = o.forward(d, h, u_in, "fft", wavelengths=[w])
        _, g, _ = o.loss(I, tau[[w]])
        o.grad(d, h, u_in, g, "fft", wavelengths=[w])

    done, t0 = 0, time.perf_counter()
    while done < W and (done < 2 * threads or time.perf_counter() - t0 < budget_s):
        batch = order[done:done + threads]
        list(pool.map(one, batch)) if pool is not None else [one(w) for w in batch]
        done += len(batch)
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=done * K / dt, unit=UNIT, cores=threads, kind="oracle", host_cpus=os.cpu_count(),
                cpu_model=model,
                sample=f"{done} wavelengths x {K} layers of the same workload, forward + loss + "
                       f"adjoint, FP64 oracle with numpy.fft (pocketfft), one wavelength per host "
                       f"thread, {threads} threads, {dt:.1f} s")


def traffic_from_profiles(pass_name, workload, all_wavelengths, column_variant, column_plan):
    """HBM bytes per launch from the committed rocprofv3 counter runs of this pass, if they were
    taken on this workload (all its wavelengths), with the same column variant and radix plan, on
    the current kernel sources; else None."""
    from paper_2604_02624_amd.profiling import kernel_source_sha
    path = os.path.join(ROOT, "profiles", f"traffic_{pass_name}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if (t.get("kernel_source_sha") != kernel_source_sha() or t.get("workload") != workload or not all_wavelengths
            or t.get("column_variant") != column_variant or t.get("column_radix_plan") != column_plan):
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=4, choices=[1, 2, 3, 4, 5, 6])
    ap.add_argument("--wavelengths", type=int, default=0,
                    help="profiling aid: keep only the first N wavelengths of each design (0: all)")
    ap.add_argument("--checkpoint-mode", type=int, default=0, choices=[0, 1])
    ap.add_argument("--wl-chunk", type=int, default=0)
    ap.add_argument("--streams", type=int, default=0, help="concurrent chunk lanes (0 automatic)")
    ap.add_argument("--transfer-table", type=int, default=0, choices=[0, 1, 2],
                    help="transfer-function tables: 0 automatic, 1 never, 2 always")
    ap.add_argument("--small-path", type=int, default=0, choices=[0, 1],
                    help="short transforms: 0 multi-pass kernels, 1 LDS-resident launches where supported")
    ap.add_argument("--schedule", type=int, default=0, choices=[0, 1, 2],
                    help="several designs: 0 automatic, 1 per design, 2 grouped launches")
    ap.add_argument("--graph", action="store_true",
                    help="replay HIP graphs of each call (per-pass timers then come from one extra "
                         "direct step after the timed region)")
    ap.add_argument("--variant", type=int, default=-1, help="column-pass variant (-1 automatic)")
    ap.add_argument("--autotune", action="store_true",
                    help="time column-pass variants and radix plans at plan creation")
    ap.add_argument("--plan", type=int, default=-1, help="radix plan of the transforms (-1 automatic)")
    ap.add_argument("--reps", type=int, default=20,
                    help="single steps and forward calls timed one by one after the timed region "
                         "(median, p10, p90); 0 skips them")
    ap.add_argument("--train-epochs", type=int, default=1,
                    help="timed training epochs (128-wavelength batches + Adam) after the step; 0 skips")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the oracle baseline (0: the CPUs this process may use, at most 16)")
    ap.add_argument("--graph-reps", type=int, default=20,
                    help="steps replayed from HIP graphs after the timed region (a second plan with "
                         "use_graph); 0 skips them")
    ap.add_argument("--plain-sample", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-loop", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "the path shards over wavelengths with one all-reduce of dL/dh, which the library does "
              "not run across GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2604_02624_amd import dpx, workloads as wk

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] workload {args.workload}: {WORKLOAD_NAMES[args.workload]}")
    w = wk.make_workload(args.workload)
    if args.wavelengths > 0:
        # profiling runs: the first wavelengths of every design only (same kernels, shorter launches)
        for i, d in enumerate(w["designs"]):
            k = min(args.wavelengths, d["n_wl"])
            w["designs"][i] = wk.subset_wavelengths(d, range(k))
            w["targets"][i] = w["targets"][i][:k]
        log(f"[bench] first {args.wavelengths} wavelengths of each design only")
    designs = w["designs"]
    plan = dpx.Plan(designs, checkpoint_mode=args.checkpoint_mode, wl_chunk=args.wl_chunk,
                    force_variant=args.variant, autotune=args.autotune, streams=args.streams,
                    use_graph=args.graph, schedule=args.schedule, transfer_table=args.transfer_table,
                    small_path=args.small_path, force_plan=args.plan)
    variant = dpx.variant_names()[plan.variant(0)]
    M0 = designs[0]["n"] * designs[0]["pad"]
    plan_names = dpx.radix_plan_names(M0)
    radix = dict(zip(("row", "column"), (plan_names[k] for k in plan.radix(0))))
    log(f"[bench] column-pass variant {variant}, radix plans {radix}")
    h = plan.pack_heights(w["h"])
    tau = plan.pack_images(w["targets"])
    # input fields (an aperture) of the designs that have one, unit plane waves elsewhere
    u = None
    if any(x is not None for x in w["u_in"]):
        u = torch.cat([torch.view_as_real(torch.as_tensor(
            np.ones((d["n"], d["n"]), np.complex64) if x is None else np.asarray(x, np.complex64))).reshape(-1)
            for d, x in zip(designs, w["u_in"])]).to(dev)
    I = torch.empty(plan.img_count, dtype=torch.float32, device=dev)
    g = torch.empty(plan.img_count, dtype=torch.float32, device=dev)
    L = torch.empty(len(designs), dtype=torch.float64, device=dev)
    dh = torch.empty(plan.h_count, dtype=torch.float32, device=dev)
    props = sum(d["n_wl"] * d["layers"] for d in designs)

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB done")

    def step():
        plan.forward(h, u, I)
        plan.loss(I, tau, L, g)
        plan.backward(h, u, g, dh)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")

    if not args.graph:
        plan.timing(True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] {args.steps} timed steps done in {wall:.3f} s")
    if args.graph:
        plan.timing(True)
        step()
        torch.cuda.synchronize()
        passes = plan.timing_read()
        passes = {k: dict(v, ms=v["ms"] * args.steps, bytes=v["bytes"] * args.steps,
                          flops=v["flops"] * args.steps, launches=v["launches"] * args.steps)
                  for k, v in passes.items()}
    else:
        passes = plan.timing_read()
    plan.timing(False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = props / (ms_step / 1e3)

    # dominant kernel: the kernel instance with the largest summed time (the full-plane column
    # passes are one instance each; the last forward and first adjoint column passes, which
    # read or keep only the window rows, are another).  The roofline is the HBM one: algorithmic
    # bytes per launch over the average launch time of that instance, against 8 TB/s.  The
    # pass issues vector instructions most of its cycles (rocprofv3 counters), so the same
    # launches are also given against the FP32 issue ceiling of a build without packed FP32
    # (78.6 TFLOP/s) at the conventional 5 M log2 M flops per transform.
    inst = {k: passes[k] for k in INSTANCE_PASSES if k in passes and passes[k]["launches"]}
    dom = max(inst, key=lambda k: inst[k]["ms"])
    pd = inst[dom]
    nl = max(pd["launches"], 1)
    per_launch_s = pd["ms"] / 1e3 / nl
    bytes_per_launch = pd["bytes"] / nl
    flops_per_launch = pd["flops"] / nl
    tfs = flops_per_launch / per_launch_s / 1e12
    gbs = bytes_per_launch / per_launch_s / 1e9
    traffic = traffic_from_profiles(dom, args.workload, args.wavelengths == 0, variant, radix["column"])
    roofline = dict(bound="hbm", kernel=dom, achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(gbs / HBM_PEAK_GBS, 4), traffic=traffic,
                    algorithmic_bytes_per_launch=int(bytes_per_launch),
                    avg_launch_ms=round(per_launch_s * 1e3, 4), launches=pd["launches"],
                    alu=dict(achieved=round(tfs, 2), peak=FP32_NONPACKED_PEAK_TFS, unit="TFLOP/s",
                             frac=round(tfs / FP32_NONPACKED_PEAK_TFS, 4),
                             algorithmic_flops_per_launch=flops_per_launch,
                             peak_note="FP32 without packed instructions; the published 157.3 counts "
                                       "packed FP32"))
    pass_summary = {k: dict(ms_per_step=round(v["ms"] / args.steps, 3),
                            ms_per_launch=round(v["ms"] / v["launches"], 4),
                            gbs=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                            tflops=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2) if v["ms"] > 0 else None)
                    for k, v in passes.items() if v["launches"]}
    all_bytes = sum(v["bytes"] for k, v in passes.items() if k not in AGGREGATE_ONLY)
    step_gbs = all_bytes / args.steps / (ms_step / 1e3) / 1e9

    # after the timed region: the spread of single steps, a forward-only rate, and the device
    # copy bandwidth of this GPU as context for the HBM fractions
    extra = {}
    if args.reps > 0:
        def timed(fn):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)
        steps_ms = sorted(timed(step) for _ in range(args.reps))
        fwd_ms = sorted(timed(lambda: plan.forward(h, u, I)) for _ in range(args.reps))
        pick = lambda v, q: v[min(len(v) - 1, int(round(q * (len(v) - 1))))]
        extra["step_ms"] = dict(median=round(pick(steps_ms, 0.5), 3), p10=round(pick(steps_ms, 0.1), 3),
                                p90=round(pick(steps_ms, 0.9), 3), reps=args.reps)
        extra["forward_only"] = dict(value=round(props / (pick(fwd_ms, 0.5) / 1e3), 1),
                                     unit="propagations/s (forward)", ms_median=round(pick(fwd_ms, 0.5), 3))
        # a misaligned step: every layer displaced by up to +-40 nm laterally and +-200 nm
        # axially (translated gaps evaluate the transfer function with their ramp)
        if (len(designs) == 1 and plan.schedule() == 1 and not plan.uses_lds_path()
                and not plan.has_transfer_tables() and plan.variant(0) != 4):
            from paper_2604_02624_amd import robustness
            lat, ax = robustness.draw_layer_offsets(np.random.default_rng(1), designs[0]["layers"],
                                                    40e-9, 200e-9)
            try:
                plan.set_misalignment(0, *robustness.gap_offsets(lat, ax))
            except dpx.DpxError as e:   # paths that cannot translate (band-limited spectrum)
                log(f"[bench] no misaligned step: {e}")
            else:
                step()
                mis_ms = sorted(timed(step) for _ in range(args.reps))
                plan.set_misalignment(0)
                extra["misaligned_step"] = dict(
                    ms_median=round(pick(mis_ms, 0.5), 3),
                    vs_aligned=round(pick(mis_ms, 0.5) / pick(steps_ms, 0.5), 3),
                    offsets="layers displaced U(+-40 nm) laterally, U(+-200 nm) axially")
        if args.graph_reps > 0 and not args.graph:
            # the same step replayed from HIP graphs (a second plan that captures each call once)
            gplan = dpx.Plan(designs, checkpoint_mode=args.checkpoint_mode, wl_chunk=args.wl_chunk,
                             force_variant=args.variant, autotune=args.autotune, streams=args.streams,
                             use_graph=True, schedule=args.schedule, transfer_table=args.transfer_table,
                             small_path=args.small_path, force_plan=args.plan)

            def gstep():
                gplan.forward(h, u, I)
                gplan.loss(I, tau, L, g)
                gplan.backward(h, u, g, dh)
            for _ in range(2):
                gstep()
            torch.cuda.synchronize()
            g_ms = sorted(timed(gstep) for _ in range(args.graph_reps))
            extra["graph_step"] = dict(ms_median=round(pick(g_ms, 0.5), 3), p10=round(pick(g_ms, 0.1), 3),
                                       p90=round(pick(g_ms, 0.9), 3), reps=args.graph_reps,
                                       vs_eager=round(pick(g_ms, 0.5) / pick(steps_ms, 0.5), 4),
                                       value=round(props / (pick(g_ms, 0.5) / 1e3), 1))
            gplan.close()
            del gplan
            torch.cuda.empty_cache()
            log(f"[bench] {args.graph_reps} graph replays of the step done")
        n = (1 << 30) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        cms = sorted(timed(lambda: dst.copy_(src)) for _ in range(5))
        extra["device_copy_gbs"] = round(2 * (1 << 30) / (pick(cms, 0.5) / 1e3) / 1e9, 1)
        del src, dst
        log(f"[bench] spread of {args.reps} steps, forward-only and copy bandwidth done")
    # training: the same design in minibatches of 128 wavelengths, one Adam step per batch
    # (forward, loss, adjoint and the update on theta), batches in shuffled order
    if args.train_epochs > 0 and len(designs) == 1:
        from paper_2604_02624_amd import train
        d0 = designs[0]
        hm = d0["h_max"]
        x = np.clip(w["h"][0] / hm, 1e-4, 1 - 1e-4)
        tr = train.Trainer(d0, w["targets"][0], hm, theta0=np.log(x / (1 - x)).astype(np.float32),
                           u_in=w["u_in"][0],
                           batch=128, plan_opts=dict(streams=args.streams))
        trng = np.random.default_rng(0)
        tr.epoch(trng)
        log("[bench] training warm-up epoch done")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        tl = [tr.epoch(trng) for _ in range(args.train_epochs)]
        e1.record(stream)
        torch.cuda.synchronize()
        ep_ms = e0.elapsed_time(e1) / args.train_epochs
        nb = len(tr.groups)
        extra["training"] = dict(
            value=round(props / (ep_ms / 1e3), 1), unit=UNIT + " (training epoch)", batch=128,
            batches_per_epoch=nb, epochs=args.train_epochs, ms_per_epoch=round(ep_ms, 3),
            ms_per_batch=round(ep_ms / nb, 3), vs_full_batch_step=round(ep_ms / ms_step, 3),
            mean_loss=tl[-1], workspace_bytes=tr.workspace_bytes())
        tr.close()
        log(f"[bench] {args.train_epochs} timed training epoch(s) done: {ep_ms:.1f} ms each")
    # sanity: the loss is finite
    Lh = L.cpu().numpy()
    if not np.isfinite(Lh).all():
        raise RuntimeError(f"non-finite loss {Lh}")

    plain = None
    if not args.no_plain_loop and len(designs) == 1:
        log(f"[bench] plain per-wavelength torch loop on {args.plain_sample} wavelengths")
        rate, dt = plain_loop_rate(torch, designs[0], w["h"][0], w["targets"][0],
                                   min(args.plain_sample, designs[0]["n_wl"]), dev, u_in=w["u_in"][0])
        plain = dict(value=round(rate, 1), unit=UNIT,
                     sample=f"{min(args.plain_sample, designs[0]['n_wl'])} wavelengths, torch.fft "
                            f"(rocFFT) + autograd, complex64, one wavelength at a time, {dt:.2f} s")

    cpu = None
    if not args.no_cpu_baseline and len(designs) == 1:
        # the host share of one GPU is 16 CPUs on the boxes this runs on, whatever the count of
        # visible CPUs says
        threads = args.cpu_threads or max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"[bench] FP64 oracle on {threads} host threads for about {args.cpu_seconds:.0f} s")
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as pool:
            cpu = cpu_baseline(designs[0], w["h"][0], w["targets"][0], args.cpu_seconds, u_in=w["u_in"][0],
                               pool=pool, threads=threads)
        cpu["value"] = round(cpu["value"], 3)

    d0 = designs[0]
    out = dict(
        metric=METRIC, value=round(value, 1), unit=UNIT, n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOAD_NAMES[args.workload] +
                    (f" (first {args.wavelengths} wavelengths only)" if args.wavelengths > 0 else ""),
                    designs=len(designs),
                    wavelengths=sum(d["n_wl"] for d in designs), layers=d0["layers"], n=d0["n"],
                    transform=d0["n"] * d0["pad"], checkpoint_mode=args.checkpoint_mode,
                    wl_chunk=args.wl_chunk, streams=args.streams, graph=args.graph,
                    schedule={1: "per-design", 2: "grouped"}[plan.schedule()],
                    transfer_tables=plan.has_transfer_tables(), lds_resident=plan.uses_lds_path(),
                    column_variant=variant, radix_plans=radix,
                    phase_args="f64"),
        roofline=roofline, cpu_baseline=cpu, plain_loop=plain,
        vs_plain_loop=(round(value / plain["value"], 2) if plain else None),
        passes=pass_summary, step_hbm=dict(achieved=round(step_gbs, 1), peak=HBM_PEAK_GBS,
                                           unit="GB/s", frac=round(step_gbs / HBM_PEAK_GBS, 4)),
        **extra,
        wall_s=round(wall, 3),
    )
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
