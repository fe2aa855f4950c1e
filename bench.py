#!/usr/bin/env python3
"""Benchmark: HSGD refinement of a 512x384 MPI with 32 planes, 4 views, 3 levels.

One step = one whole hsgd_refine: target pyramid, then per level (128x96, 256x192,
512x384) an MPI upsampling (levels > 0) and one iteration of select -> render + loss ->
restricted adjoint -> sparse update, all in the library's HIP kernels. Inputs (seeded
synthetic forward-facing scene, targets rendered by hsgd_render from the ground-truth MPI)
are resident in HBM before the timed region; each step first restores the coarse initial
MPI from a device copy (the refine updates it in place).

Other workloads: --workload c5 (1920x1080, 64 planes, 8 views, 4 levels 240x135 ->
1920x1080 with iterations [0, 1, 1, 1], k = 3, BF16 storage) and c1 (64x48x8).

Prints one JSON line. value = dense-equivalent voxel-updates per refine (sum over
iterations of D*H_l*W_l = 8,257,536 at 512x384x32) x steps / wall time of the timed region.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HSGD MPI voxel-updates/s at 512x384x32, 3 iters; p50/p99 frame latency"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=None, help="default 10 refines (100 requests for serving)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c1", "c5", "c2g", "serving", "views18", "psv", "psv5"],
                    help="c2: 512x384x32 (the headline), c1: 64x48x8, c5: 1920x1080x64 8 views, "
                         "serving: the continuous-batching mix under Poisson arrivals, "
                         "views18: 18 novel views of a refined 512x384x32 MPI per step, "
                         "psv / psv5: the 3-level plane-sweep volume of the c2 rig / the 4-level "
                         "one of the c5 rig per step, c2g: c2 with tilted cameras (general homographies)")
    ap.add_argument("--requests", type=int, default=1200, help="serving: measured requests")
    ap.add_argument("--rate", type=float, default=60.0, help="serving: mean arrivals per second")
    ap.add_argument("--dtype", default=None, choices=["fp32", "bf16"],
                    help="MPI storage (default fp32; bf16 for c5)")
    ap.add_argument("--rule", default="topk", choices=["topk", "mvs"],
                    help="sparsification: the paper's top-k by alpha gradient, or the MVS-sampling window")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run N launches of the library's plain FP32 copy kernel (256 MiB)")
    return ap.parse_args()


def kernel_source_hash(kernel="k_grad_shift"):
    from paper_2307_03017_amd.profiling import kernel_source_hash as h

    return h(kernel)


def grad_launch_bytes(D, shapes, iters, N, k, s):
    """Algorithmic bytes of the gradient kernel's launches in one refine: per launch the MPI
    read once (D*H*W*s), the targets (N*H*W*12), the plane mask (H*W*8) and the gradient of
    the active voxels written once (k*H*W*16)."""
    total = 0
    launches = 0
    for (w, h), n in zip(shapes, iters):
        HW = w * h
        total += n * (D * HW * s + N * HW * 12 + HW * 8 + k * HW * 16)
        launches += n
    return total, launches


def grad_launch_flops(D, shapes, iters, N, k):
    """Algorithmic FP32 operations of the gradient kernel's launches in one refine. Per
    (view, plane, pixel) sample: the 4-tap bilinear gather of RGBA (16 mul + 12 add), the
    over step (w = a T, C += w c, T *= 1 - a: 9), the adjoint of the over step (colour
    r w: 3; alpha T <r, c - B>: 9; behind-composite B = a c + (1 - a) B: 9) and the
    transposed bilinear into the active taps (4 taps x 4 channels x mul + add, on the k/D
    active share): 58 + 32 k / D. Per view pixel the residual and loss: 12."""
    total = 0
    for (w, h), n in zip(shapes, iters):
        total += n * N * w * h * (58 * D + 32 * k + 12)
    return total


def refine_alg_bytes(D, shapes, iters, N, k, s):
    """Algorithmic bytes of a whole refine (the method's minimum traffic): per level the
    MPI it starts from read once (the initial MPI at the coarsest level, the coarser level's
    result above it) and, above the coarsest, the upsampled MPI written; per iteration one
    dense MPI read, the FP32 targets and the read-modify-write of the active voxels with
    their int32 ids. 512x384x32 with 4 views in FP32: 345.24 MB."""
    total = 0
    for l, ((w, h), n) in enumerate(zip(shapes, iters)):
        HW = w * h
        if l > 0:
            pw, ph = shapes[l - 1]
            total += D * pw * ph * s + D * HW * s
        else:
            total += D * HW * s
        total += n * (D * HW * s + N * HW * 12 + k * HW * (4 + 2 * s))
    return total


def host_info():
    """The host the oracle is timed on: CPU model and logical core count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cores": os.cpu_count()}


def timed_runs(fn, min_s=10.0, max_runs=8):
    """Runs fn until at least min_s seconds have passed (at most max_runs times); returns the
    mean seconds per run and the number of runs."""
    runs, total = 0, 0.0
    while runs < max_runs and (runs == 0 or total < min_s):
        t0 = time.perf_counter()
        fn()
        total += time.perf_counter() - t0
        runs += 1
    return total / runs, runs


def cpu_baseline(name):
    """The FP64 oracle on the host, single-threaded: one full refine of the same workload,
    or, for the 1920x1080x64 frame, one finest-level iteration over a 1920x64 band of it
    (all planes and views), reported per dense voxel-update."""
    from threadpoolctl import threadpool_limits

    from oracle import hsgd_oracle as O
    from paper_2307_03017_amd import scenes

    sc = scenes.make_scene(name)
    G = O.view_to_ref_maps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths)
    with threadpool_limits(limits=1):
        if name == "c5":
            rng = np.random.default_rng(11)
            band = 32
            M = scenes.random_mpi(rng, sc.D, band, sc.W, 0.05, 0.95)
            I = scenes.random_images(rng, sc.N, band, sc.W)
            def one():
                S = O.select_active(M[..., 3].astype(np.float32), sc.k)
                _, g = O.loss_and_grad(M, G, I)
                O.apply_update(M, g, S, 1.0, 1.0, bf16=True)

            dt, runs = timed_runs(one)
            dense = sc.D * band * sc.W
            sample = (f"one finest-level iteration (select, render + loss, adjoint, BF16 update) "
                      f"over a {sc.W}x{band} band of the {sc.W}x{sc.H}x{sc.D} frame, {sc.N} views "
                      f"(FP64 NumPy, {runs} runs of {dt:.1f} s), per dense voxel-update")
        else:
            targets = O.render(sc.gt_mpi(), G)           # untimed input preparation
            init = sc.initial_mpi()
            dt, runs = timed_runs(lambda: O.refine(init, targets, sc.K_ref(), sc.K_views(), sc.R_views(),
                                                   sc.t_views(), sc.depths, sc.iters, sc.k, 1.0, 1.0))
            dense = sum(n * sc.D * w * h for (w, h), n in zip(sc.shapes(), sc.iters))
            sample = (f"full {len(sc.iters)}-level refines of the same {sc.W}x{sc.H}x{sc.D} scene "
                      f"(FP64 NumPy, {runs} runs of {dt:.1f} s; targets rendered by the oracle, untimed)")
    return {"value": dense / dt, "unit": "voxel-updates/s", "cores": 1, "kind": "oracle", **host_info(),
            "sample": sample}


def serving_bench(args):
    """Continuous batching of the 8-scene mix (256x192x16, 512x384x32, 1008x756x32; 3-5
    views; BF16 storage): an open-loop Poisson run (latency from arrival to completion on
    the device, after args.warmup requests), a saturated run (every request queued at
    once: the throughput ceiling of the batch), and the batched BF16 results against the
    plain FP32 single-request refine of the same inputs (PSNR)."""
    import torch

    from paper_2307_03017_amd import hsgd, serving

    torch.cuda.set_device(0)
    mix = serving.make_mix(variants=4)
    snaps = {}

    def snapshot(req, st):
        key = (req.scene, req.variant)
        if key not in snaps:
            snaps[key] = st.result.clone()

    def say(msg):
        print(msg, file=sys.stderr, flush=True)

    srv = serving.Server(mix, max_slots=8, snapshot=snapshot)
    n = args.warmup + args.requests
    reqs = serving.poisson_requests(n, args.rate, len(mix), 4)
    say(f"serving: {n} requests at {args.rate} req/s")
    done = serving.run(srv, reqs, progress=say)
    open_loop = serving.summary(done, args.warmup, mix)
    # saturation: all requests at t = 0
    sat_reqs = serving.poisson_requests(400, 1e9, len(mix), 4, seed=11)
    sat = serving.summary(serving.run(srv, sat_reqs, progress=say), 0, mix)
    # batched BF16 vs the plain FP32 single-request refine of the same initial MPI
    dps = []
    for (si_i, v), res in sorted(snaps.items()):
        si = mix[si_i]
        sc = si.sc
        f32, _ = hsgd.hsgd_refine(si.inits32[v], si.targets, sc.K_ref(), sc.K_views(), sc.R_views(),
                                  sc.t_views(), sc.depths, sc.iters, sc.k)
        table = hsgd.level_warps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths,
                                 sc.W, sc.H, sc.W, sc.H)
        ps = []
        for m in (res, f32):
            _, L = hsgd.hsgd_render(m, table, sc.N, images=si.targets, want_rgb=False, want_loss=True)
            ps.append(10.0 * np.log10(1.0 / (2.0 * L.item() / (3.0 * sc.H * sc.W))))
        dps.append(abs(ps[0] - ps[1]))
    out = {
        "metric": f"HSGD serving p50/p99 frame latency at {args.rate:g} req/s Poisson, 8-scene mix; frames/s",
        "value": open_loop["frames_per_s"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": args.warmup,
        "ms_per_step": open_loop["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": ("continuous batching, 8 persistent scenes (3x 256x192x16 k2, 3x 512x384x32 k4, "
                         "2x 1008x756x32 k4; 3-5 views; 3 levels, 1 iteration each), BF16 MPIs resident, "
                         "one hipGraph launch per batched iteration, 8 slots"),
            "arrival_rate_per_s": args.rate,
        },
        "p50_ms": open_loop["p50_ms"],
        "p99_ms": open_loop["p99_ms"],
        "open_loop": open_loop,
        "saturated": sat,
        "bf16_batched_vs_fp32_single": {"pairs": len(dps), "max_abs_dpsnr_db": max(dps) if dps else None},
    }
    print(json.dumps(out), flush=True)


def novel_rig(sc, cols=6, rows=3, a=0.1):
    """cols x rows novel view positions on a grid in [-a, a] x [-a/2, a/2]."""
    xs = np.linspace(-a, a, cols)
    ys = np.linspace(-a / 2, a / 2, rows)
    t = np.array([[x, y, 0.0] for y in ys for x in xs])
    N = len(t)
    return np.repeat(sc.K_ref()[None], N, axis=0), np.repeat(np.eye(3)[None], N, axis=0), t


def views_bench(args):
    """Novel-view rendering of a built MPI: the 512x384x32 scene refined as in the headline
    (FP32 or BF16 storage), then per step one hsgd_render of 18 views on a 6x3 grid (the
    view set a light-field display consumes), outputs [18][384][512][3] FP32."""
    import torch

    from paper_2307_03017_amd import hsgd, scenes

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sc = scenes.make_scene("c2")
    tdtype = torch.float32 if args.dtype == "fp32" else torch.bfloat16
    s_bytes = 16 if args.dtype == "fp32" else 8
    gt = torch.from_numpy(sc.gt_mpi(np.float32)).to(dev)
    table = hsgd.level_warps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths,
                             sc.W, sc.H, sc.W, sc.H, dev)
    targets, _ = hsgd.hsgd_render(gt, table, sc.N)
    init = torch.from_numpy(sc.initial_mpi().astype(np.float32)).to(dev)
    if tdtype != torch.float32:
        init = hsgd.hsgd_convert(init, tdtype)
    mpi, _ = hsgd.hsgd_refine(init, targets, sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(),
                              sc.depths, sc.iters, sc.k)
    K, R, t = novel_rig(sc)
    nv = len(t)
    novel = hsgd.level_warps(sc.K_ref(), K, R, t, sc.depths, sc.W, sc.H, sc.W, sc.H, dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        hsgd.hsgd_render(mpi, novel, nv)
    torch.cuda.synchronize()
    steps = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        hsgd.hsgd_render(mpi, novel, nv)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    with hsgd.KernelTimer([hsgd.K_RENDER]) as kt:
        for _ in range(steps):
            hsgd.hsgd_render(mpi, novel, nv)
        torch.cuda.synchronize()
    n_r, ms_r = kt.result[hsgd.K_RENDER]
    HW = sc.H * sc.W
    alg_bytes = sc.D * HW * s_bytes + nv * HW * 12
    alg_flops = nv * HW * (37 * sc.D)           # per sample: bilinear RGBA 28, over step 9
    t_launch = ms_r * 1e-3 / max(n_r, 1)
    gbs = alg_bytes / t_launch / 1e9
    tfl = alg_flops / t_launch / 1e12
    alu_bound = alg_flops / (FP32_VECTOR_PEAK_TFLOPS * 1e12) > alg_bytes / (HBM_PEAK_GBS * 1e9)
    out = {
        "metric": "novel views/s rendered from a refined 512x384x32 MPI (18-view sets); p50/p99 set latency",
        "value": nv * steps / wall,
        "unit": "views/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "fp32" else "bf16-storage/f32",
        "data": "synthetic",
        "config": {"workload": (f"hsgd_render of {nv} translated views (6x3 grid, +-0.1 x, +-0.05 y) of the "
                                f"refined {sc.W}x{sc.H}x{sc.D} MPI, {args.dtype} storage"),
                   "views_per_step": nv},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "view_sets_per_s": steps / wall,
        "roofline": {
            "kernel": "k_render_shift",
            "bound": "alu" if alu_bound else "hbm",
            "achieved": tfl if alu_bound else gbs,
            "peak": FP32_VECTOR_PEAK_TFLOPS if alu_bound else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if alu_bound else "GB/s",
            "frac": (tfl / FP32_VECTOR_PEAK_TFLOPS) if alu_bound else (gbs / HBM_PEAK_GBS),
            "traffic": None,
            "launches": n_r,
            "avg_launch_us": t_launch * 1e6,
            "alg_bytes_per_launch": alg_bytes,
            "alg_flops_per_launch": alg_flops,
            "hbm": {"achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS},
            "alu": {"achieved_tflops": tfl, "frac": tfl / FP32_VECTOR_PEAK_TFLOPS},
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = views_cpu_baseline()
    print(json.dumps(out), flush=True)


def views_cpu_baseline():
    """The FP64 oracle rendering 3 of the novel views at full size, single-threaded."""
    from threadpoolctl import threadpool_limits

    from oracle import hsgd_oracle as O
    from paper_2307_03017_amd import scenes

    sc = scenes.make_scene("c2")
    K, R, t = novel_rig(sc)
    G = O.view_to_ref_maps(sc.K_ref(), K[:3], R[:3], t[:3], sc.depths)
    M = sc.noisy_mpi(sc.W, sc.H, seed=77).astype(np.float64)
    with threadpool_limits(limits=1):
        dt, runs = timed_runs(lambda: O.render(M, G))
    return {"value": 3 / dt, "unit": "views/s", "cores": 1, "kind": "oracle", **host_info(),
            "sample": f"3 of the 18 novel views of a {sc.W}x{sc.H}x{sc.D} MPI (FP64 NumPy, {runs} runs of {dt:.1f} s)"}


def l2_hit_rate(kernel, workload):
    """The kernel's L2 hit rate from the committed counter summary of this workload, while
    the kernel's sources are unchanged since it was taken (else None)."""
    f = os.path.join(ROOT, "profiles", f"l2_hit_{workload}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash", {}).get(kernel) != kernel_source_hash(kernel):
        return None
    return rec.get("hit_rate", {}).get(kernel)


def calibrate_copy(args, out):
    """--calibrate-copy N: N launches of the library's FP32 copy over 256 MiB, whose memory
    counters scale those of the measured kernel to bytes."""
    if not args.calibrate_copy:
        return
    import torch

    from paper_2307_03017_amd import hsgd

    n = 64 * 1024 * 1024   # floats = 256 MiB
    a = torch.empty(n, dtype=torch.float32, device="cuda:0").fill_(1.0)
    for _ in range(args.calibrate_copy):
        hsgd.hsgd_convert(a, torch.float32)
    torch.cuda.synchronize()
    out["calibration_copy_bytes"] = 2 * 4 * n


PSV_RIGS = {"psv": ("c2", 3), "psv5": ("c5", 4)}


def psv_bench(args):
    """Hierarchical plane-sweep volume: per step one hsgd_plane_sweep of the rig's N source
    images (the ground truth rendered into each view) onto its D planes, all levels stored
    ([N][D][H>>l][W>>l][3] FP32)."""
    import torch

    from paper_2307_03017_amd import hsgd, scenes

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg, L = PSV_RIGS[args.workload]
    sc = scenes.make_scene(cfg)
    gt = torch.from_numpy(sc.gt_mpi(np.float32)).to(dev)
    views = hsgd.level_warps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths,
                             sc.W, sc.H, sc.W, sc.H, dev)
    images, _ = hsgd.hsgd_render(gt, views, sc.N)
    del gt
    table = hsgd.psv_warps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths, dev)
    odt = torch.bfloat16 if args.dtype == "bf16" else torch.float32
    vbytes = 6 if args.dtype == "bf16" else 12
    out = hsgd.hsgd_plane_sweep(images, table, sc.D, L, dtype=odt)
    stream = torch.cuda.current_stream()

    def step():
        hsgd.hsgd_plane_sweep(images, table, sc.D, L, out=out, dtype=odt)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    with hsgd.KernelTimer([hsgd.K_PSV]) as kt:
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
    n_k, ms_k = kt.result[hsgd.K_PSV]
    HW = sc.H * sc.W
    samples = sc.N * sc.D * HW
    wr = sum(samples // 4 ** l * vbytes for l in range(L))
    alg_bytes = sc.N * HW * 12 + wr                 # images read once, every level written once
    t_launch = ms_k * 1e-3 / max(n_k, 1)
    gbs = alg_bytes / t_launch / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"k_plane_sweep_traffic_{args.workload}_{args.dtype}.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            rec = json.load(fh)
        if rec.get("kernel_source_hash") == kernel_source_hash("k_plane_sweep"):
            traffic = rec.get("hbm_bytes_per_launch")
    res = {
        "metric": f"plane-sweep volume samples/s ({sc.W}x{sc.H}, {sc.D} planes, {sc.N} views, {L} levels)",
        "value": samples * steps / wall,
        "unit": "PSV samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "fp32" else "f32/bf16-storage",
        "data": "synthetic",
        "config": {"workload": (f"hsgd_plane_sweep of {sc.N} {sc.W}x{sc.H} source images onto {sc.D} "
                                f"planes, {L} levels {'->'.join(f'{sc.W >> l}x{sc.H >> l}' for l in range(L))}, "
                                f"translation rig, {args.dtype} output"),
                   "bytes_written_per_step": wr},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "roofline": {
            "kernel": "k_plane_sweep",
            "bound": "hbm",
            "achieved": gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "l2_hit": l2_hit_rate("k_plane_sweep", args.workload),
            "launches": n_k,
            "avg_launch_us": t_launch * 1e6,
            "alg_bytes_per_launch": alg_bytes,
        },
    }
    calibrate_copy(args, res)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = psv_cpu_baseline(cfg, L)
    print(json.dumps(res), flush=True)


def psv_cpu_baseline(cfg, L):
    """The FP64 oracle building a bounded part of the plane-sweep volume (c2: every view and
    plane; c5: 16 planes of view 0) with its levels, single-threaded, scaled to samples/s."""
    from threadpoolctl import threadpool_limits

    from oracle import hsgd_oracle as O
    from paper_2307_03017_amd import scenes

    sc = scenes.make_scene(cfg)
    nv, planes = (sc.N, sc.D) if cfg == "c2" else (1, 16)
    I = np.random.default_rng(3).uniform(size=(nv, sc.H, sc.W, 3))
    def one():
        P = O.plane_sweep(I, sc.K_ref(), sc.K_views()[:nv], sc.R_views()[:nv], sc.t_views()[:nv],
                          sc.depths[:planes])
        O.psv_pyramid(P, L)

    with threadpool_limits(limits=1):
        dt, runs = timed_runs(one)
    return {"value": nv * planes * sc.H * sc.W / dt, "unit": "PSV samples/s", "cores": 1, "kind": "oracle",
            **host_info(), "sample": (f"{nv} view(s) x {planes} planes, {L} levels at {sc.W}x{sc.H} "
                                      f"(FP64 NumPy, {runs} runs of {dt:.1f} s)")}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the HSGD path here has no multi-GPU "
              "implementation. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        args.warmup = 100 if args.warmup is None else args.warmup
        serving_bench(args)
        return
    args.warmup = 10 if args.warmup is None else args.warmup
    if args.workload == "views18":
        args.dtype = args.dtype or "fp32"
        views_bench(args)
        return
    if args.workload in PSV_RIGS:
        args.dtype = args.dtype or "fp32"
        psv_bench(args)
        return

    import torch

    from paper_2307_03017_amd import hsgd, scenes

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sc = scenes.make_scene(args.workload)
    if args.dtype is None:
        args.dtype = "bf16" if args.workload == "c5" else "fp32"
    tdtype = torch.float32 if args.dtype == "fp32" else torch.bfloat16
    s_bytes = 16 if args.dtype == "fp32" else 8
    plan = hsgd.RefinePlan(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths,
                           sc.W, sc.H, sc.iters, sc.k, lr_rgb=1.0, lr_alpha=1.0, dtype=tdtype,
                           device=dev, rule=args.rule)
    gt = torch.from_numpy(sc.gt_mpi(np.float32)).to(dev)
    targets, _ = hsgd.hsgd_render(gt, hsgd.level_warps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(),
                                                       sc.depths, sc.W, sc.H, sc.W, sc.H, dev), sc.N)
    del gt
    init32 = torch.from_numpy(sc.initial_mpi().astype(np.float32)).to(dev)
    init = init32 if tdtype == torch.float32 else hsgd.hsgd_convert(init32, tdtype)
    desc = plan.descriptors(targets)
    stream = torch.cuda.current_stream()

    def step():
        plan.levels[0].copy_(init)
        plan.run(targets, desc)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    dense = sum(n * sc.D * w * h for (w, h), n in zip(plan.shapes, sc.iters))
    active = sum(n * sc.k * w * h for (w, h), n in zip(plan.shapes, sc.iters))
    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    # timed region: K steps, events only around each refine (for p50/p99)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        plan.levels[0].copy_(init)
        ev[i][0].record(stream)
        plan.run(targets, desc)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    final_loss = plan.loss_log.cpu().numpy().tolist()

    # kernel-timing pass over the same K steps: every launch of the dominant kernel is
    # bracketed by HIP events on its stream (kept out of the headline pass: each event pair
    # costs a few microseconds)
    with hsgd.KernelTimer([hsgd.K_GRAD]) as kt:
        for i in range(K):
            plan.levels[0].copy_(init)
            plan.run(targets, desc)
        torch.cuda.synchronize()
    n_grad, ms_grad = kt.result[hsgd.K_GRAD]
    gbytes, glaunch = grad_launch_bytes(sc.D, plan.shapes, sc.iters, sc.N, sc.k, s_bytes)
    gflops = grad_launch_flops(sc.D, plan.shapes, sc.iters, sc.N, sc.k)
    t_grad = ms_grad * 1e-3 / K            # gradient-kernel seconds per refine
    achieved_gbs = gbytes / t_grad / 1e9 if ms_grad > 0 else None
    achieved_tf = gflops / t_grad / 1e12 if ms_grad > 0 else None
    # which roof binds: the larger of the ideal times at the HBM and the vector-ALU peaks
    alu_bound = gflops / (FP32_VECTOR_PEAK_TFLOPS * 1e12) > gbytes / (HBM_PEAK_GBS * 1e9)
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"k_grad_shift_traffic_{args.workload}_{args.dtype}.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            rec = json.load(fh)
        if rec.get("kernel_source_hash") == kernel_source_hash():
            traffic = rec.get("hbm_bytes_per_launch")

    out = {
        "metric": METRIC if args.workload == "c2" else
                  f"HSGD MPI voxel-updates/s at {sc.W}x{sc.H}x{sc.D}, {sum(sc.iters)} iters; p50/p99 frame latency",
        "value": dense * K / wall,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "fp32" else "bf16-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": (f"hsgd_refine {sc.W}x{sc.H}x{sc.D} planes, {sc.N} views, "
                         f"{len(sc.iters)} levels {'->'.join(f'{w}x{h}' for w, h in plan.shapes)}, "
                         f"iters {list(sc.iters)}, k={sc.k}, {args.dtype} storage"
                         + (", tilted cameras (general plane homographies)" if args.workload == "c2g" else "")
                         + ("" if args.rule == "topk" else ", MVS-sampling selection")),
            "dense_voxel_updates_per_refine": dense,
            "active_voxel_updates_per_refine": active,
        },
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "value_p50": dense / (float(np.percentile(lat, 50)) * 1e-3),
        "active_voxel_updates_per_s": active * K / wall,
        "loss_log": final_loss,
        "roofline": {
            # the translation-warp specialisation on pure-translation rigs, else the general kernel
            "kernel": "k_grad_shift" if all(w.shift_only for w in plan.warps) else "k_grad",
            "bound": "alu" if alu_bound else "hbm",
            "achieved": achieved_tf if alu_bound else achieved_gbs,
            "peak": FP32_VECTOR_PEAK_TFLOPS if alu_bound else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if alu_bound else "GB/s",
            "frac": ((achieved_tf / FP32_VECTOR_PEAK_TFLOPS) if alu_bound else
                     (achieved_gbs / HBM_PEAK_GBS)) if ms_grad > 0 else None,
            "traffic": traffic,
            "l2_hit": l2_hit_rate("k_grad_shift", f"{args.workload}_{args.dtype}"),
            "launches": n_grad,
            "avg_launch_us": ms_grad * 1e3 / max(n_grad, 1),
            "alg_bytes_per_launch": gbytes / glaunch,
            "alg_flops_per_launch": gflops / glaunch,
            "hbm": {"achieved_gbs": achieved_gbs, "frac": achieved_gbs / HBM_PEAK_GBS if achieved_gbs else None},
            "alu": {"achieved_tflops": achieved_tf,
                    "frac": achieved_tf / FP32_VECTOR_PEAK_TFLOPS if achieved_tf else None},
            "timing": "HIP events around every launch, separate pass of the same K steps",
        },
        "path_roofline": {
            "alg_bytes_per_refine": refine_alg_bytes(sc.D, plan.shapes, sc.iters, sc.N, sc.k, s_bytes),
        },
        # the paper's only speed figures: whole MPI generation (plane sweep, 3D CNNs, learned
        # iterations) on other hardware (Table 1 and the ablation of Sec. 4); context only
        "paper_context": {
            "mpi_generation_s": 0.026, "fps": 37.04, "hardware": "RTX 3090, TensorRT",
            "workload": "378x512, 40 planes, 3 views, k=5, 3 learned iterations incl. 3D CNNs",
            "dense_voxels_per_s_finest_level": 378 * 512 * 40 * 37.04,
        },
    }
    out["path_roofline"]["frac_at_p50"] = (out["path_roofline"]["alg_bytes_per_refine"]
                                           / (out["p50_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)

    calibrate_copy(args, out)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
