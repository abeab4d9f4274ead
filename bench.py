"""Benchmark of the decentralized-ADMM hot path on one MI355X.

One step = one outer iteration of Alg. 4 over every node of every slice of the
workload: E1 = 5 local steps (Joseph projection, residual, matched
backprojection, u-step) per node, the segment x-update with the quantized
exchange, and the dual update.  The iteration is launched in its batched form
(one launch per kernel for all slices and nodes) and replayed from a HIP graph;
inputs are resident on the device before timing starts.  Three forms of the
captured iteration give bit-identical iterates: the sequential one; the
pipelined one, whose last part launches the next iteration's first projection
(which reads only u and d) on a second stream, concurrently with the
consensus; and the alternating one, pipelined iterations whose local updates
alternate between the two streams.  Every step of each runs 5 projections, 5
backprojections and one consensus.  A graph holds several iterations (10 for
the single workload: each replay costs a few microseconds of launch overhead).
A few replays of each form pick the fastest, which is timed.  Workloads:

* ``single`` (default): 512 x 512, 720 angles, 725 bins, 16 nodes with
  contiguous angle blocks, Poisson data at 1e5 photons, K-means with 8 levels;
* ``batch``: 256 slices of sizes drawn from {128, ..., 1024} (angles 1.5 N,
  bins ceil(1.414 N)), 2 to 16 interleaved nodes each, K-means with 16 levels;
* ``large``: 2048 x 2048 (50 ellipses + texture), 1800 angles, 2897 bins, 64
  contiguous nodes, 8x8 DCT exchange at quality 50.

value = (ray-voxel updates in P + in P^T) per second = sum over slices of
2 E1 K N^2 / step time.  Also reported: ADMM iterations/s (summed over slices)
of the batched graph and of the plain per-slice, per-node launch loop, and the
RMSE of every slice after the same iterations in both forms (identical by
construction: a node's work decomposes the same way alone or batched); the
projector tiles picked by the autotuner; per-phase durations, the ALU roofline
of the projection phase and its HBM traffic; and, untimed, the reconstruction
RMSE against the phantom after 50, 100 and 200 iterations with the segment and
the averaging x-update (the timed configuration, segment-owned updates over
contiguous angle blocks, does not reconstruct this phantom; the averaging form
on the same data and kernels shows what the kernels reach).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload single|batch|large]
                    [--no-cpu-baseline] [--no-autotune] [--profile-kernels]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ALGO_FLOPS_PER_UPDATE = 4.0        # the two multiply-adds of the 2-tap interpolation
PEAK_FP32_TFLOPS = 157.3           # MI355X vector FP32 (published, with packed FP32 instructions)
# without packed FP32 (the library is built with it off): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_SINGLE_ISSUE_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
PHASE_KERNELS = {"project": "projection phase: k_project + k_project_reduce",
                 "backproject": "backprojection phase: k_backproject"}
# sources whose change invalidates a traffic record: the kernels, and the
# plan code that sets their launch shapes and dispatch orders
KERNEL_SOURCES = ("paper_2410_06106_amd/csrc/project.hip", "paper_2410_06106_amd/csrc/project_res.hip",
                  "paper_2410_06106_amd/csrc/backproject.hip", "paper_2410_06106_amd/csrc/common.h",
                  "paper_2410_06106_amd/csrc/api.hip")
DEFAULT_STEPS = {"single": 2000, "batch": 5, "large": 10, "diff": 4}
# untimed warm-up steps; for the single workload one whole graph (see below)
DEFAULT_WARMUP = {"single": 10, "batch": 3, "large": 3, "diff": 3}
EQUAL_RMSE_STEPS = {"single": 5, "batch": 2, "large": 2, "diff": 0}
# ADMM iterations captured per graph replay (a replay costs a few us of launch
# overhead, which matters at the 0.6 ms iteration of the single workload only)
ITERS_PER_GRAPH = {"single": 10, "batch": 1, "large": 2, "diff": 1}


def _source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str, tiles):
    """HBM bytes per launch from the committed rocprofv3 counter record of this
    workload, if it was taken on the current kernel sources with the same
    projector tiles; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}512.json") if workload == "single" else None
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != _source_sha(KERNEL_SOURCES) or not tiles:
        return None
    key = "resident" if tiles.get("kernel") == 1 else f"{tiles['band']}/{tiles['job_wgs']}"
    entry = rec.get("by_tiles", {}).get(key)
    return entry.get("hbm_bytes_per_launch") if entry else None


def _cpu_node(job):
    """One sampled node: its data, then the oracle's Alg. 2 local update, which
    alone is timed.  Returns (ray-voxel updates, seconds)."""
    import numpy as np

    import synthdata
    from oracle import admm as oadmm
    from oracle import chord, joseph

    w, si, m, model = job
    proj = chord if model == "chord" else joseph
    th = synthdata.angles(w.n_angles)
    part = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)[m]
    d = proj.project(synthdata.phantom(w, si), th[part], w.n_bins)
    u = np.random.default_rng(m).random((w.n, w.n))
    t0 = time.perf_counter()
    oadmm.local_update(u, np.zeros((w.n, w.n)), np.zeros((w.n, w.n)), d, th[part], 1.0, 1e-5, w.inner_iters,
                       proj=proj)
    return 2 * w.inner_iters * len(part) * w.n * w.n, time.perf_counter() - t0


def cpu_baseline(slices_info, sample_nodes, model="joseph"):
    """The oracle's Alg. 2 local update (E1 steps of P and P^T) on a sample of
    nodes, one after another in this process; returns ray-voxel updates/s and
    the seconds timed."""
    upd, dt = 0, 0.0
    for w, si, m in sample_nodes:
        u, t = _cpu_node((w, si, m, model))
        upd += u
        dt += t
    return upd / dt, dt


def cpu_baseline_pool(sample_nodes, model="joseph", processes=8):
    """The same sample with one worker process per node (forked before this
    process touches the GPU); the rate is the total updates over the wall time
    of the pool's work."""
    import multiprocessing as mp

    jobs = [(w, si, m, model) for w, si, m in sample_nodes]
    with mp.get_context("fork").Pool(processes) as pool:
        t0 = time.perf_counter()
        res = pool.map(_cpu_node, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    return sum(u for u, _ in res) / wall, wall


def build(which, ctx, A, T, synthdata, log):
    """Slices, quantizer and description of a workload."""
    import torch

    if which == "single":
        w = synthdata.WORKLOADS["single"]
        log(f"setup: {w.n}^2, {w.n_angles} angles, {w.n_bins} bins, {w.n_nodes} nodes")
        s = A.make_slice(ctx, w)
        s.eta1 = A.step_size(ctx, s, w.rho, 0.1)
        q = T.tomo_quant(T.TOMO_QUANT_KMEANS, w.levels, 30, 50)
        desc = ("single-GPU plain method: 512x512 random-ellipse phantom (20 ellipses), 720 angles, 725 bins, "
                "Poisson 1e5, 16 nodes contiguous, SEG x-update, K-means 8 levels, E1=5, E2=10, rho=1")
        cfg = {"n": w.n, "angles": w.n_angles, "bins": w.n_bins, "nodes": w.n_nodes}
        sample = [(w, 0, m) for m in range(8)]
        sample_desc = f"nodes 0-7 of 16 (512^2, 45 angles each)"
        return [s], [w], q, desc, cfg, sample, sample_desc
    if which == "large":
        w = synthdata.WORKLOADS["large"]
        log(f"setup: {w.n}^2, {w.n_angles} angles, {w.n_bins} bins, {w.n_nodes} nodes")
        s = A.make_slice(ctx, w)
        # contiguous angle blocks: the operator norm varies by node; the max over
        # 8 nodes spread over the angle range, 20 power iterations each
        L = max(A.operator_norm(ctx, s.angles[m], s.n, s.n_bins, iters=20) for m in range(0, w.n_nodes, 8))
        s.eta1 = 0.1 / (L + w.rho)
        q = T.tomo_quant(T.TOMO_QUANT_DCT, 0, 0, 50)
        desc = ("large: 2048x2048 random-ellipse phantom (50 ellipses + texture 0.02), 1800 angles, 2897 bins, "
                "Gaussian 1%, 64 nodes contiguous, SEG x-update, 8x8 DCT exchange at quality 50, E1=5, E2=10, rho=1")
        cfg = {"n": w.n, "angles": w.n_angles, "bins": w.n_bins, "nodes": w.n_nodes, "dct_quality": 50}
        sample = [(w, 0, 0)]
        sample_desc = "node 0 of 64 (2048^2, 29 angles)"
        return [s], [w], q, desc, cfg, sample, sample_desc
    if which == "batch":
        ws = synthdata.batch_slices(256)
        log(f"setup: 256 slices, {sum(w.n_nodes for w in ws)} nodes")
        slices = []
        for si, w in enumerate(ws):
            s = A.make_slice(ctx, w, slice_idx=si)
            # interleaved angles: every node of a slice has nearly the same
            # operator norm; node 0, 20 power iterations
            L = A.operator_norm(ctx, s.angles[0], s.n, s.n_bins, iters=20)
            s.eta1 = 0.1 / (L + w.rho)
            slices.append(s)
        torch.cuda.synchronize()
        q = T.tomo_quant(T.TOMO_QUANT_KMEANS, 16, 30, 50)
        desc = ("batch: 256 slices, N uniform over {128,256,384,512,768,1024}, 1.5N angles, ceil(1.414N) bins, "
                "2/4/8/16 interleaved nodes per slice (seed 4000), Gaussian 1%, SEG x-update, K-means 16 levels, "
                "E1=5, E2=10, rho=1")
        cfg = {"slices": len(ws), "nodes": sum(w.n_nodes for w in ws),
               "sizes": sorted({w.n for w in ws}), "node_counts": sorted({w.n_nodes for w in ws})}
        w0 = ws[0]
        sample = [(w0, 0, 0), (w0, 0, 1)]
        sample_desc = f"nodes 0-1 of slice 0 ({w0.n}^2, {w0.n_nodes} nodes, {w0.n_angles // w0.n_nodes} angles each)"
        return slices, ws, q, desc, cfg, sample, sample_desc
    raise SystemExit(f"unknown workload {which}")


def batching_line(A, T, synthdata, autotune, log, iters=2, steps=4):
    """The batching workload's comparison for the default run: 256 slices of
    sizes 128..1024 (1.5 N angles, ceil(1.414 N) bins, 2..16 interleaved nodes),
    K-means with 16 levels; ``iters`` iterations of the plain per-slice,
    per-node launch loop, then the same iterations from the same start by the
    batched one-iteration graph (same kernels, so the slices' RMSEs are equal
    bit for bit), then ``steps`` timed replays.  A context of its own, so the
    autotuned tiles of the main workload are untouched."""
    import numpy as np
    import torch

    ctx = T.Context(0)
    t0 = time.perf_counter()
    slices, ws, q, desc, cfg, _, _ = build("batch", ctx, A, T, synthdata, log)
    run = A.DADMM(ctx, slices, rho=1.0, eta2=0.2, e1=5, e2=10, mode=T.TOMO_XUPDATE_SEGMENT, quant=q)
    choice = autotune.tune(ctx, run.nodes, resident=True)
    setup_s = time.perf_counter() - t0

    def zero_all():
        for s in slices:
            s.zero()

    zero_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        run.step_plain()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / iters
    rmse_plain = [run.rmse(i) for i in range(len(slices))]
    x_plain = [s.x.clone() for s in slices]
    zero_all()
    run.step()                                   # builds the batched plans outside capture
    zero_all()
    torch.cuda.synchronize()
    g = run.capture(1)
    zero_all()
    for _ in range(iters):
        g.replay()
    torch.cuda.synchronize()
    rmse_batched = [run.rmse(i) for i in range(len(slices))]
    identical = all(bool(torch.equal(xp, s.x)) for xp, s in zip(x_plain, slices))
    del x_plain
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    batched_s = max(e0.elapsed_time(e1) * 1e-3, time.perf_counter() - t0) / steps
    n = len(slices)
    rel = max(abs(a - b) / b if b > 0 else 0.0 for a, b in zip(rmse_batched, rmse_plain))
    out = {"workload": desc, "slices": n, "nodes": cfg["nodes"], "iterations_compared": iters,
           "timed_replays": steps,
           "batched_graph": n / batched_s, "plain_loop": n / plain_s, "unit": "slice-iterations/s",
           "speedup": plain_s / batched_s, "bit_identical": identical, "max_rel_rmse_diff": rel,
           "rmse_mean_plain": float(np.mean(rmse_plain)), "rmse_mean_batched": float(np.mean(rmse_batched)),
           "updates_per_s": sum(2 * w.inner_iters * w.n_angles * w.n * w.n for w in ws) / batched_s,
           "projector_tiles": {k: choice[k] for k in ("kernel", "band", "job_wgs")}, "setup_s": setup_s}
    log(f"batching: {n} slices, batched graph {out['batched_graph']:.1f} vs plain loop {out['plain_loop']:.1f} "
        f"slice-iterations/s ({out['speedup']:.2f}x), mean rmse {out['rmse_mean_batched']:.6g} "
        f"(identical={identical})")
    del run, slices, g
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def bench_diff(args, steps, ctx, log):
    """Form (3): K = 10 unrolled ADMM iterations of the 1024^2, 1080-angle,
    32-node workload with learnable (rho_k, eta_k), trained by Adam on seeded
    phantom / sinogram pairs; the projector's backward is the hand-written
    backprojector and iterates are checkpointed every 2 iterations.  One step =
    one training step (forward, loss, backward with recomputation, Adam)."""
    import numpy as np
    import torch

    import synthdata
    from paper_2410_06106_amd import admm as A
    from paper_2410_06106_amd import autograd as AG
    from paper_2410_06106_amd import tomoadmm as T

    w = synthdata.WORKLOADS["diff"]
    n, nb, iters, e1 = w.n, w.n_bins, w.outer_iters, w.inner_iters
    th = synthdata.angles(w.n_angles)
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    segs = synthdata.segment_rows(n, w.n_nodes)
    ang_all = torch.from_numpy(th).cuda()
    angs = [ang_all[torch.from_numpy(p).cuda()].contiguous() for p in parts]
    t_setup = time.perf_counter()
    L = A.operator_norm(ctx, angs[0], n, nb, iters=20)
    model = AG.UnrolledADMM(ctx, n, nb, angs, segs, iters=iters, e1=e1, e2=w.x_iters, eta2=w.eta2,
                            eta0=0.1 / (L + 1.0), ckpt=2).cuda()
    opt = torch.optim.Adam(model.parameters(), lr=0.05)
    if args.no_autotune:
        tiles = {"kernel": 0, "band": 32, "job_wgs": 16}       # the context's defaults
    else:
        choice = model.tune_projector()
        tiles = {k: choice[k] for k in ("kernel", "band", "job_wgs")}
        log(f"autotune: band {choice['band']}, {choice['job_wgs']} workgroups per node "
            f"({choice['us']:.0f} us per batched projection)")

    from concurrent.futures import ThreadPoolExecutor

    n_pairs = args.pairs if args.pairs else steps + 1
    # phantoms are drawn on host threads ahead of the steps that use them
    gen = ThreadPoolExecutor(max_workers=8)
    phantoms = [gen.submit(synthdata.phantom, w, i) for i in range(n_pairs)]

    def pair(i):
        truth = phantoms[i].result()
        t = torch.from_numpy(truth.astype(np.float32)).cuda()
        clean = T.tomo_project(ctx, ang_all, t, nb).cpu().numpy()
        d = synthdata.add_gaussian_noise(clean, w.noise_level, synthdata.sinogram_seed(w, i))
        dd = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()
        return t, [dd[torch.from_numpy(p).cuda()].contiguous() for p in parts]

    data = {}

    def get(i):
        k = i % n_pairs
        if k not in data:
            data[k] = pair(k)
        return data[k]

    get(0)
    setup_s = time.perf_counter() - t_setup
    log(f"setup: {n}^2, {w.n_angles} angles, {w.n_nodes} nodes, {iters} unrolled iterations, {setup_s:.1f} s")

    def train_step(i):
        tgt, ds = get(i)
        opt.zero_grad()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = model(ds)
        loss = torch.mean((x - tgt) ** 2)
        loss_v = float(loss.item())
        t1 = time.perf_counter()
        loss.backward()
        opt.step()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return loss_v, t1 - t0, t2 - t1

    train_step(0)                                  # warm-up: plans, allocator
    losses, fw, bw = [], [], []
    t0 = time.perf_counter()
    for i in range(1, steps + 1):
        lv, f, b = train_step(i)
        losses.append(lv)
        fw.append(f)
        bw.append(b)
        if steps <= 20 or i % 32 == 0 or i == steps:
            log(f"step {i}: loss {lv:.6g}, forward {f * 1e3:.0f} ms, backward + Adam {b * 1e3:.0f} ms")
    wall = time.perf_counter() - t0
    fwd_updates = iters * e1 * 2 * w.n_angles * n * n       # P and P^T in the forward unroll
    upd_step = 3 * fwd_updates                               # forward, recomputation, backward
    # the training steps themselves (forward, backward, Adam), without the data
    # synthesis of pairs first used in this run
    ms = float(np.sum(fw) + np.sum(bw)) * 1e3 / steps
    out = {
        "metric": "proj+backproj ray-voxel updates/s; ADMM iter/s batched vs plain @ equal RMSE",
        "value": upd_step / (ms * 1e-3), "unit": "updates/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "differentiation: 1024x1024 random-ellipse phantoms (20 ellipses), 1080 angles, "
                               "1449 bins, Gaussian 1%, 32 nodes interleaved, 10 unrolled ADMM iterations (SEG, "
                               "no quantizer), E1=5, E2=10, learnable rho_k and eta_k (20 scalars), Adam lr 0.05, "
                               "checkpoint every 2 iterations", "n": n, "angles": w.n_angles, "bins": nb,
                   "nodes": w.n_nodes, "unrolled_iterations": iters},
        "projector_tiles": tiles,
        "training": {"pairs": n_pairs, "losses": losses, "forward_ms": float(np.mean(fw)) * 1e3,
                     "step_ms_median": float(np.median(np.array(fw) + np.array(bw))) * 1e3,
                     "backward_adam_ms": float(np.mean(bw)) * 1e3,
                     "backward_over_forward": float(np.mean(bw) / np.mean(fw)),
                     "updates_per_step": upd_step, "forward_updates": fwd_updates,
                     "rho": torch.exp(model.log_rho).tolist(), "eta": torch.exp(model.log_eta).tolist()},
        "setup_s": setup_s,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="single", choices=("single", "batch", "large", "diff"))
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tiles", default=None,
                    help="projector choice instead of autotuning: BAND/JOB_WGS (band kernel) or 'resident'")
    ap.add_argument("--model", default="joseph", choices=("joseph", "chord"),
                    help="system matrix: Joseph interpolation (default) or the chord lengths of Eq. 2")
    ap.add_argument("--xupdate", default="seg", choices=("seg", "avg"),
                    help="x-update of the consensus: Alg. 3 per segment (default) or the Eq. 9 average")
    ap.add_argument("--reg", default=None, choices=("tv", "tikhonov"),
                    help="add a regularization block (the extra ADMM sub-problem) to every slice")
    ap.add_argument("--reg-mu", type=float, default=0.02)
    ap.add_argument("--reg-iters", type=int, default=10, help="Chambolle iterations per z-update (TV)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--pairs", type=int, default=None,
                    help="differentiation workload: seeded phantom/sinogram pairs the steps cycle through "
                         "(default: one per step)")
    ap.add_argument("--no-batch-line", action="store_true",
                    help="skip the batching workload's batched-vs-plain comparison of the default run")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the untimed reconstruction-quality trajectories of the single workload")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch the projector and backprojector of the workload a few times, and a "
                         "device copy of known size (for counter runs); prints their launch counts")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every node of the workload runs on one device "
              "(no multi-GPU path is built); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    steps = args.steps if args.steps is not None else DEFAULT_STEPS[args.workload]
    if args.warmup is None:
        args.warmup = DEFAULT_WARMUP[args.workload]
    n_eq = args.plain_steps if args.plain_steps is not None else EQUAL_RMSE_STEPS[args.workload]

    import numpy as np
    import torch

    import synthdata
    from paper_2410_06106_amd import admm as A
    from paper_2410_06106_amd import autotune
    from paper_2410_06106_amd import tomoadmm as T

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    pool = None
    if args.workload == "single" and not args.no_cpu_baseline and not args.profile_kernels:
        # before anything initialises the GPU: the workers are forked
        w1 = synthdata.WORKLOADS["single"]
        procs = min(8, os.cpu_count() or 1)
        log(f"cpu baseline: oracle local update of nodes 0-7 of 16, {procs} worker processes ...")
        v_pool, wall = cpu_baseline_pool([(w1, 0, m) for m in range(8)], args.model, procs)
        pool = {"value": v_pool, "unit": "updates/s", "cores": procs, "kind": "oracle",
                "sample": f"Alg. 2 local update (E1=5: P and P^T) of nodes 0-7 of 16 (512^2, 45 angles each), "
                          f"float64 NumPy, one process per node, {wall:.1f} s wall"}
    torch.cuda.set_device(0)
    ctx = T.Context(0)
    if args.model == "chord":
        T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_MODEL, 1)
    if args.workload == "diff":
        return bench_diff(args, steps, ctx, log)
    t_setup = time.perf_counter()
    slices, ws, q, desc, cfg, sample, sample_desc = build(args.workload, ctx, A, T, synthdata, log)
    n_slices = len(slices)
    msgs = None
    km_iters = None
    if q.kind == T.TOMO_QUANT_KMEANS:
        n_nodes = sum(len(s.d) for s in slices)
        km_iters = torch.zeros((n_nodes, 1), dtype=torch.int32, device="cuda")
        msgs = T.make_msgs([dict(iters=km_iters[i]) for i in range(n_nodes)])
    reg = None
    if args.reg:
        reg = dict(kind=T.TOMO_REG_TV if args.reg == "tv" else T.TOMO_REG_TIKHONOV, mu=args.reg_mu,
                   tv_iters=args.reg_iters, tau=0.125)
    xmode = T.TOMO_XUPDATE_SEGMENT if args.xupdate == "seg" else T.TOMO_XUPDATE_AVERAGE
    run = A.DADMM(ctx, slices, rho=1.0, eta2=0.2, e1=5, e2=10, mode=xmode, quant=q, msgs=msgs,
                  reg=reg)
    updates_per_step = sum(2 * w.inner_iters * w.n_angles * w.n * w.n for w in ws)
    upd_per_launch = sum(w.n_angles * w.n * w.n for w in ws)
    tiles = None
    if args.tiles:
        if args.tiles == "resident":
            tiles = {"kernel": 1, "band": 32, "job_wgs": 16}
        else:
            band, jw = (int(v) for v in args.tiles.split("/"))
            tiles = {"kernel": 0, "band": band, "job_wgs": jw}
        autotune.apply(ctx, tiles)
    elif args.no_autotune:
        tiles = {"kernel": 0, "band": 32, "job_wgs": 16}       # the context's defaults
    else:
        choice = autotune.tune(ctx, run.nodes, resident=args.model == "joseph")
        tiles = {"kernel": choice["kernel"], "band": choice["band"], "job_wgs": choice["job_wgs"]}
        kind = ("region-resident kernel" if choice["kernel"] == 1 else
                f"band kernel, band {choice['band']}, {choice['job_wgs']} workgroups per node")
        log(f"autotune: {kind} ({choice['us']:.1f} us per projection phase; tried {len(choice['tried'])})")
    setup_s = time.perf_counter() - t_setup
    log(f"setup done in {setup_s:.1f} s")

    if args.profile_kernels:
        reps = 5
        phase_us = {}
        for phase in (0, 1):
            T.admm_local_phase(ctx, run.nodes, phase)      # builds the batched plan
        torch.cuda.synchronize()
        for phase, name in ((0, "project"), (1, "backproject")):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                T.admm_local_phase(ctx, run.nodes, phase)
            e1.record()
            torch.cuda.synchronize()
            phase_us[name] = e0.elapsed_time(e1) / reps * 1e3
        copy_bytes = 1 << 28
        a = torch.empty(copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(reps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_kernels": {"workload": args.workload, "project_launches": reps + 1,
                                              "backproject_launches": reps + 1, "copy_launches": reps,
                                              "copy_bytes": copy_bytes, "updates_per_launch": upd_per_launch,
                                              "tiles": tiles, "event_us_per_phase": phase_us}}), flush=True)
        return

    def zero_all():
        for s in slices:
            s.zero()

    # --- equal-RMSE check: plain per-slice, per-node loop vs batched graph, same iterations
    zero_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_eq):
        run.step_plain()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / n_eq
    rmse_plain = [run.rmse(i) for i in range(n_slices)]
    x_plain = [s.x.clone() for s in slices]
    zero_all()
    for _ in range(args.warmup):
        run.step()                       # builds the batched plans
    zero_all()
    torch.cuda.synchronize()
    # the forms of the captured iteration (bit-identical iterates): the
    # sequential one; the pipelined one, whose next first projection runs
    # concurrently with the consensus on a second stream; and the alternating
    # one (the local updates alternating between the two streams).  Each graph
    # holds ITERS_PER_GRAPH iterations (a replay costs a few us of launch
    # overhead); one-iteration graphs of the sequential and pipelined forms
    # cover a remainder.  A few replays of each form pick the fastest.
    G = ITERS_PER_GRAPH[args.workload]
    graphs = {"sequential": run.capture(G), "pipelined": run.capture(G, pipelined=True)}
    if G % 2 == 0:
        graphs["alternating"] = run.capture(G, pipelined=True, alternate=True)
    single = {"sequential": run.capture(1), "pipelined": run.capture(1, pipelined=True)}

    def replay_iters(form, k):
        """k iterations of a form: whole graphs, then one-iteration graphs (the
        pipelined one for both pipelined forms, which share its state convention)"""
        for _ in range(k // G):
            graphs[form].replay()
        for _ in range(k % G):
            single["sequential" if form == "sequential" else "pipelined"].replay()

    trial_us = {}
    for _ in range(2):                   # alternate the forms; each keeps its best round
        for form, g in graphs.items():
            zero_all()
            if form != "sequential":
                run.prime()
            g.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            n_trial = max(2, steps // 5 // G)
            e0.record()
            for _ in range(n_trial):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / (n_trial * G) * 1e3
            trial_us[form] = min(us, trial_us.get(form, us))
    form = min(trial_us, key=trial_us.get)
    log(f"iteration graph: {form} (trial us per iteration: "
        + ", ".join(f"{k} {v:.1f}" for k, v in trial_us.items()) + ")")
    zero_all()
    if form != "sequential":
        run.prime()
    replay_iters(form, n_eq)
    torch.cuda.synchronize()
    rmse_batched = [run.rmse(i) for i in range(n_slices)]
    identical = all(bool(torch.equal(xp, s.x)) for xp, s in zip(x_plain, slices))
    del x_plain
    log(f"plain loop {n_slices / plain_s:.1f} slice-iterations/s, rmse[0] plain {rmse_plain[0]:.6g} "
        f"batched {rmse_batched[0]:.6g} identical={identical}")

    # --- timed region: K iterations of the graph's form
    replay_iters(form, args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    replay_iters(form, steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(gpu_ms, wall * 1e3) / steps
    value = updates_per_step / (ms_per_step * 1e-3)
    rmse_final = [run.rmse(i) for i in range(n_slices)]
    log(f"batched graph: {ms_per_step:.3f} ms/iteration, {value:.4g} updates/s, rmse[0] {rmse_final[0]:.6g}")

    # --- reconstruction quality on the same data (untimed): RMSE against the
    # phantom after 50, 100 and 200 plain iterations from zero, with the timed
    # form's segment x-update and with the averaging x-update of Eq. 9 (same
    # kernels, same quantizer and step sizes)
    quality = None
    if args.workload == "single" and not args.no_quality:
        quality = {"iterations": [50, 100, 200]}
        for name, mode in (("segment", T.TOMO_XUPDATE_SEGMENT), ("average", T.TOMO_XUPDATE_AVERAGE)):
            rq = A.DADMM(ctx, slices, rho=1.0, eta2=0.2, e1=5, e2=10, mode=mode, quant=q, msgs=None, reg=reg)
            zero_all()
            traj, k = [], 0
            for target in quality["iterations"]:
                while k < target:
                    rq.step()
                    k += 1
                traj.append(rq.rmse(0))
            quality[name] = traj
        log(f"reconstruction RMSE after {quality['iterations']} iterations: segment {quality['segment']}, "
            f"average {quality['average']}")

    # --- local-update phases: average duration with HIP events on the launch stream
    kern = {}
    for phase, name in ((0, "project"), (1, "backproject")):
        T.admm_local_phase(ctx, run.nodes, phase)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.kernel_reps):
            T.admm_local_phase(ctx, run.nodes, phase)
        e1.record()
        torch.cuda.synchronize()
        kern[name] = e0.elapsed_time(e1) / args.kernel_reps
    dom = max(kern, key=kern.get)
    dur_s = kern[dom] * 1e-3
    achieved = ALGO_FLOPS_PER_UPDATE * upd_per_launch / dur_s / 1e12
    traffic = _traffic(dom, args.workload, tiles) if args.model == "joseph" else None
    log("phases: " + ", ".join(f"{k} {v * 1e3:.1f} us ({upd_per_launch / (v * 1e-3):.3g} upd/s)"
                                for k, v in kern.items()))

    lloyd = None
    if km_iters is not None:
        it = km_iters.cpu().numpy().reshape(-1)
        lloyd = {"mean": float(it.mean()), "max": int(it.max()), "min": int(it.min())}
    # --- z-update of the regularization blocks
    zinfo = None
    if run.regs is not None:
        T.admm_reg_update(ctx, run.nodes, run.regs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.kernel_reps):
            T.admm_reg_update(ctx, run.nodes, run.regs)
        e1.record()
        torch.cuda.synchronize()
        z_us = e0.elapsed_time(e1) / args.kernel_reps * 1e3
        px = sum(s.n * s.n for s in slices)
        # algorithmic (minimum) bytes per pixel: TV reads x, nu and the two-plane
        # field and writes the field, z and t_z (32 B/px); Tikhonov reads x, nu and
        # writes z, t_z (16 B/px).  The naive schedule -- one HBM pass per Chambolle
        # iteration (v formed: 12 B/px, each iteration 20 B/px, z and t_z formed:
        # 24 B/px) -- is reported beside it as an equivalent rate, not as HBM traffic.
        per_px = 32 if args.reg == "tv" else 16
        naive_px = (12 + 20 * args.reg_iters + 24) if args.reg == "tv" else 16
        zinfo = {"kind": args.reg, "mu": args.reg_mu, "tv_iters": args.reg_iters if args.reg == "tv" else None,
                 "us": z_us, "algorithmic_bytes": per_px * px,
                 "achieved_GBps": per_px * px / (z_us * 1e-6) / 1e9, "peak_GBps": PEAK_HBM_GBS,
                 "naive_schedule_equivalent_GBps": naive_px * px / (z_us * 1e-6) / 1e9}
        log(f"z-update ({args.reg}): {z_us:.1f} us, {zinfo['achieved_GBps']:.0f} GB/s of the 32 B/px minimum "
            f"({zinfo['naive_schedule_equivalent_GBps']:.0f} GB/s naive-schedule equivalent)")
    # --- consensus (quantized x-update + dual update), same stream; it moves the
    # iterates on, so it runs after everything reported above has been read
    run.consensus(run.nodes, run.msgs, run.regs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.kernel_reps):
        run.consensus(run.nodes, run.msgs, run.regs)
    e1.record()
    torch.cuda.synchronize()
    consensus_us = e0.elapsed_time(e1) / args.kernel_reps * 1e3
    log(f"consensus (x-update, quantizer, dual): {consensus_us:.1f} us")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle local update on {sample_desc} ...")
        v_cpu, dt = cpu_baseline(ws, sample, args.model)
        cpu = {"value": v_cpu, "unit": "updates/s", "cores": 1, "kind": "oracle",
               "sample": f"Alg. 2 local update (E1=5: P and P^T) of {sample_desc}, float64 NumPy, {dt:.1f} s"}

    batching = None
    if args.workload == "single" and not args.no_batch_line:
        batching = batching_line(A, T, synthdata, autotune, log)

    rel = [abs(a - b) / b if b > 0 else 0.0 for a, b in zip(rmse_batched, rmse_plain)]
    out = {
        "metric": "proj+backproj ray-voxel updates/s; ADMM iter/s batched vs plain @ equal RMSE",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict({"workload": desc if args.xupdate == "seg" else desc.replace("SEG x-update", "AVG x-update")},
                       **cfg, system_matrix=args.model,
                       **({"regularization": f"{args.reg} mu={args.reg_mu}"} if args.reg else {})),
        "admm_iters_per_s": {"batched_graph": n_slices * 1e3 / ms_per_step, "plain_loop": n_slices / plain_s,
                             "unit": "slice-iterations/s"},
        "equal_rmse": {"iterations": n_eq, "bit_identical": identical, "max_rel_rmse_diff": max(rel),
                       "plain_slice0": rmse_plain[0], "batched_slice0": rmse_batched[0]},
        "rmse_after_timed_steps": {"slice0": rmse_final[0], "mean": float(np.mean(rmse_final))},
        "reconstruction": quality,
        "batching": batching,
        "kmeans_lloyd_iters_last_step": lloyd,
        "projector_tiles": tiles,
        "iteration_graph": {"form": form, "iterations_per_graph": G, "trial_us": trial_us},
        "regularization": zinfo,
        "phases_us": dict({k: v * 1e3 for k, v in kern.items()}, consensus=consensus_us),
        "roofline": {"bound": "alu", "kernel": PHASE_KERNELS[dom], "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "peak_single_issue": PEAK_FP32_SINGLE_ISSUE_TFLOPS,
                     "frac_single_issue": achieved / PEAK_FP32_SINGLE_ISSUE_TFLOPS,
                     "algorithmic": f"{ALGO_FLOPS_PER_UPDATE:g} flop per ray-voxel update x "
                                    f"{upd_per_launch} updates per launch"},
        "hbm": ({"achieved": traffic / dur_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": traffic / dur_s / 1e9 / PEAK_HBM_GBS} if traffic else None),
        "setup_s": setup_s,
        "cpu_baseline": cpu,
        "cpu_baseline_pool": pool,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
