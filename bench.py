"""Benchmark of the decentralized-ADMM hot path on one MI355X.

One step = one outer iteration of Alg. 4 over every node of the 512 x 512,
720-angle, 725-bin, 16-node workload (contiguous angle blocks, Poisson data at
1e5 photons, SEG x-update, K-means with 8 levels): E1 = 5 local steps (Joseph
projection, residual, matched backprojection, u-step) per node, the segment
x-update with K-means exchange, and the dual update.  The iteration is launched
in its batched form and replayed from a HIP graph; inputs are resident on the
device before timing starts.

value = (ray-voxel updates in P + in P^T) per second = 2 E1 K N^2 / step time.
Also reported: ADMM iterations/s of the batched graph and of the plain
per-node launch loop, and their RMSE after the same iterations (equal by
construction: a node's work decomposes identically in both forms).

    python bench.py [--gpus 1] [--steps 100] [--warmup 3] [--no-cpu-baseline]
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
PEAK_FP32_TFLOPS = 157.3           # MI355X vector FP32 (published)
PEAK_HBM_GBS = 8000.0
PHASE_KERNELS = {"project": "projection phase: k_project + k_project_reduce",
                 "backproject": "backprojection phase: k_backproject"}
KERNEL_SOURCES = ("paper_2410_06106_amd/csrc/project.hip", "paper_2410_06106_amd/csrc/backproject.hip",
                  "paper_2410_06106_amd/csrc/common.h")


def _source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_single512.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != _source_sha(KERNEL_SOURCES):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(w, sample_nodes=8):
    """The oracle's Alg. 2 local update (E1 steps of P and P^T) on a sample of
    the workload's nodes, timed on the host; returns ray-voxel updates/s."""
    import numpy as np

    import synthdata
    from oracle import admm as oadmm
    from oracle import joseph

    th = synthdata.angles(w.n_angles)
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    truth = synthdata.phantom(w)
    rng = np.random.default_rng(0)
    n = w.n
    upd = 0
    t0 = time.perf_counter()
    for m in range(sample_nodes):
        d = joseph.project(truth, th[parts[m]], w.n_bins) if m == 0 else d0
        d0 = d
        u = rng.random((n, n))
        oadmm.local_update(u, np.zeros((n, n)), np.zeros((n, n)), d, th[parts[m]], 1.0, 1e-5, w.inner_iters)
        upd += 2 * w.inner_iters * len(parts[m]) * n * n
    dt = time.perf_counter() - t0
    return upd / dt, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch the projector and backprojector of the workload a few times, and a "
                         "device copy of known size (for counter runs); prints their launch counts")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every node of the workload runs on one device "
              "(no multi-GPU path is built); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthdata
    from paper_2410_06106_amd import admm as A
    from paper_2410_06106_amd import tomoadmm as T

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    ctx = T.Context(0)
    w = synthdata.WORKLOADS["single"]
    log(f"setup: {w.n}^2, {w.n_angles} angles, {w.n_bins} bins, {w.n_nodes} nodes")
    s = A.make_slice(ctx, w)
    rho, c_seg = w.rho, 0.1
    s.eta1 = A.step_size(ctx, s, rho, c_seg)
    q = T.tomo_quant(T.TOMO_QUANT_KMEANS, w.levels, 30, 50)
    km_iters = torch.zeros((w.n_nodes, 1), dtype=torch.int32, device="cuda")
    km_cent = torch.zeros((w.n_nodes, w.levels), dtype=torch.float32, device="cuda")
    msgs = T.make_msgs([dict(iters=km_iters[m], centroids=km_cent[m]) for m in range(w.n_nodes)])
    run = A.DADMM(ctx, [s], rho=rho, eta2=w.eta2, e1=w.inner_iters, e2=w.x_iters,
                  mode=T.TOMO_XUPDATE_SEGMENT, quant=q, msgs=msgs)
    updates_per_step = 2 * w.inner_iters * w.n_angles * w.n * w.n

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
        print(json.dumps({"profile_kernels": {"project_launches": reps + 1, "backproject_launches": reps + 1,
                                              "copy_launches": reps, "copy_bytes": copy_bytes,
                                              "updates_per_launch": w.n_angles * w.n * w.n,
                                              "event_us_per_phase": phase_us}}), flush=True)
        return

    # --- equal-RMSE check: plain per-node loop vs batched graph, same iterations
    n_eq = args.plain_steps
    s.zero()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_eq):
        run.step_plain()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / n_eq
    rmse_plain = run.rmse()
    x_plain = s.x.clone()
    s.zero()
    for _ in range(args.warmup):
        run.step()                       # builds the batched plans
    s.zero()
    torch.cuda.synchronize()
    graph = run.capture(1)
    s.zero()
    for _ in range(n_eq):
        graph.replay()
    torch.cuda.synchronize()
    rmse_batched = run.rmse()
    identical = bool(torch.equal(x_plain, s.x))
    log(f"plain loop {1.0 / plain_s:.1f} it/s, rmse plain {rmse_plain:.6g} batched {rmse_batched:.6g} "
        f"identical={identical}")

    # --- timed region: K replays of the one-iteration graph
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    value = updates_per_step / (ms_per_step * 1e-3)
    rmse_final = run.rmse()
    lloyd = km_iters.cpu().numpy().reshape(-1)
    log(f"batched graph: {ms_per_step:.3f} ms/iteration, {value:.4g} updates/s, rmse {rmse_final:.6g}")

    # --- dominant kernels: average launch duration with HIP events on the launch stream
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
    upd_per_launch = w.n_angles * w.n * w.n
    dom = max(kern, key=kern.get)
    dur_s = kern[dom] * 1e-3
    achieved = ALGO_FLOPS_PER_UPDATE * upd_per_launch / dur_s / 1e12
    traffic = _traffic(dom)
    log(f"kernels: " + ", ".join(f"{k} {v * 1e3:.1f} us ({upd_per_launch / (v * 1e-3):.3g} upd/s)"
                                  for k, v in kern.items()))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle local update on 8 of 16 nodes ...")
        v_cpu, dt = cpu_baseline(w)
        cpu = {"value": v_cpu, "unit": "updates/s", "cores": 1, "kind": "oracle",
               "sample": f"Alg. 2 local update (E1={w.inner_iters}: P and P^T) of nodes 0-7 of {w.n_nodes}, "
                         f"{w.n}^2, {w.n_angles // w.n_nodes} angles each, float64 NumPy, {dt:.1f} s"}

    out = {
        "metric": "proj+backproj ray-voxel updates/s; ADMM iter/s batched vs plain @ equal RMSE",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single-GPU plain method: 512x512 random-ellipse phantom (20 ellipses), "
                               "720 angles, 725 bins, Poisson 1e5, 16 nodes contiguous, SEG x-update, "
                               "K-means 8 levels, E1=5, E2=10, rho=1",
                   "n": w.n, "angles": w.n_angles, "bins": w.n_bins, "nodes": w.n_nodes},
        "admm_iters_per_s": {"batched_graph": 1e3 / ms_per_step, "plain_loop": 1.0 / plain_s},
        "equal_rmse": {"iterations": n_eq, "plain": rmse_plain, "batched": rmse_batched,
                       "bit_identical": identical},
        "rmse_after_timed_steps": rmse_final,
        "kmeans_lloyd_iters_last_step": {"mean": float(lloyd.mean()), "max": int(lloyd.max()),
                                          "min": int(lloyd.min())},
        "kernels_us": {k: v * 1e3 for k, v in kern.items()},
        "roofline": {"bound": "alu", "kernel": PHASE_KERNELS[dom], "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic,
                     "algorithmic": f"{ALGO_FLOPS_PER_UPDATE:g} flop per ray-voxel update x "
                                    f"{upd_per_launch} updates per launch"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
