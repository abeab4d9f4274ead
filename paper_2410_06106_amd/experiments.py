"""Reconstruction-quality studies of Section 3 on the GPU path.

* Fig. 4    the centralized baseline (Alg. 1, ``tomo_ctr_gd``) against
            decentralized ADMM without quantization on 2 and 10 nodes;
* Fig. 5    RMSE as a function of the compression level: K-means with K
            levels (the elbow method of Section 3.3) and the DCT codec at
            several quality factors;
* Fig. 6-7  robustness to Gaussian measurement noise given as NSD (Eq. 27);
* Section 4 the regularization block the discussion proposes (TV or Tikhonov
            as one more ADMM sub-problem) on the noisiest data of Fig. 6-7;
* Eq. 20    per-node traffic of each run from its real messages (K-means
            labels packed by ``tomo_pack_labels`` plus the codebook; DCT codes
            entropy-coded by ``tomo_dct_encode``; float32 segments without
            quantizer) next to the formula.

Every iteration runs in the library's kernels (projector pair, consensus,
quantizers, the centralized step) through the same batched ADMM loop as the
benchmark; the host only builds the inputs, applies the stopping rule of
Section 3.2 (relative change of x below 1e-6) and reports.  Inputs are
synthetic (``synthdata``): a piecewise-constant phantom with three gray levels
stands in for the paper's Phantom image.

    python -m paper_2410_06106_amd.experiments --study elbow [--n 256] [--iters 300] [--json out.json]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np
import torch

import synthdata

from . import admm as A
from . import tomoadmm as T

NSD_LEVELS = (0.24, 0.77, 2.43)        # percent, Section 3.3
ELBOW_LEVELS = (2, 3, 4, 5, 6, 16, 32)
DCT_QUALITIES = (10, 30, 50, 70, 90)


@dataclasses.dataclass
class Run:
    label: str
    method: str               # "ctr" | "dadmm"
    nodes: int
    quant: str                # "none" | "kmeans" | "dct"
    level: int                # K (kmeans), quality (dct), 0 otherwise
    nsd: float                # percent
    iters: int                # outer iterations run
    rmse: float               # at the last iteration
    psnr: float
    best_rmse: float
    best_iter: int
    bits_per_value: float     # exchanged bits per pixel value
    traffic_bytes: int        # per node and iteration: messages sent + received (largest node)
    eq20_bytes: float         # Eq. 20: 2 (M - 1) / M * image bytes * bits / 32
    seconds: float
    trace: list = dataclasses.field(default_factory=list, repr=False)


def _psnr(rmse: float, peak: float) -> float:
    return 20.0 * math.log10(peak / rmse) if rmse > 0 else float("inf")


def make_problem(ctx, w: synthdata.Workload, nsd: float):
    """Phantom, angles and data with Gaussian noise of sigma = nsd % of the
    clean data's peak (host arrays; the clean data come from the GPU projector)."""
    truth = synthdata.phantom(w)
    th = synthdata.angles(w.n_angles)
    clean = T.tomo_project(ctx, torch.from_numpy(th).cuda(), torch.from_numpy(truth).cuda(), w.n_bins)
    d = synthdata.add_gaussian_noise(clean.cpu().numpy(), nsd / 100.0, synthdata.sinogram_seed(w))
    return truth, th, d


class _Stopper:
    """Relative change ||x_new - x_old|| / ||x_old|| through the library's sqdiff."""

    def __init__(self, ctx, x):
        self.ctx, self.x = ctx, x
        self.prev = torch.empty_like(x)
        self.zero = torch.zeros_like(x)

    def save(self):
        self.prev.copy_(self.x)

    def rel_change(self) -> float:
        num = float(T.tomo_sqdiff(self.ctx, self.x, self.prev).item())
        den = float(T.tomo_sqdiff(self.ctx, self.prev, self.zero).item())
        return math.sqrt(num / den) if den > 0 else float("inf")


def run_ctr(ctx, w, truth, th, d, iters: int, c: float = 1.0, tol: float = 1e-6, nsd: float = 0.0,
            eta: float | None = None) -> Run:
    """Alg. 1 from u = 0 with eta = c / ||P^T P|| (or the given ``eta``), until the
    relative change of u drops below ``tol`` or after ``iters`` iterations."""
    ang = torch.from_numpy(th).cuda()
    dd = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()
    tr = torch.from_numpy(truth).cuda()
    u = torch.zeros((w.n, w.n), dtype=torch.float32, device="cuda")
    if eta is None:
        eta = c / A.operator_norm(ctx, ang, w.n, w.n_bins)
    stop, trace = _Stopper(ctx, u), []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        stop.save()
        T.tomo_ctr_gd(ctx, ang, dd, u, eta, 1)
        trace.append(math.sqrt(float(T.tomo_sqdiff(ctx, u, tr).item()) / (w.n * w.n)))
        if it > 0 and stop.rel_change() < tol:
            break
    sec = time.perf_counter() - t0
    best = int(np.argmin(trace))
    peak = float(truth.max())
    return Run("CTR", "ctr", 1, "none", 0, nsd, len(trace), trace[-1], _psnr(trace[-1], peak),
               trace[best], best + 1, 32.0, 0, 0.0, sec, trace)


def run_dadmm(ctx, w, truth, d, quant: str = "none", level: int = 0, iters: int = 1000, c: float = 0.1,
              tol: float = 1e-6, mode: int = T.TOMO_XUPDATE_SEGMENT, nsd: float = 0.0,
              eta1: float | None = None, reg: dict | None = None) -> Run:
    """Alg. 4 on ``w.n_nodes`` nodes with Q = K-means (``level`` = K), the DCT codec
    (``level`` = quality) or none, until the relative change of x drops below
    ``tol`` or after ``iters`` iterations.  eta1 = c / (L + rho) with L the largest
    ||P_m^T P_m|| unless ``eta1`` is given.  ``reg``: a regularization block
    (see ``admm.DADMM``)."""
    s = A.make_slice(ctx, w, d_host=d, truth_host=truth)
    s.eta1 = A.step_size(ctx, s, w.rho, c) if eta1 is None else eta1
    msgs, coeffs = None, []
    if quant == "kmeans":
        q = T.tomo_quant(T.TOMO_QUANT_KMEANS, level, 30, 0)
        bits = float(max(1, math.ceil(math.log2(level))))
        labels = [torch.empty(rows * w.n, dtype=torch.uint8, device="cuda") for _, rows in s.segments]
        cents = [torch.empty(level, dtype=torch.float32, device="cuda") for _ in s.segments]
        msgs = T.make_msgs([dict(labels=lb, centroids=ct) for lb, ct in zip(labels, cents)])
    elif quant == "dct":
        q = T.tomo_quant(T.TOMO_QUANT_DCT, 0, 0, level)
        coeffs = [torch.empty((rows, w.n), dtype=torch.int16, device="cuda") for _, rows in s.segments]
        lohi = [torch.empty(2, dtype=torch.float32, device="cuda") for _ in s.segments]
        msgs = T.make_msgs([dict(coeffs=cf, lohi=lh) for cf, lh in zip(coeffs, lohi)])
        bits = 0.0
    else:
        q, bits = None, 32.0
    run = A.DADMM(ctx, [s], rho=w.rho, eta2=w.eta2, e1=w.inner_iters, e2=w.x_iters, mode=mode, quant=q,
                  msgs=msgs, reg=reg)
    stop, trace = _Stopper(ctx, s.x), []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        stop.save()
        run.step()
        trace.append(run.rmse())
        if it > 0 and stop.rel_change() < tol:
            break
    sec = time.perf_counter() - t0
    rows = [r for _, r in s.segments]
    if quant == "dct":
        # the wire format: the last exchange's codes entropy-coded by
        # tomo_dct_encode, plus the restart table and the level-map range
        msg = []
        for cf, r in zip(coeffs, rows):
            _, _, total = T.tomo_dct_encode(ctx, cf)
            tb = int(total.item()) & 0xFFFFFFFF
            blocks = (r // 8) * (w.n // 8)
            msg.append(4 * ((tb + 31) // 32) + 4 * ((blocks + 63) // 64) + 8)
        bits = 8.0 * sum(msg) / (w.n * w.n)
    elif quant == "kmeans":
        # the wire format: labels packed at ceil(log2 K) bits plus the codebook
        msg = [4 * T.tomo_pack_labels(ctx, lb, int(bits)).numel() + 4 * level for lb in labels]
    else:
        msg = [4 * r * w.n for r in rows]
    m_nodes = len(msg)
    traffic = max((m_nodes - 1) * own + sum(msg) - own for own in msg)
    eq20 = 2.0 * (m_nodes - 1) / m_nodes * 4.0 * w.n * w.n * bits / 32.0
    best = int(np.argmin(trace))
    peak = float(truth.max())
    label = {"none": "dADMM", "kmeans": f"dADMM-K K={level}", "dct": f"dADMM-J q={level}"}[quant]
    if reg is not None:
        label += f" +{'TV' if reg['kind'] == T.TOMO_REG_TV else 'Tikhonov'} mu={reg['mu']:g}"
    return Run(f"{label} M={w.n_nodes}", "dadmm", w.n_nodes, quant, level, nsd, len(trace), trace[-1],
               _psnr(trace[-1], peak), trace[best], best + 1, bits, traffic, eq20, sec, trace)


def study_ctr(ctx, w, iters, nsd=0.0, node_counts=(2, 10)):
    """Fig. 4: CTR against unquantized dADMM on 2 and 10 nodes."""
    truth, th, d = make_problem(ctx, w, nsd)
    out = [run_ctr(ctx, w, truth, th, d, iters, nsd=nsd)]
    for m in node_counts:
        out.append(run_dadmm(ctx, dataclasses.replace(w, n_nodes=m), truth, d, "none", 0, iters, nsd=nsd))
    return out


def study_elbow(ctx, w, iters, nsd=0.0, levels=ELBOW_LEVELS, qualities=DCT_QUALITIES):
    """Fig. 5: RMSE against the K-means level count and the DCT quality."""
    truth, _, d = make_problem(ctx, w, nsd)
    out = [run_dadmm(ctx, w, truth, d, "kmeans", k, iters, nsd=nsd) for k in levels]
    out += [run_dadmm(ctx, w, truth, d, "dct", q, iters, nsd=nsd) for q in qualities]
    return out


def study_noise(ctx, w, iters, k=3, quality=30, nsds=(0.0,) + NSD_LEVELS):
    """Fig. 6-7: dADMM-K and dADMM-J at increasing noise."""
    out = []
    for nsd in nsds:
        truth, _, d = make_problem(ctx, w, nsd)
        out.append(run_dadmm(ctx, w, truth, d, "kmeans", k, iters, nsd=nsd))
        out.append(run_dadmm(ctx, w, truth, d, "dct", quality, iters, nsd=nsd))
    return out


def study_reg(ctx, w, iters, nsd=NSD_LEVELS[-1], k=3, mus=(0.01, 0.05, 0.2)):
    """Section 4: the regularization block on the noisiest data of Fig. 6-7,
    dADMM-K (K = 3) alone, with a TV block (10 Chambolle iterations per
    z-update) at several weights, and with a Tikhonov block."""
    truth, _, d = make_problem(ctx, w, nsd)
    out = [run_dadmm(ctx, w, truth, d, "kmeans", k, iters, nsd=nsd)]
    for mu in mus:
        out.append(run_dadmm(ctx, w, truth, d, "kmeans", k, iters, nsd=nsd,
                             reg=dict(kind=T.TOMO_REG_TV, mu=mu, tv_iters=10)))
    out.append(run_dadmm(ctx, w, truth, d, "kmeans", k, iters, nsd=nsd,
                         reg=dict(kind=T.TOMO_REG_TIKHONOV, mu=mus[1])))
    return out


STUDIES = {"ctr": study_ctr, "elbow": study_elbow, "noise": study_noise, "reg": study_reg}


def table(runs) -> str:
    rows = ["| run | NSD % | iterations | RMSE | PSNR dB | best RMSE (iteration) | bits/value | "
            "traffic/node/iter B (Eq. 20) | seconds |",
            "|---|---|---|---|---|---|---|---|---|"]
    for r in runs:
        traffic = f"{r.traffic_bytes} ({r.eq20_bytes:.0f})" if r.method == "dadmm" else "-"
        rows.append(f"| {r.label} | {r.nsd:g} | {r.iters} | {r.rmse:.4g} | {r.psnr:.2f} | "
                    f"{r.best_rmse:.4g} ({r.best_iter}) | {r.bits_per_value:.3g} | {traffic} | {r.seconds:.2f} |")
    return "\n".join(rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--study", choices=sorted(STUDIES) + ["all"], default="all")
    ap.add_argument("--n", type=int, default=None, help="image side instead of the workload's (bins and "
                    "angles scale with it)")
    ap.add_argument("--iters", type=int, default=None, help="outer iterations (default: the workload's)")
    ap.add_argument("--nsd", type=float, default=0.0, help="noise of the ctr and elbow studies, percent")
    ap.add_argument("--json", default=None, help="write every run, traces included, to this file")
    ap.add_argument("--model", default="joseph", choices=("joseph", "chord"),
                    help="system matrix: Joseph interpolation or the chord lengths of Eq. 2")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("experiments: no GPU visible; this module runs the library's kernels only")
    w = synthdata.WORKLOADS["elbow"]
    if args.n:
        scale = args.n / w.n
        w = dataclasses.replace(w, n=args.n, n_angles=max(w.n_nodes, round(w.n_angles * scale)),
                                n_bins=math.ceil(math.sqrt(2.0) * args.n))
    iters = args.iters or w.outer_iters
    ctx = T.Context()
    if args.model == "chord":
        T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_MODEL, 1)
    runs = []
    for name in (sorted(STUDIES) if args.study == "all" else [args.study]):
        print(f"== {name}: {w.n}x{w.n}, {w.n_angles} angles, {w.n_bins} bins, up to {iters} iterations, "
              f"{args.model} system matrix", flush=True)
        kw = {} if name in ("noise", "reg") else {"nsd": args.nsd}
        res = STUDIES[name](ctx, w, iters, **kw)
        print(table(res), flush=True)
        runs += res
    if args.json:
        with open(args.json, "w") as fh:
            json.dump([dataclasses.asdict(r) for r in runs], fh)


if __name__ == "__main__":
    main()
