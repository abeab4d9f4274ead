"""Autotuner of the projector's launch shape for a list of nodes.

The forward projector has two kernels and, for the band-streamed one, two
shape choices (see ``tomo_set_option`` in the C header): the band depth staged
in LDS per pass (16 or 32 image lines) and how many workgroups a node should
span before its image is split into smaller regions; the region-resident
kernel has none.  The best pair depends on the image size, the angles per node and the
number of nodes launched together, so it is measured: every candidate pair is
set on the context, the batched projection phase (``admm_local_phase`` phase 0,
which reads u and writes the residual only) is launched a few times, timed
with HIP events on the launch stream, and the fastest pair is kept.

Results are cached in a JSON file keyed by the device name and the multiset of
node shapes, so a workload is tuned once per device.  The choice changes only
the floating-point summation order of the projector (each pair is
bit-reproducible), never the set of operations.
"""
from __future__ import annotations

import json
import os
from collections import Counter

import torch

from . import tomoadmm as T

BANDS = (16, 32)
MAX_RESIDENT_N = 2048          # the region-resident kernel's largest image side
JOB_WGS = (8, 16, 32, 48, 64, 128)


def signature(nodes) -> str:
    """Device and node shapes (n, bins, angles) with multiplicities."""
    shapes = Counter((int(nd.g.n), int(nd.g.n_bins), int(nd.n_ang)) for nd in nodes)
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    body = ";".join(f"{n}x{b}x{k}*{c}" for (n, b, k), c in sorted(shapes.items()))
    return f"{dev}|{body}"


def _time_phase(ctx, nodes, reps: int) -> float:
    T.admm_local_phase(ctx, nodes, 0)          # builds the plan for these options
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        T.admm_local_phase(ctx, nodes, 0)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3      # microseconds


def apply(ctx, choice: dict):
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_KERNEL, int(choice.get("kernel", 0)))
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_BAND, int(choice["band"]))
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_JOB_WGS, int(choice["job_wgs"]))


def tune(ctx, nodes, cache_path: str | None = None, reps: int = 5, bands=BANDS, job_wgs=JOB_WGS,
         resident: bool = True) -> dict:
    """Pick and set the fastest projector (kernel, band, job_wgs) for ``nodes``
    (a ``make_nodes`` array).  ``resident`` offers the region-resident kernel too
    (it serves the Joseph model only).  Returns {"kernel", "band", "job_wgs",
    "us", "tried": {...}, "cached": bool}."""
    key = signature(nodes) + ("" if resident else "|band-only")
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        choice = dict(cache[key], cached=True)
        apply(ctx, choice)
        return choice
    tried = {}
    for band in bands:
        for jw in job_wgs:
            apply(ctx, {"kernel": 0, "band": band, "job_wgs": jw})
            tried[f"0/{band}/{jw}"] = _time_phase(ctx, nodes, reps)
    if resident and all(int(nd.g.n) <= MAX_RESIDENT_N for nd in nodes):
        apply(ctx, {"kernel": 1, "band": bands[-1], "job_wgs": job_wgs[0]})
        tried[f"1/{bands[-1]}/{job_wgs[0]}"] = _time_phase(ctx, nodes, reps)
    best = min(tried, key=tried.get)
    kernel, band, jw = (int(v) for v in best.split("/"))
    choice = {"kernel": kernel, "band": band, "job_wgs": jw, "us": tried[best], "tried": tried}
    apply(ctx, choice)
    if cache_path:
        cache[key] = choice
        d = os.path.dirname(cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return dict(choice, cached=False)


def _time_items(ctx, items, reps: int) -> float:
    T.tomo_project_many(ctx, items)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        T.tomo_project_many(ctx, items)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3      # microseconds


def tune_items(ctx, items, reps: int = 5, bands=BANDS, job_wgs=JOB_WGS, resident: bool = True) -> dict:
    """The same sweep for a ``tomo_project_many`` item list (``make_items``; the
    items' images and sinograms are read and overwritten by the trial
    launches): every (band, job_wgs) pair, and the region-resident kernel when
    ``resident`` and every image fits it, timed on the batch; the fastest is
    set on the context.  Returns {"kernel", "band", "job_wgs", "us", "tried"}."""
    tried = {}
    for band in bands:
        for jw in job_wgs:
            apply(ctx, {"kernel": 0, "band": band, "job_wgs": jw})
            tried[f"0/{band}/{jw}"] = _time_items(ctx, items, reps)
    if resident and all(int(it.g.n) <= MAX_RESIDENT_N for it in items):
        apply(ctx, {"kernel": 1, "band": bands[-1], "job_wgs": job_wgs[0]})
        tried[f"1/{bands[-1]}/{job_wgs[0]}"] = _time_items(ctx, items, reps)
    best = min(tried, key=tried.get)
    kernel, band, jw = (int(v) for v in best.split("/"))
    choice = {"kernel": kernel, "band": band, "job_wgs": jw, "us": tried[best], "tried": tried}
    apply(ctx, choice)
    return choice
