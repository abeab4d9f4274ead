"""Drivers of decentralized ADMM (Alg. 4) on one GPU.

All nodes of all slices are logical nodes on one device.  Two launch forms
compute the same iteration:

* ``step_plain``   the per-slice, per-node launch loop: one admm_local_update
                   call per node, one admm_consensus call per slice;
* ``step``         the batched form: one admm_local_update and one
                   admm_consensus call for every node of every slice, which can
                   be captured once into a HIP graph (``capture``) and replayed.

Problem set-up (phantom, data, step sizes) is host-side plumbing: phantoms come
from ``synthdata``, clean data from the GPU projector, noise from ``synthdata``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

import synthdata

from . import tomoadmm as T


@dataclass
class SliceState:
    n: int
    n_bins: int
    angles: list                 # per node: float64 cuda [K_m]
    d: list                      # per node: float32 cuda [K_m][B]
    segments: list               # per node: (row0, rows)
    u: list = field(default_factory=list)
    lam: list = field(default_factory=list)
    x: torch.Tensor | None = None
    truth: torch.Tensor | None = None
    eta1: float = 0.0
    reg: dict | None = None      # regularization block: z, nu, tz [n][n], p [2][n][n]

    def allocate(self, device):
        self.u = [torch.zeros((self.n, self.n), dtype=torch.float32, device=device) for _ in self.d]
        self.lam = [torch.zeros((self.n, self.n), dtype=torch.float32, device=device) for _ in self.d]
        self.x = torch.zeros((self.n, self.n), dtype=torch.float32, device=device)

    def allocate_reg(self):
        """Buffers of a regularization block for this slice (zero)."""
        dev = self.x.device
        self.reg = {k: torch.zeros((self.n, self.n), dtype=torch.float32, device=dev) for k in ("z", "nu", "tz")}
        self.reg["p"] = torch.zeros((2, self.n, self.n), dtype=torch.float32, device=dev)

    def zero(self):
        for t in self.u + self.lam + [self.x] + (list(self.reg.values()) if self.reg else []):
            t.zero_()


def operator_norm(ctx, angles, n, n_bins, iters=30, seed=0):
    """||P^T P||_2 by power iteration through the GPU projector pair (set-up only)."""
    dev = angles.device
    v = torch.from_numpy(np.random.default_rng(seed).standard_normal((n, n)).astype(np.float32)).to(dev)
    v /= torch.linalg.vector_norm(v)
    lam = 0.0
    sino = torch.empty((angles.numel(), n_bins), dtype=torch.float32, device=dev)
    w = torch.empty_like(v)
    for _ in range(iters):
        T.tomo_project(ctx, angles, v, n_bins, out=sino)
        T.tomo_backproject(ctx, angles, sino, n, out=w)
        lam = float(torch.sum(w.double() * v.double()))
        v = w / torch.linalg.vector_norm(w)
    return lam


def make_slice(ctx, w: synthdata.Workload, slice_idx=0, device="cuda", d_host=None, truth_host=None):
    """Build one slice on the device: phantom, angles per node, noisy data."""
    n, nb = w.n, w.n_bins
    th = synthdata.angles(w.n_angles)
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    if truth_host is None:
        truth_host = synthdata.phantom(w, slice_idx)
    truth = torch.from_numpy(np.ascontiguousarray(truth_host, dtype=np.float32)).to(device)
    ang_all = torch.from_numpy(th).to(device)
    if d_host is None:
        clean = T.tomo_project(ctx, ang_all, truth, nb).cpu().numpy()
        seed = synthdata.sinogram_seed(w, slice_idx)
        if w.noise == "poisson":
            d_host = synthdata.poisson_noisy(clean, w.noise_level, n, seed)
        else:
            d_host = synthdata.add_gaussian_noise(clean, w.noise_level, seed)
    d_all = torch.from_numpy(np.ascontiguousarray(d_host, dtype=np.float32)).to(device)
    angles = [ang_all[torch.from_numpy(p).to(device)].contiguous() for p in parts]
    d = [d_all[torch.from_numpy(p).to(device)].contiguous() for p in parts]
    s = SliceState(n, nb, angles, d, synthdata.segment_rows(n, w.n_nodes), truth=truth)
    s.allocate(device)
    return s


class DADMM:
    """Alg. 4 over one or many slices, all nodes on one GPU."""

    def __init__(self, ctx, slices, rho=1.0, eta2=0.2, e1=5, e2=10, mode=T.TOMO_XUPDATE_SEGMENT,
                 quant: T.tomo_quant | None = None, msgs=None, reg: dict | None = None):
        """``reg``: a regularization block for every slice, dict(kind=T.TOMO_REG_TV
        or T.TOMO_REG_TIKHONOV, mu, and for TV tv_iters, tau); its penalty is rho."""
        self.ctx, self.slices = ctx, slices
        self.rho, self.eta2, self.e1, self.e2, self.mode, self.quant = rho, eta2, e1, e2, mode, quant
        entries, self.slice_ranges = [], []
        for si, s in enumerate(slices):
            start = len(entries)
            for m in range(len(s.d)):
                r0, nr = s.segments[m]
                entries.append(dict(n=s.n, n_bins=s.n_bins, angles=s.angles[m], slice=si, d=s.d[m],
                                    u=s.u[m], lam=s.lam[m], x=s.x, seg_row0=r0, seg_rows=nr,
                                    rho=rho, eta1=s.eta1, eta2=eta2))
            self.slice_ranges.append((start, len(entries)))
        self.entries = entries
        self.nodes = T.make_nodes(entries)
        self.msgs = msgs
        # per-node and per-slice arrays for the plain launch loop
        self.single = [T.make_nodes([e]) for e in entries]
        self.per_slice = [T.make_nodes(entries[a:b]) for a, b in self.slice_ranges]
        self.graph = None
        self.regs, self.regs_per_slice = None, None
        if reg is not None:
            ents = []
            for si, s in enumerate(slices):
                if s.reg is None:
                    s.allocate_reg()
                ents.append(dict(slice=si, kind=reg["kind"], mu=reg["mu"], rho=rho, tv_iters=reg.get("tv_iters", 10),
                                 tau=reg.get("tau", 0.125), **s.reg))
            self.regs = T.make_regs(ents)
            self.regs_per_slice = [T.make_regs([e]) for e in ents]

    def consensus(self, nodes, msgs, regs, stream=None):
        """The consensus call of the listed nodes, with the regularization blocks if any."""
        if regs is None:
            T.admm_consensus(self.ctx, nodes, self.mode, self.e2, self.quant, msgs, stream)
        else:
            T.admm_consensus_reg(self.ctx, nodes, self.mode, self.e2, self.quant, msgs, regs, stream)

    def step(self, stream=None):
        if self.regs is not None:
            T.admm_reg_update(self.ctx, self.nodes, self.regs, stream)
        T.admm_local_update(self.ctx, self.nodes, self.e1, stream)
        self.consensus(self.nodes, self.msgs, self.regs, stream)

    def step_plain(self, stream=None):
        for si, (a, b) in enumerate(self.slice_ranges):
            if self.regs is not None:
                T.admm_reg_update(self.ctx, self.per_slice[si], self.regs_per_slice[si], stream)
            for i in range(a, b):
                T.admm_local_update(self.ctx, self.single[i], self.e1, stream)
            self.consensus(self.per_slice[si], None, None if self.regs is None else self.regs_per_slice[si],
                            stream)

    def prime(self, stream=None):
        """First projection of the next pipelined iteration (see step_pipelined);
        call it once after the state was set, before the first step_pipelined."""
        T.admm_local_phase(self.ctx, self.nodes, 0, stream)

    def step_pipelined(self, side):
        """One iteration whose first projection (residual P_m u_m - d_m) was
        launched by prime() or by the previous call.  With regularization
        blocks, their z-update runs on stream ``side`` beside the local update.  At its end the next
        iteration's first projection runs on stream ``side`` concurrently with
        this iteration's consensus: it reads only u_m and d_m, which the
        consensus (x-update, quantizer, dual update) does not write, and writes
        only the residual, which the consensus does not read.  Every kernel sees
        the same inputs as in step(), so the iterates are bit-identical."""
        if self.e1 < 1:
            raise ValueError("the pipelined iteration needs E1 >= 1")
        main = torch.cuda.current_stream()
        zdone = None
        if self.regs is not None:
            # the z-update reads x^k and nu^k, which the local update does not
            # touch: it runs on the side stream beside the local update
            side.wait_stream(main)
            with torch.cuda.stream(side):
                T.admm_reg_update(self.ctx, self.nodes, self.regs)
            zdone = torch.cuda.Event()
            zdone.record(side)
        T.admm_local_phase(self.ctx, self.nodes, 1)
        for _ in range(self.e1 - 1):
            T.admm_local_phase(self.ctx, self.nodes, 0)
            T.admm_local_phase(self.ctx, self.nodes, 1)
        if zdone is not None:
            main.wait_event(zdone)
        ready = torch.cuda.Event()
        ready.record(main)
        # the consensus is issued first so that its few large workgroups reach
        # the CUs before the projector's fill them
        self.consensus(self.nodes, self.msgs, self.regs)
        side.wait_event(ready)
        with torch.cuda.stream(side):
            T.admm_local_phase(self.ctx, self.nodes, 0)
        main.wait_stream(side)

    def step_pipelined_pair(self, a, b):
        """Two pipelined iterations whose local updates alternate between streams
        ``a`` and ``b`` (the first projection of the first was launched on ``a``
        by prime() or the previous pair; call it with ``a`` current).  Each
        next first projection runs on the other stream beside the consensus,
        and that stream then carries the next local update: it waits for the
        consensus only after its projection, when the consensus has usually
        finished, so neither stream idles at that wait (the one-stream form
        joins the side stream back at every iteration).  Bit-identical to
        step()."""
        if self.e1 < 1:
            raise ValueError("the pipelined iteration needs E1 >= 1")
        done = None
        for s, other in ((a, b), (b, a)):
            with torch.cuda.stream(s):
                if done is not None:
                    s.wait_event(done)                 # x and lambda of the last consensus
                if self.regs is not None:
                    T.admm_reg_update(self.ctx, self.nodes, self.regs)
                T.admm_local_phase(self.ctx, self.nodes, 1)
                for _ in range(self.e1 - 1):
                    T.admm_local_phase(self.ctx, self.nodes, 0)
                    T.admm_local_phase(self.ctx, self.nodes, 1)
                ready = torch.cuda.Event()
                ready.record(s)
                # consensus first: its few large workgroups reach the CUs
                # before the projector's fill them
                self.consensus(self.nodes, self.msgs, self.regs)
                done = torch.cuda.Event()
                done.record(s)
            other.wait_event(ready)
            with torch.cuda.stream(other):
                T.admm_local_phase(self.ctx, self.nodes, 0)
        a.wait_event(done)

    def capture(self, iters_per_graph=1, pipelined=False, alternate=False):
        """Capture ``iters_per_graph`` batched iterations into a HIP graph (after one
        uncaptured call has built the plans).  ``pipelined``: the iterations are
        step_pipelined ones (fork/join inside the graph), or with ``alternate``
        step_pipelined_pair ones (``iters_per_graph`` even); call prime() before
        the first replay and again whenever the state was reset."""
        if alternate and (not pipelined or iters_per_graph % 2):
            raise ValueError("the alternating form is pipelined, two iterations at a time")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        side = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                if alternate:
                    for _ in range(iters_per_graph // 2):
                        self.step_pipelined_pair(s, side)
                else:
                    for _ in range(iters_per_graph):
                        if pipelined:
                            self.step_pipelined(side)
                        else:
                            self.step()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def rmse(self, si=0):
        s = self.slices[si]
        out = T.tomo_sqdiff(self.ctx, s.x, s.truth)
        return math.sqrt(float(out.item()) / (s.n * s.n))


def step_size(ctx, s: SliceState, rho: float, c: float) -> float:
    """eta1 = c / (L + rho), L = max over nodes of ||P_m^T P_m||."""
    L = max(operator_norm(ctx, a, s.n, s.n_bins) for a in s.angles)
    return c / (L + rho)
