"""Differentiable decentralized ADMM.

* ``Project``          torch.autograd.Function  s = P u  (Eq. 2-4); backward = P^T
* ``Backproject``      torch.autograd.Function  u = P^T s;           backward = P
* ``ProjectMany``      the same for all nodes at once: U [M][n][n] -> the
                       nodes' sinograms stacked along the angle axis, one
                       launch (tomo_project_many); backward one launch of P^T
* ``BackprojectMany``  its transpose
All run the hand-written gfx950 kernels through the C ABI (float32).

``UnrolledADMM`` unrolls K iterations of Alg. 4 (without the quantizer, which
has no useful gradient) with a learnable penalty rho_k and local step eta_k per
iteration (2K scalars), and checkpoints the iterates (x, u_m, lambda_m) every
``ckpt`` iterations: only the checkpointed states are kept for the backward
pass, the iterations in between are recomputed.  The nodes' u_m and lambda_m
are stacked into [M][n][n] tensors, so every operator and every elementwise
step of an iteration is one launch for all nodes.  Every step of an iteration
is a Function whose forward and backward are HIP kernels (the tomo_unroll_*
calls): ``LocalStep`` (Alg. 2: P, the residual, P^T and the u-step; its
backward applies P^T P to the incoming gradient and forms the gradients of u,
x, lambda, rho and eta, the scalar ones as float64 sums; ``LocalSteps`` runs
E1 of them as one Function whose backward sums the gradients of x, lambda, rho
and eta over the steps in place), ``XSegment`` (Alg. 3),
``XAverage`` (Eq. 9) and ``Dual`` (Eq. 24).  (rho_k, eta_k) enter the kernels
as a two-element device tensor, so learned values never go through the host.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import tomoadmm as T


class Project(torch.autograd.Function):
    @staticmethod
    def forward(fctx, image, angles, n_bins, tctx):
        fctx.save_for_backward(angles)
        fctx.n = image.shape[-1]
        fctx.tctx = tctx
        return T.tomo_project(tctx, angles, image.contiguous(), n_bins)

    @staticmethod
    def backward(fctx, grad):
        (angles,) = fctx.saved_tensors
        g = T.tomo_backproject(fctx.tctx, angles, grad.contiguous(), fctx.n)
        return g, None, None, None


class Backproject(torch.autograd.Function):
    @staticmethod
    def forward(fctx, sino, angles, n, tctx):
        fctx.save_for_backward(angles)
        fctx.n_bins = sino.shape[-1]
        fctx.tctx = tctx
        return T.tomo_backproject(tctx, angles, sino.contiguous(), n)

    @staticmethod
    def backward(fctx, grad):
        (angles,) = fctx.saved_tensors
        g = T.tomo_project(fctx.tctx, angles, grad.contiguous(), fctx.n_bins)
        return g, None, None, None


def project(tctx, image, angles, n_bins):
    return Project.apply(image, angles, n_bins, tctx)


def backproject(tctx, sino, angles, n):
    return Backproject.apply(sino, angles, n, tctx)


def _items(angles, images, sinos, sizes):
    """tomo_proj_item array: node m's image images[m] and its rows of sinos."""
    ents, row = [], 0
    for m, (a, k) in enumerate(zip(angles, sizes)):
        ents.append(dict(angles=a, image=images[m], sino=sinos[row:row + k]))
        row += k
    return T.make_items(ents)


class ProjectMany(torch.autograd.Function):
    @staticmethod
    def forward(fctx, images, tctx, angles, n_bins):
        images = images.contiguous()
        sizes = [int(a.numel()) for a in angles]
        sinos = torch.empty((sum(sizes), n_bins), dtype=torch.float32, device=images.device)
        T.tomo_project_many(tctx, _items(angles, images, sinos, sizes))
        fctx.tctx, fctx.angles, fctx.sizes, fctx.n = tctx, angles, sizes, images.shape[-1]
        return sinos

    @staticmethod
    def backward(fctx, grad):
        grad = grad.contiguous()
        gi = torch.empty((len(fctx.angles), fctx.n, fctx.n), dtype=torch.float32, device=grad.device)
        T.tomo_backproject_many(fctx.tctx, _items(fctx.angles, gi, grad, fctx.sizes), 1.0, 0.0)
        return gi, None, None, None


class BackprojectMany(torch.autograd.Function):
    @staticmethod
    def forward(fctx, sinos, tctx, angles, n):
        sinos = sinos.contiguous()
        sizes = [int(a.numel()) for a in angles]
        images = torch.empty((len(angles), n, n), dtype=torch.float32, device=sinos.device)
        T.tomo_backproject_many(tctx, _items(angles, images, sinos, sizes), 1.0, 0.0)
        fctx.tctx, fctx.angles, fctx.sizes, fctx.n_bins = tctx, angles, sizes, sinos.shape[1]
        return images

    @staticmethod
    def backward(fctx, grad):
        grad = grad.contiguous()
        out = torch.empty((sum(fctx.sizes), fctx.n_bins), dtype=torch.float32, device=grad.device)
        T.tomo_project_many(fctx.tctx, _items(fctx.angles, grad, out, fctx.sizes))
        return out, None, None, None


class LocalStep(torch.autograd.Function):
    """One Alg. 2 step for all nodes: U' = U - eta (P^T (P U - D) + rho (U - x) + L)."""

    @staticmethod
    def forward(fctx, U, x, L, scal, D, tctx, angles, n_bins):
        U = U.contiguous()
        sizes = [int(a.numel()) for a in angles]
        R = torch.empty((sum(sizes), n_bins), dtype=torch.float32, device=U.device)
        # R = P U - D, then the u-step in the backprojector's epilogue
        Uo = T.tomo_unroll_local_step(tctx, _items(angles, U, R, sizes), U, D.contiguous(), x.contiguous(),
                                      L.contiguous(), scal.contiguous())
        fctx.save_for_backward(U, x, L, scal, R)
        fctx.tctx, fctx.angles, fctx.sizes, fctx.n_bins = tctx, angles, sizes, n_bins
        return Uo

    @staticmethod
    def backward(fctx, G):
        U, x, L, scal, R = fctx.saved_tensors
        G = G.contiguous()
        PG = torch.empty_like(R)
        T.tomo_project_many(fctx.tctx, _items(fctx.angles, G, PG, fctx.sizes))
        PtPG = torch.empty_like(U)
        T.tomo_backproject_many(fctx.tctx, _items(fctx.angles, PtPG, PG, fctx.sizes), 1.0, 0.0)
        dU, dL, dx, ds = T.tomo_unroll_ustep_grad(fctx.tctx, G, PtPG, PG, R, U, x.contiguous(), L.contiguous(),
                                                  scal.contiguous())
        return dU, dx, dL, ds, None, None, None, None


class LocalSteps(torch.autograd.Function):
    """E1 Alg. 2 steps for all nodes in one Function, U -> U after ``e1`` steps.
    It keeps every step's input and residual, and its backward runs the steps'
    backward passes in reverse order with the gradients of x, L and (rho, eta)
    summed in place over the steps (one gradient tensor each instead of one per
    step for autograd to add up)."""

    @staticmethod
    def forward(fctx, U, x, L, scal, D, tctx, angles, n_bins, e1):
        U, x, L, scal, D = U.contiguous(), x.contiguous(), L.contiguous(), scal.contiguous(), D.contiguous()
        sizes = [int(a.numel()) for a in angles]
        us, rs = [], []
        for _ in range(e1):
            R = torch.empty((sum(sizes), n_bins), dtype=torch.float32, device=U.device)
            Un = T.tomo_unroll_local_step(tctx, _items(angles, U, R, sizes), U, D, x, L, scal)
            us.append(U)
            rs.append(R)
            U = Un
        fctx.save_for_backward(x, L, scal, *us, *rs)
        fctx.tctx, fctx.angles, fctx.sizes, fctx.e1 = tctx, angles, sizes, e1
        return U

    @staticmethod
    def backward(fctx, G):
        saved = fctx.saved_tensors
        e1 = fctx.e1
        x, L, scal = saved[:3]
        us, rs = saved[3:3 + e1], saved[3 + e1:]
        G = G.contiguous()
        dL = dx = ds = None
        for k in reversed(range(e1)):
            PG = torch.empty_like(rs[k])
            T.tomo_project_many(fctx.tctx, _items(fctx.angles, G, PG, fctx.sizes))
            PtPG = torch.empty_like(G)
            T.tomo_backproject_many(fctx.tctx, _items(fctx.angles, PtPG, PG, fctx.sizes), 1.0, 0.0)
            G, dL, dx, ds = T.tomo_unroll_ustep_grad(fctx.tctx, G, PtPG, PG, rs[k], us[k], x, L, scal, dL=dL, dx=dx,
                                                     ds=ds, accumulate=k != e1 - 1)
        return G, dx, dL, ds, None, None, None, None, None


class XSegment(torch.autograd.Function):
    """Alg. 3 on every node's own rows: E2 steps x <- x - eta2 rho (x - t), t = U_o + L_o / rho."""

    @staticmethod
    def forward(fctx, U, L, x, scal, owner, tctx, eta2, e2):
        U, L, x, scal = U.contiguous(), L.contiguous(), x.contiguous(), scal.contiguous()
        xo = T.tomo_unroll_xseg(tctx, owner, U, L, x, scal, eta2, e2)
        fctx.save_for_backward(U, L, x, scal, owner)
        fctx.tctx, fctx.eta2, fctx.e2 = tctx, eta2, e2
        return xo

    @staticmethod
    def backward(fctx, G):
        U, L, x, scal, owner = fctx.saved_tensors
        dU, dL, dx, ds = T.tomo_unroll_xseg_grad(fctx.tctx, owner, G.contiguous(), U, L, x, scal, fctx.eta2, fctx.e2)
        return dU, dL, dx, ds, None, None, None, None


class SegConsensus(torch.autograd.Function):
    """Alg. 3 on every node's own rows followed by the dual update (Eq. 24), as
    one Function returning (x', L'): its backward forms the gradients of U, L,
    x and (rho, eta) of both steps in one pass (tomo_unroll_seg_dual_grad)."""

    @staticmethod
    def forward(fctx, U, L, x, scal, owner, tctx, eta2, e2):
        U, L, x, scal = U.contiguous(), L.contiguous(), x.contiguous(), scal.contiguous()
        xs = T.tomo_unroll_xseg(tctx, owner, U, L, x, scal, eta2, e2)
        Lo = T.tomo_unroll_dual(tctx, L, U, xs, scal)
        fctx.save_for_backward(U, L, x, xs, scal, owner)
        fctx.tctx, fctx.eta2, fctx.e2 = tctx, eta2, e2
        return xs, Lo

    @staticmethod
    def backward(fctx, Gx, GL):
        U, L, x, xs, scal, owner = fctx.saved_tensors
        dU, dL, dx, ds = T.tomo_unroll_seg_dual_grad(fctx.tctx, owner, Gx.contiguous(), GL.contiguous(), U, L, x, xs,
                                                     scal, fctx.eta2, fctx.e2)
        return dU, dL, dx, ds, None, None, None, None


class XAverage(torch.autograd.Function):
    """Eq. 9: x = mean_m (U_m + L_m / rho)."""

    @staticmethod
    def forward(fctx, U, L, scal, tctx):
        U, L, scal = U.contiguous(), L.contiguous(), scal.contiguous()
        fctx.save_for_backward(L, scal)
        fctx.tctx = tctx
        return T.tomo_unroll_xavg(tctx, U, L, scal)

    @staticmethod
    def backward(fctx, G):
        L, scal = fctx.saved_tensors
        dU, dL, ds = T.tomo_unroll_xavg_grad(fctx.tctx, G.contiguous(), L, scal)
        return dU, dL, ds, None


class Dual(torch.autograd.Function):
    """Eq. 24: L' = L + rho (U - x')."""

    @staticmethod
    def forward(fctx, L, U, xn, scal, tctx):
        L, U, xn, scal = L.contiguous(), U.contiguous(), xn.contiguous(), scal.contiguous()
        fctx.save_for_backward(U, xn, scal)
        fctx.tctx = tctx
        return T.tomo_unroll_dual(tctx, L, U, xn, scal)

    @staticmethod
    def backward(fctx, G):
        U, xn, scal = fctx.saved_tensors
        dL, dU, dxn, ds = T.tomo_unroll_dual_grad(fctx.tctx, G.contiguous(), U, xn, scal)
        return dL, dU, dxn, ds, None


def project_many(tctx, images, angles, n_bins):
    """images [M][n][n] -> sinograms of all nodes stacked along the angle axis."""
    return ProjectMany.apply(images, tctx, angles, n_bins)


def backproject_many(tctx, sinos, angles, n):
    """Stacked sinograms -> [M][n][n] backprojections."""
    return BackprojectMany.apply(sinos, tctx, angles, n)


class UnrolledADMM(torch.nn.Module):
    """K unrolled iterations of Alg. 4 with learnable (rho_k, eta_k).

    ``mode`` 'seg' (Alg. 3 per node segment, E2 steps of size eta2) or 'avg'
    (Eq. 9).  Parameters are stored as logarithms so they stay positive; the
    initial values are rho0 and eta0 for every iteration.
    """

    def __init__(self, tctx, n, n_bins, angles, segments, iters=10, e1=5, e2=10, eta2=0.2,
                 rho0=1.0, eta0=1e-4, mode="seg", ckpt=2):
        super().__init__()
        self.tctx, self.n, self.n_bins = tctx, n, n_bins
        self.angles, self.segments = angles, segments
        self.iters, self.e1, self.e2, self.eta2, self.mode, self.ckpt = iters, e1, e2, eta2, mode, ckpt
        self.log_rho = torch.nn.Parameter(torch.full((iters,), float(torch.log(torch.tensor(rho0)))))
        self.log_eta = torch.nn.Parameter(torch.full((iters,), float(torch.log(torch.tensor(eta0)))))
        # owner node of every image row (segments are disjoint row strips covering x)
        owner = torch.empty(n, dtype=torch.int32)
        for m, (r0, nr) in enumerate(segments):
            owner[r0:r0 + nr] = m
        self.owner = owner

    def tune_projector(self, reps: int = 5) -> dict:
        """Pick the projector launch shape for this model's node batch (the
        autotuner's sweep over tomo_project_many on scratch images) and set it
        on the context; returns the autotuner's choice."""
        from . import autotune
        m, n = len(self.angles), self.n
        sizes = [int(a.numel()) for a in self.angles]
        dev = self.angles[0].device
        U = torch.rand((m, n, n), device=dev, generator=torch.Generator(device=dev).manual_seed(0))
        R = torch.empty((sum(sizes), self.n_bins), device=dev)
        choice = autotune.tune_items(self.tctx, _items(self.angles, U, R, sizes), reps=reps)
        del U, R
        return choice

    def _iteration(self, k, D, x, U, L):
        """One iteration for all nodes: U, L [M][n][n], D the stacked data."""
        scal = torch.stack([torch.exp(self.log_rho[k]), torch.exp(self.log_eta[k])])   # (rho_k, eta_k)
        if self.e1 > 0:                                                         # Alg. 2, E1 steps
            U = LocalSteps.apply(U, x, L, scal, D, self.tctx, self.angles, self.n_bins, self.e1)
        if self.mode == "seg":                                                  # Alg. 3 (Eq. 17), Eq. 24
            x_new, L = SegConsensus.apply(U, L, x, scal, self.owner, self.tctx, self.eta2, self.e2)
        else:                                                                   # Eq. 9
            x_new = XAverage.apply(U, L, scal, self.tctx)
            L = Dual.apply(L, U, x_new, scal, self.tctx)                        # Eq. 18 / 24
        return x_new, U, L

    def _segment(self, k0, k1, D, x, U, L):
        for k in range(k0, k1):
            x, U, L = self._iteration(k, D, x, U, L)
        return x, U, L

    def forward(self, d):
        """d: list of per-node sinograms (float32 cuda).  Returns x after K iterations."""
        n, dev = self.n, d[0].device
        m = len(self.angles)
        D = torch.cat([di.reshape(-1, self.n_bins) for di in d], dim=0)
        if self.owner.device != dev:
            self.owner = self.owner.to(dev)
        x = torch.zeros((n, n), device=dev)
        U = torch.zeros((m, n, n), device=dev)
        L = torch.zeros((m, n, n), device=dev)
        span = self.ckpt if self.ckpt > 0 else self.iters
        k = 0
        while k < self.iters:
            k1 = min(self.iters, k + span)
            if self.ckpt > 0 and torch.is_grad_enabled():
                x, U, L = checkpoint(self._segment, k, k1, D, x, U, L, use_reentrant=False)
            else:
                x, U, L = self._segment(k, k1, D, x, U, L)
            k = k1
        return x
