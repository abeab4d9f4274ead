"""Differentiable decentralized ADMM.

* ``Project``      torch.autograd.Function  s = P u  (Eq. 2-4); backward = P^T
* ``Backproject``  torch.autograd.Function  u = P^T s;           backward = P
Both run the hand-written gfx950 kernels through the C ABI (float32).

``UnrolledADMM`` unrolls K iterations of Alg. 4 (without the quantizer, which
has no useful gradient) with a learnable penalty rho_k and local step eta_k per
iteration (2K scalars), and checkpoints the iterates (x, u_m, lambda_m) every
``ckpt`` iterations: only the checkpointed states are kept for the backward
pass, the iterations in between are recomputed.
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

    def _iteration(self, k, d, x, us, lams):
        rho = torch.exp(self.log_rho[k])
        eta = torch.exp(self.log_eta[k])
        new_u = []
        for m, a in enumerate(self.angles):
            u = us[m]
            for _ in range(self.e1):                                   # Alg. 2
                r = project(self.tctx, u, a, self.n_bins) - d[m]
                g = backproject(self.tctx, r, a, self.n) + rho * (u - x) + lams[m]
                u = u - eta * g
            new_u.append(u)
        if self.mode == "seg":                                          # Alg. 3
            parts = []
            for m, (r0, nr) in enumerate(self.segments):
                xs = x[r0:r0 + nr]
                t = new_u[m][r0:r0 + nr] + lams[m][r0:r0 + nr] / rho
                for _ in range(self.e2):
                    xs = xs - self.eta2 * rho * (xs - t)
                parts.append(xs)
            x_new = torch.cat(parts, dim=0)                             # Eq. 17
        else:
            x_new = sum(u + l / rho for u, l in zip(new_u, lams)) / len(new_u)   # Eq. 9
        new_l = [l + rho * (u - x_new) for u, l in zip(new_u, lams)]    # Eq. 18
        return x_new, new_u, new_l

    def _segment(self, k0, k1, d, x, *state):
        m = len(self.angles)
        us, lams = list(state[:m]), list(state[m:])
        for k in range(k0, k1):
            x, us, lams = self._iteration(k, d, x, us, lams)
        return (x, *us, *lams)

    def forward(self, d):
        """d: list of per-node sinograms (float32 cuda).  Returns x after K iterations."""
        n, dev = self.n, d[0].device
        m = len(self.angles)
        x = torch.zeros((n, n), device=dev)
        state = [torch.zeros((n, n), device=dev) for _ in range(2 * m)]
        span = self.ckpt if self.ckpt > 0 else self.iters
        k = 0
        while k < self.iters:
            k1 = min(self.iters, k + span)
            if self.ckpt > 0 and torch.is_grad_enabled():
                out = checkpoint(self._segment, k, k1, d, x, *state, use_reentrant=False)
            else:
                out = self._segment(k, k1, d, x, *state)
            x, state = out[0], list(out[1:])
            k = k1
        return x
