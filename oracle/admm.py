"""Decentralized ADMM with quantized exchange (float64 oracle).

Follows Sections 2.2-2.5 and 2.7 of the paper:

* Alg. 1  centralized gradient descent on 0.5 ||P u - d||^2 (Eq. 5).
* Alg. 2  node m's u-update: E1 gradient steps on
          0.5 ||P_m u - d_m||^2 + rho/2 ||u - x^k + lambda_m^k / rho||^2   (Eq. 15),
          gradient P_m^T (P_m u - d_m) + rho (u - (x^k - lambda_m^k / rho)).
* Alg. 3  node m's segment update: E2 gradient steps on
          rho/2 ||u_m^{k+1}[m] - x[m] + lambda_m^k[m] / rho||^2              (Eq. 16).
* Eq. 9   the averaging x-update of standard consensus ADMM,
          x = (1/M) sum_m (u_m + lambda_m / rho)  (the closed-form argmin of Eq. 9).
* Eq. 23  x^{k+1} = conc(Q(x[1]), ..., Q(x[M])).
* Eq. 24  lambda_m <- lambda_m + rho (u_m^{k+1} - x^{k+1}).
* Alg. 4  zero initialisation and K outer iterations.
* With ``reg`` (oracle/reg.py): the regularization block of the discussion
  (Section 4), its z-update before the x-update and its dual after it.

Readings where the paper is silent: u_m is zero only at k = 0 and warm-starts
afterwards; Alg. 3 starts from the current global x^k[m]; every node, the owner
included, uses the quantized segment in x^{k+1}.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Sequence

import numpy as np

from . import joseph
from . import reg as regmod
from .kmeans import kmeans_quantize
from .dct import dct_quantize
from .metrics import rmse


def ctr_gd(d, thetas, n, eta, iters, proj=joseph):
    """Alg. 1: u <- u - eta P^T (P u - d), from u = 0.  ``proj`` is the system
    matrix's module (``oracle.joseph`` or ``oracle.chord``)."""
    u = np.zeros((n, n))
    for _ in range(iters):
        u = u - eta * proj.backproject(proj.project(u, thetas, d.shape[1]) - d, thetas, n)
    return u


def local_update(u, x, lam, d_m, thetas_m, rho, eta1, e1, proj=joseph):
    """Alg. 2: E1 gradient steps of node m's u-subproblem, from the given u."""
    n = u.shape[0]
    u = np.array(u, dtype=np.float64)
    for _ in range(e1):
        resid = proj.project(u, thetas_m, d_m.shape[1]) - d_m
        grad = proj.backproject(resid, thetas_m, n) + rho * (u - (x - lam / rho))
        u = u - eta1 * grad
    return u


def local_update_exact(x, lam, d_m, thetas_m, rho, n):
    """Exact argmin of Eq. 15: (P^T P + rho I)^{-1} (P^T d + rho x - lambda) (tiny n)."""
    A = joseph.dense_matrix(n, d_m.shape[1], thetas_m)
    H = A.T @ A + rho * np.eye(n * n)
    rhs = A.T @ d_m.reshape(-1) + rho * x.reshape(-1) - lam.reshape(-1)
    return np.linalg.solve(H, rhs).reshape(n, n)


def x_update_segment(x_seg, u_seg, lam_seg, rho, eta2, e2):
    """Alg. 3: E2 gradient steps x <- x - eta2 rho (x - u - lambda/rho), from x^k[m]."""
    x = np.array(x_seg, dtype=np.float64)
    for _ in range(e2):
        x = x - eta2 * (rho * (x - u_seg - lam_seg / rho))
    return x


def x_update_average(us, lams, rho):
    """Eq. 9 closed form: x = mean_m (u_m + lambda_m / rho)."""
    return sum(u + l / rho for u, l in zip(us, lams)) / len(us)


def dual_update(lam, u, x, rho):
    """Eq. 24: lambda + rho (u - x)."""
    return lam + rho * (u - x)


@dataclass
class Quantizer:
    """Q of Eq. 23 applied to one segment: 'none', 'kmeans' (Alg. 5) or 'dct'."""

    kind: str = "none"
    levels: int = 16
    max_iter: int = 30
    quality: int = 50

    def __call__(self, seg: np.ndarray) -> np.ndarray:
        if self.kind == "none":
            return seg
        a32 = np.asarray(seg, dtype=np.float32)
        if self.kind == "kmeans":
            res = kmeans_quantize(a32.reshape(-1), self.levels, self.max_iter)
            return res.a_hat.reshape(seg.shape).astype(np.float64)
        if self.kind == "dct":
            return dct_quantize(a32, self.quality).a_hat.astype(np.float64)
        raise ValueError(self.kind)


@dataclass
class Problem:
    """One slice: sinogram rows per node, their angles, segments, geometry."""

    n: int
    n_bins: int
    thetas: Sequence[np.ndarray]          # per node, float64
    d: Sequence[np.ndarray]               # per node, [K_m][B]
    segments: Sequence[tuple]             # per node, (row0, rows)
    truth: np.ndarray | None = None


@dataclass
class Trace:
    rmse: list = field(default_factory=list)
    rel_change: list = field(default_factory=list)
    reg_state: tuple | None = None        # (z, nu, p) of the regularization block


def run(prob: Problem, iters: int, rho: float, eta1: float, e1: int, eta2: float, e2: int,
        mode: str = "seg", quant: Quantizer | None = None, exact_u: bool = False,
        state=None, cast32: bool = False, reg: "regmod.Reg | None" = None, reg_state=None):
    """Alg. 4.  ``mode`` is 'seg' (Eq. 16 per node) or 'avg' (Eq. 9).

    ``cast32`` rounds the exchanged x to float32 each iteration (the GPU keeps x
    in float32); everything else stays float64.  ``reg`` adds the
    regularization block (z, nu and, for TV, the dual field p; ``reg_state``
    continues from a given (z, nu, p)).  Returns (x, us, lams, trace); the
    block's final state is trace.reg_state.
    """
    quant = quant or Quantizer()
    n, m_nodes = prob.n, len(prob.d)
    if state is None:
        us = [np.zeros((n, n)) for _ in range(m_nodes)]
        lams = [np.zeros((n, n)) for _ in range(m_nodes)]
        x = np.zeros((n, n))
    else:
        x = np.array(state[0], dtype=np.float64)
        us = [np.array(t, dtype=np.float64) for t in state[1]]
        lams = [np.array(t, dtype=np.float64) for t in state[2]]
    tr = Trace()
    if reg is not None:
        if reg_state is None:
            z, nu, pz = np.zeros((n, n)), np.zeros((n, n)), None
        else:
            z, nu = (np.array(t, dtype=np.float64) for t in reg_state[:2])
            pz = reg_state[2]
    for _ in range(iters):
        if reg is not None:
            z, pz = regmod.z_update(reg, x, nu, pz)
            tz = z + nu / reg.rho
        for m in range(m_nodes):
            if exact_u:
                us[m] = local_update_exact(x, lams[m], prob.d[m], prob.thetas[m], rho, n)
            else:
                us[m] = local_update(us[m], x, lams[m], prob.d[m], prob.thetas[m], rho, eta1, e1)
        if mode == "seg":
            xt = x.copy()
            for m, (r0, nr) in enumerate(prob.segments):
                sl = slice(r0, r0 + nr)
                if reg is None:
                    xt[sl] = x_update_segment(x[sl], us[m][sl], lams[m][sl], rho, eta2, e2)
                else:
                    xt[sl] = regmod.x_update_segment(x[sl], us[m][sl], lams[m][sl], rho, tz[sl], reg.rho, eta2, e2)
        elif mode == "avg":
            if reg is None:
                xt = x_update_average(us, lams, rho)
            else:
                xt = regmod.x_update_average(us, lams, [rho] * m_nodes, tz, reg.rho)
        else:
            raise ValueError(mode)
        x_new = np.empty_like(xt)
        for (r0, nr) in prob.segments:
            sl = slice(r0, r0 + nr)
            x_new[sl] = quant(xt[sl])
        if cast32:
            x_new = x_new.astype(np.float32).astype(np.float64)
        for m in range(m_nodes):
            lams[m] = dual_update(lams[m], us[m], x_new, rho)
        if reg is not None:
            nu = regmod.dual_update(nu, z, x_new, reg.rho)
        denom = np.linalg.norm(x)
        tr.rel_change.append(float(np.linalg.norm(x_new - x) / denom) if denom > 0 else float("inf"))
        x = x_new
        if prob.truth is not None:
            tr.rmse.append(rmse(x, prob.truth))
    if reg is not None:
        tr.reg_state = (z, nu, pz)
    return x, us, lams, tr
