"""Regularization as one more ADMM block (float64 oracle).

Test infrastructure only: the library never imports this module.

The paper's discussion (Section 4) proposes regularization, total variation or
Tikhonov, as a separate ADMM sub-problem, and gives no formulation.  The
reading implemented here adds to the augmented Lagrangian of Eq. 7 one block
with its own copy z of the image and its own dual variable nu:

    mu R(z) + nu^T (z - x) + rho_z / 2 ||z - x||^2.

One ADMM iteration then takes, next to Eq. 15-18:

* z-update   z^{k+1} = argmin_z mu R(z) + rho_z/2 ||z - v||^2,
             v = x^k - nu^k / rho_z, i.e. the proximal map of (mu / rho_z) R at v;
* x-update   the block's copy is one more term of Eq. 9 / Eq. 16 with target
             t_z = z^{k+1} + nu^k / rho_z:
             AVG  x = (sum_m rho_m t_m + rho_z t_z) / (sum_m rho_m + rho_z),
                  t_m = u_m + lambda_m / rho_m (with equal rho, the mean of the
                  M + 1 targets);
             SEG  E2 gradient steps x <- x - eta2 (rho (x - t_m) + rho_z (x - t_z))
                  on each segment, from x^k[m] as in Alg. 3;
* dual       nu^{k+1} = nu^k + rho_z (z^{k+1} - x^{k+1})   (like Eq. 24).

R is Tikhonov, R(z) = 1/2 ||z||^2, whose proximal map is v / (1 + theta), or
isotropic total variation R(z) = sum_ij |(grad z)_ij|, grad taken with forward
differences that are zero across the last row / column.  Its proximal map is
computed with Chambolle's dual projection algorithm (A. Chambolle, "An
algorithm for total variation minimization and applications", J. Math. Imaging
Vis. 20, 2004): with theta = mu / rho_z and a dual field p = (p1, p2),

    w = div p - v / theta,
    p <- (p + tau grad w) / (1 + tau |grad w|),
    z = v - theta div p,

a fixed number of iterations from a given p (warm start across ADMM
iterations), tau <= 1/8 (the step of the convergence proof).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TIKHONOV = "tikhonov"
TV = "tv"


def grad(u):
    """Forward differences: g1 along rows (axis 0), g2 along columns (axis 1);
    zero across the last row and the last column."""
    u = np.asarray(u, dtype=np.float64)
    g1 = np.zeros_like(u)
    g2 = np.zeros_like(u)
    g1[:-1, :] = u[1:, :] - u[:-1, :]
    g2[:, :-1] = u[:, 1:] - u[:, :-1]
    return g1, g2


def div(p1, p2):
    """Divergence, the negative adjoint of ``grad``: <grad u, p> = -<u, div p>."""
    p1 = np.asarray(p1, dtype=np.float64)
    p2 = np.asarray(p2, dtype=np.float64)
    d = np.zeros_like(p1)
    # rows: p1[i] - p1[i-1], with p1[-1] = 0 and p1[last] not entering
    d[:-1, :] += p1[:-1, :]
    d[1:, :] -= p1[:-1, :]
    d[:, :-1] += p2[:, :-1]
    d[:, 1:] -= p2[:, :-1]
    return d


def tv(u):
    """Isotropic total variation sum_ij sqrt(g1^2 + g2^2)."""
    g1, g2 = grad(u)
    return float(np.sum(np.sqrt(g1 * g1 + g2 * g2)))


def prox_tikhonov(v, theta):
    """argmin_z 1/2 ||z - v||^2 + theta/2 ||z||^2."""
    return np.asarray(v, dtype=np.float64) / (1.0 + theta)


def prox_tv(v, theta, iters, tau=0.125, p=None):
    """argmin_z 1/2 ||z - v||^2 + theta TV(z) by ``iters`` Chambolle iterations
    from the dual field ``p`` (zeros if None).  Returns (z, (p1, p2))."""
    v = np.asarray(v, dtype=np.float64)
    if p is None:
        p1, p2 = np.zeros_like(v), np.zeros_like(v)
    else:
        p1, p2 = (np.array(t, dtype=np.float64) for t in p)
    if theta <= 0:
        return v.copy(), (p1, p2)
    for _ in range(iters):
        g1, g2 = grad(div(p1, p2) - v / theta)
        nrm = np.sqrt(g1 * g1 + g2 * g2)
        p1 = (p1 + tau * g1) / (1.0 + tau * nrm)
        p2 = (p2 + tau * g2) / (1.0 + tau * nrm)
    return v - theta * div(p1, p2), (p1, p2)


@dataclass
class Reg:
    """The regularization block: R ('tikhonov' or 'tv'), weight mu, penalty
    rho_z, and for TV the Chambolle iterations per z-update and their step."""

    kind: str = TV
    mu: float = 0.01
    rho: float = 1.0
    tv_iters: int = 10
    tau: float = 0.125


def z_update(reg: Reg, x, nu, p=None):
    """z^{k+1} = prox_{(mu / rho_z) R}(x^k - nu^k / rho_z); returns (z, p)."""
    v = np.asarray(x, dtype=np.float64) - np.asarray(nu, dtype=np.float64) / reg.rho
    theta = reg.mu / reg.rho
    if reg.kind == TIKHONOV:
        return prox_tikhonov(v, theta), p
    if reg.kind == TV:
        return prox_tv(v, theta, reg.tv_iters, reg.tau, p)
    raise ValueError(reg.kind)


def x_update_segment(x_seg, u_seg, lam_seg, rho, tz_seg, rho_z, eta2, e2):
    """Alg. 3 with the block's copy: E2 steps
    x <- x - eta2 (rho (x - u - lambda / rho) + rho_z (x - t_z)), from x^k[m]."""
    x = np.array(x_seg, dtype=np.float64)
    for _ in range(e2):
        x = x - eta2 * (rho * (x - u_seg - lam_seg / rho) + rho_z * (x - tz_seg))
    return x


def x_update_average(us, lams, rhos, tz, rho_z):
    """Closed-form argmin of Eq. 9 with the block's term:
    (sum_m rho_m (u_m + lambda_m / rho_m) + rho_z t_z) / (sum_m rho_m + rho_z)."""
    num = sum(r * (u + l / r) for u, l, r in zip(us, lams, rhos)) + rho_z * np.asarray(tz, dtype=np.float64)
    return num / (sum(rhos) + rho_z)


def dual_update(nu, z, x, rho_z):
    """nu + rho_z (z - x)."""
    return nu + rho_z * (z - x)
