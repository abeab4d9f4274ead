"""Step size of Alg. 2.

The paper sets the local learning rate by hand (Section 3.2).  Gradient descent
on the u-subproblem (Eq. 15) is stable for eta1 < 2 / (L_m + rho) with
L_m = ||P_m^T P_m||_2; the workloads use eta1 = c / (L + rho) with L the largest
L_m over the nodes.  L_m is estimated by power iteration from a start vector
that the caller draws (so no random numbers are drawn here).
"""
from __future__ import annotations

import numpy as np

from . import joseph


def normal_operator_norm(thetas, n: int, n_bins: int, v0: np.ndarray, iters: int = 30) -> float:
    v = np.asarray(v0, dtype=np.float64).reshape(n, n)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = joseph.backproject(joseph.project(v, thetas, n_bins), thetas, n)
        lam = float(np.sum(w * v))
        v = w / np.linalg.norm(w)
    return lam
