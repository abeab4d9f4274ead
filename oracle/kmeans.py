"""Scalar K-means quantizer (Alg. 5), fully specified so that results are bit-exact.

The paper runs K-means on the entries of a vector, replaces every entry by its
nearest cluster centre, and notes that K-means yields a locally optimal scalar
quantizer for squared error (Section 2.7).  It leaves initialisation, stopping,
tie-breaking and arithmetic open; this module fixes them so that any
implementation that follows the same steps reaches identical labels:

1. lo, hi = min, max of the float32 input (NaN or Inf rejected).  If hi == lo
   every label is 0, every centre is lo, the output equals the input, iters = 0.
2. Initial centres c_j = f32(lo + ((hi - lo) * (2j + 1)) / (2k)) in float64,
   evaluated in that order without fused multiply-add.
3. Fixed point: e = binary exponent of max(|lo|, |hi|) as returned by frexp
   (so every |a_i| < 2^e), S = 30 - e; q_i = round-half-even(a_i * 2^S) as an
   integer, |q_i| <= 2^30.  Every cluster sum of q is then exact in int64 for
   any n < 2^32.
4. Assignment: with the centres in increasing order, the nearest centre of a
   value is the number of midpoints between consecutive centres that lie below
   it: label_i = #{j < k-1 : 2 a_i > c_j + c_{j+1}}, where 2 a_i is exact in
   float64 and the sum c_j + c_{j+1} is rounded once to float64.  A value at a
   midpoint goes to the lower centre.  (This rule is monotone in the value, so
   every cluster is a run of the sorted values.)
5. Lloyd iterations t = 1..T_max: c_j <- f32(f64(sum_{label=j} q) * 2^-S / f64(count_j))
   for non-empty clusters (an empty cluster keeps its centre), then the centres
   are put in increasing order (a stable sort; Lloyd's update keeps the order
   except in degenerate cases of rounding next to an empty cluster), then
   reassign; stop as soon as the labels do not change.
Outputs: labels, the centres that produced them, a_hat_i = c_{label_i}, and the
number of Lloyd iterations run.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class KMeansResult:
    labels: np.ndarray       # uint8 [n]
    centroids: np.ndarray    # float32 [k]
    a_hat: np.ndarray        # float32 [n]
    iters: int
    shift: int               # S


def fixed_point_shift(lo: float, hi: float, n: int) -> int:
    _, e = math.frexp(max(abs(lo), abs(hi)))
    return 30 - e


def initial_centres(lo: float, hi: float, k: int) -> np.ndarray:
    lo, hi = float(lo), float(hi)
    return np.array([np.float32(lo + ((hi - lo) * (2 * j + 1)) / (2 * k)) for j in range(k)],
                    dtype=np.float32)


def midpoint_sums(c32: np.ndarray) -> np.ndarray:
    """c_j + c_{j+1} of consecutive centres, each rounded once to float64."""
    c = c32.astype(np.float64)
    return c[:-1] + c[1:]


def assign(a32: np.ndarray, c32: np.ndarray) -> np.ndarray:
    """Nearest centre of every value (centres in increasing order): the count
    of midpoints below the value, ties to the lower centre (step 4)."""
    twice = 2.0 * a32.astype(np.float64)             # exact
    return np.sum(twice[:, None] > midpoint_sums(c32)[None, :], axis=1)


def kmeans_quantize(a, k: int, max_iter: int = 30) -> KMeansResult:
    a32 = np.asarray(a, dtype=np.float32).reshape(-1)
    n = a32.size
    if not (1 <= k <= 256):
        raise ValueError("k must lie in [1, 256]")
    if n == 0:
        return KMeansResult(np.zeros(0, np.uint8), np.zeros(k, np.float32), a32.copy(), 0, 0)
    if not np.all(np.isfinite(a32)):
        raise ValueError("non-finite input")
    lo, hi = float(a32.min()), float(a32.max())
    if hi == lo:
        return KMeansResult(np.zeros(n, np.uint8), np.full(k, a32[0], np.float32), a32.copy(), 0, 0)
    S = fixed_point_shift(lo, hi, n)
    q = np.rint(np.ldexp(a32.astype(np.float64), S)).astype(np.int64)   # |q| <= 2^30
    c = initial_centres(lo, hi, k)
    labels = assign(a32, c)
    iters = 0
    for t in range(1, max_iter + 1):
        sums = np.zeros(k, dtype=np.int64)
        np.add.at(sums, labels, q)                    # exact integer sums
        counts = np.bincount(labels, minlength=k)
        for j in range(k):
            if counts[j] > 0:
                c[j] = np.float32(math.ldexp(float(int(sums[j])), -S) / float(counts[j]))
        c = np.sort(c, kind="stable")
        new = assign(a32, c)
        iters = t
        if np.array_equal(new, labels):
            break
        labels = new
    labels = assign(a32, c)
    return KMeansResult(labels.astype(np.uint8), c.copy(), c[labels].astype(np.float32), iters, S)
