"""Evaluation and resource models of the paper.

* Eq. 25  RMSE = sqrt(mean((X - O)^2)).
* Eq. 26  PSNR = 20 log10(I_max / RMSE), I_max = maximum intensity of the original.
* Eq. 27  NSD = sigma / x_peak * 100 %.
* Eq. 19  per-node memory  D/M + 3X.
* Eq. 20  per-node traffic per iteration 2 (M - 1) / M * X, scaled by the
          quantizer's bits per value over 32 (Sections 2.6 and 3.3).
"""
from __future__ import annotations

import math

import numpy as np


def rmse(x, o) -> float:
    x = np.asarray(x, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    return float(np.sqrt(np.mean((x - o) ** 2)))


def psnr(x, o, i_max: float | None = None) -> float:
    i_max = float(np.max(o)) if i_max is None else i_max
    return 20.0 * math.log10(i_max / rmse(x, o))


def nsd_percent(sigma: float, x_peak: float) -> float:
    return sigma / x_peak * 100.0


def memory_per_node(data_bytes: float, image_bytes: float, n_nodes: int) -> float:
    return data_bytes / n_nodes + 3.0 * image_bytes


def comm_per_node(image_bytes: float, n_nodes: int, bits: float = 32.0) -> float:
    return 2.0 * (n_nodes - 1) / n_nodes * image_bytes * (bits / 32.0)


def kmeans_bits(levels: int) -> int:
    """Bits per value of a K-means code (ceil(log2 K), at least 1)."""
    return max(1, math.ceil(math.log2(levels)))
