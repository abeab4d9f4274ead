"""Seeded synthetic inputs for the decentralized-ADMM tomography workloads.

This module is shared by the CPU oracle and by the GPU path.  It holds no
arithmetic of the reconstruction method itself: it draws random-ellipse
phantoms, lists the projection angles, assigns angles to nodes and image rows
to segments, and applies a measurement-noise model to a clean sinogram that the
caller computed with its own projector.

Conventions (stated once, used everywhere):

* Image ``[N][N]`` row-major, float32.  Pixel ``(r, c)`` has its centre at
  ``X = (2c + 1 - N) / N``, ``Y = (2r + 1 - N) / N`` in the square ``[-1, 1]^2``
  (Y grows with the row index).
* Angles ``theta_k = pi * k / K`` for ``k < K``: uniform over ``[0, 180)``
  degrees with the end point excluded (the paper's experiments use angles
  evenly spread from 0 to 180 degrees, Section 3.1).
* Angle partitions follow Section 3.2: with an interleaved split node ``m``
  holds ``{m, m + M, m + 2M, ...}`` so the first ``K mod M`` nodes get one
  angle more (804 angles over 10 nodes give 4 x 81 + 6 x 80).  A contiguous
  split gives node ``m`` one block of consecutive angles, again with the first
  ``K mod M`` nodes one longer.
* Segments ``x[m]`` (Eq. 13/17, ``x = conc(x[1], ..., x[M])``) are contiguous
  strips of rows of the row-major image.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "EllipseSet", "Workload", "WORKLOADS", "batch_slices",
    "ellipse_params", "rasterize", "paint_levels", "texture", "phantom", "angles",
    "partition_angles", "segment_rows", "add_gaussian_noise", "poisson_noisy",
    "standard_normal", "sinogram_seed", "phantom_seed",
]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    """One named problem shape (image size, angles, bins, nodes, solver sizes)."""

    name: str
    index: int              # used to derive seeds: phantom seed = 1000*index + slice
    n: int                  # image is n x n
    n_angles: int
    n_bins: int
    n_nodes: int
    split: str              # "interleaved" | "contiguous"
    n_ellipses: int
    noise: str              # "gaussian" | "poisson"
    noise_level: float      # relative sigma (gaussian) or incident photons I0 (poisson)
    outer_iters: int
    inner_iters: int = 5    # E1
    x_iters: int = 10       # E2
    rho: float = 1.0
    eta2: float = 0.2
    quant: str = "kmeans"   # "none" | "kmeans" | "dct"
    levels: int = 16        # K-means clusters
    quality: tuple = (50,)  # DCT quality factors
    texture_sigma: float = 0.0
    gray_levels: int = 0    # 0: additive densities; L >= 2: painted phantom with L gray values
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "tiny": Workload("tiny", 0, 64, 90, 91, 4, "interleaved", 5, "gaussian", 0.01,
                     50, quant="kmeans", levels=16),
    "single": Workload("single", 1, 512, 720, 725, 16, "contiguous", 20, "poisson", 1e5,
                       100, quant="kmeans", levels=8),
    "large": Workload("large", 2, 2048, 1800, 2897, 64, "contiguous", 50, "gaussian", 0.01,
                      50, quant="dct", quality=(25, 50, 90), texture_sigma=0.02),
    "diff": Workload("diff", 4, 1024, 1080, 1449, 32, "interleaved", 20, "gaussian", 0.01,
                     10, quant="none"),
    # quality studies of Section 3 (Fig. 4-7): 512^2 image, 804 angles, 724
    # bins (the detector spans the image diagonal, as the paper's padding to
    # 724^2 does), two interleaved nodes (odd and even angles), E1 = E2 = 10,
    # a piecewise-constant phantom with three gray levels like the paper's
    # Phantom; noise is set per run as an NSD level
    "elbow": Workload("elbow", 5, 512, 804, 724, 2, "interleaved", 10, "gaussian", 0.0,
                      1000, inner_iters=10, x_iters=10, quant="kmeans", levels=3, gray_levels=3),
}


def batch_slices(n_slices: int = 256, seed: int = 4000):
    """Slice shapes for the many-slice batching workload.

    Image sizes uniform over {128, 256, 384, 512, 768, 1024}; angles 1.5 N;
    bins ceil(1.414 N); node counts uniform over {2, 4, 8, 16}.
    Returns a list of Workload records (index 3, slice-specific seeds).
    """
    rng = np.random.default_rng(seed)
    sizes = np.array([128, 256, 384, 512, 768, 1024])
    nodes = np.array([2, 4, 8, 16])
    out = []
    for s in range(n_slices):
        n = int(rng.choice(sizes))
        m = int(rng.choice(nodes))
        out.append(Workload(f"batch{s}", 3, n, (3 * n) // 2, int(math.ceil(1.414 * n)), m,
                            "interleaved", 10, "gaussian", 0.01, 10, quant="kmeans",
                            levels=16, extra={"slice": s}))
    return out


def phantom_seed(w: Workload, slice_idx: int = 0) -> int:
    return 1000 * w.index + slice_idx


def sinogram_seed(w: Workload, slice_idx: int = 0) -> int:
    return phantom_seed(w, slice_idx) + 1


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class EllipseSet:
    """Rows of (cx, cy, a, b, phi, density), coordinates in [-1, 1]^2."""

    params: np.ndarray


def ellipse_params(n_ellipses: int, rng: np.random.Generator) -> EllipseSet:
    """Draw ellipses: centre U[-0.6,0.6]^2, semi-axes U[0.05,0.4], rotation U[0,pi),
    density U[0.1,1]; drawn per ellipse in the order (cx, cy, a, b, phi, density)."""
    rows = []
    for _ in range(n_ellipses):
        cx = rng.uniform(-0.6, 0.6)
        cy = rng.uniform(-0.6, 0.6)
        a = rng.uniform(0.05, 0.4)
        b = rng.uniform(0.05, 0.4)
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.1, 1.0)
        rows.append((cx, cy, a, b, phi, rho))
    return EllipseSet(np.array(rows, dtype=np.float64).reshape(-1, 6))


def _pixel_centres(n: int):
    g = (2.0 * np.arange(n) + 1.0 - n) / n
    return g[None, :], g[:, None]          # X (columns), Y (rows)


def rasterize(ell: EllipseSet, n: int) -> np.ndarray:
    """Additive densities sampled at pixel centres (float64 [n][n])."""
    X, Y = _pixel_centres(n)
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, phi, rho in ell.params:
        dx, dy = X - cx, Y - cy
        cp, sp = math.cos(phi), math.sin(phi)
        p = dx * cp + dy * sp
        q = -dx * sp + dy * cp
        img += np.where((p / a) ** 2 + (q / b) ** 2 <= 1.0, rho, 0.0)
    return img


def paint_levels(ell: EllipseSet, n: int, levels: int) -> np.ndarray:
    """Piecewise-constant phantom with ``levels`` gray values {0, 1/(L-1), ..., 1}
    (float64 [n][n]): background 0, a body ellipse (centre 0, semi-axes 0.85 and
    0.7) at level 1, then the drawn ellipses in order, each overwriting the
    pixels inside it with level 1 + (i mod (L-1)) for the i-th, so every level
    appears once there are L-1 ellipses or more."""
    if levels < 2:
        raise ValueError("need at least two gray levels")
    X, Y = _pixel_centres(n)
    step = 1.0 / (levels - 1)
    img = np.where((X / 0.85) ** 2 + (Y / 0.7) ** 2 <= 1.0, step, 0.0)
    for i, (cx, cy, a, b, phi, _) in enumerate(ell.params):
        dx, dy = X - cx, Y - cy
        cp, sp = math.cos(phi), math.sin(phi)
        p = dx * cp + dy * sp
        q = -dx * sp + dy * cp
        img = np.where((p / a) ** 2 + (q / b) ** 2 <= 1.0, (1 + i % (levels - 1)) * step, img)
    return img


def texture(ell: EllipseSet, n: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """I.i.d. N(0, sigma^2) inside the union of the ellipses, zero elsewhere."""
    X, Y = _pixel_centres(n)
    inside = np.zeros((n, n), dtype=bool)
    for cx, cy, a, b, phi, _ in ell.params:
        dx, dy = X - cx, Y - cy
        cp, sp = math.cos(phi), math.sin(phi)
        p = dx * cp + dy * sp
        q = -dx * sp + dy * cp
        inside |= (p / a) ** 2 + (q / b) ** 2 <= 1.0
    return np.where(inside, rng.normal(0.0, sigma, size=(n, n)), 0.0)


def phantom(w: Workload, slice_idx: int = 0, n: int | None = None) -> np.ndarray:
    """The workload's phantom (float32 [n][n]); ``n`` overrides the size."""
    n = w.n if n is None else n
    rng = np.random.default_rng(phantom_seed(w, slice_idx))
    ell = ellipse_params(w.n_ellipses, rng)
    if w.gray_levels:
        return paint_levels(ell, n, w.gray_levels).astype(np.float32)
    img = rasterize(ell, n)
    if w.texture_sigma > 0:
        img = img + texture(ell, n, w.texture_sigma, rng)
    return img.astype(np.float32)


# --------------------------------------------------------------------------
# angles, partitions, segments
# --------------------------------------------------------------------------
def angles(n_angles: int) -> np.ndarray:
    """theta_k = pi k / K, k < K (float64)."""
    return np.pi * np.arange(n_angles, dtype=np.float64) / n_angles


def partition_angles(n_angles: int, n_nodes: int, split: str = "interleaved"):
    """Index arrays of the angles each node holds (Section 3.2)."""
    if n_nodes <= 0 or n_angles < n_nodes:
        raise ValueError("need 1 <= n_nodes <= n_angles")
    if split == "interleaved":
        return [np.arange(m, n_angles, n_nodes) for m in range(n_nodes)]
    if split == "contiguous":
        base, extra = divmod(n_angles, n_nodes)
        out, start = [], 0
        for m in range(n_nodes):
            cnt = base + (1 if m < extra else 0)
            out.append(np.arange(start, start + cnt))
            start += cnt
        return out
    raise ValueError(f"unknown split {split!r}")


def segment_rows(n: int, n_nodes: int):
    """(row0, rows) of each node's segment: contiguous row strips, first n mod M one longer."""
    if n_nodes <= 0 or n < n_nodes:
        raise ValueError("need 1 <= n_nodes <= n")
    base, extra = divmod(n, n_nodes)
    out, start = [], 0
    for m in range(n_nodes):
        cnt = base + (1 if m < extra else 0)
        out.append((start, cnt))
        start += cnt
    return out


# --------------------------------------------------------------------------
# noise models applied to a clean sinogram computed by the caller
# --------------------------------------------------------------------------
def standard_normal(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


def add_gaussian_noise(clean: np.ndarray, rel_sigma: float, seed: int) -> np.ndarray:
    """clean + sigma z, sigma = rel_sigma * max(clean), z ~ N(0, 1) (float32 out)."""
    clean = np.asarray(clean, dtype=np.float64)
    sigma = rel_sigma * float(clean.max())
    return (clean + sigma * standard_normal(clean.shape, seed)).astype(np.float32)


def poisson_noisy(clean: np.ndarray, i0: float, n: int, seed: int) -> np.ndarray:
    """Photon-counting model.  ``clean`` holds line integrals in pixel units; the
    attenuation per half image width is ``p = (2/n) clean``; counts are
    Poisson(i0 exp(-p)); the returned data is ``-ln(max(counts,1)/i0) * n/2``
    (float32), i.e. back in pixel units."""
    clean = np.asarray(clean, dtype=np.float64)
    lam = i0 * np.exp(-(2.0 / n) * clean)
    counts = np.random.default_rng(seed).poisson(lam)
    return (-np.log(np.maximum(counts, 1) / i0) * (n / 2.0)).astype(np.float32)
