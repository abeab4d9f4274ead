"""JPEG-style quantizer of an exchanged segment (the paper's dADMM-J, Section 2.7).

The paper applies "standard JPEG compression" to each exchanged vector without
further detail.  This module keeps the lossy core of baseline JPEG and drops the
lossless entropy coding, which does not change the decoded values:

1. lo, hi = min, max of the float32 segment; if hi == lo the segment is sent
   as is (all coefficients zero).
2. Level map to the 8-bit sample range and level shift:
   v = (a - lo) * 255 / (hi - lo) - 128.
3. Per 8x8 block, the orthonormal 2-D DCT-II  F = C v C^T,
   C[u][x] = alpha_u cos((2x + 1) u pi / 16), alpha_0 = sqrt(1/8), alpha_u = 1/2.
4. Quantizer step Qs[u][v] = clamp(floor((T[u][v] * S + 50) / 100), 1, 255),
   with S = floor(5000 / q) for quality q < 50 and S = 200 - 2q otherwise
   (the usual quality scaling of the luminance table T).
5. Codes q = round-half-even(F / Qs) as int16; reconstruction
   a_hat = (C^T (q Qs) C + 128) * (hi - lo) / 255 + lo.

Pixel values are not rounded to 8 bits (the exchanged values are real numbers).
T is the example luminance quantization table of ITU-T Rec. T.81 (Annex K,
Table K.1), rows = vertical frequency.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LUMA_TABLE = np.array([
    [16, 11, 10, 16, 24, 40, 51, 61],
    [12, 12, 14, 19, 26, 58, 60, 55],
    [14, 13, 16, 24, 40, 57, 69, 56],
    [14, 17, 22, 29, 51, 87, 80, 62],
    [18, 22, 37, 56, 68, 109, 103, 77],
    [24, 35, 55, 64, 81, 104, 113, 92],
    [49, 64, 78, 87, 103, 121, 120, 101],
    [72, 92, 95, 98, 112, 100, 103, 99],
], dtype=np.int64)


def dct_matrix() -> np.ndarray:
    u = np.arange(8)[:, None]
    x = np.arange(8)[None, :]
    C = np.cos((2 * x + 1) * u * np.pi / 16.0) / 2.0
    C[0, :] = np.sqrt(1.0 / 8.0)
    return C


def quant_steps(quality: int) -> np.ndarray:
    if not (1 <= quality <= 100):
        raise ValueError("quality must lie in [1, 100]")
    scale = 5000 // quality if quality < 50 else 200 - 2 * quality
    return np.clip((LUMA_TABLE * scale + 50) // 100, 1, 255).astype(np.float64)


@dataclass
class DCTResult:
    coeffs: np.ndarray     # int16 [rows][cols], block layout = the image layout
    a_hat: np.ndarray      # float32 [rows][cols]
    lo: float
    hi: float
    F: np.ndarray | None = None   # float64 forward coefficients (for tie analysis)


def _blocks(a: np.ndarray) -> np.ndarray:
    r, c = a.shape
    return a.reshape(r // 8, 8, c // 8, 8).transpose(0, 2, 1, 3)      # [br][bc][y][x]


def _unblocks(b: np.ndarray) -> np.ndarray:
    br, bc = b.shape[:2]
    return b.transpose(0, 2, 1, 3).reshape(br * 8, bc * 8)


def dct_quantize(a, quality: int = 50) -> DCTResult:
    a32 = np.asarray(a, dtype=np.float32)
    if a32.ndim != 2 or a32.shape[0] % 8 or a32.shape[1] % 8:
        raise ValueError("segment must be 2-D with both sides multiples of 8")
    Qs = quant_steps(quality)
    if a32.size == 0:
        return DCTResult(np.zeros(a32.shape, np.int16), a32.copy(), 0.0, 0.0)
    if not np.all(np.isfinite(a32)):
        raise ValueError("non-finite input")
    lo, hi = float(a32.min()), float(a32.max())
    if hi == lo:
        return DCTResult(np.zeros(a32.shape, np.int16), a32.copy(), lo, hi)
    C = dct_matrix()
    v = (a32.astype(np.float64) - lo) * 255.0 / (hi - lo) - 128.0
    F = C @ _blocks(v) @ C.T
    q = np.rint(F / Qs)
    rec = C.T @ (q * Qs) @ C
    a_hat = (rec + 128.0) * (hi - lo) / 255.0 + lo
    return DCTResult(_unblocks(q).astype(np.int16), _unblocks(a_hat).astype(np.float32),
                     lo, hi, _unblocks(F))
