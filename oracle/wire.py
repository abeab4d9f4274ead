"""Wire format of a K-means message (float64-free; integers only).

Section 2.6 prices the exchange of Eq. 23 in bits per value (Eq. 20 scales the
image bytes by the quantizer's bits over 32), and Section 3.3 counts a K-level
K-means code as ceil(log2 K) bits.  The message of one segment here is its
labels packed at ``bits`` bits each plus the float32 codebook:

* value i occupies bits [i*bits, (i+1)*bits) of one bit stream, least
  significant bit of the label first;
* the stream is cut into 32-bit words, stream bit j being bit (j mod 32) of
  word floor(j / 32); the last word is padded with zero bits.

Written out bit by bit below, as the definition.
"""
from __future__ import annotations

import math

import numpy as np


def packed_words(n: int, bits: int) -> int:
    """Number of 32-bit words holding n codes of ``bits`` bits."""
    return (n * bits + 31) // 32


def message_bytes(n: int, levels: int) -> int:
    """Bytes of one segment's message: packed labels plus the float32 codebook."""
    bits = max(1, math.ceil(math.log2(levels)))
    return 4 * packed_words(n, bits) + 4 * levels


def pack_labels(labels, bits: int) -> np.ndarray:
    """uint32 words of the packed stream (only the low ``bits`` bits of a label count)."""
    lab = np.asarray(labels, dtype=np.int64).reshape(-1)
    n = lab.size
    stream = np.zeros(packed_words(n, bits) * 32, dtype=np.int64)
    for i in range(n):
        for k in range(bits):
            stream[i * bits + k] = (lab[i] >> k) & 1
    words = np.zeros(stream.size // 32, dtype=np.uint64)
    for j, bit in enumerate(stream):
        if bit:
            words[j // 32] |= np.uint64(1) << np.uint64(j % 32)
    return words.astype(np.uint32)


def unpack_labels(words, n: int, bits: int) -> np.ndarray:
    """The n labels (uint8) read back from the packed stream."""
    w = np.asarray(words, dtype=np.uint64).reshape(-1)
    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        for k in range(bits):
            j = i * bits + k
            out[i] |= int((w[j // 32] >> np.uint64(j % 32)) & np.uint64(1)) << k
    return out.astype(np.uint8)
