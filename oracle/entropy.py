"""Lossless entropy code of a segment's DCT codes (integers only; oracle).

Section 2.7 applies "standard JPEG" to the exchanged segments.  Baseline JPEG
follows its quantizer with a lossless entropy code; the paper gives no tables.
This module defines the code the library puts on the wire, so the bytes of a
DCT message can be counted for Eq. 20.  It follows baseline JPEG's sequential
layout, with universal codes instead of Huffman tables:

* blocks in row-major order over the segment; in a block the 64 codes in
  zigzag order (anti-diagonals u + v = 0 .. 14, even ones walked with u
  falling, odd ones with u rising; u = vertical frequency);
* the DC code is sent as the difference from the previous block's DC, and the
  first block of every restart interval is differenced from 0;
* the AC codes are sent as (zeros skipped, nonzero level) pairs, then an
  end-of-block symbol;
* every number is an order-0 Exp-Golomb code EG(x): floor(log2(x + 1)) zero
  bits, then x + 1 in binary, most significant bit first:
      DC difference d        EG(2d) for d >= 0, EG(-2d - 1) for d < 0
      nonzero AC level v     EG(run + 1), then EG(2 (|v| - 1) + (v < 0))
      end of block           EG(0)
* restart intervals of 64 blocks: the message carries the bit offset at which
  each interval starts, so intervals decode independently;
* bits are packed most significant first into 32-bit words: stream bit j is
  bit 31 - (j mod 32) of word j // 32; the last word is zero padded.

A message is the words, the restart offsets (uint32) and the level-map range
(two float32): 4 * words + 4 * intervals + 8 bytes.
"""
from __future__ import annotations

import numpy as np

INTERVAL = 64


def zigzag_order() -> list:
    """(u, v) of the 64 coefficients of a block in scan order."""
    out = []
    for s in range(15):
        us = range(min(s, 7), max(0, s - 7) - 1, -1) if s % 2 == 0 else range(max(0, s - 7), min(s, 7) + 1)
        out += [(u, s - u) for u in us]
    return out


def eg_bits(x: int) -> str:
    """Order-0 Exp-Golomb code of x >= 0 as a string of '0'/'1'."""
    y = x + 1
    b = bin(y)[2:]
    return "0" * (len(b) - 1) + b


def _blocks(codes):
    q = np.asarray(codes, dtype=np.int64)
    rows, cols = q.shape
    assert rows % 8 == 0 and cols % 8 == 0
    return [q[r:r + 8, c:c + 8] for r in range(0, rows, 8) for c in range(0, cols, 8)]


def encode(codes):
    """(words uint32, restart bit offsets uint32, total bits) of an int16 [rows][cols] code array."""
    zz = zigzag_order()
    bits, restart = [], []
    pos = 0
    prev_dc = 0
    for i, blk in enumerate(_blocks(codes)):
        if i % INTERVAL == 0:
            restart.append(pos)
            prev_dc = 0
        seq = [int(blk[u, v]) for u, v in zz]
        d = seq[0] - prev_dc
        prev_dc = seq[0]
        s = eg_bits(2 * d if d >= 0 else -2 * d - 1)
        run = 0
        for v in seq[1:]:
            if v == 0:
                run += 1
                continue
            s += eg_bits(run + 1) + eg_bits(2 * (abs(v) - 1) + (1 if v < 0 else 0))
            run = 0
        s += eg_bits(0)
        bits.append(s)
        pos += len(s)
    stream = "".join(bits)
    n_words = (len(stream) + 31) // 32
    stream = stream.ljust(32 * n_words, "0")
    words = np.array([int(stream[32 * w:32 * w + 32], 2) for w in range(n_words)], dtype=np.uint64)
    return words.astype(np.uint32), np.array(restart, dtype=np.uint32), pos


def decode(words, restart, rows: int, cols: int):
    """The int16 [rows][cols] code array back from encode's words and offsets."""
    w = [int(x) for x in np.asarray(words, dtype=np.uint64)]

    def bit(j):
        return (w[j // 32] >> (31 - j % 32)) & 1

    def read_eg(j):
        z = 0
        while bit(j + z) == 0:
            z += 1
        y = 0
        for k in range(z + 1):
            y = 2 * y + bit(j + z + k)
        return y - 1, j + 2 * z + 1

    zz = zigzag_order()
    out = np.zeros((rows, cols), dtype=np.int64)
    n_bc = cols // 8
    n_blocks = (rows // 8) * n_bc
    for b in range(n_blocks):
        if b % INTERVAL == 0:
            j = int(restart[b // INTERVAL])
            prev_dc = 0
        x, j = read_eg(j)
        dc = prev_dc + (x // 2 if x % 2 == 0 else -(x + 1) // 2)
        prev_dc = dc
        seq = [dc] + [0] * 63
        k = 1
        while True:
            r1, j = read_eg(j)
            if r1 == 0:
                break
            k += r1 - 1
            m, j = read_eg(j)
            seq[k] = -(m // 2 + 1) if m % 2 else m // 2 + 1
            k += 1
        br, bc = divmod(b, n_bc)
        for (u, v), val in zip(zz, seq):
            out[8 * br + u, 8 * bc + v] = val
    return out.astype(np.int16)


def message_bytes(total_bits: int, n_blocks: int) -> int:
    return 4 * ((total_bits + 31) // 32) + 4 * ((n_blocks + INTERVAL - 1) // INTERVAL) + 8
