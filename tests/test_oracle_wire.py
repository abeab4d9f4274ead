"""Pins of the oracle's K-means wire format (oracle/wire.py): a hand-packed
example, NumPy's own little-endian bit packing as an independent route, round
trips, sizes, and the bits-per-value arithmetic of Section 3.3."""
import numpy as np
import pytest

from oracle import wire


def test_hand_packed_example():
    # labels 1, 2, 3, 0, 1 at 2 bits, least significant bit first:
    # stream 1 0 | 0 1 | 1 1 | 0 0 | 1 0  ->  bits 0, 3, 4, 5, 8 set
    assert wire.pack_labels([1, 2, 3, 0, 1], 2).tolist() == [1 + 8 + 16 + 32 + 256]
    # three 3-bit codes 7, 0, 5 -> bits 0,1,2 and 6,8 -> 7 + 64 + 256
    assert wire.pack_labels([7, 0, 5], 3).tolist() == [327]


@pytest.mark.parametrize("bits", range(1, 9))
def test_matches_numpy_packbits(bits):
    rng = np.random.default_rng(bits)
    lab = rng.integers(0, 1 << bits, size=77)
    stream = ((lab[:, None] >> np.arange(bits)[None, :]) & 1).astype(np.uint8).reshape(-1)
    stream = np.concatenate([stream, np.zeros(wire.packed_words(lab.size, bits) * 32 - stream.size, np.uint8)])
    ref = np.packbits(stream, bitorder="little").view("<u4")
    np.testing.assert_array_equal(wire.pack_labels(lab, bits), ref)


@pytest.mark.parametrize("n,bits", [(1, 1), (31, 1), (32, 1), (33, 1), (11, 3), (32, 5), (100, 7), (64, 8)])
def test_round_trip_and_size(n, bits):
    lab = np.random.default_rng(n * 10 + bits).integers(0, 1 << bits, size=n)
    words = wire.pack_labels(lab, bits)
    assert words.size == -(-n * bits // 32)
    np.testing.assert_array_equal(wire.unpack_labels(words, n, bits), lab.astype(np.uint8))


def test_only_low_bits_are_stored():
    np.testing.assert_array_equal(wire.pack_labels([5, 6], 2), wire.pack_labels([1, 2], 2))


def test_message_size_follows_the_bits_per_value():
    # Section 3.3: K = 3 -> 2 bits, K = 32 -> 5 bits, K = 16 -> 4 bits per value
    n = 512 * 256
    assert wire.message_bytes(n, 3) == n * 2 // 8 + 12
    assert wire.message_bytes(n, 32) == n * 5 // 8 + 128
    assert wire.message_bytes(n, 16) == n // 2 + 64
