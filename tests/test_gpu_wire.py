"""GPU parity of the K-means wire format (tomo_pack_labels / tomo_unpack_labels)
against oracle/wire.py, and the round trip of a real consensus message: the
packed labels plus the codebook reproduce the exchanged segment of x exactly."""
import numpy as np
import pytest
import torch

from gpu_common import log, require_gpu, to_dev
from oracle import wire

pytestmark = pytest.mark.gpu

TOMO_OK, TOMO_EINVAL = 0, 1        # status codes of include/tomoadmm.h


@pytest.fixture(scope="module")
def T():
    require_gpu()
    from paper_2410_06106_amd import tomoadmm
    return tomoadmm


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


CASES = [(n, b) for b in range(1, 9) for n in (1, 31, 33, 1000)] + [(100003, 3), (100003, 8), (65536, 5)]


@pytest.mark.parametrize("n,bits", CASES)
def test_pack_and_unpack_match_oracle(T, ctx, n, bits):
    log(f"case wire n={n} bits={bits}")
    rng = np.random.default_rng(n + 17 * bits)
    lab = rng.integers(0, 1 << bits, size=n).astype(np.uint8)
    k = 1 << bits
    cent = np.sort(rng.standard_normal(k)).astype(np.float32)
    packed = T.tomo_pack_labels(ctx, to_dev(lab, torch.uint8), bits)
    want = wire.pack_labels(lab, bits)
    np.testing.assert_array_equal(packed.cpu().numpy().view(np.uint32), want)
    out_l = torch.empty(n, dtype=torch.uint8, device="cuda")
    out_a = torch.empty(n, dtype=torch.float32, device="cuda")
    T.tomo_unpack_labels(ctx, packed, n, bits, to_dev(cent), out_l, out_a)
    np.testing.assert_array_equal(out_l.cpu().numpy(), wire.unpack_labels(want, n, bits))
    np.testing.assert_array_equal(out_a.cpu().numpy(), cent[lab])


def test_pack_keeps_only_the_low_bits(T, ctx):
    lab = to_dev(np.array([5, 6, 255, 4], np.uint8), torch.uint8)
    got = T.tomo_pack_labels(ctx, lab, 2).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, wire.pack_labels([1, 2, 3, 0], 2))


def test_consensus_message_round_trip(T, ctx):
    """Labels and centroids that admm_consensus emits for each segment, packed at
    ceil(log2 K) bits and decoded, give back the quantized segment of x bit for bit;
    the message size is 4 ceil(n bits / 32) + 4 K bytes."""
    n, M, k, bits = 64, 4, 6, 3
    rng = np.random.default_rng(3)
    x = rng.random((n, n)).astype(np.float32)
    X = to_dev(x)
    U = [to_dev(rng.random((n, n)).astype(np.float32)) for _ in range(M)]
    L = [torch.zeros((n, n), dtype=torch.float32, device="cuda") for _ in range(M)]
    dummy_d = to_dev(np.zeros((1, 8), np.float32))
    labels = [torch.empty(16 * n, dtype=torch.uint8, device="cuda") for _ in range(M)]
    cents = [torch.empty(k, dtype=torch.float32, device="cuda") for _ in range(M)]
    ents = [dict(n=n, n_bins=8, angles=to_dev(np.zeros(1), torch.float64), slice=0, d=dummy_d, u=U[m],
                 lam=L[m], x=X, seg_row0=16 * m, seg_rows=16, rho=1.0, eta1=0.0, eta2=0.5) for m in range(M)]
    T.admm_consensus(ctx, T.make_nodes(ents), T.TOMO_XUPDATE_SEGMENT, 3, T.tomo_quant(T.TOMO_QUANT_KMEANS, k, 30, 0),
                     T.make_msgs([dict(labels=labels[m], centroids=cents[m]) for m in range(M)]))
    xq = X.cpu().numpy()
    for m in range(M):
        packed = T.tomo_pack_labels(ctx, labels[m], bits)
        assert 4 * packed.numel() + 4 * k == wire.message_bytes(16 * n, k)
        a_hat = torch.empty(16 * n, dtype=torch.float32, device="cuda")
        T.tomo_unpack_labels(ctx, packed, 16 * n, bits, cents[m], a_hat=a_hat)
        np.testing.assert_array_equal(a_hat.cpu().numpy(), xq[16 * m:16 * (m + 1)].reshape(-1))


def test_wire_argument_errors(T, ctx):
    lab = torch.zeros(10, dtype=torch.uint8, device="cuda")
    out = torch.zeros(3, dtype=torch.int32, device="cuda")
    lib, h = T._lib, ctx.handle
    P = lambda t: T._dev(t, t.dtype, "t")
    assert lib.tomo_pack_labels(h, P(lab), 10, 0, P(out), None) == TOMO_EINVAL
    assert lib.tomo_pack_labels(h, P(lab), 10, 9, P(out), None) == TOMO_EINVAL
    assert lib.tomo_pack_labels(h, P(lab), -1, 3, P(out), None) == TOMO_EINVAL
    assert lib.tomo_pack_labels(h, None, 10, 3, P(out), None) == TOMO_EINVAL
    assert lib.tomo_pack_labels(h, P(lab), 0, 3, None, None) == TOMO_OK
    a = torch.zeros(10, dtype=torch.float32, device="cuda")
    assert lib.tomo_unpack_labels(h, P(out), 10, 3, None, 4, None, P(a), None) == TOMO_EINVAL   # no centroids
    c = torch.zeros(4, dtype=torch.float32, device="cuda")
    assert lib.tomo_unpack_labels(h, P(out), 10, 3, P(c), 0, None, P(a), None) == TOMO_EINVAL   # k = 0
    assert lib.tomo_unpack_labels(h, P(out), 10, 3, P(c), 4, None, None, None) == TOMO_OK       # nothing asked
