"""Pins of the oracle's ADMM pieces (Alg. 1-4, Eq. 9, 15-18, 23-24).

Each check reaches the expected value by a route the oracle does not take:
dense matrices and matrix powers, numpy.linalg solves, closed forms of the
linear recursions, and least squares (numpy.linalg.lstsq) as the limit of the
averaging consensus iteration.
"""
import numpy as np
import pytest

import synthdata
from oracle import admm, joseph, stepsize


def _tiny_problem(n=8, n_angles=16, n_bins=12, n_nodes=2, noise=0.01, seed=5):
    rng = np.random.default_rng(seed)
    truth = np.zeros((n, n))
    truth[2:6, 1:5] = 1.0
    truth[4:7, 4:7] += 0.5
    th = synthdata.angles(n_angles)
    parts = synthdata.partition_angles(n_angles, n_nodes, "interleaved")
    A = joseph.dense_matrix(n, n_bins, th)
    d_full = (A @ truth.reshape(-1)).reshape(n_angles, n_bins)
    d_full = d_full + noise * d_full.max() * rng.standard_normal(d_full.shape)
    prob = admm.Problem(n, n_bins, [th[p] for p in parts], [d_full[p] for p in parts],
                        synthdata.segment_rows(n, n_nodes), truth)
    return prob, A, d_full


def test_ctr_gradient_descent_matches_dense_recursion():
    prob, A, d = _tiny_problem(n=6, n_angles=9, n_bins=9)
    th = synthdata.angles(9)
    eta, iters = 0.01, 7
    u = np.zeros(36)
    for _ in range(iters):
        u = u - eta * (A.T @ (A @ u - d.reshape(-1)))
    np.testing.assert_allclose(admm.ctr_gd(d, th, 6, eta, iters).reshape(-1), u, atol=1e-12)


def test_local_update_closed_form():
    """E1 gradient steps on the quadratic of Eq. 15 from u0:
    u_E = u* + (I - eta H)^E (u0 - u*), H = P^T P + rho I."""
    prob, _, _ = _tiny_problem()
    rng = np.random.default_rng(2)
    n = prob.n
    x, lam, u0 = (rng.standard_normal((n, n)) for _ in range(3))
    rho, eta, e1 = 1.3, 0.004, 6
    A = joseph.dense_matrix(n, prob.n_bins, prob.thetas[0])
    H = A.T @ A + rho * np.eye(n * n)
    ustar = np.linalg.solve(H, A.T @ prob.d[0].reshape(-1) + rho * x.reshape(-1) - lam.reshape(-1))
    G = np.linalg.matrix_power(np.eye(n * n) - eta * H, e1)
    ref = ustar + G @ (u0.reshape(-1) - ustar)
    got = admm.local_update(u0, x, lam, prob.d[0], prob.thetas[0], rho, eta, e1)
    np.testing.assert_allclose(got.reshape(-1), ref, atol=1e-11)
    # many steps converge to the exact argmin
    L = np.linalg.eigvalsh(A.T @ A).max()
    got = admm.local_update(u0, x, lam, prob.d[0], prob.thetas[0], rho, 1.0 / (L + rho), 3000)
    np.testing.assert_allclose(got.reshape(-1), ustar, atol=1e-8)
    ex = admm.local_update_exact(x, lam, prob.d[0], prob.thetas[0], rho, n)
    np.testing.assert_allclose(ex.reshape(-1), ustar, atol=1e-10)


def test_segment_update_closed_form():
    rng = np.random.default_rng(4)
    x0, u, lam = (rng.standard_normal((3, 8)) for _ in range(3))
    rho, eta2, e2 = 0.7, 0.2, 10
    t = u + lam / rho
    ref = t + (1 - eta2 * rho) ** e2 * (x0 - t)
    np.testing.assert_allclose(admm.x_update_segment(x0, u, lam, rho, eta2, e2), ref, atol=1e-14)
    # eta2 rho = 1 lands on the exact argmin of Eq. 16 in one step
    np.testing.assert_allclose(admm.x_update_segment(x0, u, lam, 1.0, 1.0, 1), u + lam, atol=1e-15)


@pytest.mark.slow
def test_average_consensus_converges_to_least_squares():
    """Standard consensus ADMM (Eq. 8-10 with the Eq. 9 average) with exact
    u-solves reaches the minimiser of 0.5 ||P u - d||^2 (Eq. 5)."""
    prob, A, d_full = _tiny_problem()
    x_ls = np.linalg.lstsq(A, d_full.reshape(-1), rcond=None)[0].reshape(prob.n, prob.n)
    # factor each node's system once: exact solves through numpy.linalg
    x, us, lams, _ = admm.run(prob, 3000, 1.0, 0.0, 0, 0.2, 10, mode="avg", exact_u=True)
    assert np.linalg.norm(x - x_ls) / np.linalg.norm(x_ls) <= 1e-9


def test_segment_mode_single_iteration_by_dense_algebra():
    """One dADMM iteration (Alg. 4) from zero state, reproduced with dense
    matrices: u_m = (I - (I - eta1 H_m)^E1) H_m^{-1} P_m^T d_m, then the Alg. 3
    closed form on each segment, then Eq. 24."""
    prob, _, _ = _tiny_problem(n=6, n_angles=8, n_bins=9, n_nodes=2)
    n, rho, eta1, e1, eta2, e2 = prob.n, 1.0, 0.01, 5, 0.2, 10
    x, us, lams, _ = admm.run(prob, 1, rho, eta1, e1, eta2, e2, mode="seg")
    xr = np.zeros(n * n)
    ur = []
    for m in range(2):
        A = joseph.dense_matrix(n, prob.n_bins, prob.thetas[m])
        H = A.T @ A + rho * np.eye(n * n)
        G = np.eye(n * n) - np.linalg.matrix_power(np.eye(n * n) - eta1 * H, e1)
        ur.append(G @ np.linalg.solve(H, A.T @ prob.d[m].reshape(-1)))
    for m, (r0, nr) in enumerate(prob.segments):
        sl = slice(r0 * n, (r0 + nr) * n)
        t = ur[m][sl]                      # lambda^0 = 0
        xr[sl] = t + (1 - eta2 * rho) ** e2 * (0.0 - t)
    np.testing.assert_allclose(x.reshape(-1), xr, atol=1e-12)
    for m in range(2):
        np.testing.assert_allclose(us[m].reshape(-1), ur[m], atol=1e-12)
        np.testing.assert_allclose(lams[m].reshape(-1), rho * (ur[m] - xr), atol=1e-12)


def test_segment_mode_fixed_point_on_consistent_data():
    """Noise-free data: x = u_m = truth, lambda_m = 0 is a fixed point of
    Eq. 15-18 (every gradient vanishes)."""
    prob, _, _ = _tiny_problem(noise=0.0)
    n = prob.n
    state = (prob.truth, [prob.truth] * 2, [np.zeros((n, n))] * 2)
    x, us, lams, _ = admm.run(prob, 3, 1.0, 0.003, 5, 0.2, 10, mode="seg", state=state)
    np.testing.assert_allclose(x, prob.truth, atol=1e-12)
    for m in range(2):
        np.testing.assert_allclose(lams[m], 0.0, atol=1e-11)


def test_power_iteration_matches_eigvalsh():
    prob, _, _ = _tiny_problem()
    A = joseph.dense_matrix(prob.n, prob.n_bins, prob.thetas[1])
    ref = np.linalg.eigvalsh(A.T @ A).max()
    v0 = np.random.default_rng(0).standard_normal((prob.n, prob.n))
    got = stepsize.normal_operator_norm(prob.thetas[1], prob.n, prob.n_bins, v0, iters=200)
    assert abs(got - ref) <= 1e-6 * ref


def _dense_quantized_iterations(prob, iters, rho, eta1, e1, eta2, e2, mode, q):
    """Alg. 4 with the exchange of Eq. 23-24 written with dense matrices: the
    local update by its closed form u* + (I - eta1 H)^E1 (u - u*), the segment
    x-update by t + (1 - eta2 rho)^E2 (x[m] - t) (or the Eq. 9 average), then Q
    on every segment of the concatenation, the owner's segment included
    (reading R11), and the dual with the quantized x."""
    n, M = prob.n, len(prob.d)
    I = np.eye(n * n)
    ops = []
    for m in range(M):
        A = joseph.dense_matrix(n, prob.n_bins, prob.thetas[m])
        H = A.T @ A + rho * I
        ops.append((A, H, np.linalg.matrix_power(I - eta1 * H, e1)))
    x = np.zeros(n * n)
    us = [np.zeros(n * n) for _ in range(M)]
    lams = [np.zeros(n * n) for _ in range(M)]
    for _ in range(iters):
        for m, (A, H, G) in enumerate(ops):
            ustar = np.linalg.solve(H, A.T @ prob.d[m].reshape(-1) + rho * x - lams[m])
            us[m] = ustar + G @ (us[m] - ustar)
        if mode == "seg":
            xt = x.copy()
            for m, (r0, nr) in enumerate(prob.segments):
                sl = slice(r0 * n, (r0 + nr) * n)
                t = us[m][sl] + lams[m][sl] / rho
                xt[sl] = t + (1 - eta2 * rho) ** e2 * (x[sl] - t)
        else:
            xt = sum(u + l / rho for u, l in zip(us, lams)) / M
        xq = np.empty_like(xt)
        for r0, nr in prob.segments:
            sl = slice(r0 * n, (r0 + nr) * n)
            xq[sl] = q(xt[sl].reshape(nr, n)).reshape(-1)
        x = xq
        lams = [l + rho * (u - x) for u, l in zip(us, lams)]
    return x.reshape(n, n), [u.reshape(n, n) for u in us], [l.reshape(n, n) for l in lams]


@pytest.mark.parametrize("mode", ["seg", "avg"])
@pytest.mark.parametrize("kind", ["kmeans", "dct"])
def test_quantized_iterations_by_dense_algebra(mode, kind):
    """Three dADMM iterations with a quantizer in the exchange (Eq. 23-24,
    Alg. 5 or the DCT codec) against the dense-matrix restatement above.  A
    quantizer applied to the whole image instead of per segment, before the
    x-update, or skipped on the owner's segment, or a dual formed with the
    unquantized x, fails this (the quantized x is far from x~ at 4 levels /
    quality 10)."""
    if kind == "kmeans":
        prob, _, _ = _tiny_problem(n=6, n_angles=9, n_bins=9, n_nodes=2)
        from oracle.kmeans import kmeans_quantize
        levels = 4

        def q(seg):
            return kmeans_quantize(seg.astype(np.float32).reshape(-1), levels, 30).a_hat.reshape(seg.shape)
        oq = admm.Quantizer("kmeans", levels, 30, 50)
    else:
        prob, _, _ = _tiny_problem(n=16, n_angles=20, n_bins=23, n_nodes=2)
        from oracle.dct import dct_quantize

        def q(seg):
            return dct_quantize(seg.astype(np.float32), 10).a_hat
        oq = admm.Quantizer("dct", 16, 30, 10)
    rho, eta1, e1, eta2, e2 = 1.0, 0.01, 5, 0.2, 10
    x, us, lams, _ = admm.run(prob, 3, rho, eta1, e1, eta2, e2, mode=mode, quant=oq)
    xr, ur, lr = _dense_quantized_iterations(prob, 3, rho, eta1, e1, eta2, e2, mode, q)
    np.testing.assert_allclose(x, xr, atol=1e-10)
    for m in range(2):
        np.testing.assert_allclose(us[m], ur[m], atol=1e-10)
        np.testing.assert_allclose(lams[m], lr[m], atol=1e-10)
    # the quantizer changed the exchanged image (the test is not vacuous)
    xn, _, _, _ = admm.run(prob, 3, rho, eta1, e1, eta2, e2, mode=mode)
    assert np.abs(x - xn).max() > 1e-3
    # every segment of x^K holds at most `levels` values (K-means) and each is
    # its own quantization (Q is idempotent on a quantized segment only approximately
    # for DCT, so this part is K-means only)
    if kind == "kmeans":
        for r0, nr in prob.segments:
            assert np.unique(x[r0:r0 + nr].astype(np.float32)).size <= levels
