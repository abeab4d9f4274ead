"""Pins of the regularization block's oracle (oracle/reg.py) against closed
forms, brute-force minimization and an independent algorithm."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import admm as oadmm
from oracle import joseph
from oracle import reg


def test_grad_on_ramps_and_div_adjoint():
    n, m = 5, 7
    ii, jj = np.meshgrid(np.arange(n, dtype=float), np.arange(m, dtype=float), indexing="ij")
    g1, g2 = reg.grad(3.0 * ii + 2.0 * jj)
    # a ramp's forward differences are its slopes, zero across the last row / column
    np.testing.assert_array_equal(g1[:-1], 3.0)
    np.testing.assert_array_equal(g1[-1], 0.0)
    np.testing.assert_array_equal(g2[:, :-1], 2.0)
    np.testing.assert_array_equal(g2[:, -1], 0.0)
    rng = np.random.default_rng(0)
    for _ in range(5):
        u = rng.standard_normal((n, m))
        p1, p2 = rng.standard_normal((n, m)), rng.standard_normal((n, m))
        a1, a2 = reg.grad(u)
        lhs = np.sum(a1 * p1) + np.sum(a2 * p2)
        assert abs(lhs + np.sum(u * reg.div(p1, p2))) <= 1e-12 * (1 + abs(lhs))


def test_tv_of_step_and_ramp():
    n = 8
    step = np.zeros((n, n))
    step[:, n // 2:] = 1.0
    assert reg.tv(step) == pytest.approx(n)             # one unit jump per row
    ramp = np.tile(np.arange(n, dtype=float)[:, None], (1, n))
    assert reg.tv(ramp) == pytest.approx((n - 1) * n)   # unit slope down every column
    assert reg.tv(np.full((n, n), 3.5)) == 0.0


def test_prox_tikhonov_minimizes_its_objective():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(6)
    theta = 0.7
    obj = lambda z: 0.5 * np.sum((z - v) ** 2) + 0.5 * theta * np.sum(z * z)
    ref = minimize(obj, np.zeros(6), method="BFGS", options={"gtol": 1e-12}).x
    np.testing.assert_allclose(reg.prox_tikhonov(v, theta), ref, atol=1e-7)


@pytest.mark.parametrize("a,b,theta", [(1.0, 0.2, 0.1), (1.0, 0.9, 0.1), (-0.3, 0.5, 0.25), (2.0, -1.0, 2.0)])
def test_prox_tv_two_pixels_closed_form(a, b, theta):
    """Two pixels in one column: TV = |z1 - z0|, so the prox shrinks the pair
    towards each other by theta, or merges them at their mean."""
    v = np.array([[a], [b]])
    z, _ = reg.prox_tv(v, theta, iters=4000)
    if abs(a - b) <= 2 * theta:
        ref = np.full(2, 0.5 * (a + b))
    else:
        s = np.sign(a - b)
        ref = np.array([a - theta * s, b + theta * s])
    np.testing.assert_allclose(z.reshape(-1), ref, atol=1e-6)


def test_prox_tv_matches_primal_dual_solver():
    """6x6 image: the prox against the primal-dual method of Chambolle and Pock
    (J. Math. Imaging Vis. 40, 2011) on the primal problem
    min_z 1/2 ||z - v||^2 + theta ||grad z||_{2,1}, an independent method."""
    rng = np.random.default_rng(2)
    theta = 0.3
    v = rng.standard_normal((6, 6))
    z = v.copy()
    zb = v.copy()
    y1, y2 = np.zeros_like(v), np.zeros_like(v)
    tau = sigma = 0.3                                   # tau sigma ||grad||^2 <= 0.72 < 1
    for _ in range(20000):
        g1, g2 = reg.grad(zb)
        y1, y2 = y1 + sigma * g1, y2 + sigma * g2
        scale = np.maximum(1.0, np.sqrt(y1 * y1 + y2 * y2) / theta)   # project onto |y| <= theta
        y1, y2 = y1 / scale, y2 / scale
        z_new = (z + tau * reg.div(y1, y2) + tau * v) / (1.0 + tau)
        zb = 2.0 * z_new - z
        z = z_new
    zc, _ = reg.prox_tv(v, theta, iters=20000)
    prox_obj = lambda w: 0.5 * np.sum((w - v) ** 2) + theta * reg.tv(w)
    assert prox_obj(zc) == pytest.approx(prox_obj(z), rel=1e-9, abs=1e-9)
    np.testing.assert_allclose(zc, z, atol=1e-5)


def test_prox_tv_limits():
    rng = np.random.default_rng(3)
    c = np.full((4, 5), 1.25)
    z, (p1, p2) = reg.prox_tv(c, 0.5, iters=50)
    np.testing.assert_array_equal(z, c)                  # TV(constant) = 0
    assert not p1.any() and not p2.any()
    v = rng.standard_normal((4, 4))
    z, _ = reg.prox_tv(v, 50.0, iters=20000)             # huge weight: the constant of the same mean
    np.testing.assert_allclose(z, np.full_like(v, v.mean()), atol=1e-3)
    z0, _ = reg.prox_tv(v, 0.0, iters=10)
    np.testing.assert_array_equal(z0, v)


def test_segment_update_with_block_tends_to_weighted_target():
    rng = np.random.default_rng(4)
    x, u, lam, tz = (rng.standard_normal(10) for _ in range(4))
    rho, rho_z = 1.5, 0.5
    out = reg.x_update_segment(x, u, lam, rho, tz, rho_z, eta2=0.2, e2=400)
    # the segment objective rho/2 ||x - t_m||^2 + rho_z/2 ||x - t_z||^2 has its minimum
    # at the rho-weighted mean of the two targets
    ref = minimize(lambda y: 0.5 * rho * np.sum((y - u - lam / rho) ** 2) + 0.5 * rho_z * np.sum((y - tz) ** 2),
                   np.zeros(10), method="BFGS", options={"gtol": 1e-12}).x
    np.testing.assert_allclose(out, ref, atol=1e-7)


def test_segment_update_with_block_closed_form():
    """E2 steps on the block's quadratic: a linear recurrence with factor
    1 - eta2 (rho + rho_z) towards the rho-weighted mean of the two targets."""
    rng = np.random.default_rng(6)
    x, u, lam, tz = (rng.standard_normal((3, 7)) for _ in range(4))
    rho, rho_z, eta2 = 0.8, 0.3, 0.25
    t = (rho * (u + lam / rho) + rho_z * tz) / (rho + rho_z)
    for e2 in (0, 1, 3, 10):
        ref = t + (1 - eta2 * (rho + rho_z)) ** e2 * (x - t)
        np.testing.assert_allclose(reg.x_update_segment(x, u, lam, rho, tz, rho_z, eta2, e2), ref, atol=1e-14)


def _tiny_problem(n=6, n_ang=8, nodes=2, seed=5):
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(0, np.pi, n_ang))
    nb = int(np.ceil(np.sqrt(2) * n)) + 1
    truth = np.zeros((n, n))
    truth[1:4, 2:5] = 1.0
    truth[3:5, 1:3] = 0.5
    d = joseph.project(truth, th, nb) + 0.01 * rng.standard_normal((n_ang, nb))
    parts = [np.arange(m, n_ang, nodes) for m in range(nodes)]
    rows = n // nodes
    segs = [(m * rows, rows if m < nodes - 1 else n - m * rows) for m in range(nodes)]
    prob = oadmm.Problem(n, nb, [th[p] for p in parts], [d[p] for p in parts], segs, truth)
    A = [joseph.dense_matrix(n, nb, th[p]) for p in parts]
    return prob, A, [d[p] for p in parts]


def test_admm_with_tikhonov_block_reaches_regularized_least_squares():
    """Exact u-updates and the averaging x-update: the iterates converge to the
    minimizer of 1/2 sum_m ||P_m x - d_m||^2 + mu/2 ||x||^2, the solution of
    (sum_m P_m^T P_m + mu I) x = sum_m P_m^T d_m."""
    prob, A, d = _tiny_problem()
    mu = 0.5
    H = sum(a.T @ a for a in A) + mu * np.eye(prob.n ** 2)
    rhs = sum(a.T @ dm.reshape(-1) for a, dm in zip(A, d))
    ref = np.linalg.solve(H, rhs).reshape(prob.n, prob.n)
    r = reg.Reg(kind=reg.TIKHONOV, mu=mu, rho=1.0)
    x, _, _, tr = oadmm.run(prob, 400, 1.0, 0.0, 0, 0.0, 0, mode="avg", exact_u=True, reg=r)
    np.testing.assert_allclose(x, ref, atol=1e-6)
    z, nu, _ = tr.reg_state
    np.testing.assert_allclose(z, x, atol=1e-6)          # the block's copy agrees with x


def test_admm_with_tv_block_matches_fista():
    """TV: the same fixed point as accelerated proximal gradient (FISTA) on
    F(x) = 1/2 sum_m ||P_m x - d_m||^2 + mu TV(x), an independent method."""
    prob, A, d = _tiny_problem()
    mu = 0.05
    At = np.vstack(A)
    dt = np.concatenate([dm.reshape(-1) for dm in d])
    F = lambda x: 0.5 * np.sum((At @ x.reshape(-1) - dt) ** 2) + mu * reg.tv(x)
    L = np.linalg.norm(At.T @ At, 2)
    n = prob.n
    x = y = np.zeros((n, n))
    t, p = 1.0, None
    for _ in range(400):
        g = (At.T @ (At @ y.reshape(-1) - dt)).reshape(n, n)
        x_new, p = reg.prox_tv(y - g / L, mu / L, iters=60, p=p)
        t_new = 0.5 * (1 + np.sqrt(1 + 4 * t * t))
        y = x_new + ((t - 1) / t_new) * (x_new - x)
        x, t = x_new, t_new
    r = reg.Reg(kind=reg.TV, mu=mu, rho=1.0, tv_iters=60)
    xa, _, _, _ = oadmm.run(prob, 500, 1.0, 0.0, 0, 0.0, 0, mode="avg", exact_u=True, reg=r)
    assert F(xa) == pytest.approx(F(x), rel=2e-5)
    np.testing.assert_allclose(xa, x, atol=2e-3)


def test_dual_update_of_block():
    z, x, nu = np.array([1.0, 2.0]), np.array([0.5, 2.5]), np.array([0.1, -0.1])
    np.testing.assert_allclose(reg.dual_update(nu, z, x, 2.0), [1.1, -1.1])
