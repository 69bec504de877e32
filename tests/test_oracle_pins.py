"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each uses an independent route
(explicit constraint matrices built row by row, SVD, the NNLS dual of the QP,
brute-force active sets, hand-derived closed forms, finite differences, bounds
from the paper, exact symmetries of the problem).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import refqp

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_problem(N, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(N, n))
    y = rng.normal(size=N)
    xi = rng.normal(size=(N, n))
    theta = np.abs(rng.normal(size=(N, N)))
    return X, y, xi, theta


# --------------------------------------------------------------------------
# Operators (eq. "original_compact"; Sec. II-E matrix-free products)
# --------------------------------------------------------------------------

def test_forward_matches_explicit_rows():
    X, y, xi, _ = _rand_problem(7, 3, 1)
    A1, A2 = refqp.explicit_A(X)
    r = A1 @ y + A2 @ xi.ravel()
    R = oracle.forward(X, y, xi)
    np.testing.assert_allclose(refqp.matrix_to_pairs(R), r, rtol=0, atol=1e-13)
    assert np.all(np.diag(R) == 0.0)


def test_adjoint_matches_explicit_transpose():
    X, _, _, Z = _rand_problem(8, 3, 2)
    A1, A2 = refqp.explicit_A(X)
    z = refqp.matrix_to_pairs(Z)
    u, v = oracle.adjoint(X, Z)
    np.testing.assert_allclose(u, A1.T @ z, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v.ravel(), A2.T @ z, rtol=0, atol=1e-12)


def test_adjoint_ignores_diagonal_and_sums_to_zero():
    X, _, _, Z = _rand_problem(40, 4, 3)
    u, v = oracle.adjoint(X, Z)
    Z2 = Z.copy()
    np.fill_diagonal(Z2, 1e6)
    u2, v2 = oracle.adjoint(X, Z2)
    np.testing.assert_array_equal(u, u2)
    np.testing.assert_array_equal(v, v2)
    # 1^T A1 = 0: every A1 row holds one +1 and one -1
    assert abs(u.sum()) < 1e-10 * np.abs(u).sum()


def test_dot_product_identity_at_moderate_size():
    X, y, xi, Z = _rand_problem(120, 5, 4)
    np.fill_diagonal(Z, 0.0)
    R = oracle.forward(X, y, xi)
    u, v = oracle.adjoint(X, Z)
    lhs = float(np.sum(R * Z))
    rhs = float(y @ u + np.sum(xi * v))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.abs(R * Z).sum())


def test_single_entry_helpers_match_full():
    X, y, xi, Z = _rand_problem(30, 3, 5)
    R = oracle.forward(X, y, xi)
    u, v = oracle.adjoint(X, Z)
    for (i, j) in [(0, 1), (5, 29), (17, 3)]:
        assert oracle.pair_residual(X, y, xi, i, j) == R[i, j]
    for m in [0, 13, 29]:
        um, vm = oracle.adjoint_one(X, m, Z[m], Z[:, m])
        assert abs(um - u[m]) < 1e-12
        np.testing.assert_allclose(vm, v[m], atol=1e-12)
        # the sampled-output checker of the full-size tests: row m and column m of R
        row, col = oracle.residual_row_col(X, y, xi, m)
        np.testing.assert_allclose(row, R[m], rtol=0, atol=1e-13)
        np.testing.assert_allclose(col, R[:, m], rtol=0, atol=1e-13)
        assert row[m] == 0.0 and col[m] == 0.0


# --------------------------------------------------------------------------
# sigma_max closed forms (used for L^y, L^xi in Fig. 3 step 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,n,seed", [(9, 3, 0), (25, 2, 1), (12, 1, 2)])
def test_sigma2_closed_forms_match_svd(N, n, seed):
    X = np.random.default_rng(seed).uniform(-1, 1, size=(N, n))
    A1, A2 = refqp.explicit_A(X)
    s1 = np.linalg.svd(A1, compute_uv=False)[0] ** 2
    s2 = np.linalg.svd(A2, compute_uv=False)[0] ** 2
    assert abs(oracle.sigma2_A1(N) - s1) <= 1e-10 * s1
    assert abs(oracle.sigma2_A2(X) - s2) <= 1e-10 * s2


# --------------------------------------------------------------------------
# Gradient of P_k (eq. "subproblem" and the formulas after it)
# --------------------------------------------------------------------------

def test_grad_P_central_differences():
    N, n = 10, 2
    X, y, xi, theta = _rand_problem(N, n, 6)
    theta *= 0.5
    gamma, mu = 0.3, 0.7
    ybar = np.random.default_rng(7).normal(size=N)
    gy, gxi = oracle.grad_P(X, ybar, gamma, mu, theta, y, xi)
    h = 1e-6
    for m in range(N):
        e = np.zeros(N); e[m] = h
        fd = (oracle.P_value(X, ybar, gamma, mu, theta, y + e, xi)
              - oracle.P_value(X, ybar, gamma, mu, theta, y - e, xi)) / (2 * h)
        assert abs(fd - gy[m]) < 1e-6 * (1 + abs(gy[m]))
    for m in range(N):
        for k in range(n):
            E = np.zeros((N, n)); E[m, k] = h
            fd = (oracle.P_value(X, ybar, gamma, mu, theta, y, xi + E)
                  - oracle.P_value(X, ybar, gamma, mu, theta, y, xi - E)) / (2 * h)
            assert abs(fd - gxi[m, k]) < 1e-6 * (1 + abs(gxi[m, k]))


def test_grad_h_explicit_matrices():
    N, n = 6, 2
    X, y, xi, theta = _rand_problem(N, n, 8)
    A1, A2 = refqp.explicit_A(X)
    w = np.maximum(refqp.matrix_to_pairs(theta) - (A1 @ y + A2 @ xi.ravel()), 0.0)
    mu, gamma = 1.0, 1.0
    ybar = y.copy()
    gy, gxi = oracle.grad_P(X, ybar, gamma, mu, theta, y, xi)
    np.testing.assert_allclose(gy, -(A1.T @ w), atol=1e-12)
    np.testing.assert_allclose(gxi.ravel() - gamma * xi.ravel(), -(A2.T @ w), atol=1e-12)


# --------------------------------------------------------------------------
# The converged ALCC solve against exact solutions of eq. "regularize"
# --------------------------------------------------------------------------

def _tight(**kw):
    base = dict(kkt_tol=1e-9, max_outer=40, max_inner=20000)
    base.update(kw)
    return oracle.Params(**base)


@pytest.mark.parametrize("case", json.load(open(os.path.join(HERE, "golden", "closed_forms.json")))["cases"],
                         ids=lambda c: c["name"])
def test_alcc_closed_form_cases(case):
    X = np.array(case["X"]); ybar = np.array(case["ybar"])
    res = oracle.alcc(X, ybar, _tight(gamma=case["gamma"]))
    np.testing.assert_allclose(res.y, case["y"], atol=2e-6)
    np.testing.assert_allclose(res.xi, case["xi"], atol=2e-5)


@pytest.mark.parametrize("step_scale", [0.5, 1.0])
@pytest.mark.parametrize("N,n,seed", [(4, 1, 0), (4, 2, 1)])
def test_alcc_matches_active_set_brute_force(N, n, seed, step_scale):
    """step_scale 1.0 is Fig. 4's step 1/L as printed, 0.5 the default reading."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(N, n))
    ybar = np.sum(X ** 2, axis=1) + 0.3 * rng.normal(size=N)
    gamma = 0.05
    y_ref, xi_ref = refqp.solve_qp_active_set(X, ybar, gamma)
    res = oracle.alcc(X, ybar, _tight(gamma=gamma, step_scale=step_scale))
    np.testing.assert_allclose(res.y, y_ref, atol=1e-5)
    np.testing.assert_allclose(res.xi, xi_ref, atol=1e-4)


@pytest.mark.parametrize("step_scale", [0.5, 1.0])
def test_alcc_matches_nnls_dual_qp(step_scale):
    p = synth.quadratic_uniform(30, 2, 0.1, seed=3)
    gamma = 1e-2
    y_ref, xi_ref, lam = refqp.solve_qp_nnls(p.X, p.ybar, gamma)
    # the reference itself satisfies the KKT conditions
    m = oracle.kkt_measures(p.X, p.ybar, gamma, y_ref, xi_ref, refqp.pairs_to_matrix(lam, 30))
    assert m["kkt"] < 1e-8
    res = oracle.alcc(p.X, p.ybar, _tight(gamma=gamma, kkt_tol=1e-7, step_scale=step_scale))
    assert res.converged
    assert np.linalg.norm(res.y - y_ref) <= 1e-4 * np.linalg.norm(y_ref)
    assert np.linalg.norm(res.xi - xi_ref) <= 1e-3 * np.linalg.norm(xi_ref)


def test_brute_force_and_nnls_agree():
    # the two references pin each other on a tiny case
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, size=(4, 2))
    ybar = rng.normal(size=4)
    y1, xi1 = refqp.solve_qp_active_set(X, ybar, 0.1)
    y2, xi2, _ = refqp.solve_qp_nnls(X, ybar, 0.1)
    np.testing.assert_allclose(y1, y2, atol=1e-9)
    np.testing.assert_allclose(xi1, xi2, atol=1e-9)


# --------------------------------------------------------------------------
# Bounds and special cases
# --------------------------------------------------------------------------

def test_exact_recovery_bound_noise_free():
    # (ybar, grad f0) is feasible for noise-free convex data, so the optimum has
    # 1/2||y - ybar||^2 + gamma/2||xi||^2 <= gamma/2 ||grad f0||_F^2 (form of Lemma 1).
    p = synth.quadratic_uniform(40, 2, sigma=0.0, seed=5)
    gamma = 1e-3
    res = oracle.alcc(p.X, p.ybar, _tight(gamma=gamma, kkt_tol=1e-8))
    bound = math.sqrt(gamma) * np.linalg.norm(p.grad_f0)
    assert np.linalg.norm(res.y - p.ybar) <= bound * 1.001
    obj = 0.5 * np.sum((res.y - p.ybar) ** 2) + 0.5 * gamma * np.sum(res.xi ** 2)
    assert obj <= 0.5 * gamma * np.sum(p.grad_f0 ** 2) * 1.001


def test_objective_no_larger_than_affine_fit():
    p = synth.logsumexp_gaussian(60, 3, seed=2)
    gamma = 1e-3
    res = oracle.alcc(p.X, p.ybar, _tight(gamma=gamma, kkt_tol=1e-7))
    M = np.hstack([p.X, np.ones((60, 1))])
    coef = np.linalg.lstsq(M, p.ybar, rcond=None)[0]
    aff = 0.5 * np.sum((M @ coef - p.ybar) ** 2) + 0.5 * gamma * 60 * np.sum(coef[:3] ** 2)
    obj = 0.5 * np.sum((res.y - p.ybar) ** 2) + 0.5 * gamma * np.sum(res.xi ** 2)
    assert obj <= aff * (1 + 1e-6)


def test_constant_data_is_a_fixed_point():
    p = synth.constant_data(25, 3, value=1.5)
    res = oracle.alcc(p.X, p.ybar, oracle.Params(inner_iters=30, max_outer=3))
    np.testing.assert_allclose(res.y, p.ybar, atol=1e-12)
    assert np.max(np.abs(res.xi)) < 1e-12
    assert np.max(np.abs(res.theta)) < 1e-12


def test_n1_small_gamma_matches_slope_formulation():
    # n = 1: with the points sorted, convexity is nondecreasing slopes (a QP on y only);
    # Lemma 1 bounds ||y(gamma) - y*|| <= B_xi sqrt(gamma).
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, size=25)
    ybar = x ** 2 + 0.2 * rng.normal(size=25)
    y_star = refqp.convex_1d_ls(x, ybar)
    gamma = 1e-6
    res = oracle.alcc(x[:, None], ybar, _tight(gamma=gamma, kkt_tol=1e-8, max_outer=60))
    slopes = np.diff(y_star[np.argsort(x)]) / np.diff(np.sort(x))
    B_xi = math.sqrt(np.sum(slopes ** 2) * 2 + 4 * np.max(slopes ** 2))  # loose bound on ||xi*||
    assert np.linalg.norm(res.y - y_star) <= B_xi * math.sqrt(gamma) + 1e-3


def test_kkt_converged_run_is_feasible():
    p = synth.workload("small_quadratic")
    res = oracle.alcc(p.X[:60], p.ybar[:60], oracle.Params(kkt_tol=1e-5))
    assert res.converged
    last = res.history[-1]
    assert last["kkt"] <= 1e-5
    assert last["infeas_norm"] < 1e-1   # the paper's termination threshold (Sec. III)


# --------------------------------------------------------------------------
# Exact symmetries of a fixed schedule
# --------------------------------------------------------------------------

FIXED = oracle.Params(inner_iters=20, max_outer=3)


def test_translation_equivariance():
    p = synth.quadratic_uniform(30, 2, seed=4)
    a = oracle.alcc(p.X, p.ybar, FIXED)
    b = oracle.alcc(p.X, p.ybar + 3.25, FIXED)
    np.testing.assert_allclose(b.y, a.y + 3.25, atol=1e-11)
    np.testing.assert_allclose(b.xi, a.xi, atol=1e-10)


def test_positive_homogeneity():
    p = synth.quadratic_uniform(30, 2, seed=4)
    a = oracle.alcc(p.X, p.ybar, FIXED)
    b = oracle.alcc(p.X, 2.5 * p.ybar, FIXED)
    np.testing.assert_allclose(b.y, 2.5 * a.y, rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(b.xi, 2.5 * a.xi, rtol=1e-9, atol=1e-10)


def test_permutation_equivariance():
    p = synth.quadratic_uniform(30, 2, seed=4)
    perm = np.random.default_rng(0).permutation(30)
    a = oracle.alcc(p.X, p.ybar, FIXED)
    b = oracle.alcc(p.X[perm], p.ybar[perm], FIXED)
    np.testing.assert_allclose(b.y, a.y[perm], atol=1e-11)
    np.testing.assert_allclose(b.xi, a.xi[perm], atol=1e-10)


# --------------------------------------------------------------------------
# MAPG rate (Sec. II-E, bound after Lemma 3)
# --------------------------------------------------------------------------

def test_mapg_rate_bound():
    p = synth.quadratic_uniform(20, 2, seed=6)
    X, ybar = p.X, p.ybar
    gamma, mu = 1e-2, 0.05
    theta = 0.01 * np.abs(np.random.default_rng(1).normal(size=(20, 20)))
    yhat, xihat, Bbar, By, Bxi = oracle.affine_fit(X, ybar, gamma)
    Ly = 1 / mu + oracle.sigma2_A1(20)
    Lxi = gamma / mu + oracle.sigma2_A2(X)
    ys, xs, _ = oracle.mapg(X, ybar, gamma, mu, theta, Ly, Lxi, yhat, xihat, By, Bxi,
                            0, 0, 30000, adaptive=False)
    Pstar = oracle.P_value(X, ybar, gamma, mu, theta, ys, xs)
    d0 = Ly * np.sum((yhat - ys) ** 2) + Lxi * np.sum((xihat - xs) ** 2)
    for l in [1, 3, 10, 30, 100, 300]:
        yl, xl, _ = oracle.mapg(X, ybar, gamma, mu, theta, Ly, Lxi, yhat, xihat, By, Bxi,
                                0, 0, l, adaptive=False)
        gap = oracle.P_value(X, ybar, gamma, mu, theta, yl, xl) - Pstar
        assert gap >= -1e-9
        assert gap <= 4 * d0 / (l + 1) ** 2 + 1e-9


def test_affine_fit_full_rank_and_degenerate():
    """The start point: with N > n and points in general position the fit is
    the ordinary least-squares fit on [X 1] (numpy's solver on the uncentred
    system); with N <= n it interpolates, and its slope is the shortest one,
    i.e. it lies in the span of the centred points."""
    rng = np.random.default_rng(0)
    X = rng.normal(size=(30, 4))
    ybar = rng.normal(size=30)
    yhat, xihat, Bbar, By, Bxi = oracle.affine_fit(X, ybar, 1e-3)
    M = np.hstack([X, np.ones((30, 1))])
    coef = np.linalg.lstsq(M, ybar, rcond=None)[0]
    np.testing.assert_allclose(yhat, M @ coef, rtol=0, atol=1e-12)
    np.testing.assert_allclose(xihat[7], coef[:4], rtol=0, atol=1e-12)
    # feasibility: every residual of the affine point is zero
    assert np.abs(oracle.forward(X, yhat, xihat)).max() < 1e-12
    # degenerate: 3 points in 5 dimensions
    X = rng.normal(size=(3, 5))
    ybar = rng.normal(size=3)
    yhat, xihat, Bbar, By, Bxi = oracle.affine_fit(X, ybar, 1e-3)
    np.testing.assert_allclose(yhat, ybar, rtol=0, atol=1e-12)
    Xc = X - X.mean(axis=0)
    a = xihat[0]
    # a is in the row space of Xc: its component orthogonal to it vanishes
    P = np.linalg.pinv(Xc) @ Xc
    np.testing.assert_allclose(P @ a, a, rtol=0, atol=1e-12)
    assert abs(Bbar - np.sqrt(1e-3 * 3 * a @ a)) < 1e-12


# --------------------------------------------------------------------------
# MAPG steps (Fig. 4) on a hand-derived example, and the ball projection
# --------------------------------------------------------------------------

def _mapg_golden():
    g = json.load(open(os.path.join(HERE, "golden", "mapg_momentum.json")))
    pr = g["problem"]
    args = dict(X=np.array(pr["X"]), ybar=np.array(pr["ybar"]), gamma=pr["gamma"], mu=pr["mu"],
                theta=np.array(pr["theta"]), Ly=pr["Ly"], Lxi=pr["Lxi"], y0=np.array(pr["y0"]),
                xi0=np.array(pr["xi0"]), By=pr["ball_radius"], Bxi=pr["ball_radius"])
    return g, args, pr["step_scale"]


def test_mapg_momentum_hand_example():
    """t_l, the extrapolation weights and every iterate of the first five MAPG
    steps against their hand derivation (the penalty stays idle, so the run is
    the accelerated method on a known quadratic)."""
    g, a, s = _mapg_golden()
    for lmax in range(1, 6):
        trace = []
        y, xi, used = oracle.mapg(a["X"], a["ybar"], a["gamma"], a["mu"], a["theta"], a["Ly"], a["Lxi"],
                                  a["y0"], a["xi0"], a["By"], a["Bxi"], 0.0, 0.0, lmax, step_scale=s,
                                  adaptive=False, trace=trace)
        assert used == lmax
        np.testing.assert_array_equal(y, a["ybar"])
        b = g["b1"][lmax - 1]
        np.testing.assert_allclose(xi.ravel(), [-b, b], rtol=1e-14, atol=0)
    assert [row[0] for row in trace] == [1, 2, 3, 4, 5]
    np.testing.assert_allclose([row[3] for row in trace], g["t"], rtol=1e-15, atol=0)
    np.testing.assert_allclose([row[4] for row in trace], g["beta"], rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose([row[2] for row in trace], g["xi_move"], rtol=1e-14, atol=0)
    assert all(row[1] == 0.0 for row in trace)


@pytest.mark.parametrize("alpha_xi,stop", [(0.36, 1), (0.2, 3), (0.11, 4), (0.1074868, 5), (0.01, 5)])
def test_mapg_alpha_stop_returns_that_steps_iterate(alpha_xi, stop):
    """The adaptive test stops after the first step whose two block moves are
    within alpha and returns that step's projected iterate (not the
    extrapolated one); otherwise the run ends at l_max = 5."""
    g, a, s = _mapg_golden()
    y, xi, used = oracle.mapg(a["X"], a["ybar"], a["gamma"], a["mu"], a["theta"], a["Ly"], a["Lxi"],
                              a["y0"], a["xi0"], a["By"], a["Bxi"], 0.0, alpha_xi, 5, step_scale=s,
                              adaptive=True)
    assert used == stop
    b = g["b1"][stop - 1]
    np.testing.assert_allclose(xi.ravel(), [-b, b], rtol=1e-14, atol=0)
    np.testing.assert_array_equal(y, a["ybar"])


def test_project_ball_hand_values_and_variational_inequality():
    """Euclidean projection onto a ball (Q_y, Q_xi of Sec. II-E): hand values
    inside, outside and on the sphere, and the characterisation of the
    projection onto a closed convex set: P(v) lies in the ball and
    <v - P(v), z - P(v)> <= 0 for every z in it."""
    o = np.zeros(2)
    np.testing.assert_allclose(oracle.project_ball(np.array([3.0, 4.0]), o, 1.0), [0.6, 0.8], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(oracle.project_ball(np.array([0.1, -0.2]), o, 1.0), [0.1, -0.2])
    c = np.array([1.0, 1.0])
    np.testing.assert_allclose(oracle.project_ball(np.array([1.0, 5.0]), c, 2.0), [1.0, 3.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.project_ball(np.array([-2.0, -3.0]), c, 2.5), [-0.5, -1.0], rtol=0,
                               atol=1e-15)
    np.testing.assert_array_equal(oracle.project_ball(np.array([1.0, 3.0]), c, 2.0), [1.0, 3.0])
    rng = np.random.default_rng(8)
    for trial in range(60):
        shape = (7,) if trial % 2 else (4, 3)          # vectors and slope arrays alike
        cen = rng.normal(size=shape)
        v = cen + rng.normal(size=shape) * rng.choice([0.1, 1.0, 5.0])
        r = float(rng.uniform(0.2, 3.0))
        p = oracle.project_ball(v, cen, r)
        assert p.shape == v.shape
        assert np.linalg.norm(p - cen) <= r * (1 + 1e-13)
        if np.linalg.norm(v - cen) <= r:
            np.testing.assert_array_equal(p, v)
        d = rng.normal(size=(200,) + shape)
        norms = np.sqrt(np.sum(d.reshape(200, -1) ** 2, axis=1)).reshape((200,) + (1,) * len(shape))
        u = rng.uniform(0, 1, size=(200,) + (1,) * len(shape)) ** (1.0 / v.size)
        Z = cen + d / norms * r * u
        Z[0] = cen + (p - cen)                          # a point on the sphere next to P(v)
        vi = np.sum((Z - p) * (v - p), axis=tuple(range(1, 1 + len(shape))))
        assert np.all(vi <= 1e-12 * (1 + np.linalg.norm(v - cen) * r))
