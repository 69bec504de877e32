"""Pins of the P-APG oracle (oracle/papg.py) and of the shifted-slope ALCC it
calls for step 1 of Fig. 2.

Each test checks a fact that does not come from the oracle itself:
* C^T is the adjoint of C (eq. "C"): <C eta, theta> = <eta, C^T theta>;
* completing the square (eq. "g_gamma"): the Lagrangian and the block
  objective 1/2||y - (ybar + u)||^2 + gamma/2||xi - v/gamma||^2 differ by a
  constant that does not depend on eta;
* adding an affine function to the data moves the solution of eq.
  "regularize" by that function, so ALCC with a constant slope shift a on data
  ybar must match ALCC on ybar - X a, shifted back;
* the projection onto Q2 (eq. "lambda_dual") satisfies the variational
  inequality of a Euclidean projection;
* with K = 1 there are no cross-block pairs, so P-APG is one ALCC solve.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import papg as pp


def _data(N, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(N, n))
    yb = (X ** 2).sum(axis=1) + 0.1 * rng.normal(size=N)
    return X, yb


def test_block_partition_and_cross_mask():
    b = pp.block_of(12, 3)
    np.testing.assert_array_equal(b, [0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2])
    m = pp.cross_mask(12, 3)
    # K (K - 1) Nbar^2 cross pairs (the size of theta, Sec. II-B)
    assert m.sum() == 3 * 2 * 16
    assert not m[0, 3] and m[0, 4] and m[11, 0]
    with pytest.raises(ValueError):
        pp.block_of(10, 3)


def test_C_adjoint_is_the_adjoint_of_C():
    rng = np.random.default_rng(1)
    N, n, K = 12, 3, 3
    X = rng.normal(size=(N, n))
    y, xi = rng.normal(size=N), rng.normal(size=(N, n))
    Th, th_y = rng.normal(size=(N, N)), rng.normal(size=N)
    R, yy = pp.C_apply(X, y, xi, K)
    u, v = pp.C_adjoint(X, Th, th_y, K)
    lhs = float(np.sum(np.where(pp.cross_mask(N, K), Th, 0.0) * R)) + float(th_y @ yy)
    rhs = float(u @ y) + float(np.sum(v * xi))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # C eta is zero inside the diagonal blocks
    assert np.all(R[~pp.cross_mask(N, K)] == 0.0)


def test_completing_the_square_of_the_lagrangian():
    rng = np.random.default_rng(2)
    N, n, K, gamma = 10, 2, 2, 0.3
    X, yb = _data(N, n, 3)
    Th, th_y = np.abs(rng.normal(size=(N, N))), np.abs(rng.normal(size=N))
    u, v = pp.C_adjoint(X, Th, th_y, K)
    consts = []
    for s in range(5):
        y, xi = rng.normal(size=N), rng.normal(size=(N, n))
        Lval = pp.lagrangian(X, yb, gamma, K, Th, th_y, y, xi)
        block = 0.5 * np.sum((y - (yb + u)) ** 2) + 0.5 * gamma * np.sum((xi - v / gamma) ** 2)
        consts.append(Lval - block)
    expect = -float(u @ yb) - 0.5 * float(u @ u) - 0.5 * float(np.sum(v * v)) / gamma
    np.testing.assert_allclose(consts, expect, rtol=1e-12, atol=1e-12)


def test_zero_shift_is_the_plain_run():
    X, yb = _data(9, 2, 4)
    p = oracle.Params(gamma=0.05, inner_iters=30, max_outer=4)
    a = oracle.alcc(X, yb, p)
    b = oracle.alcc(X, yb, p, xi_shift=np.zeros_like(X))
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.xi, b.xi)


def test_constant_shift_equals_affine_change_of_data():
    # with xi = xi' + a for every point, the problem in (y, xi') on data ybar is
    # the plain problem in (y - X a, xi') on data ybar - X a
    X, yb = _data(10, 3, 5)
    a = np.array([0.7, -1.2, 0.4])
    p = oracle.Params(gamma=0.1, inner_iters=60, max_outer=5)
    sh = oracle.alcc(X, yb, p, xi_shift=np.tile(a, (10, 1)))
    pl = oracle.alcc(X, yb - X @ a, p)
    np.testing.assert_allclose(sh.y - X @ a, pl.y, rtol=0, atol=1e-10)
    np.testing.assert_allclose(sh.xi, pl.xi, rtol=0, atol=1e-10)


def test_projection_onto_Q2():
    rng = np.random.default_rng(6)
    N = 8
    for B in (math.inf, 3.0, 0.5):
        Th, th_y = rng.normal(size=(N, N)), rng.normal(size=N)
        P, p = pp.project_Q2(Th, th_y, B)
        assert np.all(P >= 0) and np.all(p >= 0)
        nrm = math.sqrt(np.sum(P * P) + np.sum(p * p))
        assert nrm <= B * (1 + 1e-12)
        for _ in range(20):
            Z, z = np.abs(rng.normal(size=(N, N))), np.abs(rng.normal(size=N))
            zn = math.sqrt(np.sum(Z * Z) + np.sum(z * z))
            if zn > B:
                Z, z = Z * (B / zn), z * (B / zn)
            # <v - Pi(v), z - Pi(v)> <= 0 for every z in Q2
            ip = np.sum((Th - P) * (Z - P)) + np.sum((th_y - p) * (z - p))
            assert ip <= 1e-10


def test_single_block_is_one_alcc_solve():
    X, yb = _data(10, 2, 7)
    p = oracle.Params(gamma=0.1, inner_iters=40, max_outer=4)
    r = pp.papg(X, yb, 1, 0.1, 2, p)
    d = oracle.alcc(X, yb, p)
    # no cross pairs; y > 0 after the shift keeps the y >= 0 multipliers at zero
    assert r.y_shift > 0 and np.all(r.th_y == 0.0)
    np.testing.assert_allclose(r.y, d.y, rtol=0, atol=1e-9)
    np.testing.assert_allclose(r.xi, d.xi, rtol=0, atol=1e-9)


def test_first_iteration_is_the_block_diagonal_problem():
    # theta^(2)_1 = 0: step 1 solves the K blocks with their own data and no shift
    X, yb = _data(12, 2, 8)
    p = oracle.Params(gamma=0.1, inner_iters=40, max_outer=4)
    r = pp.papg(X, yb, 2, 0.1, 1, p, y_shift=0.0)
    for i in range(2):
        s = slice(6 * i, 6 * i + 6)
        d = oracle.alcc(X[s], yb[s], p)
        np.testing.assert_array_equal(r.y[s], d.y)
        np.testing.assert_array_equal(r.xi[s], d.xi)
    # theta^(1)_1 = max(-C eta_1 / L, 0) on the cross pairs
    R, yy = pp.C_apply(X, r.y, r.xi, 2)
    np.testing.assert_allclose(r.Th, np.where(pp.cross_mask(12, 2), np.maximum(-R / r.L, 0.0), 0.0), rtol=0,
                               atol=1e-15)


def test_lipschitz_bound_dominates_sigma_max_of_C():
    # L_g = sigma_max(C)^2 / gamma (eq. "lischitz"), C built densely for a tiny case
    rng = np.random.default_rng(9)
    N, n, K, gamma = 6, 2, 2, 0.2
    X = rng.normal(size=(N, n))
    mask = pp.cross_mask(N, K)
    rows = []
    for i in range(N):
        for j in range(N):
            if mask[i, j]:
                r = np.zeros(N + N * n)
                r[i] += 1.0
                r[j] -= 1.0
                r[N + j * n:N + (j + 1) * n] = -(X[i] - X[j])
                rows.append(r)
    for i in range(N):
        r = np.zeros(N + N * n)
        r[i] = 1.0
        rows.append(r)
    C = np.array(rows)
    s2 = np.linalg.norm(C, 2) ** 2
    Lb = pp.lipschitz_bound(X, gamma)
    assert s2 / gamma <= Lb
    # and C_apply agrees with the dense matrix
    y, xi = rng.normal(size=N), rng.normal(size=(N, n))
    R, yy = pp.C_apply(X, y, xi, K)
    dense = C @ np.concatenate([y, xi.reshape(-1)])
    np.testing.assert_allclose(dense, np.concatenate([R[mask], yy]), rtol=0, atol=1e-12)


def test_step1_minimises_the_lagrangian_slsqp():
    # eq. "g_gamma" at a nonzero theta on a tiny instance, minimised directly by
    # scipy's SLSQP over Q1 (the within-block constraints); the block ALCC runs
    # a long fixed schedule, so the two agree to the ALCC's accuracy
    from scipy.optimize import minimize
    rng = np.random.default_rng(10)
    N, n, K, gamma = 6, 1, 2, 0.5
    X = np.sort(rng.uniform(-1, 1, size=(N, n)), axis=0)
    yb = (X[:, 0] ** 2) + 0.05 * rng.normal(size=N) + 2.0
    Th = np.where(pp.cross_mask(N, K), np.abs(rng.normal(size=(N, N))) * 0.3, 0.0)
    th_y = np.abs(rng.normal(size=N)) * 0.1
    p = oracle.Params(gamma=gamma, inner_iters=400, max_outer=14)
    y, xi, _, _ = pp.step1(X, yb, gamma, K, Th, th_y, p)

    def f(z):
        return pp.lagrangian(X, yb, gamma, K, Th, th_y, z[:N], z[N:].reshape(N, n))

    blk = pp.block_of(N, K)
    cons = []
    for i in range(N):
        for j in range(N):
            if i != j and blk[i] == blk[j]:
                cons.append({"type": "ineq",
                             "fun": (lambda z, i=i, j=j: z[i] - z[j] - z[N + j] * (X[i, 0] - X[j, 0]))})
    z0 = np.concatenate([yb, np.zeros(N)])
    res = minimize(f, z0, method="SLSQP", constraints=cons, options={"ftol": 1e-14, "maxiter": 500})
    assert res.success
    np.testing.assert_allclose(y, res.x[:N], rtol=0, atol=2e-3)
    np.testing.assert_allclose(xi[:, 0], res.x[N:], rtol=0, atol=2e-2)
    assert f(np.concatenate([y, xi[:, 0]])) <= res.fun + 1e-4


def test_trace_identity_and_gradient_variant():
    # gap = theta2^T C eta is the primal objective minus the Lagrangian
    # (eq. "g_gamma"); without momentum the first two iterations coincide with
    # P-APG (beta_1 = (t_1 - 1)/t_2 = 0) and the third differs
    X, yb = _data(12, 2, 11)
    p = oracle.Params(gamma=0.1, inner_iters=30, max_outer=3)
    a = pp.papg(X, yb, 2, 0.1, 3, p, record=True)
    b = pp.papg(X, yb, 2, 0.1, 3, p, record=True, accelerate=False)
    for t in a.trace + b.trace:
        assert abs((t["primal"] - t["g"]) - t["gap"]) <= 1e-10 * (1 + abs(t["primal"]))
    for k in ("theta_norm", "infeas_cross", "gap"):
        assert a.trace[0][k] == b.trace[0][k] and a.trace[1][k] == b.trace[1][k]
    assert a.trace[2]["theta_norm"] != b.trace[2]["theta_norm"]
