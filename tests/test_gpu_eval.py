"""GPU parity of the estimator evaluation (cr_eval) against the FP64 oracle.

Every case prints its name, sizes and seed before touching the GPU."""
import sys

import numpy as np
import pytest

from oracle import estimator
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_7220_amd as cr
    return cr


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _planes(N, n, seed, feasible=False):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(N, n))
    if feasible:
        # tangent planes of the convex f(x) = log sum_k exp(a_k^T x): every constraint holds
        A = rng.normal(size=(9, n))
        Z = X @ A.T
        zmax = Z.max(axis=1, keepdims=True)
        E = np.exp(Z - zmax)
        y = zmax[:, 0] + np.log(E.sum(axis=1))
        xi = (E / E.sum(axis=1, keepdims=True)) @ A
    else:
        y = rng.normal(size=N)
        xi = rng.normal(size=(N, n))
    return X, y, xi


# Tolerance: the device forms d_l + xi_l^T q with FP64 fused multiply-adds, the
# oracle y_l + xi_l^T (q - x_l); both round within a few ulps of the terms'
# magnitude (|y| + |xi| (|q| + |x|) <= ~50 here).
TOL = 1e-12


def _check(cr, X, y, xi, Q, sample=None):
    f, arg = cr.evaluate(dev(X), dev(y), dev(xi), dev(Q))
    f, arg = host(f), host(arg)
    idx = np.arange(Q.shape[0]) if sample is None else sample
    fo, ao = estimator.evaluate(X, y, xi, Q[idx])
    scale = 1.0 + np.abs(y).max() + np.abs(xi).max() * (np.abs(Q).max() + np.abs(X).max()) * X.shape[1]
    err = np.abs(f[idx] - fo).max() / scale
    assert err < TOL, err
    # the returned plane attains the maximum (up to rounding); it is the
    # oracle's plane unless the two are within rounding of each other
    for j, m in enumerate(idx):
        pv = estimator.plane_values(X, y, xi, Q[m])
        assert 0 <= arg[m] < X.shape[0]
        assert pv[arg[m]] >= fo[j] - TOL * scale
        if arg[m] != ao[j]:
            assert abs(pv[arg[m]] - pv[ao[j]]) <= TOL * scale
    return f, arg, err


@pytest.mark.parametrize("N,n,M,seed", [(1, 1, 5, 1), (37, 3, 70, 2), (64, 2, 64, 3), (333, 10, 129, 4),
                                        (1000, 20, 300, 5), (517, 31, 91, 6), (2049, 5, 33, 7)])
def test_eval_matches_oracle(cr, N, n, M, seed):
    say("eval N=%d n=%d M=%d seed=%d" % (N, n, M, seed))
    X, y, xi = _planes(N, n, seed)
    Q = np.random.default_rng(seed + 100).uniform(-1.5, 1.5, size=(M, n))
    _, _, err = _check(cr, X, y, xi, Q)
    say("  max relative error %.2e" % err)


def test_eval_tie_rule_and_hand_example(cr):
    say("eval hand example N=3 n=1 M=5")
    X = np.array([[0.0], [1.0], [0.5]])
    y = np.array([0.0, 0.0, -0.25])
    xi = np.array([[-1.0], [1.0], [0.0]])
    Q = np.array([[0.25], [2.0], [-1.0], [0.625], [0.5]])
    f, arg = cr.evaluate(dev(X), dev(y), dev(xi), dev(Q))
    np.testing.assert_array_equal(host(f), [-0.25, 1.0, 1.0, -0.25, -0.25])
    np.testing.assert_array_equal(host(arg), [0, 1, 0, 2, 2])


def test_eval_interpolates_feasible_planes(cr):
    say("eval at the points of feasible planes N=3000 n=8")
    X, y, xi = _planes(3000, 8, 9, feasible=True)
    f, arg = cr.evaluate(dev(X), dev(y), dev(xi), dev(X))
    f = host(f)
    assert np.abs(f - y).max() < 1e-12 * (1 + np.abs(y).max())


def test_eval_edge_cases(cr):
    say("eval edge cases: M = 0, without arg, repeated calls on one workspace")
    X, y, xi = _planes(100, 4, 10)
    est = cr.Estimator(dev(X), dev(y), dev(xi))
    f, arg = est(dev(np.zeros((0, 4))))
    assert f.shape == (0,) and arg.shape == (0,)
    Q = np.random.default_rng(11).normal(size=(50, 4))
    f1, none = est(dev(Q), with_arg=False)
    assert none is None
    f2, _ = est(dev(Q[:17]))
    fo, _ = estimator.evaluate(X, y, xi, Q)
    np.testing.assert_allclose(host(f1), fo, rtol=0, atol=1e-12 * 50)
    np.testing.assert_allclose(host(f2), fo[:17], rtol=0, atol=1e-12 * 50)


def test_eval_of_a_solver_output(cr):
    say("eval of a fixed-schedule solve, small_quadratic (N=200, n=2)")
    p = synth.workload("small_quadratic")
    y, xi, _ = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=0, inner_iters=50, max_outer=10))
    y, xi = host(y), host(xi)
    Q = np.random.default_rng(12).uniform(-1, 1, size=(400, 2))
    _check(cr, p.X, y, xi, np.vstack([Q, p.X]))


def test_eval_full_size_sampled(cr):
    # the evaluation benchmark's shapes: 20000 planes in 20 dimensions, 20000 queries
    say("eval full size N=20000 n=20 M=20000, 96 sampled queries")
    X, y, xi = _planes(20000, 20, 13)
    Q = np.random.default_rng(14).uniform(-1, 1, size=(20000, 20))
    sample = np.random.default_rng(15).choice(20000, size=96, replace=False)
    sample = np.concatenate([sample, [0, 19999]])
    _, _, err = _check(cr, X, y, xi, Q, sample=sample)
    say("  max relative error %.2e" % err)
    # and at the planes' own points for a feasible set of the same size
    Xf, yf, xif = _planes(20000, 20, 16, feasible=True)
    f, _ = cr.evaluate(dev(Xf), dev(yf), dev(xif), dev(Xf))
    assert np.abs(host(f) - yf).max() < 1e-12 * (1 + np.abs(yf).max())
