"""Pins of the estimator-evaluation oracle (oracle/estimator.py).

The evaluated function is the piecewise-linear convex estimator of Sec. I:
the largest of the supporting hyperplanes y_l + xi_l^T (x - x_l).  Each test
checks it against a fact that does not come from the oracle itself:
interpolation of feasible data, exact reproduction of affine data, a
hand-computed one-dimensional example (with the tie rule), the tangent-plane
bounds of a convex function, convexity, and brute force over the planes.
"""
import numpy as np

from oracle import estimator


def _logsumexp_data(N, n, seed):
    # y_l = f(x_l) and xi_l = grad f(x_l) for the convex f(x) = log sum_k exp(a_k^T x):
    # tangent planes of a convex function satisfy every constraint of eq. "original"
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(7, n)) / np.sqrt(n)
    X = rng.normal(size=(N, n))
    Z = X @ A.T
    zmax = Z.max(axis=1, keepdims=True)
    E = np.exp(Z - zmax)
    y = (zmax[:, 0] + np.log(E.sum(axis=1)))
    P = E / E.sum(axis=1, keepdims=True)
    xi = P @ A
    return X, y, xi, A


def _lse(A, Q):
    Z = Q @ A.T
    zmax = Z.max(axis=1, keepdims=True)
    return zmax[:, 0] + np.log(np.exp(Z - zmax).sum(axis=1))


def test_interpolates_feasible_points():
    # Sec. I: the estimator takes the value y_l at x_l when (y, xi) is feasible
    X, y, xi, _ = _logsumexp_data(200, 5, 1)
    f, arg = estimator.evaluate(X, y, xi, X)
    np.testing.assert_allclose(f, y, rtol=0, atol=1e-12)
    # the maximiser is the point itself or a plane with the same value there
    vals = np.array([estimator.plane_values(X, y, xi, X[m])[arg[m]] for m in range(len(y))])
    np.testing.assert_allclose(vals, y, rtol=0, atol=1e-12)


def test_affine_data_is_reproduced():
    rng = np.random.default_rng(2)
    n = 4
    a, b = rng.normal(size=n), 0.7
    X = rng.normal(size=(50, n))
    y = X @ a + b
    xi = np.tile(a, (50, 1))
    Q = rng.normal(size=(30, n)) * 3
    f, _ = estimator.evaluate(X, y, xi, Q)
    np.testing.assert_allclose(f, Q @ a + b, rtol=0, atol=1e-12)


def test_hand_example_one_dimension():
    # tangents of f(x) = x^2 - x at x = 0, 1, 1/2: lines -x, x - 1, -1/4
    X = np.array([[0.0], [1.0], [0.5]])
    y = np.array([0.0, 0.0, -0.25])
    xi = np.array([[-1.0], [1.0], [0.0]])
    Q = np.array([[0.25], [2.0], [-1.0], [0.625], [0.5]])
    f, arg = estimator.evaluate(X, y, xi, Q)
    # q = 1/4: planes give -1/4, -3/4, -1/4 (tie: the smaller index, 0); q = 2: -2, 1, -1/4;
    # q = -1: 1, -2, -1/4; q = 5/8: -5/8, -3/8, -1/4; q = 1/2: -1/2, -1/2, -1/4
    np.testing.assert_array_equal(f, [-0.25, 1.0, 1.0, -0.25, -0.25])
    np.testing.assert_array_equal(arg, [0, 1, 0, 2, 2])


def test_tangent_plane_bounds_of_a_convex_function():
    # max of tangent planes of a convex f lies below f, above every plane,
    # and equals f at the tangent points
    X, y, xi, A = _logsumexp_data(300, 3, 3)
    rng = np.random.default_rng(4)
    Q = rng.normal(size=(100, 3)) * 1.5
    f, _ = estimator.evaluate(X, y, xi, Q)
    assert np.all(f <= _lse(A, Q) + 1e-12)
    for m in range(0, 100, 9):
        assert np.all(f[m] >= estimator.plane_values(X, y, xi, Q[m]) - 1e-12)


def test_convex_along_segments():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(80, 3))
    y = rng.normal(size=80)
    xi = rng.normal(size=(80, 3))
    a, b = rng.normal(size=(20, 3)), rng.normal(size=(20, 3))
    lam = 0.3
    fa, _ = estimator.evaluate(X, y, xi, a)
    fb, _ = estimator.evaluate(X, y, xi, b)
    fm, _ = estimator.evaluate(X, y, xi, lam * a + (1 - lam) * b)
    assert np.all(fm <= lam * fa + (1 - lam) * fb + 1e-12)


def test_brute_force_and_blocking():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(37, 2))
    y = rng.normal(size=37)
    xi = rng.normal(size=(37, 2))
    Q = rng.normal(size=(70, 2))
    f, arg = estimator.evaluate(X, y, xi, Q, block=64)
    for m in range(70):
        best, bl = -np.inf, -1
        for l in range(37):
            v = y[l] + xi[l, 0] * (Q[m, 0] - X[l, 0]) + xi[l, 1] * (Q[m, 1] - X[l, 1])
            if v > best:
                best, bl = v, l
        assert abs(best - f[m]) <= 1e-14 * max(1.0, abs(best))
        assert bl == arg[m]
    f7, arg7 = estimator.evaluate(X, y, xi, Q, block=7)
    np.testing.assert_array_equal(f7, f)
    np.testing.assert_array_equal(arg7, arg)
