"""Pins of the differentiated-map oracle (oracle/diff.py) on the CPU.

The forward written with torch pair arrays must reproduce ``oracle.alcc``
(numpy + the C operators) on a fixed schedule, and its autograd gradient must
match central finite differences of ``oracle.alcc`` itself, in random
directions of every input, both with the ball projections idle and with them
active.  A wrong sign, a dropped term or a transposed index in either the
forward or the chain rule moves one of these far beyond the tolerances.
"""
import numpy as np
import pytest

import oracle
from oracle import diff as odiff
import synth


def _problem(N, n, seed):
    p = synth.quadratic_uniform(N, n, 0.1, seed=seed)
    return p.X, p.ybar


def _params(K, L, By=0.0, Bxi=0.0, Lxi=0.0):
    return oracle.Params(inner_iters=L, max_outer=K, By_override=By, Bxi_override=Bxi, Lxi_override=Lxi)


def _alcc_y(X, ybar, params, y0, xi0):
    return oracle.alcc(X, ybar, params, y0=y0, xi0=xi0, record_kkt=False)


@pytest.mark.parametrize("start", ["data", "random"])
def test_unrolled_forward_matches_alcc(start):
    X, ybar = _problem(17, 3, 5)
    N, n = X.shape
    rng = np.random.default_rng(3)
    if start == "data":
        y0, xi0 = ybar.copy(), np.zeros((N, n))
    else:
        y0, xi0 = ybar + 0.1 * rng.normal(size=N), 0.3 * rng.normal(size=(N, n))
    params = _params(3, 7)
    ref = _alcc_y(X, ybar, params, y0, xi0)
    sch = odiff.schedule(X, ybar, params)
    gy = rng.normal(size=N)
    _, _, _, _, y, xi = odiff.unrolled_vjp(X, ybar, y0, xi0, sch, gy)
    np.testing.assert_allclose(y, ref.y, rtol=0, atol=1e-12 * (1 + np.abs(ref.y).max()))
    np.testing.assert_allclose(xi, ref.xi, rtol=0, atol=1e-12 * (1 + np.abs(ref.xi).max()))
    # the run must have used the penalty: theta_{K+1} is not all zero
    assert np.abs(ref.theta).max() > 0


def _fd_check(X, ybar, y0, xi0, params, seed, h=1e-6, rtol=2e-6):
    N, n = X.shape
    rng = np.random.default_rng(seed)
    gy = rng.normal(size=N)
    gxi = rng.normal(size=(N, n))
    sch = odiff.schedule(X, ybar, params)
    dX, dyb, dy0, dxi0, _, _ = odiff.unrolled_vjp(X, ybar, y0, xi0, sch, gy, gxi)

    def f(X_, yb_, y0_, xi0_):
        r = _alcc_y(X_, yb_, params, y0_, xi0_)
        return float(gy @ r.y + np.sum(gxi * r.xi))

    for _ in range(2):
        dirs = [rng.normal(size=X.shape), rng.normal(size=N), rng.normal(size=N), rng.normal(size=(N, n))]
        ana = float(np.sum(dX * dirs[0]) + dyb @ dirs[1] + dy0 @ dirs[2] + np.sum(dxi0 * dirs[3]))
        plus = f(X + h * dirs[0], ybar + h * dirs[1], y0 + h * dirs[2], xi0 + h * dirs[3])
        minus = f(X - h * dirs[0], ybar - h * dirs[1], y0 - h * dirs[2], xi0 - h * dirs[3])
        fd = (plus - minus) / (2 * h)
        assert abs(fd - ana) <= rtol * max(1.0, abs(fd)), (fd, ana)
        # and each input alone, so that one input's term cannot hide another's
        for which in range(4):
            d = [np.zeros_like(a) for a in dirs]
            d[which] = dirs[which]
            ana1 = [float(np.sum(dX * d[0])), float(dyb @ d[1]), float(dy0 @ d[2]), float(np.sum(dxi0 * d[3]))][which]
            fd1 = (f(X + h * d[0], ybar + h * d[1], y0 + h * d[2], xi0 + h * d[3])
                   - f(X - h * d[0], ybar - h * d[1], y0 - h * d[2], xi0 - h * d[3])) / (2 * h)
            assert abs(fd1 - ana1) <= rtol * max(1.0, abs(fd1)), (which, fd1, ana1)


def test_unrolled_grad_matches_central_differences():
    X, ybar = _problem(11, 2, 7)
    N, n = X.shape
    # the constants that depend on the data are frozen (overrides), as the
    # derivative assumes; the balls are large enough never to bind
    params = _params(3, 5, By=50.0, Bxi=500.0, Lxi=1e-3 * 2 * N + 40.0)
    _fd_check(X, ybar, ybar.copy(), np.zeros((N, n)), params, seed=1)


def test_unrolled_grad_with_active_projections():
    X, ybar = _problem(9, 2, 8)
    N, n = X.shape
    rng = np.random.default_rng(4)
    y0 = ybar + 0.05 * rng.normal(size=N)
    xi0 = 0.2 * rng.normal(size=(N, n))
    # small radii: both projections bind in most iterations
    params = _params(2, 6, By=0.08, Bxi=0.3, Lxi=1e-3 * 2 * N + 40.0)
    sch = odiff.schedule(X, ybar, params)
    import torch
    hits = [0, 0]
    orig = odiff._proj_ball

    def counting(v, centre, radius):
        d = (v - centre).detach().numpy()
        if np.sqrt(np.sum(d * d)) > radius:
            hits[0 if radius == sch.By else 1] += 1
        return orig(v, centre, radius)

    odiff._proj_ball = counting
    try:
        odiff.unrolled(torch.tensor(X), torch.tensor(ybar), torch.tensor(y0), torch.tensor(xi0), sch)
    finally:
        odiff._proj_ball = orig
    assert hits[0] >= 3 and hits[1] >= 3, hits
    _fd_check(X, ybar, y0, xi0, params, seed=2)


def test_linear_regime_closed_form():
    """With every pair strictly feasible along the whole run (theta = 0 and the
    residuals stay positive), the penalty is idle and one MAPG step is the
    affine map y -> y - s (y - ybar)/mu: then y_K - ybar is (y0 - ybar) times
    a product of scalars, so dy_K/dybar = 1 - c_K and dy_K/dy0 = c_K with
    c_K = that product, independent of X."""
    N, n = 8, 2
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, size=(N, n))
    # strictly convex data on the points, interpolated exactly: r_ij > 0
    f = np.sum(X * X, axis=1)
    xi0 = 2 * X
    y0 = f.copy()
    ybar = f + 1e-9 * rng.normal(size=N)     # ybar ~ y0: the iterates barely move
    params = _params(1, 4, By=100.0, Bxi=1000.0, Lxi=1.0)
    sch = odiff.schedule(X, ybar, params)
    gy = rng.normal(size=N)
    dX, dyb, dy0, dxi0, y, xi = odiff.unrolled_vjp(X, ybar, y0, xi0, sch, gy)
    # scalar recursion of the y block: e_l = y - ybar
    mu, s = sch.mu[0], sch.sy[0]
    a = 1.0 - s / mu
    e1p, e2, cK = 1.0, 1.0, None
    for l in range(sch.L):
        e1 = a * e2
        e2 = e1 + sch.beta[l] * (e1 - e1p)
        e1p = e1
    cK = e1p
    R = oracle.forward(X, y, xi)
    np.fill_diagonal(R, 1.0)
    assert R.min() > 0      # the penalty stayed idle
    np.testing.assert_allclose(dy0, cK * gy, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(dyb, (1 - cK) * gy, rtol=1e-12, atol=1e-15)
    assert np.abs(dX).max() < 1e-12 and np.abs(dxi0).max() < 1e-12
