"""GPU parity of the differentiable form (cr_diff_*): the reverse pass of the
fixed-schedule map against the oracle's gradient (torch-CPU FP64 autograd of
the same map, oracle/diff.py), against central finite differences, across
checkpoint intervals, through torch.autograd, and at the full 10000-point
size against the FP64 path and finite differences."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cr():
    import paper_1407_7220_amd as cr
    return cr


def _oracle():
    import oracle
    from oracle import diff as odiff
    return oracle, odiff


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _run(cr, X, ybar, y0, xi0, gy, gxi, prec, K, L, C, **over):
    params = cr.Params(precision=prec, inner_iters=L, max_outer=K, **over)
    d = cr.Diff(_dev(X), _dev(ybar), params, checkpoint_every=C)
    y, xi, info = d.forward(_dev(y0), _dev(xi0))
    g = d.backward(_dev(gy), _dev(gxi) if gxi is not None else None)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in g] + [y.cpu().numpy(), xi.cpu().numpy()]
    d.close()
    return out, info


def _ref(X, ybar, y0, xi0, gy, gxi, K, L, **over):
    oracle, odiff = _oracle()
    p = oracle.Params(inner_iters=L, max_outer=K, **over)
    sch = odiff.schedule(X, ybar, p)
    return odiff.unrolled_vjp(X, ybar, y0, xi0, sch, gy, gxi)


def _problem(N, n, seed):
    p = synth.quadratic_uniform(N, n, 0.1, seed=seed)
    rng = np.random.default_rng(seed + 100)
    return p.X, p.ybar, rng.normal(size=N), rng.normal(size=(N, n))


# FP64: every pass, reduction and vector step is FP64; the tolerance is the
# forward's 1e-9 relative bar (measured: about 1e-15).  FP32: pair terms in
# FP32 (unit roundoff u = 6e-8) summed over up to N terms per point, through
# 10-200 chained steps, with the masks taken from the FP32 residuals (as the
# FP32 forward does), so pairs within rounding of a kink may flip relative to
# the FP64 oracle.  Measured: below 1e-7 at N <= 333 and 6.3e-5 at N = 10000
# (against the FP64 path); the bound 2e-4 is about N u / 3 at N = 10000.
TOL_GRAD = {0: 1e-9, 1: 2e-4}
TOL_FWD = {0: 1e-9, 1: 1e-5}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("N,n,K,L,C", [(150, 3, 3, 8, 3), (97, 1, 2, 5, 5), (70, 6, 1, 7, 2), (2, 2, 2, 3, 1),
                                       (333, 10, 2, 6, 4)])
def test_adjoint_matches_oracle(prec, N, n, K, L, C):
    cr = _cr()
    X, ybar, gy, gxi = _problem(N, n, 7 + N)
    y0, xi0 = ybar.copy(), np.zeros((N, n))
    print("case prec=%d N=%d n=%d K=%d L=%d C=%d" % (prec, N, n, K, L, C), flush=True)
    (dX, dyb, dy0, dxi0, y, xi), _ = _run(cr, X, ybar, y0, xi0, gy, gxi, prec, K, L, C)
    rdX, rdyb, rdy0, rdxi0, ry, rxi = _ref(X, ybar, y0, xi0, gy, gxi, K, L)
    assert _rel(y, ry) <= TOL_FWD[prec] and _rel(xi, rxi) <= TOL_FWD[prec]
    errs = [_rel(dX, rdX), _rel(dyb, rdyb), _rel(dy0, rdy0), _rel(dxi0, rdxi0)]
    print("  rel errors dX %.2e dybar %.2e dy0 %.2e dxi0 %.2e" % tuple(errs), flush=True)
    assert max(errs) <= TOL_GRAD[prec], errs


@pytest.mark.parametrize("prec", [0, 1])
def test_adjoint_with_active_projections_and_random_start(prec):
    cr = _cr()
    N, n = 120, 4
    X, ybar, gy, gxi = _problem(N, n, 21)
    rng = np.random.default_rng(5)
    y0 = ybar + 0.05 * rng.normal(size=N)
    xi0 = 0.2 * rng.normal(size=(N, n))
    over = dict(By_override=0.3, Bxi_override=1.5)
    (dX, dyb, dy0, dxi0, y, xi), _ = _run(cr, X, ybar, y0, xi0, gy, gxi, prec, 3, 6, 4, **over)
    rdX, rdyb, rdy0, rdxi0, ry, rxi = _ref(X, ybar, y0, xi0, gy, gxi, 3, 6, **over)
    # the radii bind: without them the run ends elsewhere
    free = _ref(X, ybar, y0, xi0, gy, gxi, 3, 6, By_override=1e3, Bxi_override=1e4)
    assert np.abs(free[4] - ry).max() > 1e-3 and np.abs(free[5] - rxi).max() > 1e-3
    assert np.linalg.norm(ry - ybar) <= 0.3 + 1e-9
    errs = [_rel(dX, rdX), _rel(dyb, rdyb), _rel(dy0, rdy0), _rel(dxi0, rdxi0)]
    print("prec %d rel errors dX %.2e dybar %.2e dy0 %.2e dxi0 %.2e" % ((prec,) + tuple(errs)), flush=True)
    assert max(errs) <= TOL_GRAD[prec], errs


def test_checkpoint_interval_does_not_change_the_gradient():
    """Recomputation from checkpoints is exact: any interval gives identical bits."""
    cr = _cr()
    N, n = 140, 3
    X, ybar, gy, gxi = _problem(N, n, 3)
    y0, xi0 = ybar.copy(), np.zeros((N, n))
    outs = [_run(cr, X, ybar, y0, xi0, gy, gxi, 1, 2, 9, C)[0] for C in (1, 4, 9, 50)]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_backward_twice_and_without_gxi():
    cr = _cr()
    N, n = 90, 2
    X, ybar, gy, gxi = _problem(N, n, 4)
    params = cr.Params(precision=0, inner_iters=5, max_outer=2)
    d = cr.Diff(_dev(X), _dev(ybar), params, checkpoint_every=2)
    d.forward(_dev(ybar), None)
    g1 = [t.cpu().numpy() for t in d.backward(_dev(gy))]
    g2 = [t.cpu().numpy() for t in d.backward(_dev(2.0 * gy), _dev(np.zeros((N, n))))]
    for a, b in zip(g1, g2):
        np.testing.assert_allclose(b, 2.0 * a, rtol=1e-12, atol=1e-14)
    r = _ref(X, ybar, ybar, np.zeros((N, n)), gy, None, 2, 5)
    for a, b in zip(g1, r[:4]):
        assert _rel(a, b) <= 1e-9
    d.close()


def test_backward_before_forward_is_an_error():
    cr = _cr()
    X, ybar, gy, _ = _problem(40, 2, 9)
    d = cr.Diff(_dev(X), _dev(ybar), cr.Params(precision=1, inner_iters=3, max_outer=1))
    with pytest.raises(cr.CRError) as e:
        d.backward(_dev(gy))
    assert e.value.status == 6     # CR_ERR_STATE
    d.close()


def test_adjoint_central_differences():
    """Directional central differences of the FP64 GPU forward (constants
    frozen by the overrides) against the FP64 adjoint, at h = 1e-3 and 1e-6.
    The map is piecewise smooth: a perturbation of size h moves O(h N^2) pairs
    across the kink of (.)_-, each changing the difference quotient by O(h),
    so the quotient's error is first order in h.  On this case the oracle's
    own quotient (numpy + C forward) is off by 3.5e-3 relative at h = 1e-3,
    8.5e-4 at 1e-4 and 3.3e-6 at 1e-6 in the X direction, converging to the
    oracle's autograd gradient.  At h = 1e-3 the four directions (X, ybar,
    y0, xi0) measure 3.5e-3, 2.0e-3, 2.4e-3 and 2.5e-2 (the xi0 direction
    moves every pair's residual from the data start, where theta = 0 puts
    the kinks at r = ybar_i - ybar_j); at h = 1e-6 they fall to 1e-5 or less.
    Bounds: 5e-2 at h = 1e-3, 1e-4 at h = 1e-6."""
    cr = _cr()
    N, n, K, L = 400, 5, 3, 10
    X, ybar, gy, gxi = _problem(N, n, 12)
    over = dict(By_override=100.0, Bxi_override=1000.0, Lxi_override=1e-3 * 2 * N + 60.0)
    params = cr.Params(precision=0, inner_iters=L, max_outer=K, **over)
    Xd, ybd = _dev(X), _dev(ybar)
    d = cr.Diff(Xd, ybd, params, checkpoint_every=4)
    d.forward(ybd, None)
    dX, dyb, dy0, dxi0 = [t.cpu().numpy() for t in d.backward(_dev(gy), _dev(gxi))]
    d.close()
    rng = np.random.default_rng(1)

    def f(X_, yb_, y0_, xi0_):
        dd = cr.Diff(_dev(X_), _dev(yb_), params, checkpoint_every=L)
        y, xi, _ = dd.forward(_dev(y0_), _dev(xi0_))
        v = float(gy @ y.cpu().numpy() + np.sum(gxi * xi.cpu().numpy()))
        dd.close()
        return v

    for which in range(4):
        dirs = [np.zeros_like(X), np.zeros(N), np.zeros(N), np.zeros((N, n))]
        dirs[which] = rng.normal(size=dirs[which].shape)
        ana = float(np.sum(dX * dirs[0]) + dyb @ dirs[1] + dy0 @ dirs[2] + np.sum(dxi0 * dirs[3]))
        xi0 = np.zeros((N, n))
        for h, tol in ((1e-3, 5e-2), (1e-6, 1e-4)):
            fd = (f(X + h * dirs[0], ybar + h * dirs[1], ybar + h * dirs[2], xi0 + h * dirs[3])
                  - f(X - h * dirs[0], ybar - h * dirs[1], ybar - h * dirs[2], xi0 - h * dirs[3])) / (2 * h)
            rel = abs(fd - ana) / max(1.0, abs(fd))
            print("input %d h %.0e: fd %.10e adjoint %.10e rel %.2e" % (which, h, fd, ana, rel), flush=True)
            assert rel <= tol


def test_autograd_function():
    cr = _cr()
    N, n = 110, 3
    X, ybar, gy, gxi = _problem(N, n, 14)
    params = cr.Params(precision=0, inner_iters=6, max_outer=2)
    Xt = _dev(X).requires_grad_(True)
    ybt = _dev(ybar).requires_grad_(True)
    y, xi = cr.solve_unrolled(Xt, ybt, params, checkpoint_every=3)
    loss = (y * _dev(gy)).sum() + (xi * _dev(gxi)).sum()
    dX, dyb = torch.autograd.grad(loss, (Xt, ybt))
    r = _ref(X, ybar, ybar, np.zeros((N, n)), gy, gxi, 2, 6)
    assert _rel(dX.cpu().numpy(), r[0]) <= 1e-9
    # the start is ybar itself: both paths reach ybar
    assert _rel(dyb.cpu().numpy(), r[1] + r[2]) <= 1e-9


def test_full_size_10000_fp32_against_fp64_and_differences():
    """The differentiable workload at full size: N = 10000, n = 10,
    x ~ U[-1,1]^10, f0 = ||x||^2, noise N(0, 0.1^2), 10 ALCC iterations of 20
    MAPG steps, checkpoints every 20; d(sum w_l y_l)/d(ybar, X) for
    w ~ N(0, 1).  The FP32 gradient against the FP64 one, and the FP64 one
    against central differences (h = 1e-3) in two random directions."""
    cr = _cr()
    p = synth.quadratic_uniform(10000, 10, 0.1, seed=5)
    X, ybar = p.X, p.ybar
    N, n = X.shape
    w = synth.weights(N)
    res = {}
    info64 = None
    for prec in (1, 0):
        print("full size prec %d" % prec, flush=True)
        (dX, dyb, dy0, dxi0, y, xi), info = _run(cr, X, ybar, ybar, np.zeros((N, n)), w, None, prec, 10, 20, 20)
        res[prec] = (dX, dyb + dy0, y)
        info64 = info
        print("  forward %.3fs" % info.seconds, flush=True)
    e_y = _rel(res[1][2], res[0][2])
    e_dX, e_dyb = _rel(res[1][0], res[0][0]), _rel(res[1][1], res[0][1])
    print("FP32 vs FP64: y %.2e dX %.2e dybar %.2e" % (e_y, e_dX, e_dyb), flush=True)
    assert e_y <= 1e-5
    assert e_dX <= TOL_GRAD[1] and e_dyb <= TOL_GRAD[1]

    # central differences need the data-dependent constants frozen: the
    # first ALCC iteration's L^xi and the radii, as overrides
    over = dict(Lxi_override=1e-3 * 2.0 * N + info64.sigma2_A2, By_override=info64.Bbar_y,
                Bxi_override=info64.Bbar_xi)
    params = cr.Params(precision=0, inner_iters=20, max_outer=10, **over)
    d = cr.Diff(_dev(X), _dev(ybar), params, checkpoint_every=20)
    d.forward(_dev(ybar), None)
    dX, dyb, dy0, _ = [t.cpu().numpy() for t in d.backward(_dev(w))]
    d.close()
    rng = np.random.default_rng(2)
    h = 1e-3
    for which in range(2):
        dXd = rng.normal(size=X.shape) if which == 0 else np.zeros_like(X)
        dyd = rng.normal(size=N) if which == 1 else np.zeros(N)
        vals = []
        for sgn in (1.0, -1.0):
            dd = cr.Diff(_dev(X + sgn * h * dXd), _dev(ybar + sgn * h * dyd), params, checkpoint_every=20)
            yv, _, _ = dd.forward(_dev(ybar + sgn * h * dyd), None)
            vals.append(float(w @ yv.cpu().numpy()))
            dd.close()
        fd = (vals[0] - vals[1]) / (2 * h)
        ana = float(np.sum(dX * dXd) + (dyb + dy0) @ dyd)
        print("direction %d: fd %.10e adjoint %.10e rel %.2e" % (which, fd, ana, abs(fd - ana) / abs(fd)), flush=True)
        assert abs(fd - ana) <= 1e-3 * max(1.0, abs(fd))
