"""GPU parity of the HIP pair engine against the FP64 oracle (through the C ABI).

Every case prints its name, sizes and seed before touching the GPU."""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
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


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# Tolerances: FP64 pass vs FP64 oracle differs only by summation order (~1e-15
# per term); the FP32 pass rounds theta, r and every in-tile sum to 24 bits.
TOL_PASS = {0: 1e-12, 1: 3e-5, 2: 3e-4}
# After a fixed schedule: the spec bars for FP64 and FP32 (y and Xi
# alike); the mixed form's bar is its measured error level (below 1e-5 on
# every case here), stated rather than derived.
TOL_SOLVE = {0: 1e-9, 1: 1e-5, 2: 3e-5}
PREC_NAME = {0: "f64", 1: "f32", 2: "mixed_bf16"}


def _random_state(N, n, seed, theta_scale=0.3):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(N, n))
    ybar = np.sum(X * X, axis=1) + 0.1 * rng.normal(size=N)
    y = ybar + 0.2 * rng.normal(size=N)
    xi = rng.normal(size=(N, n))
    theta = theta_scale * np.abs(rng.normal(size=(N, N)))
    np.fill_diagonal(theta, 0.0)
    return X, ybar, y, xi, theta


SHAPES = [(2, 1), (37, 3), (64, 2), (200, 2), (333, 10), (1000, 5), (517, 20), (300, 31)]


@pytest.mark.parametrize("N,n", [(37, 3), (200, 2), (1000, 10), (517, 20), (300, 31)])
def test_setup_constants(cr, N, n):
    say("setup_constants N=%d n=%d" % (N, n))
    p = synth.quadratic_uniform(N, n, seed=N + n)
    ctx = cr.Context(dev(p.X), dev(p.ybar), cr.Params(gamma=1e-3))
    info = ctx.info()
    yhat, xihat, Bbar, By, Bxi = oracle.affine_fit(p.X, p.ybar, 1e-3)
    assert info.sigma2_A1 == 2.0 * N
    assert abs(info.sigma2_A2 - oracle.sigma2_A2(p.X)) <= 1e-11 * oracle.sigma2_A2(p.X)
    assert abs(info.Bbar_y - By) <= 1e-10 * By
    assert abs(info.Bbar_xi - Bxi) <= 1e-10 * Bxi
    y0, xi0 = ctx.get_start()
    assert rel(host(y0), yhat) < 1e-11
    assert rel(host(xi0), xihat) < 1e-10


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
@pytest.mark.parametrize("N,n", SHAPES)
def test_grad_pass(cr, prec, N, n):
    say("grad_pass %s N=%d n=%d" % (PREC_NAME[prec], N, n))
    X, ybar, y, xi, theta = _random_state(N, n, seed=10 * N + n)
    gamma, mu = 1e-2, 0.37
    ctx = cr.Context(dev(X), dev(ybar), cr.Params(gamma=gamma, precision=prec))
    ctx.set_theta(dev(theta))
    gy, gxi = ctx.pairwise_step(cr.GRAD, dev(y), dev(xi), mu)
    ey, exi = oracle.grad_P(X, ybar, gamma, mu, theta, y, xi)
    # compare the pair part (the (y - ybar)/mu term is exact on both sides)
    hy, hxi = host(gy), host(gxi)
    e1 = rel(hy - (y - ybar) / mu, ey - (y - ybar) / mu)
    e2 = rel(hxi - gamma / mu * xi, exi - gamma / mu * xi)
    say("  pass relative error: grad_y %.3e  grad_xi %.3e" % (e1, e2))
    assert e1 < TOL_PASS[prec]
    assert e2 < TOL_PASS[prec]


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
@pytest.mark.parametrize("N,n", [(37, 3), (200, 2), (640, 10), (517, 20)])
def test_theta_pass(cr, prec, N, n):
    say("theta_pass %s N=%d n=%d" % (PREC_NAME[prec], N, n))
    X, ybar, y, xi, theta = _random_state(N, n, seed=7 * N + n)
    gamma, mu, mu_next = 1e-2, 0.25, 1.0
    ctx = cr.Context(dev(X), dev(ybar), cr.Params(gamma=gamma, precision=prec))
    ctx.set_theta(dev(theta))
    sy, sxi = ctx.pairwise_step(cr.THETA_UPDATE, dev(y), dev(xi), mu, mu_next)
    th_new = host(ctx.get_theta())
    W = oracle.penalty_weights(X, y, xi, theta)
    assert rel(th_new, (mu / mu_next) * W) < TOL_PASS[prec]
    lam = mu * W
    u, v = oracle.adjoint(X, lam)
    assert rel(host(sy), y - ybar - u) < TOL_PASS[prec] * 10
    assert rel(host(sxi), gamma * xi - v) < TOL_PASS[prec] * 10
    m = oracle.kkt_measures(X, ybar, gamma, y, xi, lam)
    info = ctx.info()
    t = {0: 1e-10, 1: 1e-4, 2: 1e-3}[prec]
    assert abs(info.infeas - m["infeas"]) <= t * max(1.0, m["infeas"])
    assert abs(info.compl - m["compl"]) <= t * max(1.0, m["compl"])
    assert abs(info.stat_y - m["stat_y"]) <= 10 * t * max(1.0, m["stat_y"])
    assert abs(info.stat_xi - m["stat_xi"]) <= 10 * t * max(1.0, m["stat_xi"])
    assert abs(info.infeas_norm - m["infeas_norm"]) <= t * max(1.0, m["infeas_norm"])
    assert abs(info.gap_norm - m["gap_norm"]) <= t * max(1e-3, abs(m["gap_norm"]))


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("tile_rows", [64, 128, 512])
def test_passes_across_tile_heights(cr, prec, tile_rows):
    """Gradient and multiplier passes against the oracle when a workgroup's
    wave owns one tile (64 rows per workgroup), two tiles, or eight, with the
    ragged last chunk of N = 1000."""
    say("tile heights %s tile_rows=%d" % (PREC_NAME[prec], tile_rows))
    N, n = 1000, 5
    X, ybar, y, xi, theta = _random_state(N, n, seed=11)
    gamma, mu, mu_next = 1e-2, 0.25, 1.0
    ctx = cr.Context(dev(X), dev(ybar), cr.Params(gamma=gamma, precision=prec, tile_rows=tile_rows))
    ctx.set_theta(dev(theta))
    gy, gxi = ctx.pairwise_step(cr.GRAD, dev(y), dev(xi), mu)
    ry, rxi = oracle.grad_P(X, ybar, gamma, mu, theta, y, xi)
    assert rel(host(gy), ry) < TOL_PASS[prec] and rel(host(gxi), rxi) < TOL_PASS[prec]
    ctx.pairwise_step(cr.THETA_UPDATE, dev(y), dev(xi), mu, mu_next)
    W = oracle.penalty_weights(X, y, xi, theta)
    assert rel(host(ctx.get_theta()), (mu / mu_next) * W) < TOL_PASS[prec]


def test_pass_is_deterministic(cr):
    say("deterministic N=700 n=10")
    X, ybar, y, xi, theta = _random_state(700, 10, seed=3)
    ctx = cr.Context(dev(X), dev(ybar), cr.Params(precision=1))
    ctx.set_theta(dev(theta))
    a = [host(t) for t in ctx.pairwise_step(cr.GRAD, dev(y), dev(xi), 0.5)]
    b = [host(t) for t in ctx.pairwise_step(cr.GRAD, dev(y), dev(xi), 0.5)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


FIXED_C1 = dict(inner_iters=50, max_outer=10)


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
def test_fixed_schedule_small_quadratic(cr, prec):
    say("fixed schedule small_quadratic N=200 n=2 10x50 %s" % PREC_NAME[prec])
    p = synth.workload("small_quadratic")
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**FIXED_C1), record_kkt=False)
    y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=prec, **FIXED_C1))
    assert info.inner_iters == 500 and info.outer_iters == 10
    ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
    say("  relative error vs FP64 oracle: y %.3e  xi %.3e" % (ey, exi))
    assert ey < TOL_SOLVE[prec]
    assert exi < TOL_SOLVE[prec]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_fixed_schedule_step_as_printed(cr, prec):
    """Fig. 4 with the step 1/L exactly as printed (step_scale = 1) on both
    sides: the default reading takes half of it."""
    say("fixed schedule small_quadratic N=200 n=2 10x50 step_scale=1 %s" % PREC_NAME[prec])
    p = synth.workload("small_quadratic")
    sched = dict(inner_iters=50, max_outer=10, step_scale=1.0)
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
    y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=prec, **sched))
    assert info.inner_iters == 500 and info.outer_iters == 10
    ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
    say("  relative error vs FP64 oracle: y %.3e  xi %.3e" % (ey, exi))
    assert ey < TOL_SOLVE[prec]
    assert exi < TOL_SOLVE[prec]


def _alpha_margin(traces):
    """Smallest relative distance of a MAPG step's block moves from the alpha
    thresholds over a whole oracle run (the adaptive test's rounding margin)."""
    worst = math.inf
    for ay, axi, steps in traces:
        for (_, dy, dxi, _, _) in steps:
            worst = min(worst, abs(dy - ay) / ay, abs(dxi - axi) / axi)
    return worst


# Adaptive schedules (Fig. 3 l_max and tau/alpha decay, Fig. 4 alpha test) in
# FP64: lazy passes with alpha stops and l_max caps, and tall chunks (the update
# kernel) with capped runs.  Every step's block moves stay at least 1e-6
# (relative) away from the thresholds, so both sides take the same branches.
ADAPTIVE_CASES = [
    # N, n, seed, max_inner, max_outer, tile_rows
    (60, 2, 0, 20000, 30, 0),
    (90, 5, 2, 3000, 6, 0),
    (1600, 3, 4, 300, 4, 1600),
]


@pytest.mark.parametrize("N,n,seed,max_inner,max_outer,tile_rows", ADAPTIVE_CASES,
                         ids=["N60-lazy", "N90-lazy-capped", "N1600-tall-chunks"])
def test_adaptive_schedule_matches_oracle(cr, N, n, seed, max_inner, max_outer, tile_rows):
    say("adaptive f64 N=%d n=%d seed=%d max_inner=%d max_outer=%d tile_rows=%d"
        % (N, n, seed, max_inner, max_outer, tile_rows))
    p = synth.quad_l1_gaussian(N, n, seed=seed)
    sched = dict(kkt_tol=1e-4, max_inner=max_inner, max_outer=max_outer)
    traces = []
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), mapg_traces=traces)
    margin = _alpha_margin(traces)
    say("  oracle: inner %s converged %s, alpha margin %.2e" % (ref.inner_per_outer, ref.converged, margin))
    assert margin > 1e-6
    ctx = cr.Context(dev(p.X), dev(p.ybar), cr.Params(precision=0, tile_rows=tile_rows, **sched))
    y, xi, info = ctx.run()
    inner, kkt = ctx.outer_history()
    ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
    say("  gpu: inner %s, y %.3e xi %.3e" % (inner, ey, exi))
    assert inner == ref.inner_per_outer
    assert info.outer_iters == ref.outer and info.inner_iters == ref.inner_total
    assert (info.status == 0) == ref.converged
    np.testing.assert_allclose(kkt, [h["kkt"] for h in ref.history], rtol=1e-6, atol=1e-12)
    assert ey < TOL_SOLVE[0]
    assert exi < TOL_SOLVE[0]


# MAPG run lengths around the 32-iteration replay: a run that a reduce kernel
# stops (last iterate odd or even) and one that ends with the last replay
# (l^max a multiple of 32, finished after the replays), plus the shortest runs.
@pytest.mark.parametrize("prec,inner", [(0, 1), (0, 2), (0, 31), (0, 32), (0, 33), (0, 64), (1, 32), (1, 33),
                                        (2, 32), (2, 31)])
def test_fixed_schedule_run_lengths(cr, prec, inner):
    say("fixed schedule run length %s inner=%d N=130 n=5" % (PREC_NAME[prec], inner))
    p = synth.quad_l1_gaussian(130, 5, seed=7)
    sched = dict(inner_iters=inner, max_outer=3)
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
    y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=prec, **sched))
    assert info.inner_iters == 3 * inner and info.outer_iters == 3
    ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
    say("  y %.2e xi %.2e" % (ey, exi))
    assert ey < TOL_SOLVE[prec]
    assert exi < TOL_SOLVE[prec]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_tall_chunks_match_short_chunks(cr, prec):
    # 4096-row chunks leave no LDS room for the staged operands of a lazy
    # pass, so that solve completes each step with the update kernel; 256-row
    # chunks use lazy passes.  Both follow the same iteration.
    N = 1700 if prec == 0 else 3100
    say("tall vs short chunks %s N=%d n=3" % (PREC_NAME[prec], N))
    p = synth.quad_l1_gaussian(N, 3, seed=8)
    sched = dict(inner_iters=20, max_outer=2)
    out = {}
    for tr in (256, 4096):
        y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=prec, tile_rows=tr, **sched))
        out[tr] = (host(y), host(xi))
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
    for tr, (y, xi) in out.items():
        say("  tile_rows %d: y %.2e xi %.2e" % (tr, rel(y, ref.y), rel(xi, ref.xi)))
        assert rel(y, ref.y) < TOL_SOLVE[prec]
        assert rel(xi, ref.xi) < TOL_SOLVE[prec]
    tol = 1e-12 if prec == 0 else 1e-5
    assert rel(out[256][0], out[4096][0]) < tol


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
def test_time_pass_then_solve(cr, prec):
    # the timing hook runs the solve's pass kernel on scratch state; a solve
    # on the same context afterwards is unaffected
    say("time_pass then solve %s N=200 n=2" % PREC_NAME[prec])
    p = synth.workload("small_quadratic")
    sched = dict(inner_iters=20, max_outer=2)
    ctx = cr.Context(dev(p.X), dev(p.ybar), cr.Params(precision=prec, **sched))
    ms = ctx.time_pass(3)
    assert ms > 0
    y, xi, info = ctx.run()
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
    assert rel(host(y), ref.y) < TOL_SOLVE[prec]


@pytest.mark.parametrize("N,n,seed", [(37, 3, 1), (130, 5, 2), (96, 20, 3)])
def test_fixed_schedule_ragged(cr, N, n, seed):
    say("fixed schedule ragged N=%d n=%d seed=%d" % (N, n, seed))
    p = synth.quad_l1_gaussian(N, n, seed=seed)
    sched = dict(inner_iters=20, max_outer=4)
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
    y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=0, **sched))
    assert rel(host(y), ref.y) < 1e-9
    assert rel(host(xi), ref.xi) < 1e-9


def test_nonfinite_inputs_rejected(cr):
    say("non-finite X / ybar at set-up: CR_ERR_NONFINITE")
    p = synth.quad_l1_gaussian(50, 3, seed=30)
    yb = p.ybar.copy(); yb[17] = np.nan
    with pytest.raises(cr.CRError) as e:
        cr.Context(dev(p.X), dev(yb), cr.Params(precision=1))
    assert e.value.status == 4
    X = p.X.copy(); X[3, 1] = np.inf
    with pytest.raises(cr.CRError) as e:
        cr.solve(dev(X), dev(p.ybar), cr.Params(precision=0, inner_iters=5, max_outer=1))
    assert e.value.status == 4


@pytest.mark.parametrize("N,n,prec", [(2, 1, 0), (2, 3, 1), (5, 10, 0), (40, 31, 0), (40, 31, 1)],
                         ids=["N2n1-f64", "N2n3-f32", "N5n10-f64", "N40n31-f64", "N40n31-f32"])
def test_degenerate_and_widest_shapes(cr, N, n, prec):
    # two points (two constraints), fewer points than dimensions (the
    # minimum-norm affine start of R16), and the widest supported n
    say("fixed schedule N=%d n=%d %s" % (N, n, PREC_NAME[prec]))
    p = synth.quad_l1_gaussian(N, n, seed=31 + N + n)
    sched = dict(inner_iters=30, max_outer=3)
    ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
    y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=prec, **sched))
    ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
    say("  y %.2e xi %.2e" % (ey, exi))
    assert ey < TOL_SOLVE[prec]
    assert exi < TOL_SOLVE[prec]


def test_constant_data_fixed_point(cr):
    say("constant data N=50 n=3")
    p = synth.constant_data(50, 3, value=1.5)
    y, xi, info = cr.solve(dev(p.X), dev(p.ybar), cr.Params(inner_iters=10, max_outer=2))
    assert np.max(np.abs(host(y) - 1.5)) < 1e-12
    assert np.max(np.abs(host(xi))) < 1e-12


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_adaptive_reaches_kkt(cr, prec):
    say("adaptive N=60 n=2 %s" % PREC_NAME[prec])
    p = synth.workload("small_quadratic")
    X, ybar = p.X[:60], p.ybar[:60]
    y, xi, info = cr.solve(dev(X), dev(ybar), cr.Params(precision=prec, kkt_tol=1e-4))
    assert info.status == 0 and info.kkt <= 1e-4
    ref = oracle.alcc(X, ybar, oracle.Params(kkt_tol=1e-6))
    assert rel(host(y), ref.y) < 1e-3


def test_mixed_adaptive_against_fp64_at_the_same_kkt(cr):
    """The mixed BF16 form solved to KKT <= 1e-4 at n = 20 (the mixed form's
    dimension), against the FP64 form solved to the same tolerance and to
    1e-7: both land within the KKT-level distance of the optimum."""
    p = synth.max_affine_uniform(1500, 20, 50, 0.1, seed=3)
    say("adaptive mixed vs f64 N=1500 n=20 maxaffine seed 3")
    X, yb = dev(p.X), dev(p.ybar)
    ym, xim, im = cr.solve(X, yb, cr.Params(precision=2, kkt_tol=1e-4))
    yd, xid, idd = cr.solve(X, yb, cr.Params(precision=0, kkt_tol=1e-4))
    yt, xit, it = cr.solve(X, yb, cr.Params(precision=0, kkt_tol=1e-7, max_outer=40))
    say("  KKT mixed %.2e (%d MAPG), f64 %.2e (%d MAPG), tight f64 %.2e" % (im.kkt, im.inner_iters, idd.kkt,
                                                                          idd.inner_iters, it.kkt))
    assert im.status == 0 and im.kkt <= 1e-4 and idd.status == 0
    em, ed = rel(host(ym), host(yt)), rel(host(yd), host(yt))
    exm, exd = rel(host(xim), host(xit)), rel(host(xid), host(xit))
    say("  distance to the tight solution: mixed y %.2e xi %.2e, f64 y %.2e xi %.2e" % (em, exm, ed, exd))
    assert em < 1e-3 and ed < 1e-3 and exm < 1e-2 and exd < 1e-2


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
def test_full_size_pass_sampled(cr, prec):
    """One gradient pass at the 5000-point, n=10 workload, in the launch
    configuration the benchmark uses; sampled outputs recomputed by the oracle."""
    say("full-size sampled logsumexp_5000 %s" % PREC_NAME[prec])
    p = synth.workload("logsumexp_5000")
    N, n = p.N, p.n
    rng = np.random.default_rng(5)
    y = p.ybar + 0.05 * rng.normal(size=N)
    xi = 0.3 * rng.normal(size=(N, n))
    theta = 0.02 * np.abs(rng.normal(size=(N, N)))
    np.fill_diagonal(theta, 0.0)
    gamma, mu = 1e-3, 1e-4
    ctx = cr.Context(dev(p.X), dev(p.ybar), cr.Params(gamma=gamma, precision=prec))
    ctx.set_theta(dev(theta))
    gy, gxi = ctx.pairwise_step(cr.GRAD, dev(y), dev(xi), mu)
    hy, hxi = host(gy), host(gxi)
    tol = {0: 1e-11, 1: 2e-4, 2: 2e-3}[prec]
    for m in [0, 1, 17, 2500, 4095, 4096, 4998, 4999]:
        row, col = oracle.residual_row_col(p.X, y, xi, m)
        wrow = np.maximum(theta[m] - row, 0.0); wrow[m] = 0.0
        wcol = np.maximum(theta[:, m] - col, 0.0); wcol[m] = 0.0
        u, v = oracle.adjoint_one(p.X, m, wrow, wcol)
        scale = wrow.sum() + wcol.sum()
        assert abs((hy[m] - (y[m] - p.ybar[m]) / mu) - (-u)) <= tol * scale
        assert np.max(np.abs((hxi[m] - gamma / mu * xi[m]) - (-v))) <= tol * scale * (1 + np.abs(p.X).max())


@pytest.mark.parametrize("prec,N", [(1, 131072), (0, 65536)], ids=["f32-131072", "f64-65536"])
def test_large_n_pass_sampled(cr, prec, N):
    """One gradient pass far beyond the benchmark sizes (theta of 64 GiB in FP32,
    32 GiB in FP64, as the context allocates it): the 32-bit buffer offsets of
    the pass and the partial sums at their largest here.  theta = 0 after set-up,
    so w = (r)_-; sampled rows and columns recomputed by the oracle."""
    n = 3
    say("large-N pass %s N=%d n=%d" % (PREC_NAME[prec], N, n))
    rng = np.random.default_rng(21)
    X = rng.uniform(-1, 1, size=(N, n))
    ybar = np.sum(X * X, axis=1)
    y = ybar + 0.05 * rng.normal(size=N)
    xi = 2.0 * X + 0.1 * rng.normal(size=(N, n))
    gamma, mu = 1e-3, 1e-4
    ctx = cr.Context(dev(X), dev(ybar), cr.Params(gamma=gamma, precision=prec))
    gy, gxi = ctx.pairwise_step(cr.GRAD, dev(y), dev(xi), mu)
    hy, hxi = host(gy), host(gxi)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    tol = {0: 1e-11, 1: 3e-4}[prec]
    for m in [0, 1, 4095, 4096, N // 2 + 7, N - 65, N - 1]:
        row, col = oracle.residual_row_col(X, y, xi, m)
        wrow = np.maximum(-row, 0.0); wrow[m] = 0.0
        wcol = np.maximum(-col, 0.0); wcol[m] = 0.0
        u, v = oracle.adjoint_one(X, m, wrow, wcol)
        scale = wrow.sum() + wcol.sum() + 1.0
        assert abs((hy[m] - (y[m] - ybar[m]) / mu) - (-u)) <= tol * scale, m
        assert np.max(np.abs((hxi[m] - gamma / mu * xi[m]) - (-v))) <= tol * scale * 2, m


_FULL_REF = {}


def _full_size_reference():
    # the oracle's 2 x 33 run on the 5000-point workload, shared by both precisions
    if "ref" not in _FULL_REF:
        p = synth.workload("logsumexp_5000")
        _FULL_REF["ref"] = oracle.alcc(p.X, p.ybar, oracle.Params(inner_iters=33, max_outer=2), record_kkt=False)
    return _FULL_REF["ref"]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_full_size_fixed_schedule_benchmark_launch(cr, prec):
    """The 5000-point workload through whole MAPG runs in the benchmark's launch
    configuration (the tuned chunk height: lazy passes, two kernels per
    iteration), 2 ALCC iterations of 33 MAPG steps (an odd run length, so the
    last iterate sits in the second parity buffer), against the oracle."""
    from paper_1407_7220_amd import autotune
    p = synth.workload("logsumexp_5000")
    X, yb = dev(p.X), dev(p.ybar)
    tile = autotune.tile_rows_for(X, yb, prec, tune_if_missing=False)
    say("full-size fixed schedule logsumexp_5000 %s tile_rows %d, 2 x 33" % (PREC_NAME[prec], tile))
    sched = dict(inner_iters=33, max_outer=2)
    y, xi, info = cr.solve(X, yb, cr.Params(precision=prec, tile_rows=tile, **sched))
    assert info.inner_iters == 66 and info.outer_iters == 2
    ref = _full_size_reference()
    ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
    say("  relative error vs FP64 oracle: y %.3e  xi %.3e" % (ey, exi))
    assert ey < TOL_SOLVE[prec]
    assert exi < TOL_SOLVE[prec]


_C3_FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "maxaffine_20000_2x25.npz")


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
def test_maxaffine_20000_fixed_schedule_against_oracle(cr, prec):
    """The 20000-point, n = 20 workload (the mixed form's configuration) after 2
    ALCC iterations of 25 MAPG steps, in the benchmark's launch configuration,
    against the FP64 oracle's iterate stored by tests/golden/make_maxaffine_20000.py:
    element by element (largest deviation relative to the largest entry) and in
    norm.  FP64 and FP32 at the spec bars; the mixed BF16 form at its
    measured level (the split drops only the lo*lo products, and W is split
    hi/lo too): 1.9e-8 (y) and 1.1e-7 (Xi) in norm, 2.3e-7 at the largest entry."""
    from paper_1407_7220_amd import autotune
    d = np.load(_C3_FIXTURE)
    meta = json.loads(str(d["meta"]))
    p = synth.workload("maxaffine_20000")
    assert hashlib.sha256(p.X.tobytes() + p.ybar.tobytes()).hexdigest() == meta["input_sha256"]
    X, yb = dev(p.X), dev(p.ybar)
    tile = autotune.tile_rows_for(X, yb, prec, tune_if_missing=False)
    sched = meta["schedule"]
    say("maxaffine_20000 %s tile_rows %d, %d x %d against the stored oracle iterate"
        % (PREC_NAME[prec], tile, sched["max_outer"], sched["inner_iters"]))
    y, xi, info = cr.solve(X, yb, cr.Params(precision=prec, tile_rows=tile, **sched))
    assert info.inner_iters == sched["max_outer"] * sched["inner_iters"]
    hy, hxi = host(y), host(xi)
    del X, yb, y, xi
    torch.cuda.empty_cache()
    ey, exi = rel(hy, d["y"]), rel(hxi, d["xi"])
    my = np.max(np.abs(hy - d["y"])) / np.max(np.abs(d["y"]))
    mxi = np.max(np.abs(hxi - d["xi"])) / np.max(np.abs(d["xi"]))
    say("  relative error vs FP64 oracle: y %.3e  xi %.3e (norm); y %.3e  xi %.3e (largest entry)"
        % (ey, exi, my, mxi))
    tol = {0: 1e-9, 1: 1e-5, 2: 1e-6}[prec]
    assert ey < tol and exi < tol
    assert my < tol and mxi < tol


# --------------------------------------------------------------------------
# Batched form
# --------------------------------------------------------------------------

BATCH_SHAPES = [(37, 3), (150, 5), (300, 10), (64, 2), (513, 20), (90, 10)]


def _batch_problems(shapes, seed0=100):
    return [synth.quad_l1_gaussian(N, n, 0.1, seed=seed0 + i) for i, (N, n) in enumerate(shapes)]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_batched_fixed_schedule_matches_oracle(cr, prec):
    say("batched fixed schedule %s shapes %s" % (PREC_NAME[prec], BATCH_SHAPES))
    probs = _batch_problems(BATCH_SHAPES)
    sched = dict(inner_iters=20, max_outer=3)
    outs, infos = cr.solve_batched([(dev(p.X), dev(p.ybar)) for p in probs], cr.Params(precision=prec, **sched))
    for p, (y, xi), info in zip(probs, outs, infos):
        ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
        assert info.inner_iters == 60 and info.outer_iters == 3
        ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
        say("  N=%d n=%d: y %.2e xi %.2e" % (p.N, p.n, ey, exi))
        assert ey < TOL_SOLVE[prec]
        assert exi < TOL_SOLVE[prec]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_batched_update_form_with_a_large_problem_matches_oracle(cr, prec):
    """A batch holding a problem past the lazy form's 2048-point limit runs the
    update-kernel form for every problem; both sizes against the oracle."""
    shapes = [(2300, 5), (700, 10)]
    say("batched update form %s shapes %s" % (PREC_NAME[prec], shapes))
    probs = _batch_problems(shapes, seed0=600)
    sched = dict(inner_iters=10, max_outer=2)
    outs, infos = cr.solve_batched([(dev(p.X), dev(p.ybar)) for p in probs], cr.Params(precision=prec, **sched))
    for p, (y, xi), info in zip(probs, outs, infos):
        ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
        assert info.inner_iters == 20 and info.outer_iters == 2
        ey, exi = rel(host(y), ref.y), rel(host(xi), ref.xi)
        say("  N=%d n=%d: y %.2e xi %.2e" % (p.N, p.n, ey, exi))
        assert ey < TOL_SOLVE[prec]
        assert exi < TOL_SOLVE[prec]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_batched_lazy_form_over_several_tiles_matches_oracle(cr, prec):
    """A batch of problems up to 2048 points runs lazy passes; with tile heights
    that give several chunks and strips per problem (and a ragged last chunk)."""
    shapes = [(1800, 10), (1100, 3), (333, 20)]
    tiles = [256, 384, 128]
    say("batched lazy form %s shapes %s tiles %s" % (PREC_NAME[prec], shapes, tiles))
    probs = _batch_problems(shapes, seed0=700)
    sched = dict(inner_iters=12, max_outer=2)
    b = cr.Batch([(dev(p.X), dev(p.ybar)) for p in probs], cr.Params(precision=prec, **sched), tile_rows=tiles)
    try:
        outs, infos, _ = b.run()
        outs = [(host(y), host(xi)) for y, xi in outs]
    finally:
        b.close()
    for p, (y, xi), info in zip(probs, outs, infos):
        ref = oracle.alcc(p.X, p.ybar, oracle.Params(**sched), record_kkt=False)
        assert info.inner_iters == 24 and info.outer_iters == 2
        ey, exi = rel(y, ref.y), rel(xi, ref.xi)
        say("  N=%d n=%d: y %.2e xi %.2e" % (p.N, p.n, ey, exi))
        assert ey < TOL_SOLVE[prec]
        assert exi < TOL_SOLVE[prec]


def test_batched_equals_single_problem_solves(cr):
    say("batched vs single-problem solves, f64")
    probs = _batch_problems(BATCH_SHAPES[:4], seed0=200)
    sched = dict(inner_iters=25, max_outer=2)
    outs, _ = cr.solve_batched([(dev(p.X), dev(p.ybar)) for p in probs], cr.Params(precision=0, **sched))
    for p, (y, xi) in zip(probs, outs):
        ys, xis, _ = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=0, **sched))
        assert rel(host(y), host(ys)) < 1e-12
        assert rel(host(xi), host(xis)) < 1e-11


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_batched_equals_single_problem_bitwise_in_deterministic_mode(cr, prec):
    """With deterministic = 1 a problem solved alone runs the batched form's
    kernels; with the same tile heights its result has the same bits as inside
    the batch (fixed and adaptive schedules)."""
    shapes = [(37, 3), (150, 5), (300, 10), (513, 20)]
    tiles = [64, 128, 192, 256]
    say("batched vs single, bitwise, %s shapes %s tiles %s" % (PREC_NAME[prec], shapes, tiles))
    probs = _batch_problems(shapes, seed0=400)
    for sched in (dict(inner_iters=25, max_outer=3), dict(kkt_tol=1e-3, max_inner=400, max_outer=4)):
        prm = cr.Params(precision=prec, deterministic=1, **sched)
        b = cr.Batch([(dev(p.X), dev(p.ybar)) for p in probs], prm, tile_rows=tiles)
        try:
            outs, infos, _ = b.run()
            outs = [(host(y), host(xi)) for y, xi in outs]
        finally:
            b.close()
        for p, t, (y, xi), info in zip(probs, tiles, outs, infos):
            ys, xis, infs = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=prec, deterministic=1,
                                                                     tile_rows=t, **sched))
            say("  N=%d n=%d %s: inner %d / %d" % (p.N, p.n, sched, info.inner_iters, infs.inner_iters))
            assert info.inner_iters == infs.inner_iters and info.outer_iters == infs.outer_iters
            np.testing.assert_array_equal(y, host(ys))
            np.testing.assert_array_equal(xi, host(xis))


def test_batched_in_bounded_pieces_equals_one_run(cr):
    """cr_batch_start / cr_batch_advance (a few replays at a time) / cr_batch_finish
    give the bits of one cr_batch_run, for an adaptive and a fixed schedule."""
    say("batched run in pieces vs one run, f64")
    probs = _batch_problems([(40, 2), (90, 5), (130, 3)], seed0=500)
    pairs = [(dev(p.X), dev(p.ybar)) for p in probs]
    for sched in (dict(kkt_tol=1e-4, max_inner=300, max_outer=6), dict(inner_iters=40, max_outer=3)):
        b = cr.Batch(pairs, cr.Params(precision=0, **sched))
        try:
            outs, infos, _ = b.run()
            ref = [(host(y).copy(), host(xi).copy()) for y, xi in outs]
            ref_inner = [i.inner_iters for i in infos]
            b.start()
            steps = 0
            while b.advance(3):
                steps += 1
            outs, infos, _ = b.finish()
        finally:
            b.close()
        say("  %s: %d advance calls, inner %s" % (sched, steps + 1, ref_inner))
        assert [i.inner_iters for i in infos] == ref_inner
        for (y, xi), (ry, rxi) in zip(outs, ref):
            np.testing.assert_array_equal(host(y), ry)
            np.testing.assert_array_equal(host(xi), rxi)


def test_batched_adaptive_converges_and_freezes(cr):
    say("batched adaptive f32")
    probs = _batch_problems([(40, 2), (60, 3), (80, 5)], seed0=300)
    outs, infos = cr.solve_batched([(dev(p.X), dev(p.ybar)) for p in probs], cr.Params(precision=1, kkt_tol=1e-4))
    outers = []
    for p, (y, xi), info in zip(probs, outs, infos):
        assert info.status == 0 and info.kkt <= 1e-4, info
        outers.append(info.outer_iters)
        ref = oracle.alcc(p.X, p.ybar, oracle.Params(kkt_tol=1e-6))
        assert rel(host(y), ref.y) < 1e-3
    say("  ALCC iterations per problem: %s" % outers)
