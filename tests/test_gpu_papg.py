"""GPU parity of P-APG (cr_papg, Fig. 2) against the FP64 oracle (oracle/papg.py).

Both sides run the same fixed schedules: `iters` P-APG iterations, each
solving the K block problems with ALCC for max_outer x inner_iters MAPG steps,
and the same constants (L and y_shift are passed where a case pins them).
Every case prints its name, sizes and schedule before touching the GPU."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import papg as opapg
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


# FP64 block solves against the FP64 oracle: the two differ by summation order
# in every reduction (the same bound as the fixed-schedule ALCC parity, 1e-9),
# and P-APG's multiplier step adds O(N) sums of such values per iteration.
TOL = 1e-9


def _run(cr, p, K, iters, inner, outer, gamma, L=0.0, B=math.inf, y_shift=None, prec=0, accelerate=True):
    sched = dict(gamma=gamma, inner_iters=inner, max_outer=outer)
    ref = opapg.papg(p.X, p.ybar, K, gamma, iters, oracle.Params(**sched), L=L, B_theta=B, y_shift=y_shift,
                     record=True, accelerate=accelerate)
    pp = cr.PapgParams(K=K, iters=iters, L=L, B_theta=B, y_shift=-1.0 if y_shift is None else y_shift,
                       method=cr.PAPG_ACCELERATED if accelerate else cr.PAPG_GRADIENT)
    y, xi, info, th, thy = cr.papg(dev(p.X), dev(p.ybar), pp, cr.Params(precision=prec, **sched), with_theta=True)
    return ref, host(y), host(xi), info, host(th), host(thy)


CASES = [
    # (name, problem, K, iters, inner, outer, gamma)
    ("gaussian_quadratic N=12 n=2 K=2", lambda: synth.gaussian_quadratic(12, 2, seed=3), 2, 4, 40, 4, 0.1),
    ("gaussian_quadratic N=100 n=5 K=2 (Sec. III study)", lambda: synth.gaussian_quadratic(100, 5, seed=0), 2, 3,
     40, 4, 0.05),
    ("quadratic_uniform N=90 n=3 K=3", lambda: synth.quadratic_uniform(90, 3, seed=4), 3, 3, 33, 3, 0.1),
    ("quad_l1_gaussian N=96 n=7 K=4", lambda: synth.quad_l1_gaussian(96, 7, seed=5), 4, 2, 31, 3, 0.2),
    # the widest points (n = CR_MAX_DIM), two-point blocks, and a ragged size spanning several tiles
    ("quadratic_uniform N=64 n=31 K=2", lambda: synth.quadratic_uniform(64, 31, seed=95), 2, 2, 20, 2, 0.1),
    ("quadratic_uniform N=24 n=2 K=12", lambda: synth.quadratic_uniform(24, 2, seed=26), 12, 3, 20, 3, 0.1),
    ("quadratic_uniform N=1000 n=10 K=4", lambda: synth.quadratic_uniform(1000, 10, seed=1010), 4, 2, 32, 2, 0.1),
    # above 4096 points the column sums take longer row chunks (72 rows here, 58 chunks); ragged tiles
    ("quadratic_uniform N=4160 n=6 K=4", lambda: synth.quadratic_uniform(4160, 6, seed=4166), 4, 2, 5, 2, 0.1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_papg_matches_oracle(cr, case):
    name, mk, K, iters, inner, outer, gamma = case
    p = mk()
    say("papg %s: %d iterations of %d x %d MAPG steps per block, gamma %g" % (name, iters, outer, inner, gamma))
    ref, y, xi, info, th, thy = _run(cr, p, K, iters, inner, outer, gamma)
    assert abs(info["L"] - ref.L) <= 1e-10 * ref.L
    assert info["y_shift"] == ref.y_shift
    ey, exi, eth = rel(y, ref.y), rel(xi, ref.xi), rel(th, ref.Th)
    say("  relative error vs FP64 oracle: y %.3e  xi %.3e  theta %.3e  (||theta|| %.3e)"
        % (ey, exi, eth, info["theta_norm"]))
    assert ey < TOL and exi < TOL and eth < TOL
    np.testing.assert_allclose(thy, ref.th_y, rtol=0, atol=TOL * (1 + np.abs(ref.Th).max()))
    # structure: zero inside the diagonal blocks, nonnegative everywhere
    assert np.all(th[~opapg.cross_mask(p.N, K)] == 0.0) and np.all(th >= 0.0) and np.all(thy >= 0.0)
    assert info["inner_iters"] == iters * K * inner * outer
    nrm = math.sqrt(float(np.sum(th * th) + np.sum(thy * thy)))
    assert abs(info["theta_norm"] - nrm) <= 1e-12 * max(nrm, 1.0)


def test_papg_ball_active_and_given_constants(cr):
    # data moved down by 5 and no shift: the rows y >= 0 bind (theta_y > 0), and
    # the radius 0.02 is below the unprojected ||theta|| (0.0236 with the oracle)
    p = synth.gaussian_quadratic(60, 3, seed=6)
    p.ybar = p.ybar - 5.0
    L = 0.5 * opapg.lipschitz_bound(p.X, 0.1)
    B = 0.02
    say("papg ball radius %g, L %.3e, y_shift 0: N=60 n=3 K=3, 3 iterations of 3 x 30" % (B, L))
    ref, y, xi, info, th, thy = _run(cr, p, 3, 3, 30, 3, 0.1, L=L, B=B, y_shift=0.0)
    assert info["L"] == L and info["y_shift"] == 0.0
    assert abs(info["theta_norm"] - B) <= 1e-12      # the ball is active
    assert np.count_nonzero(ref.th_y) > 0
    ey, eth = rel(y, ref.y), rel(th, ref.Th)
    say("  relative error vs FP64 oracle: y %.3e  theta %.3e  theta_y %.3e" % (ey, eth, rel(thy, ref.th_y)))
    assert ey < TOL and eth < TOL and rel(thy, ref.th_y) < TOL


def test_papg_single_block_is_a_batched_solve(cr):
    # K = 1: no cross pairs; theta_y stays 0 once y > 0, so eta is one ALCC solve
    p = synth.quadratic_uniform(80, 4, seed=8)
    sched = dict(gamma=0.1, inner_iters=32, max_outer=3)
    say("papg K=1 N=80 n=4, 2 iterations of 3 x 32, against cr.solve")
    y, xi, info = cr.papg(dev(p.X), dev(p.ybar), cr.PapgParams(K=1, iters=2), cr.Params(precision=0, **sched))
    ys, xis, _ = cr.solve(dev(p.X), dev(p.ybar), cr.Params(precision=0, **sched))
    assert rel(host(y), host(ys)) < TOL and rel(host(xi), host(xis)) < TOL
    assert info["theta_norm"] == 0.0


def test_papg_f32_blocks(cr):
    p = synth.gaussian_quadratic(100, 5, seed=0)
    say("papg f32 block solves N=100 n=5 K=2, 2 iterations of 4 x 40")
    ref, y, xi, info, th, thy = _run(cr, p, 2, 2, 40, 4, 0.05, prec=1)
    ey, eth = rel(y, ref.y), rel(th, ref.Th)
    say("  relative error vs FP64 oracle: y %.3e  theta %.3e" % (ey, eth))
    assert ey < 1e-5 and eth < 1e-4


def test_papg_rejects_bad_arguments(cr):
    p = synth.gaussian_quadratic(12, 2, seed=3)
    say("papg argument errors (host-side)")
    with pytest.raises(cr.CRError) as e:
        cr.papg(dev(p.X), dev(p.ybar), cr.PapgParams(K=5, iters=1), cr.Params(precision=0, inner_iters=5))
    assert e.value.status == 1
    bad = p.ybar.copy()
    bad[3] = np.nan
    with pytest.raises(cr.CRError) as e:
        cr.papg(dev(p.X), dev(bad), cr.PapgParams(K=2, iters=1), cr.Params(precision=0, inner_iters=5))
    assert e.value.status == 4


def _check_trace(trace, ref):
    # per iteration: ||theta^(1)_l||, cross-block infeasibility at eta_l, theta^(2)_l^T C eta_l
    for col, key in enumerate(("theta_norm", "infeas_cross", "gap")):
        r = np.array([t[key] for t in ref.trace])
        scale = max(np.abs(r).max(), 1e-300)
        assert np.abs(trace[:, col] - r).max() <= 1e-9 * scale, key


def test_gradient_ascent_matches_oracle(cr):
    p = synth.quadratic_uniform(64, 3, seed=11)
    say("projected gradient ascent (no momentum) N=64 n=3 K=4, 4 iterations of 3 x 32")
    ref, y, xi, info, th, thy = _run(cr, p, 4, 4, 32, 3, 0.1, accelerate=False)
    ey, eth = rel(y, ref.y), rel(th, ref.Th)
    say("  relative error vs FP64 oracle: y %.3e  theta %.3e" % (ey, eth))
    assert ey < TOL and eth < TOL
    _check_trace(info["trace"], ref)


def test_small_study_accelerated_against_gradient_ascent(cr):
    # the comparison of Sec. III on its problem: n = 5, N = 100, K = 2,
    # f0 = 1/2 x^T Q x with Q = Lambda^T Lambda, Lambda, x, eps ~ N(0, 1)
    p = synth.gaussian_quadratic(100, 5, seed=0)
    say("Sec. III study N=100 n=5 K=2: P-APG and gradient ascent, 40 iterations of 4 x 40")
    out = {}
    for acc in (True, False):
        ref, y, xi, info, th, thy = _run(cr, p, 2, 40, 40, 4, 0.05, accelerate=acc)
        _check_trace(info["trace"], ref)
        assert rel(y, ref.y) < TOL and rel(th, ref.Th) < TOL
        out[acc] = info["trace"]
        say("  %s: infeasibility %.4e -> %.4e, ||theta|| %.4e"
            % ("P-APG" if acc else "ascent", info["trace"][0, 1], info["trace"][-1, 1], info["trace"][-1, 0]))
    # the accelerated dual iterates move further: lower cross-block infeasibility
    assert out[True][-1, 1] < out[False][-1, 1]
    assert out[True][-1, 0] > out[False][-1, 0]


def test_papg_approaches_the_direct_solution(cr):
    # A property at any size: as the dual iterates improve, eta(theta) approaches
    # the solution y(gamma) of eq. "regularize" (which eq. "omega_primal" equals
    # once y >= 0 is inactive), and the cross-block constraints are met better.
    p = synth.quadratic_uniform(40, 2, seed=21)
    X, yb = dev(p.X), dev(p.ybar)
    say("papg convergence N=40 n=2 K=2: 25, 100, 400 iterations of 8 x 100 against a direct solve to KKT 1e-5")
    yd, _, info = cr.solve(X, yb, cr.Params(precision=0, gamma=0.1, kkt_tol=1e-5, max_outer=30))
    assert info.status == 0 and info.kkt <= 1e-5
    yd = host(yd)
    err, inf = [], []
    for it in (25, 100, 400):
        y, xi, pinfo = cr.papg(X, yb, cr.PapgParams(K=2, iters=it),
                               cr.Params(precision=0, gamma=0.1, inner_iters=100, max_outer=8))
        err.append(float(np.linalg.norm(host(y) - yd)))
        inf.append(pinfo["infeas_cross"])
        say("  %3d iterations: |y - y(gamma)| %.3e  cross infeasibility %.3e" % (it, err[-1], inf[-1]))
    assert err[0] > err[1] > err[2] and inf[0] > inf[1] > inf[2]
    assert inf[2] < inf[0] / 10 and err[2] < err[0] / 4


def test_papg_with_adaptive_block_solves(cr):
    # block solves to KKT <= 1e-4 instead of a fixed schedule: no parity (the
    # stopping tests are discontinuous), but the run must improve on the
    # block-diagonal start as with fixed schedules
    p = synth.quadratic_uniform(40, 2, seed=21)
    X, yb = dev(p.X), dev(p.ybar)
    say("papg with adaptive block solves (KKT 1e-4, at most 1000 MAPG steps per ALCC iteration) N=40 n=2 K=2, "
        "1 and 20 iterations")
    adaptive = cr.Params(precision=0, gamma=0.1, kkt_tol=1e-4, max_outer=30, max_inner=1000)
    yd, _, info = cr.solve(X, yb, cr.Params(precision=0, gamma=0.1, kkt_tol=1e-5, max_outer=30))
    assert info.status == 0
    yd = host(yd)
    y1, _, i1 = cr.papg(X, yb, cr.PapgParams(K=2, iters=1), adaptive)
    y20, _, i20 = cr.papg(X, yb, cr.PapgParams(K=2, iters=20), adaptive)
    e1, e20 = np.linalg.norm(host(y1) - yd), np.linalg.norm(host(y20) - yd)
    say("  |y - y(gamma)|: %.3e after 1, %.3e after 20; cross infeasibility %.3e -> %.3e; MAPG steps %d, %d"
        % (e1, e20, i1["infeas_cross"], i20["infeas_cross"], i1["inner_iters"], i20["inner_iters"]))
    assert np.all(np.isfinite(host(y20)))
    assert e20 < e1 and i20["infeas_cross"] < i1["infeas_cross"] / 1.2
    assert i1["inner_iters"] > 0 and i20["inner_iters"] > 10 * i1["inner_iters"]


def _dense_C(X, K):
    # C = [A3 A4; I 0] (eq. "C") row by row, for sigma_max(C) of a small case
    N, n = X.shape
    mask = opapg.cross_mask(N, K)
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
    return np.array(rows)


def test_theorem1_bounds_on_the_dual_iterates(cr):
    # Theorem 1 through its intermediate bound eq. "mixed_bound": for a
    # delta-optimal theta_delta in Q2 and eta_delta minimising the Lagrangian
    # there, ||y_delta - y(gamma)|| and ||(A3 y_delta + A4 xi_delta)_-|| are at most
    # sqrt(2 delta / gamma) sigma_max(C).  Gradient ascent keeps theta^(2) in Q2;
    # g* = the optimal value of eq. "regularize" (strong duality, y >= 0
    # inactive after the shift) from a direct solve, g(theta^(2)_l) = the
    # objective at eta_l minus the reported theta^(2)_l^T C eta_l.  Ascent with
    # step 1/L >= 1/L_g also increases g monotonically, and P-APG's delta falls
    # faster (the accelerated rate).
    N, n, K, gamma = 40, 2, 2, 0.1
    p = synth.quadratic_uniform(N, n, seed=21)
    X, yb = dev(p.X), dev(p.ybar)
    say("Theorem 1 bounds: N=40 n=2 K=2, gradient ascent 20 / 100 / 300 iterations and P-APG 300, blocks 8 x 100")
    yd, xid, info = cr.solve(X, yb, cr.Params(precision=0, gamma=gamma, kkt_tol=1e-6, max_outer=30))
    assert info.status == 0
    yd, xid = host(yd), host(xid)
    gstar = 0.5 * np.sum((yd - p.ybar) ** 2) + 0.5 * gamma * np.sum(xid ** 2)
    smax = np.linalg.norm(_dense_C(p.X, K), 2)
    blocks = cr.Params(precision=0, gamma=gamma, inner_iters=100, max_outer=8)

    def run(it, method):
        y, xi, pinfo = cr.papg(X, yb, cr.PapgParams(K=K, iters=it, method=method), blocks)
        y, xi = host(y), host(xi)
        gval = 0.5 * np.sum((y - p.ybar) ** 2) + 0.5 * gamma * np.sum(xi ** 2) - pinfo["trace"][-1, 2]
        return gstar - gval, float(np.linalg.norm(y - yd)), pinfo["infeas_cross"]

    deltas = []
    for it in (20, 100, 300):
        delta, dy, infx = run(it, cr.PAPG_GRADIENT)
        rhs = math.sqrt(max(2.0 * delta / gamma, 0.0)) * smax
        say("  ascent %3d iterations: delta %.3e  |y - y(gamma)| %.3e  cross infeasibility %.3e  bound %.3e"
            % (it, delta, dy, infx, rhs))
        assert delta > 0.0
        assert dy <= rhs and infx <= rhs
        deltas.append(delta)
    assert deltas[0] > deltas[1] > deltas[2]
    delta, dy, infx = run(300, cr.PAPG_ACCELERATED)
    say("  P-APG  300 iterations: delta %.3e  |y - y(gamma)| %.3e  cross infeasibility %.3e" % (delta, dy, infx))
    assert 0.0 < delta < deltas[2] / 5


def test_power_iteration_step_constant(cr):
    # sigma_max(C)^2 by power iteration on C^T C: the step constant must not fall
    # below L_g = sigma_max(C)^2 / gamma (eq. "lischitz", dense SVD here) and is
    # at most 5% above it once converged; ascent with it gains more per
    # iteration than with the bound (2N + sigma_max(A2)^2 + 1) / gamma
    N, n, K, gamma = 40, 2, 2, 0.1
    p = synth.quadratic_uniform(N, n, seed=21)
    X, yb = dev(p.X), dev(p.ybar)
    say("power iteration for L_g: N=40 n=2 K=2, 200 iterations; ascent 60 iterations with each constant")
    s2 = np.linalg.norm(_dense_C(p.X, K), 2) ** 2
    Lg = s2 / gamma
    blocks = cr.Params(precision=0, gamma=gamma, inner_iters=100, max_outer=8)
    _, _, ib = cr.papg(X, yb, cr.PapgParams(K=K, iters=60, method=cr.PAPG_GRADIENT), blocks)
    _, _, ip = cr.papg(X, yb, cr.PapgParams(K=K, iters=60, method=cr.PAPG_GRADIENT, power_iters=200), blocks)
    say("  L_g %.4f  bound %.4f  power %.4f; cross infeasibility after 60: %.3e (bound) %.3e (power)"
        % (Lg, ib["L"], ip["L"], ib["infeas_cross"], ip["infeas_cross"]))
    assert Lg <= ip["L"] <= 1.05 * Lg * (1 + 1e-9)
    assert ip["L"] < ib["L"]
    assert ip["infeas_cross"] < ib["infeas_cross"]
