"""Throughput benchmark: constraint-pair updates per second of the ALCC/MAPG
solve run to KKT <= 1e-4, on one MI355X.

A step is one whole solve (every stage of the hot path: pair passes, MAPG
steps, multiplier steps and KKT checks) of the 5000-point, n = 10 workload
(x ~ N(0, I), f0 = log-sum-exp of 20 random affine maps, noise N(0, 0.05^2)),
in FP64, the paper's arithmetic, with the inputs already resident in device
memory.  value = sum over the timed steps of N (N - 1) x MAPG iterations /
wall seconds.

Also reported on the same JSON line:
  roofline      the dominant kernel (the gradient pair pass): algorithmic bytes
                (one theta read per pair) / its average device time, measured
                with HIP events on the library's stream, against 8 TB/s HBM;
                traffic = HBM bytes per launch from the committed rocprofv3
                counter summary when it matches the current kernel sources;
  cpu_baseline  the FP64 CPU oracle timed on the host cores on a bounded
                sample of the same workload (a fixed number of MAPG
                iterations), on all cores and on one thread;
  variants      the same metric, each with its pass roofline, for the FP32
                solve of the same workload, the mixed BF16 form on the
                20000-point, n = 20 workload solved to KKT <= 1e-4 and the FP32
                form there over a fixed 2 x 25 schedule (both with their error
                against the FP64 oracle's stored iterate after 2 x 25 MAPG
                iterations), the 64-problem batched form solved to
                KKT <= 1e-4, the differentiable form (10000 points, 10 x 20
                unrolled iterations, forward + reverse pass), the estimator
                evaluation and P-APG (4096 points, K = 4).
The pass tile height comes from the autotuner (paper_1407_7220_amd.autotune).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f64|f32]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "constraint-pair updates/s (N(N-1)·iters/s) at KKT<=1e-4, plain vs mixed/batched"
HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFS = 78.6       # MI355X dense FP64 matrix peak
WORKLOAD = "logsumexp_5000"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("cr_kernels.hip", "cr_ops.h", "cr_device.h", "cr_api.hip"):
        with open(os.path.join(ROOT, "paper_1407_7220_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str):
    """HBM bytes per pass launch from the committed rocprofv3 counter summary
    profiles/<name>_counters.json, only if it was taken on the current kernel
    sources (else None)."""
    path = os.path.join(ROOT, "profiles", name + "_counters.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def progress(msg: str) -> None:
    """A line on stderr after each finished piece of work (the JSON line goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def pass_roofline(ms: float, pairs: float, esz: int, kernel: str, traffic_name: str):
    """Roofline block of a pass: algorithmic bytes (one theta read per pair) over
    its HIP-event time, against the HBM peak."""
    alg = pairs * esz
    achieved = alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(traffic_name),
            "kernel": kernel, "avg_ms": ms, "bytes_per_launch": alg}


def _one_thread():
    """Limit the oracle's OpenMP operators to one thread (same process); returns
    a function that restores the previous count."""
    import ctypes
    import oracle
    oracle._load()
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(1)
    return lambda: gomp.omp_set_num_threads(prev)


def cpu_baseline(p, budget_s: float, one_thread_s: float):
    """Oracle MAPG iterations (FP64, C operators + numpy) on the same workload,
    from the same starting point, until about budget_s seconds have passed; then
    the same on one thread for about one_thread_s seconds."""
    import numpy as np
    import oracle
    gamma = 1e-3
    yhat, xihat, Bbar, By, Bxi = oracle.affine_fit(p.X, p.ybar, gamma)
    N = p.N
    mu = 1.0 / (2.0 * N)
    Ly = 1.0 / mu + oracle.sigma2_A1(N)
    Lxi = gamma / mu + oracle.sigma2_A2(p.X)
    theta = np.zeros((N, N))

    def run(budget):
        y, xi = yhat, xihat
        oracle.mapg(p.X, p.ybar, gamma, mu, theta, Ly, Lxi, y, xi, By, Bxi, 0, 0, 1, adaptive=False)
        t0 = time.perf_counter()
        iters = 0
        while time.perf_counter() - t0 < budget:
            y, xi, _ = oracle.mapg(p.X, p.ybar, gamma, mu, theta, Ly, Lxi, y, xi, By, Bxi, 0, 0, 1, adaptive=False)
            iters += 1
        return iters, time.perf_counter() - t0

    iters, secs = run(budget_s)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    out = {"value": N * (N - 1) * iters / secs, "unit": "pair-updates/s", "cores": cores, "kind": "oracle",
           "sample": "%d MAPG iterations of the FP64 oracle on %s (N=%d, n=%d), %.1f s" % (
               iters, WORKLOAD, N, p.n, secs)}
    restore = _one_thread() if one_thread_s > 0 else None
    if restore is not None:
        try:
            it1, s1 = run(one_thread_s)
        finally:
            restore()
        out["one_thread"] = {"value": N * (N - 1) * it1 / s1, "unit": "pair-updates/s", "cores": 1,
                             "sample": "%d MAPG iterations, %.1f s" % (it1, s1)}
    return out


def solve_rate(cr, p, prec, tile_rows, steps=1, warmup=0, name=None, max_outer=None):
    """Pair-updates/s of whole solves to KKT <= 1e-4 on workload p, with the pass
    roofline (HIP events) of the solve's gradient pass."""
    import torch
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    kw = {} if max_outer is None else {"max_outer": max_outer}
    ctx = cr.Context(X, yb, cr.Params(precision=prec, kkt_tol=1e-4, tile_rows=tile_rows, **kw))
    pname = {cr.F64: "f64", cr.F32: "f32", cr.MIXED_BF16: "mixed_bf16"}[prec]
    for _ in range(warmup):
        ctx.run()
        progress("%s %s warm-up solve done" % (pname, name or p.name))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(ctx.run()[2])
        progress("%s %s solve done: %d MAPG iterations, KKT %.2e" % (pname, name or p.name, infos[-1].inner_iters,
                                                                    infos[-1].kkt))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms = ctx.time_pass(20)
    ctx.close()
    esz = 8 if prec == cr.F64 else 4
    return {"value": sum(i.pair_updates for i in infos) / wall, "unit": "pair-updates/s",
            "N": p.N, "n": p.n, "solves": steps, "seconds_per_solve": wall / steps,
            "mapg_iters_per_solve": infos[-1].inner_iters, "alcc_iters_per_solve": infos[-1].outer_iters,
            "final_kkt": infos[-1].kkt, "converged": all(i.status == 0 for i in infos), "tile_rows": tile_rows,
            "roofline": pass_roofline(pass_ms, p.N * (p.N - 1), esz, "k_pair_pass",
                                      "pair_pass_%s_%s" % (pname, name or p.name))}


def fixed_rate(cr, p, prec, tile_rows, inner=25, outer=2, name=None):
    """Steady-state pair-updates/s over a fixed schedule (outer x inner MAPG
    iterations from the affine start, after one untimed run), with the pass
    roofline."""
    import torch
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    ctx = cr.Context(X, yb, cr.Params(precision=prec, inner_iters=inner, max_outer=outer, tile_rows=tile_rows))
    ctx.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = ctx.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms = ctx.time_pass(10)
    ctx.close()
    esz = 8 if prec == cr.F64 else 4
    pname = {cr.F64: "f64", cr.F32: "f32", cr.MIXED_BF16: "mixed_bf16"}[prec]
    return {"value": info.pair_updates / wall, "unit": "pair-updates/s",
            "schedule": "%d x %d MAPG (fixed; steady-state rate)" % (outer, inner), "N": p.N, "n": p.n,
            "tile_rows": tile_rows,
            "roofline": pass_roofline(pass_ms, p.N * (p.N - 1), esz, "k_pair_pass",
                                      "pair_pass_%s_%s" % (pname, name or p.name))}


def fixture_error(cr, p, prec, tile_rows):
    """Relative error in y and xi (2-norm, and largest entry over the largest
    stored entry) against the FP64 oracle's iterate after 2 x 25 MAPG steps,
    stored by tests/golden/make_maxaffine_20000.py (None if absent)."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", "maxaffine_20000_2x25.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path)
    meta = json.loads(str(d["meta"]))
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    y, xi, info = cr.solve(X, yb, cr.Params(precision=prec, tile_rows=tile_rows, **meta["schedule"]))
    torch.cuda.synchronize()
    hy, hxi = y.cpu().numpy(), xi.cpu().numpy()
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    big = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return {"schedule": "%d x %d MAPG from the affine start" % (meta["schedule"]["max_outer"],
                                                               meta["schedule"]["inner_iters"]),
            "rel_err_y": rel(hy, d["y"]), "rel_err_xi": rel(hxi, d["xi"]),
            "max_err_y": big(hy, d["y"]), "max_err_xi": big(hxi, d["xi"]),
            "reference": "FP64 oracle, tests/golden/maxaffine_20000_2x25.npz"}


def batched_rate(cr, autotune):
    """The 64-problem FP32 batch (N_p ~ U{500..8000}, n_p in {5, 10, 20}) solved to
    KKT <= 1e-4 per problem, with the roofline of its batched pass."""
    import torch
    import synth
    probs = synth.batched_workload()
    pairs = [(torch.from_numpy(q.X).cuda(), torch.from_numpy(q.ybar).cuda()) for q in probs]
    tiles = [autotune.tile_rows_for(X, yb, cr.F32, form="batched") for X, yb in pairs]
    b = cr.Batch(pairs, cr.Params(precision=cr.F32, kkt_tol=1e-4), tile_rows=tiles)
    b.start()
    replays = 0
    while b.advance(400):
        replays += 400
        progress("batched: %d graph replays so far" % replays)
    _, infos, secs = b.finish()
    progress("batched solve done: %.1f s" % secs)
    ms = b.time_pass(10)
    b.close()
    npairs = float(sum(q.N * (q.N - 1) for q in probs))
    return {"value": sum(i.pair_updates for i in infos) / secs, "unit": "pair-updates/s",
            "problems": len(probs), "seconds": secs, "converged": all(i.status == 0 for i in infos),
            "max_final_kkt": max(i.kkt for i in infos),
            "mapg_iters_per_problem": [i.inner_iters for i in infos], "pairs_per_iteration": npairs,
            "roofline": pass_roofline(ms, npairs, 4, "k_pair_pass_batched (all operand classes)",
                                      "pair_pass_batched_f32_64_problems")}


def diff_rate(cr, K=10, L=20, C=20):
    """The differentiable workload: N = 10000, n = 10, x ~ U[-1,1]^10,
    f0 = ||x||^2, noise N(0, 0.1^2), FP32, K x L unrolled MAPG iterations
    checkpointed every C, gradient of sum_l w_l y_l (w ~ N(0, 1))."""
    import torch
    import synth
    p = synth.workload("quadratic_10000")
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    w = torch.from_numpy(synth.weights(p.N)).cuda()
    params = cr.Params(precision=cr.F32, inner_iters=L, max_outer=K)
    d = cr.Diff(X, yb, params, checkpoint_every=C)
    d.forward(yb, None)
    d.backward(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.forward(yb, None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d.backward(w)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    adj_ms = d.time_adjoint_pass(10)
    d.close()
    pairs = p.N * (p.N - 1)
    iters = K * L
    adj_bytes = pairs * 4 * 3          # theta read, theta-bar read and write
    return {"value": pairs * iters / (t2 - t0), "unit": "pair-updates/s (forward + reverse, per unrolled iteration)",
            "N": p.N, "n": p.n, "schedule": "%d x %d MAPG, checkpoint every %d" % (K, L, C),
            "forward_s": t1 - t0, "backward_s": t2 - t1,
            "adjoint_pass": {"avg_ms": adj_ms, "bytes_per_launch": adj_bytes,
                             "achieved_GBs": adj_bytes / (adj_ms * 1e-3) / 1e9,
                             "frac": adj_bytes / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def eval_rate(cr, reps=10):
    """Estimator evaluation (cr_eval, FP64): the 20000 tangent planes
    (f0(x_l), grad f0(x_l)) of the maxaffine_20000 workload at 20000 query
    points q ~ U[-1,1]^20.  Device time from HIP events on the stream the
    kernels run on; algorithmic work 2(n+1) flops per (query, plane)."""
    import torch
    import synth
    p = synth.workload("maxaffine_20000")
    Q = torch.from_numpy(synth.query_points(p.N, p.n)).cuda()
    est = cr.Estimator(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.f0).cuda(), torch.from_numpy(p.grad_f0).cuda())
    for _ in range(2):
        est(Q)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        est(Q)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pairs = float(Q.shape[0]) * p.N
    tflops = 2.0 * (p.n + 1) * pairs / (ms * 1e-3) / 1e12
    return {"value": pairs / (ms * 1e-3), "unit": "query-plane evaluations/s", "M": int(Q.shape[0]), "N": p.N,
            "n": p.n, "ms": ms, "roofline": {"bound": "mfma", "achieved": tflops, "peak": MFMA_F64_PEAK_TFS,
                                             "unit": "TFLOP/s", "frac": tflops / MFMA_F64_PEAK_TFS}}


def papg_rate(cr, N=4096, n=5, K=4, iters=5, inner=40, outer=4):
    """P-APG (Fig. 2) on the problem of the Sec. III study scaled up: x ~ N(0, I_5),
    f0 = 1/2 x^T Q x with Q = Lambda^T Lambda, Lambda ~ N(0, 1), noise N(0, 1),
    N = 4096 points in K = 4 index sets; FP32 block solves of outer x inner MAPG
    steps, `iters` P-APG iterations after one untimed run."""
    import torch
    import synth
    p = synth.gaussian_quadratic(N, n, seed=0)
    X, yb = torch.from_numpy(p.X).cuda(), torch.from_numpy(p.ybar).cuda()
    params = cr.Params(precision=cr.F32, gamma=0.05, inner_iters=inner, max_outer=outer)
    pp = cr.PapgParams(K=K, iters=iters)
    cr.papg(X, yb, pp, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = cr.papg(X, yb, pp, params)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    nb = N // K
    block_pairs = float(K * nb * (nb - 1)) * inner * outer
    cross_pairs = float(N * N - K * nb * nb)
    return {"value": iters / secs, "unit": "P-APG iterations/s", "N": N, "n": n, "K": K,
            "schedule": "%d P-APG iterations, blocks %d x %d MAPG" % (iters, outer, inner),
            "ms_per_iteration": secs / iters * 1e3,
            "pair_updates_per_s": (block_pairs + cross_pairs) * iters / secs,
            "final_infeas_cross": info["infeas_cross"], "theta_norm": info["theta_norm"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=("f32", "f64"), default="f64")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-one-thread", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the pair engine runs on a single device "
              "(the multi-GPU sharding is described in the design notes, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1407_7220_amd as cr
    from paper_1407_7220_amd import autotune
    import synth

    p = synth.workload(WORKLOAD)
    prec = cr.F32 if args.precision == "f32" else cr.F64
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    tile_rows = autotune.tile_rows_for(X, yb, prec)
    params = cr.Params(precision=prec, kkt_tol=1e-4, tile_rows=tile_rows)
    ctx = cr.Context(X, yb, params)

    for w in range(args.warmup):
        ctx.run()
        progress("warm-up solve %d/%d done" % (w + 1, args.warmup))
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, _, info = ctx.run()
        infos.append(info)
        progress("step %d/%d: %d MAPG iterations, KKT %.2e" % (k + 1, args.steps, info.inner_iters, info.kkt))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pair_updates = sum(i.pair_updates for i in infos)
    value = pair_updates / wall
    converged = all(i.status == 0 and i.kkt <= 1e-4 for i in infos)

    # dominant kernel: the gradient pair pass, timed with HIP events on its own stream
    pass_ms = ctx.time_pass(50)
    esz = 4 if prec == cr.F32 else 8
    roof = pass_roofline(pass_ms, p.N * (p.N - 1), esz, "k_pair_pass",
                         "pair_pass_%s_%s" % (args.precision, WORKLOAD))

    line = {
        "metric": METRIC, "value": value, "unit": "pair-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": WORKLOAD, "N": p.N, "n": p.n, "precision": args.precision, "kkt_tol": 1e-4,
                   "mapg_iters_per_solve": infos[-1].inner_iters, "alcc_iters_per_solve": infos[-1].outer_iters,
                   "final_kkt": infos[-1].kkt, "converged": converged, "gamma": 1e-3, "tile_rows": tile_rows},
        "roofline": roof,
    }
    ctx.close()
    del X, yb
    torch.cuda.empty_cache()
    if not args.no_variants:
        v = {}
        other = cr.F64 if prec == cr.F32 else cr.F32
        Xo, ybo = torch.from_numpy(p.X).cuda(), torch.from_numpy(p.ybar).cuda()
        v[("f64" if other == cr.F64 else "f32") + "_" + WORKLOAD] = solve_rate(
            cr, p, other, autotune.tile_rows_for(Xo, ybo, other), steps=2, warmup=1, name=WORKLOAD)
        del Xo, ybo
        big = synth.workload("maxaffine_20000")
        Xb, ybb = torch.from_numpy(big.X).cuda(), torch.from_numpy(big.ybar).cuda()
        tr = autotune.tile_rows_for(Xb, ybb, cr.MIXED_BF16)
        leg = solve_rate(cr, big, cr.MIXED_BF16, tr, steps=1, warmup=0, name="maxaffine_20000")
        leg["error_vs_oracle"] = fixture_error(cr, big, cr.MIXED_BF16, tr)
        v["mixed_bf16_maxaffine_20000"] = leg
        torch.cuda.empty_cache()
        tr = autotune.tile_rows_for(Xb, ybb, cr.F32)
        leg = fixed_rate(cr, big, cr.F32, tr, name="maxaffine_20000")
        leg["error_vs_oracle"] = fixture_error(cr, big, cr.F32, tr)
        v["f32_maxaffine_20000"] = leg
        torch.cuda.empty_cache()
        del Xb, ybb
        torch.cuda.empty_cache()
        v["batched_f32_64_problems"] = batched_rate(cr, autotune)
        torch.cuda.empty_cache()
        progress("batched leg done")
        v["differentiable_f32_quadratic_10000"] = diff_rate(cr)
        torch.cuda.empty_cache()
        v["estimator_eval_f64_20000x20000"] = eval_rate(cr)
        torch.cuda.empty_cache()
        v["papg_f32_gaussian_quadratic_4096_K4"] = papg_rate(cr)
        progress("differentiable, estimator and P-APG legs done")
        line["variants"] = v
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_budget, args.cpu_one_thread)
        progress("CPU baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
