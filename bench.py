"""Throughput benchmark: constraint-pair updates per second of the ALCC/MAPG
solve run to KKT <= 1e-4, on one MI355X.

A step is one whole solve (every stage of the hot path: pair passes, MAPG
steps, multiplier steps and KKT checks) of the 5000-point, n = 10 workload
(x ~ N(0, I), f0 = log-sum-exp of 20 random affine maps, noise N(0, 0.05^2)),
with the inputs already resident in device memory.  value = sum over the timed
steps of N (N - 1) x MAPG iterations / wall seconds.

Also reported on the same JSON line:
  roofline      the dominant kernel (the gradient pair pass): algorithmic bytes
                (one theta read per pair) / its average device time, measured
                with HIP events on the library's stream, against 8 TB/s HBM;
  cpu_baseline  the FP64 CPU oracle timed on the host cores on a bounded
                sample of the same workload (a fixed number of MAPG iterations);
  variants      the same metric for the FP64 solve of the same workload, and the
                steady-state MAPG throughput (fixed iteration count, stated) of
                the mixed BF16 form on the 20000-point workload and of the
                64-problem batched form, the differentiable form (10000
                points, 10 x 20 unrolled iterations, forward + reverse pass),
                the estimator evaluation and P-APG (4096 points, K = 4).
The pass tile height comes from the autotuner (paper_1407_7220_amd.autotune).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f32|f64]
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


def load_traffic(prec_name: str):
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "pair_pass_%s_%s_counters.json" % (prec_name, WORKLOAD))
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(p, budget_s: float):
    """Oracle MAPG iterations (FP64, C operators + numpy) on the same workload,
    from the same starting point, until about budget_s seconds have passed."""
    import numpy as np
    import oracle
    gamma = 1e-3
    yhat, xihat, Bbar, By, Bxi = oracle.affine_fit(p.X, p.ybar, gamma)
    N = p.N
    mu = 1.0 / (2.0 * N)
    Ly = 1.0 / mu + oracle.sigma2_A1(N)
    Lxi = gamma / mu + oracle.sigma2_A2(p.X)
    theta = np.zeros((N, N))
    oracle.mapg(p.X, p.ybar, gamma, mu, theta, Ly, Lxi, yhat, xihat, By, Bxi, 0, 0, 1, adaptive=False)
    t0 = time.perf_counter()
    iters = 0
    y, xi = yhat, xihat
    while time.perf_counter() - t0 < budget_s:
        y, xi, _ = oracle.mapg(p.X, p.ybar, gamma, mu, theta, Ly, Lxi, y, xi, By, Bxi, 0, 0, 1, adaptive=False)
        iters += 1
    secs = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": N * (N - 1) * iters / secs, "unit": "pair-updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d MAPG iterations of the FP64 oracle on %s (N=%d, n=%d), %.1f s" % (
                iters, WORKLOAD, N, p.n, secs)}


def solve_rate(cr, p, prec, tile_rows, steps=1, warmup=0):
    """Pair-updates/s of whole solves to KKT <= 1e-4 on workload p."""
    import torch
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    ctx = cr.Context(X, yb, cr.Params(precision=prec, kkt_tol=1e-4, tile_rows=tile_rows))
    for _ in range(warmup):
        ctx.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [ctx.run()[2] for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms = ctx.time_pass(20)
    ctx.close()
    return {"value": sum(i.pair_updates for i in infos) / wall, "unit": "pair-updates/s",
            "mapg_iters_per_solve": infos[-1].inner_iters, "final_kkt": infos[-1].kkt,
            "converged": all(i.status == 0 for i in infos), "pass_us": pass_ms * 1e3, "tile_rows": tile_rows}


def fixed_rate(cr, p, prec, tile_rows, inner=100, outer=2):
    """Steady-state pair-updates/s over a fixed schedule (outer x inner MAPG iterations)."""
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
    return {"value": info.pair_updates / wall, "unit": "pair-updates/s", "schedule": "%d x %d MAPG" % (outer, inner),
            "N": p.N, "n": p.n, "pass_us": pass_ms * 1e3, "tile_rows": tile_rows,
            "pass_hbm_frac": p.N * (p.N - 1) * esz / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def batched_rate(cr, autotune, inner=100, outer=2):
    import torch
    import synth
    probs = synth.batched_workload()
    pairs = [(torch.from_numpy(q.X).cuda(), torch.from_numpy(q.ybar).cuda()) for q in probs]
    tiles = [autotune.tile_rows_for(X, yb, cr.F32, form="batched") for X, yb in pairs]
    b = cr.Batch(pairs, cr.Params(precision=cr.F32, inner_iters=inner, max_outer=outer), tile_rows=tiles)
    b.run()
    _, infos, secs = b.run()
    b.close()
    return {"value": sum(i.pair_updates for i in infos) / secs, "unit": "pair-updates/s",
            "schedule": "%d x %d MAPG, every problem" % (outer, inner), "problems": len(probs),
            "pairs_per_iteration": float(sum(q.N * (q.N - 1) for q in probs))}


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
    ap.add_argument("--precision", choices=("f32", "f64"), default="f32")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
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

    for _ in range(args.warmup):
        ctx.run()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, info = ctx.run()
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pair_updates = sum(i.pair_updates for i in infos)
    value = pair_updates / wall
    converged = all(i.status == 0 and i.kkt <= 1e-4 for i in infos)

    # dominant kernel: the gradient pair pass, timed with HIP events on its own stream
    pass_ms = ctx.time_pass(50)
    esz = 4 if prec == cr.F32 else 8
    alg_bytes = p.N * (p.N - 1) * esz
    achieved = alg_bytes / (pass_ms * 1e-3) / 1e9
    traffic = load_traffic(args.precision)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_pair_pass", "avg_ms": pass_ms, "bytes_per_launch": alg_bytes}

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
    if not args.no_variants:
        other = cr.F64 if prec == cr.F32 else cr.F32
        v = {("f64" if other == cr.F64 else "f32") + "_" + WORKLOAD:
             solve_rate(cr, p, other, autotune.tile_rows_for(X, yb, other))}
        big = synth.workload("maxaffine_20000")
        Xb, ybb = torch.from_numpy(big.X).cuda(), torch.from_numpy(big.ybar).cuda()
        v["mixed_bf16_maxaffine_20000"] = fixed_rate(cr, big, cr.MIXED_BF16,
                                                     autotune.tile_rows_for(Xb, ybb, cr.MIXED_BF16))
        v["f32_maxaffine_20000"] = fixed_rate(cr, big, cr.F32, autotune.tile_rows_for(Xb, ybb, cr.F32))
        del Xb, ybb
        torch.cuda.empty_cache()
        v["batched_f32_64_problems"] = batched_rate(cr, autotune)
        torch.cuda.empty_cache()
        v["differentiable_f32_quadratic_10000"] = diff_rate(cr)
        torch.cuda.empty_cache()
        v["estimator_eval_f64_20000x20000"] = eval_rate(cr)
        torch.cuda.empty_cache()
        v["papg_f32_gaussian_quadratic_4096_K4"] = papg_rate(cr)
        line["variants"] = v
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
