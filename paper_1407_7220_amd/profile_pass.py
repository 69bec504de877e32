"""Profiling driver: repeated pair passes on a named workload, then one theta
export (k_theta_export: reads the N x N pass-precision theta once and writes
it as N x N doubles), a plain copy of known size that serves as the reference
for scaling hardware byte counters.  Run it under rocprofv3, e.g.

    rocprofv3 --kernel-trace --stats -d OUT -- python -u paper_1407_7220_amd/profile_pass.py
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -u paper_1407_7220_amd/profile_pass.py --reps 5

--kernel pass     gradient pair passes (k_pair_pass) with the tile height the
                  autotuner cached for the workload (the benchmark's launch);
--kernel adjoint  adjoint pair passes of a MAPG step (k_adj_pass) after one
                  forward and reverse run of 2 x 2 unrolled iterations;
--kernel eval     estimator evaluations (k_eval) of the workload's tangent planes
                  (f0(x_l), grad f0(x_l)) at N query points q ~ U[-1,1]^n;
--kernel batched  batched solves (k_pair_pass_batched, k_reduce_batched,
                  k_update_batched) of the 64-problem FP32 workload
                  (N_p ~ U{500..8000}, n_p in {5, 10, 20}) with the tuned
                  tile heights, a fixed schedule of 1 x --reps MAPG steps per
                  problem after one untimed run;
--kernel solve    one fixed-schedule solve (2 ALCC iterations of --reps MAPG
                  steps) in the benchmark's launch configuration: the MAPG
                  iteration's kernels (lazy pass, reduce) and the multiplier step's;
--kernel papg     P-APG runs (cr_papg: k_papg_lin, k_papg_step2 and the batched
                  block solves) on the Sec. III study problem at N = 4096,
                  n = 5, K = 4, FP32 blocks of 4 x 40 MAPG steps, --reps
                  iterations after one untimed run of the same length.
"""
import argparse
import os
import time
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", choices=("pass", "adjoint", "eval", "papg", "batched", "solve"), default="pass")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--precision", choices=("f32", "f64", "mixed_bf16"), default="f32")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    import torch
    import paper_1407_7220_amd as cr
    from paper_1407_7220_amd import autotune
    import synth
    if args.kernel == "papg":
        q = synth.gaussian_quadratic(4096, 5, seed=0)
        X, yb = torch.from_numpy(q.X).cuda(), torch.from_numpy(q.ybar).cuda()
        params = cr.Params(precision=cr.F32, gamma=0.05, inner_iters=40, max_outer=4)
        pp = cr.PapgParams(K=4, iters=args.reps)
        cr.papg(X, yb, pp, params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = cr.papg(X, yb, pp, params)
        torch.cuda.synchronize()
        print("workload gaussian_quadratic N=4096 n=5 K=4: %d P-APG iterations, %.3f ms each"
              % (args.reps, (time.perf_counter() - t0) / args.reps * 1e3), flush=True)
        return
    if args.kernel == "batched":
        probs = synth.batched_workload()
        pairs = [(torch.from_numpy(q.X).cuda(), torch.from_numpy(q.ybar).cuda()) for q in probs]
        tiles = [autotune.tile_rows_for(X, yb, cr.F32, form="batched", tune_if_missing=False) for X, yb in pairs]
        b = cr.Batch(pairs, cr.Params(precision=cr.F32, inner_iters=args.reps, max_outer=1), tile_rows=tiles)
        b.run()
        _, infos, secs = b.run()
        b.close()
        pairs_per_it = sum(q.N * (q.N - 1) for q in probs)
        print("workload batched (64 problems, %d pairs per MAPG iteration): %d MAPG iterations, %.3f ms each"
              % (pairs_per_it, args.reps, secs / args.reps * 1e3), flush=True)
        return
    workload = args.workload or {"pass": "logsumexp_5000", "adjoint": "quadratic_10000",
                                 "eval": "maxaffine_20000", "solve": "logsumexp_5000"}[args.kernel]
    p = synth.workload(workload)
    if args.kernel == "eval":
        Q = torch.from_numpy(synth.query_points(p.N, p.n)).cuda()
        est = cr.Estimator(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.f0).cuda(),
                           torch.from_numpy(p.grad_f0).cuda())
        est(Q)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            est(Q)
        e1.record()
        torch.cuda.synchronize()
        print("workload %s N=%d n=%d queries %d: %d evaluations, avg %.3f us"
              % (workload, p.N, p.n, Q.shape[0], args.reps, e0.elapsed_time(e1) / args.reps * 1e3), flush=True)
        return
    prec = {"f32": cr.F32, "f64": cr.F64, "mixed_bf16": cr.MIXED_BF16}[args.precision]
    X = torch.from_numpy(p.X).cuda()
    yb = torch.from_numpy(p.ybar).cuda()
    tile = autotune.tile_rows_for(X, yb, prec, tune_if_missing=False)
    esz = 8 if prec == cr.F64 else 4
    if args.kernel == "solve":
        ctx = cr.Context(X, yb, cr.Params(precision=prec, tile_rows=tile, inner_iters=args.reps, max_outer=2))
        ctx.run()
        _, _, info = ctx.run()
        print("workload %s N=%d n=%d precision %s tile_rows %d: 2 x %d MAPG iterations, %.3f us each"
              % (workload, p.N, p.n, args.precision, tile, args.reps, info.seconds / info.inner_iters * 1e6), flush=True)
        return
    if args.kernel == "pass":
        ctx = cr.Context(X, yb, cr.Params(precision=prec, tile_rows=tile))
        ms = ctx.time_pass(args.reps)
        ctx.get_theta()
        what = "pair passes"
    else:
        d = cr.Diff(X, yb, cr.Params(precision=prec, inner_iters=2, max_outer=2, tile_rows=tile), checkpoint_every=2)
        d.forward(yb, None)
        d.backward(torch.from_numpy(synth.weights(p.N)).cuda())
        ms = d.time_adjoint_pass(args.reps)
        d.close()
        # the calibration copy on a context of the same size
        cr.Context(X, yb, cr.Params(precision=prec, tile_rows=tile)).get_theta()
        what = "adjoint pair passes"
    torch.cuda.synchronize()
    print("workload %s N=%d n=%d precision %s tile_rows %d: %d %s, avg %.3f us; theta export reads %d B, writes %d B"
          % (workload, p.N, p.n, args.precision, tile, args.reps, what, ms * 1e3, p.N * p.N * esz, p.N * p.N * 8),
          flush=True)


if __name__ == "__main__":
    main()
