"""Profiling driver: repeated gradient pair passes on a named workload, then one
theta export (k_theta_export: reads the N x N pass-precision theta once and
writes it as N x N doubles), a plain copy of known size that serves as the
reference for scaling hardware byte counters.  Run it under rocprofv3, e.g.

    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_1407_7220_amd.profile_pass
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_1407_7220_amd.profile_pass
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="logsumexp_5000")
    ap.add_argument("--precision", choices=("f32", "f64"), default="f32")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    import torch
    import paper_1407_7220_amd as cr
    import synth
    p = synth.workload(args.workload)
    prec = cr.F32 if args.precision == "f32" else cr.F64
    ctx = cr.Context(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.ybar).cuda(), cr.Params(precision=prec))
    ms = ctx.time_pass(args.reps)
    ctx.get_theta()
    torch.cuda.synchronize()
    esz = 4 if prec == cr.F32 else 8
    print("workload %s N=%d n=%d precision %s: %d pair passes, avg %.3f us; theta export reads %d B, writes %d B" % (
        args.workload, p.N, p.n, args.precision, args.reps, ms * 1e3, p.N * p.N * esz, p.N * p.N * 8), flush=True)


if __name__ == "__main__":
    main()
