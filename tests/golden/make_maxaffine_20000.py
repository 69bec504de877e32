"""Writes the FP64 oracle's iterate of the 20000-point, n = 20 max-affine
workload after a fixed ALCC schedule of 2 x 25 MAPG iterations (Fig. 3 with
Fig. 4, default parameters, gamma = 1e-3) to maxaffine_20000_2x25.npz.

The GPU parity tests of that workload (FP32 and the mixed BF16 form) and the
benchmark's mixed-precision leg compare against it; the oracle itself needs
about half an hour on 8 cores here, too long for a test.  Only ``oracle`` and
``synth`` are called.  Stored: y (N), xi (N x n), the SHA-256 of the inputs
(X then ybar, float64 bytes) and the schedule.

Command (from the repository root):
    python tests/golden/make_maxaffine_20000.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

SCHEDULE = dict(inner_iters=25, max_outer=2)
OUT = os.path.join(HERE, "maxaffine_20000_2x25.npz")


def input_hash(p) -> str:
    return hashlib.sha256(p.X.tobytes() + p.ybar.tobytes()).hexdigest()


def main():
    p = synth.workload("maxaffine_20000")
    t0 = time.time()
    res = oracle.alcc(p.X, p.ybar, oracle.Params(**SCHEDULE), record_kkt=False)
    meta = dict(workload=p.name, N=p.N, n=p.n, schedule=SCHEDULE, gamma=oracle.Params().gamma,
                input_sha256=input_hash(p), seconds=round(time.time() - t0, 1),
                command="python tests/golden/make_maxaffine_20000.py")
    np.savez(OUT, y=res.y, xi=res.xi, meta=json.dumps(meta))
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
