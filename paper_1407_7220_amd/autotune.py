"""Tile autotuner of the pair pass.

The one free tile dimension of the pass is the number of theta rows a
workgroup sweeps (``tile_rows``): taller tiles amortise the per-workgroup
prologue (in a MAPG run, the completion of the previous step for the
workgroup's rows and columns) and the column-partial writes, shorter ones give
the scheduler more workgroups.  For single-problem solves the tuner times whole
MAPG iterations (a short fixed-schedule run: pair pass plus reductions, since
the tile height also sets the reduction's work and whether the pass can
complete the previous step itself); for the batched form, whose graph runs the
plain pass and its own update, it times the gradient pass alone (HIP events
inside the library, ``Context.time_pass``).  Candidates run on the caller's
own data and the fastest is kept.  Choices are cached in a JSON file keyed on
(form, n, precision, N bucket), the bucket being N rounded to the nearest
quarter octave.  The cache path is ``tile_cache.json`` next to this file
unless ``CR_TILE_CACHE`` names another.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional

if __package__ in (None, ""):
    import sys as _sys
    _sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1407_7220_amd import Context, Params, F64, F32, MIXED_BF16
else:
    from . import Context, Params, F64, F32, MIXED_BF16

CANDIDATES = (128, 256, 384, 512, 640, 768, 896, 1024, 1536, 2048, 2560, 3072, 4096)
_PREC = {F64: "f64", F32: "f32", MIXED_BF16: "mixed_bf16"}


def cache_path() -> str:
    return os.environ.get("CR_TILE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "tile_cache.json"))


def bucket(N: int) -> int:
    """N rounded to the nearest quarter octave, 2^(k/4)."""
    return int(round(2.0 ** (round(4.0 * math.log2(max(2, int(N)))) / 4.0)))


FORMS = ("solve", "batched")


def key(N: int, n: int, precision: int, form: str = "solve") -> str:
    k = "n%d-%s-N%d" % (int(n), _PREC[int(precision)], bucket(N))
    return k if form == "solve" else form + "-" + k


def load_cache() -> Dict[str, dict]:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict]) -> None:
    path = cache_path()
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(N: int, n: int, precision: int, form: str = "solve") -> Optional[int]:
    entry = load_cache().get(key(N, n, precision, form))
    return int(entry["tile_rows"]) if entry else None


def _time(X, ybar, precision: int, r: int, form: str, reps: int) -> float:
    """Milliseconds per MAPG iteration (form 'solve') or per gradient pass ('batched')."""
    if form == "batched":
        ctx = Context(X, ybar, Params(precision=precision, tile_rows=int(r)))
        ctx.time_pass(3)
        ms = ctx.time_pass(reps)
    else:
        iters = max(32, 2 * reps)
        ctx = Context(X, ybar, Params(precision=precision, tile_rows=int(r), inner_iters=iters, max_outer=1))
        ctx.run()                                  # captures the iteration graph
        ms = min(1e3 * ctx.run()[2].seconds / iters for _ in range(2))
    ctx.close()
    return ms


def tune(X, ybar, precision: int, reps: int = 20, candidates=CANDIDATES, save: bool = True,
         form: str = "solve") -> int:
    """Time each candidate tile height on (X, ybar); return and cache the fastest."""
    N, n = int(X.shape[0]), int(X.shape[1])
    rows = ((N + 63) // 64) * 64
    timings = {}
    for r in candidates:
        if r > rows and timings:
            continue
        timings[int(r)] = _time(X, ybar, precision, r, form, reps)
    best = min(timings, key=timings.get)
    if save:
        cache = load_cache()
        cache[key(N, n, precision, form)] = {
            "tile_rows": best, "ms": timings[best], "N": N,
            "metric": "ms per MAPG iteration" if form == "solve" else "ms per gradient pass",
            "timings_ms": {str(k): v for k, v in sorted(timings.items())}}
        save_cache(cache)
    return best


def tile_rows_for(X, ybar, precision: int, tune_if_missing: bool = True, form: str = "solve") -> int:
    """Cached tile height for this (form, n, precision, N bucket), tuning on (X, ybar) if
    absent (0, the library's heuristic, when tuning is not allowed)."""
    N, n = int(X.shape[0]), int(X.shape[1])
    found = lookup(N, n, precision, form)
    if found is not None:
        return found
    return tune(X, ybar, precision, form=form) if tune_if_missing else 0


def _main(argv=None) -> int:
    """Tune the named synthetic workloads (the seeded generators beside the
    package) and write their entries to the cache:
    python paper_1407_7220_amd/autotune.py logsumexp_5000:f32 maxaffine_20000:mixed_bf16 batched:f32"""
    import argparse
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("targets", nargs="+", help="workload:precision, workload 'batched' = the 64-problem set")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--force", action="store_true", help="re-tune keys that the cache already holds")
    args = ap.parse_args(argv)
    names = {v: k for k, v in _PREC.items()}
    done = set()       # keys tuned in this run: the first target to reach a key keeps it
    for t in args.targets:
        wl, pn = t.split(":")
        prec = names[pn]
        form = "batched" if wl == "batched" else "solve"
        probs = synth.batched_workload() if wl == "batched" else [synth.workload(wl)]
        for p in probs:
            k = key(p.N, p.n, prec, form)
            if k in done or (not args.force and k in load_cache()):
                continue
            done.add(k)
            X = torch.from_numpy(p.X).cuda()
            yb = torch.from_numpy(p.ybar).cuda()
            best = tune(X, yb, prec, reps=args.reps, form=form)
            e = load_cache()[k]
            print("%-36s N=%-6d tile_rows=%-5d %.4f %s  (%s)" % (
                k, p.N, best, e["ms"], e["metric"], " ".join("%s:%.4f" % kv for kv in e["timings_ms"].items())),
                flush=True)
            del X, yb
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
