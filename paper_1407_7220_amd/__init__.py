"""MI355X (gfx950) engine for least-squares convex regression.

A thin ctypes binding of the C ABI in ``include/cr.h`` (``libcr.so``, built
from ``csrc/``).  It only marshals arguments: every step of the solver runs in
the HIP kernels of the library.  PyTorch supplies device memory and the
stream; importing this package fails loudly when the library is missing.

Problem (Aybat & Wang, Sec. II-C, eq. "regularize"):
    min 1/2||y - ybar||^2 + gamma/2||xi||^2
    s.t. y_i >= y_j + xi_j^T (x_i - x_j) for all i != j,
solved by ALCC (Fig. 3) with MAPG (Fig. 4) as the inner solver.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Optional

__all__ = [
    "Params", "Info", "CRError", "Context", "solve", "workspace_bytes", "lib_path",
    "F64", "F32", "MIXED_BF16", "GRAD", "THETA_UPDATE", "MAX_DIM", "Batch", "solve_batched",
    "Diff", "diff_workspace_bytes", "solve_unrolled", "Estimator", "evaluate", "eval_workspace_bytes",
    "PapgParams", "papg_workspace_bytes", "papg",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcr.so")

F64, F32, MIXED_BF16 = 0, 1, 2
PAPG_ACCELERATED, PAPG_GRADIENT = 0, 1
GRAD, THETA_UPDATE = 0, 1
MAX_DIM = 31

OK, ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_NONFINITE, NOT_CONVERGED, ERR_STATE, ERR_UNSUPPORTED = range(8)


class _CParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("gamma", "mu1", "c", "kappa", "tau1", "alpha_y1", "alpha_xi1", "step_scale", "kkt_tol")] + \
               [(k, ctypes.c_int32) for k in ("max_outer", "inner_iters", "max_inner", "precision",
                                              "tile_rows", "deterministic")] + \
               [(k, ctypes.c_double) for k in ("Ly_override", "Lxi_override", "By_override", "Bxi_override")]


class _CProblem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("X_dev", ctypes.c_void_p), ("ybar_dev", ctypes.c_void_p),
                ("y_dev", ctypes.c_void_p), ("xi_dev", ctypes.c_void_p)]


class _CPapgParams(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("iters", ctypes.c_int32), ("L", ctypes.c_double),
                ("B_theta", ctypes.c_double), ("y_shift", ctypes.c_double), ("method", ctypes.c_int32),
                ("power_iters", ctypes.c_int32)]


class _CPapgInfo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("y_shift", ctypes.c_double), ("theta_norm", ctypes.c_double),
                ("infeas_cross", ctypes.c_double), ("inner_iters", ctypes.c_int64), ("seconds", ctypes.c_double)]


class _CInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("status", ctypes.c_int32), ("inner_iters", ctypes.c_int64)] + \
               [(k, ctypes.c_double) for k in
                ("objective", "kkt", "stat_y", "stat_xi", "infeas", "compl_", "infeas_norm", "gap_norm",
                 "seconds", "pair_updates", "sigma2_A1", "sigma2_A2", "Bbar_y", "Bbar_xi")]


def lib_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            "libcr.so is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_1407_7220_amd/build.py` first")
    # torch first: its HIP runtime then serves this library too (one runtime per
    # process; loading the library first binds a second copy that sees no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pp, pi = ctypes.POINTER(_CParams), ctypes.POINTER(_CInfo)
    sig = {
        "cr_params_default": (i32, [pp]),
        "cr_status_string": (ctypes.c_char_p, [i32]),
        "cr_last_error": (ctypes.c_char_p, [vp]),
        "cr_workspace_bytes": (i32, [i64, i32, pp, ctypes.POINTER(ctypes.c_size_t)]),
        "cr_init": (i32, [ctypes.POINTER(vp), i64, i32, pp, vp, vp, vp, ctypes.c_size_t, vp]),
        "cr_destroy": (i32, [vp]),
        "cr_pairwise_step": (i32, [vp, i32, vp, vp, vp, vp, dbl, dbl]),
        "cr_run": (i32, [vp, vp, vp, pi]),
        "cr_solve": (i32, [vp, vp, i64, i32, pp, vp, vp, vp, ctypes.c_size_t, pi, vp]),
        "cr_get_theta": (i32, [vp, vp]),
        "cr_set_theta": (i32, [vp, vp]),
        "cr_get_start": (i32, [vp, vp, vp]),
        "cr_get_info": (i32, [vp, pi]),
        "cr_time_pass": (i32, [vp, i32, i32, ctypes.POINTER(dbl)]),
        "cr_pass_layout": (i32, [i64, i32, pp, ctypes.POINTER(i64)]),
        "cr_get_outer_history": (i32, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(i32)]),
        "cr_batch_workspace_bytes": (i32, [ctypes.POINTER(_CProblem), i32, pp, ctypes.POINTER(ctypes.c_size_t)]),
        "cr_batch_init": (i32, [ctypes.POINTER(vp), ctypes.POINTER(_CProblem), i32, pp, vp, ctypes.c_size_t, vp]),
        "cr_batch_run": (i32, [vp, pi, ctypes.POINTER(dbl)]),
        "cr_batch_destroy": (i32, [vp]),
        "cr_batch_time_pass": (i32, [vp, i32, ctypes.POINTER(dbl)]),
        "cr_batch_start": (i32, [vp]),
        "cr_batch_advance": (i32, [vp, i32, ctypes.POINTER(i32)]),
        "cr_batch_finish": (i32, [vp, pi, ctypes.POINTER(dbl)]),
        "cr_solve_batched": (i32, [ctypes.POINTER(_CProblem), i32, pp, vp, ctypes.c_size_t, pi, vp]),
        "cr_diff_workspace_bytes": (i32, [i64, i32, pp, i32, ctypes.POINTER(ctypes.c_size_t)]),
        "cr_diff_init": (i32, [ctypes.POINTER(vp), i64, i32, pp, i32, vp, vp, vp, ctypes.c_size_t, vp]),
        "cr_diff_forward": (i32, [vp, vp, vp, vp, vp, pi]),
        "cr_diff_backward": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "cr_diff_destroy": (i32, [vp]),
        "cr_diff_time_adjoint_pass": (i32, [vp, i32, ctypes.POINTER(dbl)]),
        "cr_eval_workspace_bytes": (i32, [i64, i32, ctypes.POINTER(ctypes.c_size_t)]),
        "cr_eval": (i32, [vp, vp, vp, i64, i32, vp, i64, vp, vp, vp, ctypes.c_size_t, vp]),
        "cr_eval_noalloc": (i32, [vp, vp, vp, i64, i32, vp, i64, vp, vp, vp]),
        "cr_papg_workspace_bytes": (i32, [i64, i32, pp, ctypes.POINTER(_CPapgParams), ctypes.POINTER(ctypes.c_size_t)]),
        "cr_papg": (i32, [vp, vp, i64, i32, pp, ctypes.POINTER(_CPapgParams), vp, vp, vp, vp,
                          ctypes.POINTER(dbl), vp, ctypes.c_size_t, ctypes.POINTER(_CPapgInfo), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()

EXPORTED = ("cr_params_default", "cr_status_string", "cr_last_error", "cr_workspace_bytes", "cr_init",
            "cr_destroy", "cr_pairwise_step", "cr_run", "cr_solve", "cr_get_theta", "cr_set_theta",
            "cr_get_start", "cr_get_info", "cr_time_pass", "cr_get_outer_history", "cr_pass_layout", "cr_batch_workspace_bytes", "cr_batch_init",
            "cr_batch_run", "cr_batch_destroy", "cr_batch_time_pass", "cr_batch_start", "cr_batch_advance", "cr_batch_finish", "cr_solve_batched", "cr_diff_workspace_bytes", "cr_diff_init",
            "cr_diff_forward", "cr_diff_backward", "cr_diff_destroy", "cr_diff_time_adjoint_pass",
            "cr_eval_workspace_bytes", "cr_eval", "cr_eval_noalloc", "cr_papg_workspace_bytes", "cr_papg")


class CRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_lib.cr_status_string(status).decode(), msg))
        self.status = status


def _check(status: int, ctx=None, allow=(OK,)):
    if status not in allow:
        raise CRError(status, (_lib.cr_last_error(ctx) or b"").decode())
    return status


@dataclasses.dataclass
class Params:
    """ALCC/MAPG parameters (see ``include/cr.h``); None keeps the library default."""
    gamma: Optional[float] = None
    mu1: Optional[float] = None
    c: Optional[float] = None
    kappa: Optional[float] = None
    tau1: Optional[float] = None
    alpha_y1: Optional[float] = None
    alpha_xi1: Optional[float] = None
    step_scale: Optional[float] = None
    kkt_tol: Optional[float] = None
    max_outer: Optional[int] = None
    inner_iters: Optional[int] = None
    max_inner: Optional[int] = None
    precision: Optional[int] = None
    tile_rows: Optional[int] = None
    deterministic: Optional[int] = None
    Ly_override: Optional[float] = None
    Lxi_override: Optional[float] = None
    By_override: Optional[float] = None
    Bxi_override: Optional[float] = None

    def to_c(self) -> _CParams:
        p = _CParams()
        _check(_lib.cr_params_default(ctypes.byref(p)))
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if v is not None:
                setattr(p, f.name, v)
        return p


@dataclasses.dataclass
class Info:
    outer_iters: int
    status: int
    inner_iters: int
    objective: float
    kkt: float
    stat_y: float
    stat_xi: float
    infeas: float
    compl: float
    infeas_norm: float
    gap_norm: float
    seconds: float
    pair_updates: float
    sigma2_A1: float
    sigma2_A2: float
    Bbar_y: float
    Bbar_xi: float

    @classmethod
    def from_c(cls, ci: _CInfo) -> "Info":
        d = {f: getattr(ci, f) for f, _ in _CInfo._fields_}
        d["compl"] = d.pop("compl_")
        return cls(**d)


def workspace_bytes(N: int, n: int, params: Optional[Params] = None) -> int:
    out = ctypes.c_size_t(0)
    cp = (params or Params()).to_c()
    _check(_lib.cr_workspace_bytes(int(N), int(n), ctypes.byref(cp), ctypes.byref(out)))
    return int(out.value)


def _torch():
    import torch
    return torch


def _dev_f64(t, shape, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous float64 CUDA tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


class Context:
    """A solver context bound to (X, ybar) on the current CUDA/HIP device and stream.

    Keeps references to X, ybar and the workspace tensor for its lifetime."""

    def __init__(self, X, ybar, params: Optional[Params] = None):
        torch = _torch()
        self.N, self.n = int(X.shape[0]), int(X.shape[1])
        self.params = params or Params()
        self._X = X
        self._ybar = ybar
        px = _dev_f64(X, (self.N, self.n), "X")
        py = _dev_f64(ybar, (self.N,), "ybar")
        nbytes = workspace_bytes(self.N, self.n, self.params)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        self._cp = self.params.to_c()
        h = ctypes.c_void_p()
        _check(_lib.cr_init(ctypes.byref(h), self.N, self.n, ctypes.byref(self._cp), px, py,
                            ctypes.c_void_p(self._ws.data_ptr()), nbytes, _stream()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.cr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, *shape):
        torch = _torch()
        return torch.empty(*shape, dtype=torch.float64, device=self._X.device)

    def pairwise_step(self, mode: int, y, xi, mu: float, mu_next: float = 0.0):
        """One pass over all pairs (CR_GRAD or CR_THETA_UPDATE); returns (gy, gxi)."""
        gy, gxi = self._new(self.N), self._new(self.N, self.n)
        _check(_lib.cr_pairwise_step(self._h, int(mode), _dev_f64(y, (self.N,), "y"),
                                     _dev_f64(xi, (self.N, self.n), "xi"), ctypes.c_void_p(gy.data_ptr()),
                                     ctypes.c_void_p(gxi.data_ptr()), float(mu), float(mu_next)), self._h)
        return gy, gxi

    def run(self):
        """ALCC/MAPG to kkt_tol (or the fixed schedule); returns (y, xi, Info)."""
        y, xi = self._new(self.N), self._new(self.N, self.n)
        ci = _CInfo()
        _check(_lib.cr_run(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(xi.data_ptr()),
                           ctypes.byref(ci)), self._h, allow=(OK, NOT_CONVERGED))
        return y, xi, Info.from_c(ci)

    def get_theta(self):
        th = self._new(self.N, self.N)
        _check(_lib.cr_get_theta(self._h, ctypes.c_void_p(th.data_ptr())), self._h)
        return th

    def set_theta(self, theta):
        _check(_lib.cr_set_theta(self._h, _dev_f64(theta, (self.N, self.N), "theta")), self._h)

    def get_start(self):
        y, xi = self._new(self.N), self._new(self.N, self.n)
        _check(_lib.cr_get_start(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(xi.data_ptr())), self._h)
        return y, xi

    def time_pass(self, reps: int = 20) -> float:
        """Average device milliseconds of one gradient pair pass (HIP events)."""
        out = ctypes.c_double(0.0)
        _check(_lib.cr_time_pass(self._h, GRAD, int(reps), ctypes.byref(out)), self._h)
        return float(out.value)

    def info(self) -> Info:
        ci = _CInfo()
        _check(_lib.cr_get_info(self._h, ctypes.byref(ci)), self._h)
        return Info.from_c(ci)

    def outer_history(self):
        """(MAPG iterations, KKT measure) of every ALCC iteration of the last run."""
        cnt = ctypes.c_int32(0)
        _check(_lib.cr_get_outer_history(self._h, 0, None, None, ctypes.byref(cnt)), self._h)
        m = cnt.value
        inner = (ctypes.c_int64 * max(m, 1))()
        kkt = (ctypes.c_double * max(m, 1))()
        _check(_lib.cr_get_outer_history(self._h, m, inner, kkt, ctypes.byref(cnt)), self._h)
        return [int(inner[k]) for k in range(m)], [float(kkt[k]) for k in range(m)]


def solve(X, ybar, params: Optional[Params] = None):
    """cr_solve: returns (y, xi, Info) for float64 CUDA tensors X (N x n) and ybar (N)."""
    torch = _torch()
    N, n = int(X.shape[0]), int(X.shape[1])
    p = params or Params()
    cp = p.to_c()
    px = _dev_f64(X, (N, n), "X")
    py = _dev_f64(ybar, (N,), "ybar")
    nbytes = workspace_bytes(N, n, p)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    y = torch.empty(N, dtype=torch.float64, device=X.device)
    xi = torch.empty(N, n, dtype=torch.float64, device=X.device)
    ci = _CInfo()
    _check(_lib.cr_solve(px, py, N, n, ctypes.byref(cp), ctypes.c_void_p(y.data_ptr()),
                         ctypes.c_void_p(xi.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes,
                         ctypes.byref(ci), _stream()), None, allow=(OK, NOT_CONVERGED))
    return y, xi, Info.from_c(ci)


class Batch:
    """Many independent problems solved together (cr_batch_*): problems is a list
    of (X, ybar) float64 CUDA tensor pairs with their own N and n."""

    def __init__(self, problems, params: Optional[Params] = None, tile_rows=None):
        torch = _torch()
        self.params = params or Params()
        self._keep = []
        self.P = len(problems)
        arr = (_CProblem * self.P)()
        self.outputs = []
        for p, (X, ybar) in enumerate(problems):
            N, n = int(X.shape[0]), int(X.shape[1])
            px = _dev_f64(X, (N, n), "X[%d]" % p)
            py = _dev_f64(ybar, (N,), "ybar[%d]" % p)
            y = torch.empty(N, dtype=torch.float64, device=X.device)
            xi = torch.empty(N, n, dtype=torch.float64, device=X.device)
            self._keep += [X, ybar]
            self.outputs.append((y, xi))
            tr = int(tile_rows[p]) if tile_rows is not None else 0
            arr[p] = _CProblem(N, n, tr, px.value, py.value, y.data_ptr(), xi.data_ptr())
        self._arr = arr
        self._cp = self.params.to_c()
        nbytes = ctypes.c_size_t(0)
        _check(_lib.cr_batch_workspace_bytes(arr, self.P, ctypes.byref(self._cp), ctypes.byref(nbytes)))
        self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=problems[0][0].device)
        h = ctypes.c_void_p()
        _check(_lib.cr_batch_init(ctypes.byref(h), arr, self.P, ctypes.byref(self._cp),
                                  ctypes.c_void_p(self._ws.data_ptr()), int(nbytes.value), _stream()))
        self._h = h

    def run(self):
        """Solve every problem; returns ([(y, xi), ...], [Info, ...], wall seconds)."""
        infos = (_CInfo * self.P)()
        secs = ctypes.c_double(0.0)
        _check(_lib.cr_batch_run(self._h, infos, ctypes.byref(secs)), None, allow=(OK, NOT_CONVERGED))
        return self.outputs, [Info.from_c(infos[p]) for p in range(self.P)], float(secs.value)

    def start(self):
        """cr_batch_start: restart every problem (asynchronous)."""
        _check(_lib.cr_batch_start(self._h), None)

    def advance(self, max_replays: int) -> bool:
        """cr_batch_advance: at most max_replays graph replays; True while a problem still runs."""
        running = ctypes.c_int32(1)
        _check(_lib.cr_batch_advance(self._h, int(max_replays), ctypes.byref(running)), None)
        return bool(running.value)

    def finish(self):
        """cr_batch_finish: ([(y, xi), ...], [Info, ...], seconds since start)."""
        infos = (_CInfo * self.P)()
        secs = ctypes.c_double(0.0)
        _check(_lib.cr_batch_finish(self._h, infos, ctypes.byref(secs)), None, allow=(OK, NOT_CONVERGED))
        return self.outputs, [Info.from_c(infos[p]) for p in range(self.P)], float(secs.value)

    def time_pass(self, reps: int = 10) -> float:
        """Average device milliseconds of one batched pair pass over every problem."""
        out = ctypes.c_double(0.0)
        _check(_lib.cr_batch_time_pass(self._h, int(reps), ctypes.byref(out)), None)
        return float(out.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.cr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(problems, params: Optional[Params] = None):
    """cr_solve_batched: returns ([(y, xi), ...], [Info, ...]) for a list of (X, ybar) pairs."""
    b = Batch(problems, params)
    try:
        outs, infos, _ = b.run()
    finally:
        b.close()
    return outs, infos


# ---------------------------------------------------------------------------
# Differentiable form (cr_diff_*)
# ---------------------------------------------------------------------------

def diff_workspace_bytes(N: int, n: int, params: Params, checkpoint_every: int = 20) -> int:
    out = ctypes.c_size_t(0)
    cp = params.to_c()
    _check(_lib.cr_diff_workspace_bytes(int(N), int(n), ctypes.byref(cp), int(checkpoint_every), ctypes.byref(out)))
    return int(out.value)


class Diff:
    """The fixed-schedule ALCC/MAPG map (params.max_outer ALCC iterations of
    params.inner_iters MAPG steps) and its reverse pass, bound to (X, ybar).
    forward(y0, xi0) -> (y_K, xi_K, Info); backward(gy, gxi) -> (dX, dybar, dy0, dxi0),
    the gradients of <gy, y_K> + <gxi, xi_K> for the last forward."""

    def __init__(self, X, ybar, params: Params, checkpoint_every: int = 20):
        torch = _torch()
        self.N, self.n = int(X.shape[0]), int(X.shape[1])
        self.params = params
        self._X, self._ybar = X, ybar
        px = _dev_f64(X, (self.N, self.n), "X")
        py = _dev_f64(ybar, (self.N,), "ybar")
        nbytes = diff_workspace_bytes(self.N, self.n, params, checkpoint_every)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        self._cp = params.to_c()
        h = ctypes.c_void_p()
        _check(_lib.cr_diff_init(ctypes.byref(h), self.N, self.n, ctypes.byref(self._cp), int(checkpoint_every),
                                 px, py, ctypes.c_void_p(self._ws.data_ptr()), nbytes, _stream()))
        self._h = h

    def _new(self, *shape):
        torch = _torch()
        return torch.empty(*shape, dtype=torch.float64, device=self._X.device)

    def forward(self, y0=None, xi0=None):
        y, xi = self._new(self.N), self._new(self.N, self.n)
        py0 = _dev_f64(y0, (self.N,), "y0") if y0 is not None else None
        pxi0 = _dev_f64(xi0, (self.N, self.n), "xi0") if xi0 is not None else None
        self._start = (y0, xi0)
        ci = _CInfo()
        _check(_lib.cr_diff_forward(self._h, py0, pxi0, ctypes.c_void_p(y.data_ptr()),
                                    ctypes.c_void_p(xi.data_ptr()), ctypes.byref(ci)), None)
        return y, xi, Info.from_c(ci)

    def backward(self, gy, gxi=None):
        dX, dyb = self._new(self.N, self.n), self._new(self.N)
        dy0, dxi0 = self._new(self.N), self._new(self.N, self.n)
        pgxi = _dev_f64(gxi, (self.N, self.n), "gxi") if gxi is not None else None
        _check(_lib.cr_diff_backward(self._h, _dev_f64(gy, (self.N,), "gy"), pgxi,
                                     ctypes.c_void_p(dX.data_ptr()), ctypes.c_void_p(dyb.data_ptr()),
                                     ctypes.c_void_p(dy0.data_ptr()), ctypes.c_void_p(dxi0.data_ptr())), None)
        return dX, dyb, dy0, dxi0

    def time_adjoint_pass(self, reps: int = 20) -> float:
        """Average device milliseconds of one adjoint pair pass (HIP events),
        at the operands of the last backward."""
        out = ctypes.c_double(0.0)
        _check(_lib.cr_diff_time_adjoint_pass(self._h, int(reps), ctypes.byref(out)), None)
        return float(out.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.cr_diff_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _unrolled_function():
    torch = _torch()

    class UnrolledSolve(torch.autograd.Function):
        """torch.autograd.Function over cr_diff: forward runs the map, backward
        the library's reverse pass (checkpointed recomputation + adjoint kernels)."""

        @staticmethod
        def forward(ctx, X, ybar, y0, xi0, params, checkpoint_every):
            d = Diff(X.detach().contiguous(), ybar.detach().contiguous(), params, checkpoint_every)
            y, xi, info = d.forward(y0.detach().contiguous(), xi0.detach().contiguous())
            ctx.diff = d
            ctx.info = info
            return y, xi

        @staticmethod
        def backward(ctx, gy, gxi):
            d = ctx.diff
            if gy is None:
                gy = torch.zeros(d.N, dtype=torch.float64, device=d._X.device)
            dX, dyb, dy0, dxi0 = d.backward(gy.contiguous(), gxi.contiguous() if gxi is not None else None)
            return dX, dyb, dy0, dxi0, None, None

    return UnrolledSolve


_UNROLLED = None


def solve_unrolled(X, ybar, params: Params, y0=None, xi0=None, checkpoint_every: int = 20):
    """(y_K, xi_K) of the fixed-schedule map, differentiable with respect to X,
    ybar, y0 and xi0 through torch autograd.  y0 defaults to ybar itself (so its
    gradient reaches ybar), xi0 to zeros."""
    global _UNROLLED
    torch = _torch()
    if _UNROLLED is None:
        _UNROLLED = _unrolled_function()
    if y0 is None:
        y0 = ybar
    if xi0 is None:
        xi0 = torch.zeros(X.shape[0], X.shape[1], dtype=torch.float64, device=X.device)
    return _UNROLLED.apply(X, ybar, y0, xi0, params, int(checkpoint_every))


def pass_layout(N: int, n: int, params: Optional[Params] = None) -> dict:
    """The pair-pass launch layout cr_init would choose (host arithmetic only)."""
    out = (ctypes.c_int64 * 6)()
    cp = (params or Params()).to_c()
    _check(_lib.cr_pass_layout(int(N), int(n), ctypes.byref(cp), out))
    return dict(Nrow=out[0], ld=out[1], rows_per_chunk=out[2], chunks=out[3], strips=out[4], lazy=bool(out[5]))


def eval_workspace_bytes(N: int, n: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.cr_eval_workspace_bytes(int(N), int(n), ctypes.byref(out)))
    return int(out.value)


class Estimator:
    """The fitted estimator (X, y, xi) of Sec. I, evaluated at query points on the
    device: fhat(q) = max_l (y_l + xi_l^T (q - x_l)) and the maximising plane
    (``cr_eval``).  Keeps references to its inputs and a workspace tensor."""

    def __init__(self, X, y, xi):
        torch = _torch()
        self.N, self.n = int(X.shape[0]), int(X.shape[1])
        self._X = _dev_f64(X, (self.N, self.n), "X")
        self._y = _dev_f64(y, (self.N,), "y")
        self._xi = _dev_f64(xi, (self.N, self.n), "xi")
        self._keep = (X, y, xi)
        self._ws = torch.empty(eval_workspace_bytes(self.N, self.n), dtype=torch.uint8, device=X.device)

    def __call__(self, Q, with_arg: bool = True):
        """(fhat (M,) float64, arg (M,) int64 or None) at the rows of Q (M x n)."""
        torch = _torch()
        M = int(Q.shape[0])
        q = _dev_f64(Q, (M, self.n), "Q")
        f = torch.empty(M, dtype=torch.float64, device=Q.device)
        arg = torch.empty(M, dtype=torch.int64, device=Q.device) if with_arg else None
        _check(_lib.cr_eval(self._X, self._y, self._xi, self.N, self.n, q, M, ctypes.c_void_p(f.data_ptr()),
                            ctypes.c_void_p(arg.data_ptr()) if arg is not None else None,
                            ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(), _stream()))
        return f, arg


def evaluate(X, y, xi, Q, with_arg: bool = True):
    """One-shot ``Estimator(X, y, xi)(Q)``."""
    return Estimator(X, y, xi)(Q, with_arg)


def evaluate_noalloc(X, y, xi, Q, fhat, arg=None):
    """``cr_eval_noalloc``: the estimator at the rows of Q into the caller's
    fhat (M,) float64 and arg (M,) int64 (or None) tensors, with no device
    allocation by the library (a static 32 MiB scratch per GPU; calls that
    overlap on one GPU race)."""
    N, n = int(X.shape[0]), int(X.shape[1])
    M = int(Q.shape[0])
    _check(_lib.cr_eval_noalloc(_dev_f64(X, (N, n), "X"), _dev_f64(y, (N,), "y"), _dev_f64(xi, (N, n), "xi"),
                                N, n, _dev_f64(Q, (M, n), "Q"), M, _dev_f64(fhat, (M,), "fhat"),
                                ctypes.c_void_p(arg.data_ptr()) if arg is not None else None, _stream()))
    return fhat, arg



# ---------------------------------------------------------------------------
# P-APG on the partial dual (cr_papg)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PapgParams:
    """cr_papg_params: K index sets, iterations, step constant L (<= 0: the
    bound (2N + sigma_max(A2)^2 + 1)/gamma), radius of Q2 (inf: none), the
    data shift (< 0: the library's default), the method (PAPG_ACCELERATED,
    Fig. 2, or PAPG_GRADIENT, projected gradient ascent) and, with L <= 0,
    the number of power iterations that estimate sigma_max(C) (0: the bound)."""
    K: int = 2
    iters: int = 10
    L: float = 0.0
    B_theta: float = math.inf
    y_shift: float = -1.0
    method: int = 0
    power_iters: int = 0

    def to_c(self):
        return _CPapgParams(int(self.K), int(self.iters), float(self.L),
                            float(self.B_theta) if math.isfinite(self.B_theta) else 0.0, float(self.y_shift),
                            int(self.method), int(self.power_iters))


def papg_workspace_bytes(N: int, n: int, params: Params, pp: PapgParams) -> int:
    out = ctypes.c_size_t(0)
    cp, cpp = params.to_c(), pp.to_c()
    _check(_lib.cr_papg_workspace_bytes(int(N), int(n), ctypes.byref(cp), ctypes.byref(cpp), ctypes.byref(out)))
    return int(out.value)


def papg(X, ybar, pp: PapgParams, params: Optional[Params] = None, with_theta: bool = False):
    """cr_papg: returns (y, xi, info dict[, theta (N x N), theta_y (N)]).
    info["trace"] is an iters x 3 numpy array: ||theta^(1)_l||, the cross-block
    infeasibility at eta_l and theta^(2)_l^T C eta_l."""
    import numpy as np
    torch = _torch()
    params = params or Params()
    N, n = int(X.shape[0]), int(X.shape[1])
    px = _dev_f64(X, (N, n), "X")
    py = _dev_f64(ybar, (N,), "ybar")
    nbytes = papg_workspace_bytes(N, n, params, pp)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    y = torch.empty(N, dtype=torch.float64, device=X.device)
    xi = torch.empty(N, n, dtype=torch.float64, device=X.device)
    th = torch.empty(N, N, dtype=torch.float64, device=X.device) if with_theta else None
    thy = torch.empty(N, dtype=torch.float64, device=X.device) if with_theta else None
    cp, cpp, ci = params.to_c(), pp.to_c(), _CPapgInfo()
    trace = np.zeros((int(pp.iters), 3), dtype=np.float64)
    _check(_lib.cr_papg(px, py, N, n, ctypes.byref(cp), ctypes.byref(cpp), ctypes.c_void_p(y.data_ptr()),
                        ctypes.c_void_p(xi.data_ptr()), ctypes.c_void_p(th.data_ptr()) if th is not None else None,
                        ctypes.c_void_p(thy.data_ptr()) if thy is not None else None,
                        trace.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(ws.data_ptr()),
                        nbytes, ctypes.byref(ci), _stream()))
    info = {k: getattr(ci, k) for k, _ in _CPapgInfo._fields_}
    info["trace"] = trace
    if with_theta:
        return y, xi, info, th, thy
    return y, xi, info
