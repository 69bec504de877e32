"""FP64 CPU oracle of the ALCC/MAPG iteration for least-squares convex regression.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check and
by the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library; the two meet only in the seeded inputs of ``synth``.

The O(N^2) constraint operators A1, A2, A1^T, A2^T are plain C loops
(``cr_oracle.c``); everything else is numpy float64, written in the order and
notation of the paper (Aybat & Wang, "A Parallel Method for Large Scale Convex
Regression Problems"):

* problem: eq. "regularize" (Sec. II-C), min 1/2||y-ybar||^2 + gamma/2||xi||^2
  s.t. A1 y + A2 xi >= 0;
* ALCC: the augmented-Lagrangian outer loop of Fig. 3 (Sec. II-E);
* MAPG: the block-wise accelerated projected gradient inner loop of Fig. 4;
* P_k, h_k and their gradients: eq. "subproblem" and the gradient formulas
  that follow it (Sec. II-E);
* bounding balls Q_y, Q_xi from a feasible point: first paragraph of Sec. II-E.

Readings of passages the paper leaves open are listed in the design notes and
repeated next to the code that takes them.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cr_oracle.c")
_LIB = os.path.join(_HERE, "libcr_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C operators with gcc (-O2 -fopenmp).  Returns the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.cro_forward.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp]
        lib.cro_forward.restype = None
        lib.cro_adjoint.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp]
        lib.cro_adjoint.restype = None
        lib.cro_pair_residual.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int64, ctypes.c_int64]
        lib.cro_pair_residual.restype = ctypes.c_double
        lib.cro_adjoint_one.argtypes = [ctypes.c_int64, ctypes.c_int, dp, ctypes.c_int64,
                                        dp, dp, dp, dp]
        lib.cro_adjoint_one.restype = None
        lib.cro_residual_row_col.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, dp, ctypes.c_int64, dp, dp]
        lib.cro_residual_row_col.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Constraint operators (eq. "original_compact"; matrix-free, Sec. II-E)
# ---------------------------------------------------------------------------

def forward(X, y, xi) -> np.ndarray:
    """R = A1 y + A2 xi as an N x N array, R[i, j] = y_i - y_j - xi_j^T (x_i - x_j); R[i, i] = 0."""
    X, y, xi = _f64(X), _f64(y), _f64(xi)
    N, n = X.shape
    R = np.empty((N, N), dtype=np.float64)
    _load().cro_forward(N, n, _p(X), _p(y), _p(xi.reshape(N, n)), _p(R))
    return R


def adjoint(X, Z):
    """(A1^T z, A2^T z) for a pair array Z[i, j] (diagonal ignored); A2^T z is N x n."""
    X, Z = _f64(X), _f64(Z)
    N, n = X.shape
    u = np.empty(N)
    v = np.empty((N, n))
    _load().cro_adjoint(N, n, _p(X), _p(Z), _p(u), _p(v))
    return u, v


def pair_residual(X, y, xi, i: int, j: int) -> float:
    X, y, xi = _f64(X), _f64(y), _f64(xi)
    return float(_load().cro_pair_residual(X.shape[1], _p(X), _p(y), _p(xi), i, j))


def adjoint_one(X, m: int, zrow, zcol):
    """Entry m of A1^T z and block m of A2^T z from row m (z_mj) and column m (z_im) of z."""
    X, zrow, zcol = _f64(X), _f64(zrow), _f64(zcol)
    N, n = X.shape
    u = np.empty(1)
    v = np.empty(n)
    _load().cro_adjoint_one(N, n, _p(X), m, _p(zrow), _p(zcol), _p(u), _p(v))
    return float(u[0]), v


def residual_row_col(X, y, xi, m: int):
    """(row m, column m) of R = A1 y + A2 xi (pairs (m, j) and (i, m)); entry m is 0."""
    X, y, xi = _f64(X), _f64(y), _f64(xi)
    N, n = X.shape
    row, col = np.empty(N), np.empty(N)
    _load().cro_residual_row_col(N, n, _p(X), _p(y), _p(xi.reshape(N, n)), m, _p(row), _p(col))
    return row, col


def neg_part(v):
    """(v)_- := max(-v, 0), taken elementwise (the paper's notation, Sec. II-D)."""
    return np.maximum(-v, 0.0)


# ---------------------------------------------------------------------------
# Problem constants
# ---------------------------------------------------------------------------

def sigma2_A1(N: int) -> float:
    """sigma_max(A1)^2.  A1^T A1 = 2(N I - 1 1^T) (every pair contributes e_i - e_j
    twice, once per order), whose largest eigenvalue is 2N."""
    return 2.0 * N


def sigma2_A2(X) -> float:
    """sigma_max(A2)^2.  Row (i,j) of A2 touches only block j, so A2^T A2 is block
    diagonal with blocks S_j = sum_{i != j} (x_i - x_j)(x_i - x_j)^T; the answer is
    max_j lambda_max(S_j) (numpy eigvalsh per block)."""
    X = _f64(X)
    N, n = X.shape
    best = 0.0
    step = max(1, 4_000_000 // max(1, N * n))
    for j0 in range(0, N, step):
        D = X[None, :, :] - X[j0:j0 + step, None, :]          # (b, N, n): x_i - x_j
        S = np.einsum("bik,bil->bkl", D, D)
        best = max(best, float(np.linalg.eigvalsh(S)[:, -1].max()))
    return best


def affine_fit(X, ybar, gamma: float):
    """Feasible starting point and bounding radii (Sec. II-E, first paragraph).

    The least-squares affine fit yhat = X a + b with xi_l = a for every l has
    A1 yhat + A2 xihat = 0, so it is feasible.  The slope a is the
    minimum-norm least-squares solution of the centred problem (numpy lstsq on
    X - mean(X) against ybar - mean(ybar)) and b = mean(ybar) - mean(X)^T a;
    when the fit is not unique (N <= n, or collinear points) this picks the
    shortest slope, the intercept being free.  Then
    Bbar = sqrt(||yhat - ybar||^2 + gamma ||xihat||^2), Bbar_y = Bbar and
    Bbar_xi = Bbar / sqrt(gamma).
    """
    X, ybar = _f64(X), _f64(ybar)
    N, n = X.shape
    xm = X.mean(axis=0)
    ym = float(ybar.mean())
    a, *_ = np.linalg.lstsq(X - xm, ybar - ym, rcond=None)
    b = ym - float(xm @ a)
    yhat = X @ a + b
    xihat = np.tile(a, (N, 1))
    Bbar = math.sqrt(float(np.sum((yhat - ybar) ** 2)) + gamma * float(np.sum(xihat ** 2)))
    return yhat, xihat, Bbar, Bbar, Bbar / math.sqrt(gamma)


# ---------------------------------------------------------------------------
# ALCC subproblem P_k (eq. "subproblem") and its gradient
# ---------------------------------------------------------------------------

def _shifted(xi, shift):
    """The slopes that enter the constraints: xi itself, or xi + shift when the
    problem is posed in shifted coordinates (see `alcc`)."""
    return xi if shift is None else xi + shift


def penalty_weights(X, y, xi, theta, shift=None):
    """w = (A1 y + A2 (xi + shift) - theta)_- for every pair, diagonal 0."""
    R = forward(X, y, _shifted(xi, shift))
    W = neg_part(R - theta)
    np.fill_diagonal(W, 0.0)
    return W


def grad_P(X, ybar, gamma, mu, theta, y, xi, shift=None):
    """(grad_y P_k, grad_xi P_k) at (y, xi):
    grad_y  = (y - ybar)/mu      - A1^T (A1 y + A2 xi - theta)_-
    grad_xi = (gamma/mu) xi      - A2^T (A1 y + A2 xi - theta)_-
    (with xi + shift in the constraints when a shift is given)."""
    W = penalty_weights(X, y, xi, theta, shift)
    u, v = adjoint(X, W)
    return (y - ybar) / mu - u, (gamma / mu) * xi - v


def P_value(X, ybar, gamma, mu, theta, y, xi, shift=None) -> float:
    W = penalty_weights(X, y, xi, theta, shift)
    return (0.5 / mu) * float(np.sum((y - ybar) ** 2)) + (0.5 * gamma / mu) * float(np.sum(xi ** 2)) \
        + 0.5 * float(np.sum(W * W))


def project_ball(v, center, radius):
    """Euclidean projection onto {z : ||z - center||_2 <= radius}."""
    d = v - center
    nrm = float(np.sqrt(np.sum(d * d)))
    if nrm <= radius:
        return v.copy()
    return center + d * (radius / nrm)


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    """ALCC/MAPG parameters.  The paper gives no values for any of them; the
    defaults are this implementation's readings (see the design notes)."""
    gamma: float = 1e-3          # Tikhonov weight (eq. "regularize")
    mu1: float = 0.0             # <= 0: 1/sigma_max(A1)^2 = 1/(2N)
    c: float = 4.0               # mu_{k+1} = c mu_k, c > 1
    kappa: float = 0.1           # kappa > 0 in the tau/alpha decay
    tau1: float = 1.0            # first subproblem tolerance
    alpha_y1: float = 0.0        # <= 0: 1e-2 * Bbar_y
    alpha_xi1: float = 0.0       # <= 0: 1e-2 * Bbar
    step_scale: float = 0.5      # MAPG step = step_scale / L (reading of Lemma 3)
    kkt_tol: float = 1e-4
    max_outer: int = 30
    inner_iters: int = 0         # > 0: fixed schedule, exactly this many MAPG steps per outer
    max_inner: int = 20000       # cap on l_max when the schedule is adaptive
    Ly_override: float = 0.0
    Lxi_override: float = 0.0
    By_override: float = 0.0
    Bxi_override: float = 0.0


def resolve(params: Params, N: int, Bbar: float, gamma: float):
    mu1 = params.mu1 if params.mu1 > 0 else 1.0 / (2.0 * N)
    ay = params.alpha_y1 if params.alpha_y1 > 0 else 1e-2 * Bbar
    axi = params.alpha_xi1 if params.alpha_xi1 > 0 else 1e-2 * Bbar
    return mu1, ay, axi


# ---------------------------------------------------------------------------
# MAPG (Fig. 4) and ALCC (Fig. 3)
# ---------------------------------------------------------------------------

def mapg(X, ybar, gamma, mu, theta, Ly, Lxi, y0, xi0, By, Bxi, alpha_y, alpha_xi,
         lmax, step_scale=0.5, adaptive=True, trace=None, shift=None):
    """MAPG (Fig. 4): accelerated projected gradient on P_k over Q_y x Q_xi.

    Each step takes a projected gradient step from the extrapolated point,
    one block at a time (y with step_scale/Ly onto the ball around ybar, xi
    with step_scale/Lxi onto the ball around 0), then extrapolates from the
    new iterate along its change since the previous iterate with the weight
    (t - 1)/t+ of the accelerated method, where t starts at 1 and
    t+ = (1 + sqrt(1 + 4 t^2))/2.  The run begins at (y0, xi0) with no
    momentum and returns the last projected iterate: after the first step
    whose two block moves are both within alpha (adaptive) or after lmax
    steps.  A list passed as `trace` receives (l, ||y1 - y2||, ||xi1 - xi2||,
    t_l, weight_l) per step.  Returns (y, xi, steps)."""
    y1_prev, xi1_prev = y0.copy(), xi0.copy()
    y2, xi2 = y0.copy(), xi0.copy()
    t = 1.0
    zero = np.zeros_like(xi0)
    for l in range(1, lmax + 1):
        gy, gxi = grad_P(X, ybar, gamma, mu, theta, y2, xi2, shift)
        y1 = project_ball(y2 - (step_scale / Ly) * gy, ybar, By)
        xi1 = project_ball(xi2 - (step_scale / Lxi) * gxi, zero, Bxi)
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_next
        dy = float(np.sqrt(np.sum((y1 - y2) ** 2)))
        dxi = float(np.sqrt(np.sum((xi1 - xi2) ** 2)))
        if trace is not None:
            trace.append((l, dy, dxi, t, beta))
        y2 = y1 + beta * (y1 - y1_prev)
        xi2 = xi1 + beta * (xi1 - xi1_prev)
        y1_prev, xi1_prev = y1, xi1
        t = t_next
        if adaptive and dy <= alpha_y and dxi <= alpha_xi:
            return y1, xi1, l
    return y1_prev, xi1_prev, lmax


def kkt_measures(X, ybar, gamma, y, xi, lam, shift=None):
    """First-order optimality residuals of eq. "regularize" at (y, xi) with a
    multiplier estimate lam >= 0 (one entry per pair):
      stationarity  y - ybar - A1^T lam,  gamma xi - A2^T lam   (inf-norms)
      infeasibility max_ij (r_ij)_-  with r = A1 y + A2 xi
      complementarity max_ij lam_ij |r_ij|
    and the combined KKT = max of the four / (1 + ||ybar||_inf).
    Also the paper's normalized infeasibility ||(r)_-||_2 / sqrt(N^2-N) and
    normalized gap lam^T r / (N^2-N) (Sec. III)."""
    N = X.shape[0]
    R = forward(X, y, _shifted(xi, shift))
    u, v = adjoint(X, lam)
    st_y = float(np.max(np.abs(y - ybar - u)))
    st_xi = float(np.max(np.abs(gamma * xi - v)))
    rneg = neg_part(R)
    np.fill_diagonal(rneg, 0.0)
    infeas = float(rneg.max())
    LR = lam * R
    np.fill_diagonal(LR, 0.0)
    compl = float(np.max(np.abs(LR)))
    scale = 1.0 + float(np.max(np.abs(ybar)))
    return dict(stat_y=st_y, stat_xi=st_xi, infeas=infeas, compl=compl,
                kkt=max(st_y, st_xi, infeas, compl) / scale,
                infeas_norm=float(np.sqrt(np.sum(rneg * rneg))) / math.sqrt(N * N - N),
                gap_norm=float(np.sum(LR)) / (N * N - N),
                objective=0.5 * float(np.sum((y - ybar) ** 2)))


class _Schedule:
    """The scalars ALCC carries from one outer iteration to the next (Fig. 3):
    the penalty parameter mu_k, the subproblem tolerance tau_k and the two
    MAPG stopping thresholds alpha^y_k, alpha^xi_k."""

    def __init__(self, p: Params, N: int, Bbar: float, s2A1: float, s2A2: float, By: float, Bxi: float):
        self.p, self.s2A1, self.s2A2, self.By, self.Bxi = p, s2A1, s2A2, By, Bxi
        self.mu, self.ay, self.axi = resolve(p, N, Bbar, p.gamma)
        self.tau = p.tau1

    def constants(self):
        """Block Lipschitz constants of grad P_k and the MAPG step budget l_max:
        ceil(4 sqrt((L^y By^2 + L^xi Bxi^2)/tau_k)) clipped to [1, max_inner],
        or the fixed count of a fixed schedule."""
        p = self.p
        Ly = p.Ly_override if p.Ly_override > 0 else 1.0 / self.mu + self.s2A1
        Lxi = p.Lxi_override if p.Lxi_override > 0 else p.gamma / self.mu + self.s2A2
        if p.inner_iters > 0:
            return Ly, Lxi, p.inner_iters
        lmax = int(math.ceil(4.0 * math.sqrt((Ly * self.By ** 2 + Lxi * self.Bxi ** 2) / self.tau)))
        return Ly, Lxi, max(1, min(lmax, p.max_inner))

    def advance(self, k: int):
        """After outer iteration k: mu grows by c; tau and both alpha thresholds
        shrink by (c k^{1+kappa})^2."""
        p = self.p
        decay = (p.c * k ** (1.0 + p.kappa)) ** 2
        self.mu, self.tau = p.c * self.mu, self.tau / decay
        self.ay, self.axi = self.ay / decay, self.axi / decay


def multiplier_step(X, y, xi_c, theta, ratio):
    """The ALCC multiplier update at the MAPG output: theta_{k+1} =
    (mu_k/mu_{k+1}) (A1 y + A2 xi_c - theta_k)_- with ratio = mu_k/mu_{k+1};
    xi_c are the slopes that enter the constraints.  Diagonal 0."""
    Wk = neg_part(forward(X, y, xi_c) - theta)
    np.fill_diagonal(Wk, 0.0)
    return ratio * Wk


@dataclasses.dataclass
class Result:
    y: np.ndarray
    xi: np.ndarray
    theta: np.ndarray
    outer: int
    inner_total: int
    inner_per_outer: list
    history: list
    converged: bool


def alcc(X, ybar, params: Optional[Params] = None, y0=None, xi0=None,
         record_kkt: bool = True, xi_shift=None, mapg_traces: Optional[list] = None) -> Result:
    """ALCC (Fig. 3) on eq. "regularize", with MAPG (Fig. 4) as the inner solver.

    The multipliers start at zero and the iterate at the affine fit.  Each
    outer iteration minimises the penalty function P_k of eq. "subproblem"
    approximately with MAPG, warm-started at the previous outer iterate, with
    block Lipschitz constants 1/mu_k + sigma_max(A1)^2 and
    gamma/mu_k + sigma_max(A2)^2 and a step budget that grows with the square
    root of the constants over the tolerance tau_k (a fixed count instead when
    params.inner_iters > 0; capped by params.max_inner).  The multipliers are
    then moved to (mu_k/mu_{k+1}) (r - theta_k)_- at the MAPG output, the
    penalty weight grows by c, and tau and both alpha thresholds shrink by
    (c k^{1+kappa})^2.  The multiplier estimate of outer iteration k is
    mu_{k+1} theta_{k+1}; the run stops after the first outer iteration whose
    KKT measure is within params.kkt_tol (adaptive schedule only) or after
    params.max_outer.

    xi_shift (N x n, optional) poses the problem in shifted slopes: with
    xi = xi' + shift the run solves
      min 1/2||y - ybar||^2 + gamma/2||xi'||^2  s.t.  A1 y + A2 (xi' + shift) >= 0,
    i.e. eq. "regularize" with the slope term gamma/2||xi - shift||^2, the form
    of each block subproblem of P-APG step 1 (Fig. 2, eq. "g_gamma").  The run
    returns xi'.  The affine fit stays the start; in shifted slopes it is
    (yhat, a - shift), feasible for the shifted constraints, and Bbar is the
    objective there: Bbar^2 = ||yhat - ybar||^2 + gamma ||a - shift||^2.

    A list passed as `mapg_traces` receives, per outer iteration, the
    thresholds (alpha_y, alpha_xi) and the MAPG trace (see `mapg`)."""
    p = params or Params()
    X, ybar = _f64(X), _f64(ybar)
    N, n = X.shape
    gamma = p.gamma
    yhat, xihat, Bbar, By, Bxi = affine_fit(X, ybar, gamma)
    shift = None
    if xi_shift is not None:
        shift = _f64(xi_shift).reshape(N, n)
        xihat = xihat - shift
        Bbar = math.sqrt(float(np.sum((yhat - ybar) ** 2)) + gamma * float(np.sum(xihat ** 2)))
        By, Bxi = Bbar, Bbar / math.sqrt(gamma)
    if p.By_override > 0:
        By = p.By_override
    if p.Bxi_override > 0:
        Bxi = p.Bxi_override
    sched = _Schedule(p, N, Bbar, sigma2_A1(N), sigma2_A2(X), By, Bxi)
    y = yhat if y0 is None else _f64(y0).copy()
    xi = xihat if xi0 is None else _f64(xi0).reshape(N, n).copy()
    theta = np.zeros((N, N))
    fixed = p.inner_iters > 0
    inner_list, hist = [], []
    converged = False
    k = 0
    for k in range(1, p.max_outer + 1):
        Ly, Lxi, lmax = sched.constants()
        mu = sched.mu
        tr = None
        if mapg_traces is not None:
            tr = []
            mapg_traces.append((sched.ay, sched.axi, tr))
        y, xi, used = mapg(X, ybar, gamma, mu, theta, Ly, Lxi, y, xi, By, Bxi, sched.ay, sched.axi,
                           lmax, p.step_scale, adaptive=not fixed, trace=tr, shift=shift)
        inner_list.append(used)
        mu_next = p.c * mu
        theta = multiplier_step(X, y, _shifted(xi, shift), theta, mu / mu_next)
        if record_kkt:
            m = kkt_measures(X, ybar, gamma, y, xi, mu_next * theta, shift)
            m.update(k=k, inner=used, mu=mu)
            hist.append(m)
            converged = not fixed and m["kkt"] <= p.kkt_tol
        sched.advance(k)
        if converged:
            break
    return Result(y, xi, theta, k, int(sum(inner_list)), inner_list, hist, converged)
