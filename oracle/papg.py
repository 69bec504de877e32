"""FP64 CPU oracle of P-APG, the parallel accelerated proximal gradient method
on the partial dual (Aybat & Wang, Sec. II-B to II-D, Fig. 2).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's
CPU-baseline leg, never by the product path; it shares no code with the HIP
library.

Notation.  The N points are split into K contiguous index sets C_i of
Nbar = N / K points each (Sec. II-B).  Pair (i, j) is a cross-block pair when
i and j lie in different sets.  The method poses eq. "omega_primal":

    min 1/2 ||y - ybar||^2 + gamma/2 ||xi||^2   over eta = (y, xi) in Q1,
    s.t.  C eta >= 0,   C = [A3 A4; I 0]   (eq. "C"),

where Q1 holds the within-block constraints and A3, A4 are the cross-block
rows of A1, A2; the rows I 0 ask y >= 0, which holds at the solution once the
observations are shifted up (the shift is `y_shift` below).  Its dual
(eq. "lambda_dual") maximises g_gamma over Q2 = {theta >= 0, ||theta||_2 <= B_theta},
and by eq. "g_gamma" and eq. "dual gradient",

    g_gamma(theta) = min_{eta in Q1} 1/2||y - ybar||^2 + gamma/2||xi||^2 - theta^T C eta,
    grad g_gamma(theta) = -C eta(theta),  Lipschitz with L_g = sigma_max(C)^2 / gamma.

Storage: the cross-block multipliers are the off-diagonal blocks of an N x N
array Th (Th[i, j] for pair (i, j), zero inside the diagonal blocks), the
multipliers of y >= 0 a vector th_y of N entries.

Step 1 of Fig. 2 separates into K block problems (eq. "subgradient_split").
With u = A3^T Th + th_y and v = A4^T Th, completing the squares gives, up to
a constant, 1/2||y - (ybar + u)||^2 + gamma/2||xi - v/gamma||^2 over Q1, so
block i is eq. "regularize" on its own points with data ybar_i + u_i and the
slope term centred at c_i = v_i / gamma.  The oracle's ALCC solves it in
shifted slopes (`oracle.alcc(..., xi_shift=c_i)`), and xi_i = xi'_i + c_i.

Readings (listed in the design notes):
* L: the bound (2N + sigma_max(A2)^2 + 1) / gamma >= L_g unless given, from
  ||C||^2 <= ||A3||^2 + ||A4||^2 + 1, ||A3||^2 <= ||A1||^2 = 2N and
  ||A4||^2 <= ||A2||^2.
* B_theta: +inf unless given (Q2 is then the nonnegative orthant);
  projection onto Q2 = clip at zero, then scale into the ball (the ball is
  centred at the origin and the orthant is a cone, so this is exact).
* y_shift: max(0, max(ybar) - 2 min(ybar)) unless given, which puts the
  shifted data at or above the data range; the results are shifted back.
* Step 1 starts every block's ALCC from its affine fit with zero within-block
  multipliers (no warm start), and returns eta_l computed at theta^(2)_l.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

import oracle as _o


def block_of(N: int, K: int) -> np.ndarray:
    """Block index of every point: C_i = {(i-1) Nbar + 1, ..., i Nbar} (Sec. II-B)."""
    if K < 1 or N % K != 0:
        raise ValueError("N must be a multiple of K")
    return np.arange(N) // (N // K)


def cross_mask(N: int, K: int) -> np.ndarray:
    """True for the cross-block pairs (i, j): i, j in different index sets."""
    b = block_of(N, K)
    return b[:, None] != b[None, :]


def C_apply(X, y, xi, K: int):
    """C eta = (A3 y + A4 xi, y): the cross-block residuals r_ij as an N x N
    array (zero inside the diagonal blocks) and the rows I y."""
    X, y, xi = _o._f64(X), _o._f64(y), _o._f64(xi)
    R = _o.forward(X, y, xi)
    R[~cross_mask(X.shape[0], K)] = 0.0
    return R, y.copy()


def C_adjoint(X, Th, th_y, K: int):
    """C^T (Th, th_y) = (A3^T Th + th_y, A4^T Th)."""
    X = _o._f64(X)
    T = np.where(cross_mask(X.shape[0], K), _o._f64(Th), 0.0)
    u, v = _o.adjoint(X, T)
    return u + _o._f64(th_y), v


def lipschitz_bound(X, gamma: float) -> float:
    """(2N + sigma_max(A2)^2 + 1) / gamma, an upper bound of L_g (eq. "lischitz")."""
    X = _o._f64(X)
    return (_o.sigma2_A1(X.shape[0]) + _o.sigma2_A2(X) + 1.0) / gamma


def default_y_shift(ybar) -> float:
    ybar = _o._f64(ybar)
    return max(0.0, float(ybar.max()) - 2.0 * float(ybar.min()))


def project_Q2(Th, th_y, B_theta: float):
    """Euclidean projection onto Q2 = {theta >= 0, ||theta||_2 <= B_theta}
    (the cross entries and the y >= 0 entries form one vector theta)."""
    P = np.maximum(Th, 0.0)
    p = np.maximum(th_y, 0.0)
    if math.isfinite(B_theta):
        nrm = math.sqrt(float(np.sum(P * P)) + float(np.sum(p * p)))
        if nrm > B_theta:
            s = B_theta / nrm
            P, p = P * s, p * s
    return P, p


def step1(X, ybar_s, gamma: float, K: int, Th, th_y, params: _o.Params):
    """eta(theta) of eq. "g_gamma": K block problems solved by ALCC in shifted
    slopes.  Returns (y, xi, u, v) with u = A3^T Th + th_y, v = A4^T Th."""
    X, ybar_s = _o._f64(X), _o._f64(ybar_s)
    N, n = X.shape
    u, v = C_adjoint(X, Th, th_y, K)
    yb = ybar_s + u
    c = v / gamma
    y = np.empty(N)
    xi = np.empty((N, n))
    p = dataclasses.replace(params, gamma=gamma)
    nb = N // K
    for i in range(K):
        s = slice(i * nb, (i + 1) * nb)
        r = _o.alcc(X[s], yb[s], p, xi_shift=c[s], record_kkt=False)
        y[s] = r.y
        xi[s] = r.xi + c[s]
    return y, xi, u, v


def lagrangian(X, ybar_s, gamma, K, Th, th_y, y, xi) -> float:
    """1/2||y - ybar||^2 + gamma/2||xi||^2 - theta^T C eta (the function minimised in eq. "g_gamma")."""
    R, yy = C_apply(X, y, xi, K)
    return (0.5 * float(np.sum((y - ybar_s) ** 2)) + 0.5 * gamma * float(np.sum(xi * xi))
            - float(np.sum(np.where(cross_mask(X.shape[0], K), Th, 0.0) * R)) - float(np.dot(th_y, yy)))


@dataclasses.dataclass
class PapgResult:
    y: np.ndarray          # y of the last step 1, shifted back by y_shift
    xi: np.ndarray
    Th: np.ndarray         # theta^(1) of the last iteration (cross entries)
    th_y: np.ndarray
    L: float
    y_shift: float
    trace: list            # per iteration: dict(l, g (Lagrangian at eta_l), infeas, ...)


def papg(X, ybar, K: int, gamma: float, iters: int, params: Optional[_o.Params] = None,
         L: float = 0.0, B_theta: float = math.inf, y_shift: Optional[float] = None,
         record: bool = False, accelerate: bool = True) -> PapgResult:
    """P-APG (Fig. 2) for `iters` iterations: accelerated projected gradient
    ascent on the dual of eq. "omega_primal".

    The multipliers start at zero with no momentum.  Each iteration solves the
    K block problems at the extrapolated multipliers theta^(2) (step1, which
    gives eta and hence the dual gradient -C eta), takes a projected step
    theta^(1) = Pi_Q2(theta^(2) - C eta / L), and extrapolates the next
    theta^(2) from theta^(1) along its change since the previous iteration
    with the accelerated weight (t - 1)/t+, t+ = (1 + sqrt(1 + 4 t^2))/2,
    t starting at 1.  `params` is the block ALCC's schedule (its gamma is
    replaced by `gamma`).  With accelerate=False the weight is 0:
    projected gradient ascent on the same dual, the method P-APG is compared
    with in Sec. III.

    With record=True every iteration appends theta_norm = ||theta^(1)_l||,
    infeas_cross = ||(A3 y + A4 xi)_-||_2 at eta_l, gap = theta^(2)_l^T C eta_l
    (the objective of eq. "omega_primal" at eta_l minus the Lagrangian there,
    i.e. minus g_gamma(theta^(2)_l) when eta_l is exact), the Lagrangian g,
    the all-pairs infeasibility and the primal objective."""
    X, ybar = _o._f64(X), _o._f64(ybar)
    N, n = X.shape
    block_of(N, K)
    p = params or _o.Params()
    Lg = L if L > 0 else lipschitz_bound(X, gamma)
    s = default_y_shift(ybar) if y_shift is None else float(y_shift)
    ybs = ybar + s
    mask = cross_mask(N, K)
    T1p = np.zeros((N, N)); t1p = np.zeros(N)        # theta^(1)_{l-1}
    T2 = np.zeros((N, N)); t2 = np.zeros(N)          # theta^(2)_l
    t = 1.0
    trace = []
    y = xi = None
    for l in range(1, iters + 1):
        y, xi, u, v = step1(X, ybs, gamma, K, T2, t2, p)
        R, yy = C_apply(X, y, xi, K)
        T1, t1 = project_Q2(np.where(mask, T2 - R / Lg, 0.0), t2 - yy / Lg, B_theta)
        if record:
            Rall = _o.forward(X, y, xi)
            neg = _o.neg_part(Rall)
            np.fill_diagonal(neg, 0.0)
            trace.append(dict(l=l, g=lagrangian(X, ybs, gamma, K, T2, t2, y, xi),
                              theta_norm=math.sqrt(float(np.sum(T1 * T1)) + float(np.sum(t1 * t1))),
                              gap=float(np.sum(np.where(mask, T2, 0.0) * R)) + float(np.dot(t2, yy)),
                              infeas=float(np.sqrt(np.sum(neg * neg))),
                              infeas_cross=float(np.sqrt(np.sum(np.where(mask, neg, 0.0) ** 2))),
                              primal=0.5 * float(np.sum((y - ybs) ** 2)) + 0.5 * gamma * float(np.sum(xi * xi))))
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_next if accelerate else 0.0
        T2 = T1 + beta * (T1 - T1p)
        t2 = t1 + beta * (t1 - t1p)
        T1p, t1p = T1, t1
        t = t_next
    return PapgResult(y - s, xi, T1p, t1p, Lg, s, trace)
