"""Independent references for the convex-regression QP, used to pin the oracle.

Nothing here calls the oracle or the HIP library.  The constraint matrices are
built row by row from the constraint list of eq. "original"
(y_i >= y_j + xi_j^T (x_i - x_j) for every ordered pair i != j), and the
regularized QP (eq. "regularize") is solved through its Lagrange dual, which is
a nonnegative least-squares problem (scipy's Lawson-Hanson ``nnls``):

    min 1/2 (z - z0)^T H (z - z0)  s.t.  A z >= 0,   z = (y, xi), z0 = (ybar, 0),
    H = diag(I_N, gamma I_Nn).
    Stationarity gives z = z0 + H^{-1} A^T lam; the dual is
    min_{lam >= 0} 1/2 || H^{-1/2} A^T lam + H^{1/2} z0 ||^2.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import nnls


def pairs(N):
    return [(i, j) for i in range(N) for j in range(N) if i != j]


def explicit_A(X):
    """(A1, A2) with one row per ordered pair (i, j), i != j, in row-major pair order."""
    X = np.asarray(X, dtype=np.float64)
    N, n = X.shape
    P = pairs(N)
    A1 = np.zeros((len(P), N))
    A2 = np.zeros((len(P), N * n))
    for r, (i, j) in enumerate(P):
        A1[r, i] += 1.0
        A1[r, j] -= 1.0
        A2[r, j * n:(j + 1) * n] = -(X[i] - X[j])
    return A1, A2


def pairs_to_matrix(v, N):
    """Scatter a per-pair vector (row-major pair order) into an N x N array with 0 diagonal."""
    M = np.zeros((N, N))
    for r, (i, j) in enumerate(pairs(N)):
        M[i, j] = v[r]
    return M


def matrix_to_pairs(M):
    N = M.shape[0]
    return np.array([M[i, j] for (i, j) in pairs(N)])


def solve_qp_nnls(X, ybar, gamma):
    """Exact minimizer (y, xi) of eq. "regularize" and a multiplier lam >= 0 (per pair)."""
    X = np.asarray(X, dtype=np.float64)
    ybar = np.asarray(ybar, dtype=np.float64)
    N, n = X.shape
    A1, A2 = explicit_A(X)
    A = np.hstack([A1, A2])
    h = np.concatenate([np.ones(N), np.full(N * n, gamma)])
    z0 = np.concatenate([ybar, np.zeros(N * n)])
    M = (A / np.sqrt(h)[None, :]).T           # H^{-1/2} A^T
    b = -np.sqrt(h) * z0                       # -H^{1/2} z0
    lam, _ = nnls(M, b, maxiter=50 * M.shape[1])
    z = z0 + (A.T @ lam) / h
    return z[:N], z[N:].reshape(N, n), lam


def solve_qp_active_set(X, ybar, gamma):
    """Brute force over every active set (tiny N only): solve the equality-constrained
    KKT system for each subset and keep the primal- and dual-feasible solution."""
    X = np.asarray(X, dtype=np.float64)
    ybar = np.asarray(ybar, dtype=np.float64)
    N, n = X.shape
    A1, A2 = explicit_A(X)
    A = np.hstack([A1, A2])
    m, d = A.shape
    H = np.diag(np.concatenate([np.ones(N), np.full(N * n, gamma)]))
    q = -np.concatenate([ybar, np.zeros(N * n)])
    best = None
    for size in range(0, m + 1):
        for S in itertools.combinations(range(m), size):
            S = list(S)
            AS = A[S]
            K = np.block([[H, -AS.T], [AS, np.zeros((len(S), len(S)))]])
            rhs = np.concatenate([-q, np.zeros(len(S))])
            sol, *_ = np.linalg.lstsq(K, rhs, rcond=None)
            if np.linalg.norm(K @ sol - rhs) > 1e-9:
                continue
            z, lam = sol[:d], sol[d:]
            if np.all(A @ z >= -1e-10) and np.all(lam >= -1e-10):
                return z[:N], z[N:].reshape(N, n)
    return best


def convex_1d_ls(x, ybar):
    """n = 1 least-squares convex fit without regularization: with x sorted, convexity of
    the fitted values is nondecreasing consecutive slopes (N-2 constraints).  Solved via
    the NNLS dual of min 1/2||y - ybar||^2 s.t. D y >= 0."""
    order = np.argsort(x)
    xs, ys = np.asarray(x, float)[order], np.asarray(ybar, float)[order]
    N = len(xs)
    D = np.zeros((N - 2, N))
    for k in range(N - 2):
        h0, h1 = xs[k + 1] - xs[k], xs[k + 2] - xs[k + 1]
        D[k, k] = 1.0 / h0
        D[k, k + 1] = -1.0 / h0 - 1.0 / h1
        D[k, k + 2] = 1.0 / h1
    lam, _ = nnls(D.T, -ys, maxiter=50 * N)
    y = ys + D.T @ lam
    out = np.empty(N)
    out[order] = y
    return out
