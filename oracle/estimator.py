"""FP64 CPU oracle of the fitted estimator's evaluation at new points.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's
CPU-baseline leg, never by the product path; it shares no code with the HIP
library.

Sec. I of Aybat & Wang: the least-squares estimator f_N of eq. "infinite_dim"
takes the value y*_l at x_l and has xi*_l in its subdifferential there; the
method fits a piecewise-linear convex function.  Read (the design notes list
it): f_N is evaluated at any x as the largest of the N supporting hyperplanes
that the solution (y, xi) defines,

    f(x) = max_l ( y_l + xi_l^T (x - x_l) ),

with the maximising l (the smallest such l on exact ties) identifying a
subgradient xi_l of f at x.  The definition is written out directly: no
rearrangement of the hyperplanes into a matrix product.
"""
from __future__ import annotations

import numpy as np


def evaluate(X, y, xi, Q, block: int = 64):
    """f(q_m) and the maximising plane index for every row q_m of Q.

    X, xi: N x n; y: N; Q: M x n.  Returns (f (M,), arg (M,) int64).  Queries
    are taken in blocks of `block` rows only to bound memory."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    xi = np.asarray(xi, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    M = Q.shape[0]
    f = np.empty(M)
    arg = np.empty(M, dtype=np.int64)
    for m0 in range(0, M, block):
        q = Q[m0:m0 + block]
        # plane l at query m: y_l + sum_k xi_lk (q_mk - x_lk)
        d = q[:, None, :] - X[None, :, :]
        v = y[None, :] + np.sum(xi[None, :, :] * d, axis=2)
        a = np.argmax(v, axis=1)                       # first maximiser: smallest l on ties
        arg[m0:m0 + block] = a
        f[m0:m0 + block] = v[np.arange(v.shape[0]), a]
    return f, arg


def plane_values(X, y, xi, q):
    """All N hyperplane values y_l + xi_l^T (q - x_l) at one query point q."""
    X = np.asarray(X, dtype=np.float64)
    return np.asarray(y, dtype=np.float64) + np.sum(np.asarray(xi, dtype=np.float64) * (np.asarray(q)[None, :] - X),
                                                    axis=1)
