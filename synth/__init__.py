"""Seeded synthetic inputs for the convex-regression pair pass.

This module only draws data: points x_l, observations ybar_l = f0(x_l) + eps_l
(the data model of the paper's Introduction, eq. "data") and auxiliary random
vectors.  It holds none of the method's arithmetic, so both the oracle and the
GPU path can take their inputs from it without sharing any solver code.

Every generator uses ``numpy.random.default_rng(seed)`` and draws, in order,
the points X, then the parameters of f0, then the noise eps.  All arrays are
float64, C-contiguous, X row-major (N x n).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Problem",
    "quadratic_uniform",
    "logsumexp_gaussian",
    "max_affine_uniform",
    "quad_l1_gaussian",
    "constant_data",
    "gaussian_quadratic",
    "workload",
    "batched_workload",
    "WORKLOADS",
]


@dataclasses.dataclass
class Problem:
    """One convex-regression instance: N points in R^n with observations."""

    name: str
    X: np.ndarray          # (N, n) float64, row l is x_l
    ybar: np.ndarray       # (N,)  float64 noisy observations
    f0: np.ndarray         # (N,)  float64 noise-free values f0(x_l)
    grad_f0: np.ndarray    # (N, n) float64, a (sub)gradient of f0 at x_l
    seed: int

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def n(self) -> int:
        return int(self.X.shape[1])


def _finish(name, X, f0, g0, eps, seed) -> Problem:
    X = np.ascontiguousarray(X, dtype=np.float64)
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    return Problem(name, X, np.ascontiguousarray(f0 + eps), f0,
                   np.ascontiguousarray(g0, dtype=np.float64), seed)


def quadratic_uniform(N: int, n: int, sigma: float = 0.1, seed: int = 0,
                      name: str = "quadratic_uniform") -> Problem:
    """x ~ U[-1,1]^n, f0(x) = ||x||^2, eps ~ N(0, sigma^2)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(N, n))
    f0 = np.sum(X * X, axis=1)
    eps = rng.normal(0.0, 1.0, size=N) * sigma
    return _finish(name, X, f0, 2.0 * X, eps, seed)


def gaussian_quadratic(N: int = 100, n: int = 5, seed: int = 0, name: str = "gaussian_quadratic") -> Problem:
    """The small study of Sec. III: x ~ N(0, I_n), f0(x) = 1/2 x^T Q x with
    Q = Lambda^T Lambda, Lambda_ij ~ N(0, 1), eps ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(N, n))
    Lam = rng.normal(size=(n, n))
    Q = Lam.T @ Lam
    f0 = 0.5 * np.einsum("li,ij,lj->l", X, Q, X)
    eps = rng.normal(size=N)
    return _finish(name, X, f0, X @ Q, eps, seed)


def logsumexp_gaussian(N: int, n: int, pieces: int = 20, sigma: float = 0.05,
                       seed: int = 0) -> Problem:
    """x ~ N(0, I_n), f0(x) = log sum_k exp(a_k^T x), a_k ~ N(0, I/n)."""
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, size=(N, n))
    A = rng.normal(0.0, 1.0, size=(pieces, n)) / np.sqrt(n)
    Z = X @ A.T
    zmax = Z.max(axis=1, keepdims=True)
    E = np.exp(Z - zmax)
    f0 = zmax[:, 0] + np.log(E.sum(axis=1))
    P = E / E.sum(axis=1, keepdims=True)
    g0 = P @ A
    eps = rng.normal(0.0, 1.0, size=N) * sigma
    return _finish("logsumexp_gaussian", X, f0, g0, eps, seed)


def max_affine_uniform(N: int, n: int, pieces: int = 50, sigma: float = 0.1,
                       seed: int = 0) -> Problem:
    """x ~ U[-1,1]^n, f0(x) = max_k (a_k^T x + b_k), a_k ~ N(0,I), b_k ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(N, n))
    A = rng.normal(0.0, 1.0, size=(pieces, n))
    b = rng.uniform(0.0, 1.0, size=pieces)
    V = X @ A.T + b[None, :]
    k = np.argmax(V, axis=1)
    f0 = V[np.arange(N), k]
    g0 = A[k]
    eps = rng.normal(0.0, 1.0, size=N) * sigma
    return _finish("max_affine_uniform", X, f0, g0, eps, seed)


def quad_l1_gaussian(N: int, n: int, sigma: float = 0.1, seed: int = 0) -> Problem:
    """x ~ N(0, I), f0(x) = ||x||^2 + 0.5 ||x||_1."""
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, size=(N, n))
    f0 = np.sum(X * X, axis=1) + 0.5 * np.sum(np.abs(X), axis=1)
    g0 = 2.0 * X + 0.5 * np.sign(X)
    eps = rng.normal(0.0, 1.0, size=N) * sigma
    return _finish("quad_l1_gaussian", X, f0, g0, eps, seed)


def constant_data(N: int, n: int, value: float = 1.5, seed: int = 0) -> Problem:
    """x ~ U[-1,1]^n with ybar = value for every point (f0 constant, no noise)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(N, n))
    f0 = np.full(N, float(value))
    return _finish("constant_data", X, f0, np.zeros((N, n)), np.zeros(N), seed)


def workload(name: str) -> Problem:
    """The named single-problem workloads (sizes and laws of the benchmark configs).

    small_quadratic   N=200,   n=2   x~U[-1,1]^2, f0=||x||^2,          eps~N(0,0.1^2)
    logsumexp_5000    N=5000,  n=10  x~N(0,I),    f0=logsumexp of 20,   eps~N(0,0.05^2)
    maxaffine_20000   N=20000, n=20  x~U[-1,1]^20, f0=max of 50 pieces, eps~N(0,0.1^2)
    quadratic_10000   N=10000, n=10  x~U[-1,1]^10, f0=||x||^2,          eps~N(0,0.1^2)
    """
    if name == "small_quadratic":
        return quadratic_uniform(200, 2, 0.1, seed=0, name=name)
    if name == "logsumexp_5000":
        return logsumexp_gaussian(5000, 10, 20, 0.05, seed=0)
    if name == "maxaffine_20000":
        return max_affine_uniform(20000, 20, 50, 0.1, seed=0)
    if name == "quadratic_10000":
        return quadratic_uniform(10000, 10, 0.1, seed=0, name=name)
    raise KeyError(name)


WORKLOADS = ("small_quadratic", "logsumexp_5000", "maxaffine_20000", "quadratic_10000")


def batched_workload(P: int = 64, n_min: int = 500, n_max: int = 8000,
                     dims=(5, 10, 20), meta_seed: int = 0):
    """P independent problems: N_p ~ U{n_min..n_max}, n_p uniform on dims,
    x ~ N(0, I), f0 = ||x||^2 + 0.5||x||_1, eps ~ N(0, 0.1^2); problem p is
    drawn with seed 1000 + p."""
    rng = np.random.default_rng(meta_seed)
    Ns = rng.integers(n_min, n_max + 1, size=P)
    ns = rng.choice(np.asarray(dims), size=P)
    return [quad_l1_gaussian(int(Ns[p]), int(ns[p]), 0.1, seed=1000 + p) for p in range(P)]


def weights(N: int, seed: int = 1) -> np.ndarray:
    """Random output weights w ~ N(0,1)^N for the scalar sum_l w_l y_l."""
    return np.random.default_rng(seed).normal(0.0, 1.0, size=N)


def query_points(M: int, n: int, seed: int = 2, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    """Points at which a fitted estimator is evaluated: q ~ U[low, high]^n (the
    distribution of the uniform workloads' x)."""
    return np.random.default_rng(seed).uniform(low, high, size=(M, n))
