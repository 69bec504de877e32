"""FP64 CPU oracle of the differentiated fixed-schedule ALCC/MAPG map.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/``,
never by the product path, and sharing no code with the HIP library.

The map.  With K ALCC iterations (Fig. 3) of exactly L MAPG iterations each
(Fig. 4), all step constants fixed, and a given start (y0, xi0):

    theta_1 = 0
    for k = 1..K:
        MAPG on P_k from (y_{k-1}, xi_{k-1}):  t_1 = 1, y^(1)_0 = y^(2)_1 = y_{k-1}
            for l = 1..L:
                g    = grad P_k at (y^(2)_l, xi^(2)_l)
                y^(1)_l  = Proj_{Q_y}(y^(2)_l - s^y_k g_y)      (ball around ybar, radius Bbar_y)
                xi^(1)_l = Proj_{Q_xi}(xi^(2)_l - s^xi_k g_xi)  (ball around 0, radius Bbar_xi)
                t_{l+1} = (1 + sqrt(1 + 4 t_l^2)) / 2,  beta_l = (t_l - 1) / t_{l+1}
                y^(2)_{l+1} = y^(1)_l + beta_l (y^(1)_l - y^(1)_{l-1})       (same for xi)
            (y_k, xi_k) = (y^(1)_L, xi^(1)_L)
        theta_{k+1} = (mu_k / mu_{k+1}) (A1 y_k + A2 xi_k - theta_k)_-

and the output is (y_K, xi_K).  mu_k, the steps s = step_scale / L_k and the
ball radii enter as constants: the derivative holds them fixed (they depend on
the data only through sigma_max(A2)^2 and Bbar, which a caller fixes through
the overrides when comparing with finite differences).

The gradient is the plain definition: reverse-mode automatic differentiation
(torch autograd, CPU, float64) of the map written out with dense N x N pair
arrays.  The pair map (v)_- has derivative -1 where its argument is negative
and 0 elsewhere (the HIP path takes the same branch at v = 0), which matters
only on a set of measure zero.  The forward is checked against
``oracle.alcc`` and the gradient against central finite differences of
``oracle.alcc`` in ``tests/test_oracle_diff_pins.py``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

from . import Params, resolve, affine_fit, sigma2_A2


@dataclasses.dataclass
class Schedule:
    """Constants of the fixed schedule (Fig. 3 steps 1 and 5, Fig. 4 momentum)."""
    gamma: float
    mu: List[float]          # mu_k, k = 1..K
    sy: List[float]          # step_scale / L^y_k
    sxi: List[float]         # step_scale / L^xi_k
    By: float
    Bxi: float
    beta: List[float]        # beta_l, l = 1..L (the same in every MAPG run)
    theta_scale: List[float]  # mu_k / mu_{k+1}
    K: int
    L: int


def schedule(X, ybar, params: Params) -> Schedule:
    """The constants that ``oracle.alcc`` uses for a fixed schedule
    (params.inner_iters = L > 0, params.max_outer = K)."""
    p = params
    if p.inner_iters <= 0:
        raise ValueError("the differentiated map needs a fixed schedule (inner_iters > 0)")
    X = np.asarray(X, dtype=np.float64)
    ybar = np.asarray(ybar, dtype=np.float64)
    N = X.shape[0]
    _, _, Bbar, By, Bxi = affine_fit(X, ybar, p.gamma)
    if p.By_override > 0:
        By = p.By_override
    if p.Bxi_override > 0:
        Bxi = p.Bxi_override
    mu, _, _ = resolve(p, N, Bbar, p.gamma)
    s2A1 = 2.0 * N
    s2A2 = sigma2_A2(X) if p.Lxi_override <= 0 else 0.0
    mus, sys, sxis, scales = [], [], [], []
    for _ in range(p.max_outer):
        Ly = p.Ly_override if p.Ly_override > 0 else 1.0 / mu + s2A1
        Lxi = p.Lxi_override if p.Lxi_override > 0 else p.gamma / mu + s2A2
        mus.append(mu)
        sys.append(p.step_scale / Ly)
        sxis.append(p.step_scale / Lxi)
        scales.append(1.0 / p.c)
        mu = p.c * mu
    betas, t = [], 1.0
    for _ in range(p.inner_iters):
        tn = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        betas.append((t - 1.0) / tn)
        t = tn
    return Schedule(p.gamma, mus, sys, sxis, By, Bxi, betas, scales, p.max_outer, p.inner_iters)


def _torch():
    import torch
    return torch


def _residuals(X, y, xi):
    """r_ij = y_i - y_j - xi_j^T (x_i - x_j) for every ordered pair (row i, column j)."""
    torch = _torch()
    d = (X * xi).sum(1)                     # xi_j^T x_j
    return y[:, None] - y[None, :] - X @ xi.T + d[None, :]


def _neg_part(v):
    """(v)_- = max(-v, 0), derivative -1 where v < 0 and 0 elsewhere."""
    torch = _torch()
    return torch.where(v < 0, -v, torch.zeros_like(v))


def _adjoint_ops(X, W):
    """(A1^T W, A2^T W): u_m = sum_j W_mj - sum_i W_im,
    v_m = -sum_i W_im (x_i - x_m)."""
    cs = W.sum(0)
    u = W.sum(1) - cs
    v = -(W.T @ X) + cs[:, None] * X
    return u, v


def _proj_ball(v, centre, radius: float):
    torch = _torch()
    d = v - centre
    nrm = torch.sqrt((d * d).sum())
    if float(nrm.detach()) <= radius:
        return v
    return centre + d * (radius / nrm)


def unrolled(X, ybar, y0, xi0, sch: Schedule):
    """The map (y_K, xi_K) of (X, ybar, y0, xi0), torch float64 tensors on the CPU."""
    torch = _torch()
    N = X.shape[0]
    off = 1.0 - torch.eye(N, dtype=torch.float64)
    theta = torch.zeros(N, N, dtype=torch.float64)
    y, xi = y0, xi0
    for k in range(sch.K):
        mu = sch.mu[k]
        y1p, xi1p, y2, xi2 = y, xi, y, xi
        for l in range(sch.L):
            W = _neg_part(_residuals(X, y2, xi2) - theta) * off
            u, v = _adjoint_ops(X, W)
            gy = (y2 - ybar) / mu - u
            gxi = (sch.gamma / mu) * xi2 - v
            y1 = _proj_ball(y2 - sch.sy[k] * gy, ybar, sch.By)
            xi1 = _proj_ball(xi2 - sch.sxi[k] * gxi, torch.zeros_like(xi2), sch.Bxi)
            b = sch.beta[l]
            y2 = y1 + b * (y1 - y1p)
            xi2 = xi1 + b * (xi1 - xi1p)
            y1p, xi1p = y1, xi1
        y, xi = y1p, xi1p
        theta = sch.theta_scale[k] * _neg_part(_residuals(X, y, xi) - theta) * off
    return y, xi


def unrolled_vjp(X, ybar, y0, xi0, sch: Schedule, gy, gxi=None):
    """Vector-Jacobian product of the map: for the scalar
    sum_l gy_l y_K,l + sum gxi * xi_K, its gradients (dX, dybar, dy0, dxi0)
    (numpy float64) with respect to X, ybar, y0 and xi0 as independent inputs,
    and the outputs (y_K, xi_K)."""
    torch = _torch()
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), dtype=torch.float64, requires_grad=True)
    Xt, ybt, y0t, xi0t = t(X), t(ybar), t(y0), t(np.asarray(xi0).reshape(np.asarray(X).shape))
    y, xi = unrolled(Xt, ybt, y0t, xi0t, sch)
    s = (y * torch.tensor(np.asarray(gy, dtype=np.float64))).sum()
    if gxi is not None:
        s = s + (xi * torch.tensor(np.asarray(gxi, dtype=np.float64).reshape(xi.shape))).sum()
    dX, dyb, dy0, dxi0 = torch.autograd.grad(s, (Xt, ybt, y0t, xi0t), allow_unused=True)
    z = lambda g, ref: np.zeros(ref.shape) if g is None else g.detach().numpy()
    return (z(dX, Xt), z(dyb, ybt), z(dy0, y0t), z(dxi0, xi0t),
            y.detach().numpy(), xi.detach().numpy())
