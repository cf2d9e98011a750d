"""Gradients of both bounds with respect to the input measures (oracle side).

The paper does not differentiate its bounds; the contract used here (a
reading of ours, not the paper's) is:

* the coarse solution (coupling pi~ and potential f~) is frozen;
* lower bound: f^ = R(f~) does not depend on (mu, nu), so neither do the
  c-transforms g, f; S = <f, mu> + <g, nu> gives dS/dmu = f, dS/dnu = g and
  d(S^(1/p)) = (1/p) S^(1/p - 1) dS;
* upper bound: the derivative of W^ = <pi^_xi, C>^(1/p) through exactly the
  T proportional-fitting iterations the forward pass took; the total
  variation terms are constants (their 1/p-th root has infinite slope at 0).

The upper-bound gradient is taken by PyTorch autograd in float64 on the CPU,
through a literal transcription of Algorithm 4 (fine-level sparse coupling).
"""
from __future__ import annotations

import numpy as np
import torch

from .grid import coords
from .upper import upscale_plan


def lower_grad(f: np.ndarray, g: np.ndarray, S: float, p: int):
    """(d lower / d mu, d lower / d nu) for lower = S^(1/p), S > 0."""
    if S <= 0:
        return np.zeros_like(f, dtype=np.float64), np.zeros_like(g, dtype=np.float64)
    s = (1.0 / p) * S ** (1.0 / p - 1.0)
    return s * np.asarray(f, dtype=np.float64), s * np.asarray(g, dtype=np.float64)


def _safe_div(x, y):
    pos = y > 0
    return torch.where(pos, x / torch.where(pos, y, torch.ones_like(y)), torch.zeros_like(x))


def plan_cost_fn(mu, nu, rows, cols, vals, k: int, p: int, iters: int, kernel=None):
    """Returns a closure (mu_t, nu_t) -> W^ as a torch float64 scalar
    (``kernel``: the coupling upscaling kernel, None = uniform)."""
    d, N = mu.ndim, mu.shape[0]
    I, J, V = upscale_plan(rows, cols, vals, N, d, k, kernel)
    X = coords(N, d)
    diff = X[I] - X[J]
    d2 = (diff * diff).sum(1).astype(np.float64)
    c = torch.from_numpy(d2 if p == 2 else d2 ** (p / 2.0))
    It, Jt, Vt = torch.from_numpy(I), torch.from_numpy(J), torch.from_numpy(V)
    P = N ** d

    def mv(rows_, cols_, x):
        return torch.zeros(P, dtype=torch.float64).index_add(0, rows_, Vt * x[cols_])

    def W(mu_t, nu_t):
        b = torch.ones(P, dtype=torch.float64)
        a = None
        for _ in range(iters):
            a = _safe_div(mu_t, mv(It, Jt, b))
            b = _safe_div(nu_t, mv(Jt, It, a))
        cost = (a[It] * Vt * b[Jt] * c).sum()
        return cost.clamp_min(0.0) ** (1.0 / p)

    return W


def upper_grad(mu, nu, rows, cols, vals, k: int, p: int, iters: int, kernel=None):
    """(d W^/d mu, d W^/d nu) with the coarse coupling and T = ``iters`` frozen."""
    W = plan_cost_fn(mu, nu, rows, cols, vals, k, p, iters, kernel)
    mu_t = torch.tensor(mu.reshape(-1), dtype=torch.float64, requires_grad=True)
    nu_t = torch.tensor(nu.reshape(-1), dtype=torch.float64, requires_grad=True)
    val = W(mu_t, nu_t)
    val.backward()
    return mu_t.grad.numpy().copy(), nu_t.grad.numpy().copy(), float(val.detach())
