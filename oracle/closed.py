"""Closed forms that pin the bounds at any grid size (standard optimal-transport
facts, not from the paper):

* one-dimensional W_p by the quantile formula
  W_p^p = int_0^1 |F^-1(t) - G^-1(t)|^p dt;
* measures that vary along one axis only: W_p equals the one-dimensional W_p
  of the profiles (projection onto that axis is 1-Lipschitz, and moving mass
  along that axis alone attains it);
* an exact translate: W_p(mu, mu(. - t)) = |t|;
* two Diracs: W_p = |x - y|.
"""
from __future__ import annotations

import math

import numpy as np


def w1d(a: np.ndarray, b: np.ndarray, p: int) -> float:
    """W_p between two measures on the integer points 0..len-1 (quantile formula)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a = a / a.sum()
    b = b / b.sum()
    ca, cb = np.cumsum(a), np.cumsum(b)
    ca[-1] = cb[-1] = 1.0
    ts = np.union1d(ca, cb)
    ts = ts[(ts > 0) & (ts <= 1.0)]
    lo = np.concatenate([[0.0], ts[:-1]])
    mid = 0.5 * (lo + ts)
    xa = np.searchsorted(ca, mid, side="left")
    xb = np.searchsorted(cb, mid, side="left")
    return math.fsum(((ts - lo) * np.abs(xa - xb).astype(np.float64) ** p).tolist()) ** (1.0 / p)


def axis_constant_w(mu: np.ndarray, nu: np.ndarray, p: int) -> float:
    """W_p for measures that vary only along the last axis."""
    ax = tuple(range(mu.ndim - 1))
    return w1d(mu.sum(axis=ax), nu.sum(axis=ax), p)
