"""Coarsening and coarse cost matrices.

* ``sumpool`` / ``centres``: Section 2.2 - the grid is cut into n^d hypercubes
  X_k of side kappa; the coarse measure puts mu(X_k) at the block's centre
  mean(X_k) (SumPool of the measure, AvgPool of the coordinates, size and
  stride kappa).
* ``centre_cost``: C~_kl = rho(x~_k, x~_l)^p, the coarse cost of Algorithms 4
  and 5.
* ``cbar``: the marginally weighted coarse cost of Section 3.2,
  C-bar_kl = sum_{x in X_k, y in Y_l} rho(x, y)^p mu(x) nu(y) / (mu(X_k) nu(Y_l)),
  evaluated by its definition.  Where mu(X_k) nu(Y_l) = 0 the entry is 0/0;
  we set it to C~_kl (reading: any finite value is fine because the coarse LP
  cannot put mass on that pair).
* ``cmin``: the locally minimal cost of Section 3.3,
  C^min_kl = min_{x in X_k, y in Y_l} rho(x, y)^p, by its definition.
"""
from __future__ import annotations

import numpy as np

from .grid import coords, cost64


def block_of(N: int, d: int, k: int) -> np.ndarray:
    """Coarse block (flat C order over [n]^d) of every fine pixel, in fine flat order."""
    n = N // k
    X = coords(N, d) // k
    out = np.zeros(len(X), dtype=np.int64)
    for a in range(d):
        out = out * n + X[:, a]
    return out


def sumpool(m: np.ndarray, k: int) -> np.ndarray:
    """SumPool with size and stride k; returns the coarse measure in flat order."""
    m = np.asarray(m, dtype=np.float64)
    d, N = m.ndim, m.shape[0]
    if N % k:
        raise ValueError("N must be a multiple of k")
    n = N // k
    shp = []
    for _ in range(d):
        shp += [n, k]
    r = m.reshape(shp)
    return r.sum(axis=tuple(range(1, 2 * d, 2))).reshape(-1)


def centres(N: int, d: int, k: int) -> np.ndarray:
    """Coarse grid points x~_k = mean(X_k) = k*K + (k-1)/2 per axis, shape (n^d, d)."""
    n = N // k
    return coords(n, d).astype(np.float64) * k + (k - 1) / 2.0


def centre_cost(N: int, d: int, k: int, p: int) -> np.ndarray:
    c = centres(N, d, k)
    diff = c[:, None, :] - c[None, :, :]
    d2 = (diff * diff).sum(-1)
    return d2 if p == 2 else d2 ** (p / 2.0)


def cbar_numerator(mu: np.ndarray, nu: np.ndarray, k: int, p: int) -> np.ndarray:
    """S_kl = sum_{x in X_k, y in Y_l} rho(x, y)^p mu(x) nu(y), by brute force."""
    d, N = mu.ndim, mu.shape[0]
    n = N // k
    Q = n ** d
    X = coords(N, d)
    blk = block_of(N, d, k)
    muf, nuf = mu.reshape(-1), nu.reshape(-1)
    S = np.zeros((Q, Q))
    for kb in range(Q):
        rows = np.nonzero(blk == kb)[0]
        c = cost64(X[rows], X, p)                  # (k^d, N^d)
        w = (muf[rows][:, None] * c).sum(0) * nuf  # sum over x in X_k, times nu(y)
        S[kb] = np.bincount(blk, weights=w, minlength=Q)
    return S


def cbar(mu: np.ndarray, nu: np.ndarray, k: int, p: int) -> np.ndarray:
    d, N = mu.ndim, mu.shape[0]
    S = cbar_numerator(mu, nu, k, p)
    mt, nt = sumpool(mu, k), sumpool(nu, k)
    den = mt[:, None] * nt[None, :]
    Ct = centre_cost(N, d, k, p)
    out = Ct.copy()
    pos = den > 0
    out[pos] = S[pos] / den[pos]
    return out


def cmin(N: int, d: int, k: int, p: int) -> np.ndarray:
    """C^min by its definition (brute force over the pixels of each block pair)."""
    n = N // k
    Q = n ** d
    X = coords(N, d)
    blk = block_of(N, d, k)
    out = np.full((Q, Q), np.inf)
    for kb in range(Q):
        rows = np.nonzero(blk == kb)[0]
        c = cost64(X[rows], X, p).min(0)
        np.minimum.at(out[kb], blk, c)
    return out
