"""The regular grid X = [N]^d and the ground cost (Section 2.1, Section 2.2).

Conventions (readings of the paper where it leaves them open):

* Pixels sit at integer coordinates 0..N-1 along every axis, spacing 1.  The
  paper uses [N] = {1..N}; the cost is translation invariant, so the shift
  changes nothing.
* A measure on [N]^d is a C-contiguous array of shape (N,)*d.  Its flat index
  is the C order index, i.e. the paper's row index of the reshape in Section
  3.4 with the *last* tensor axis playing the paper's first (fastest) axis.
  Ties in a c-transform's arg-min are broken towards the lowest flat index.
* The ground cost is C_ij = rho(x_i, y_j)^p with rho the Euclidean distance
  (the paper's experiments use rho = L2 with p in {1, 2}).
"""
from __future__ import annotations

import numpy as np


def coords(N: int, d: int) -> np.ndarray:
    """Integer coordinates of all N^d pixels in flat (C) order, shape (N^d, d)."""
    axes = np.meshgrid(*([np.arange(N, dtype=np.int64)] * d), indexing="ij")
    return np.stack([a.reshape(-1) for a in axes], axis=1)


def sqdist(xa: np.ndarray, xb: np.ndarray) -> np.ndarray:
    """Exact integer squared distances between two coordinate lists, shape (len(xa), len(xb))."""
    diff = xa[:, None, :] - xb[None, :, :]
    return (diff * diff).sum(-1)


def cost64(xa: np.ndarray, xb: np.ndarray, p: int) -> np.ndarray:
    """rho(x, y)^p in float64.  For p = 2 the value is an exact integer."""
    d2 = sqdist(xa, xb).astype(np.float64)
    if p == 2:
        return d2
    if p == 1:
        return np.sqrt(d2)
    return d2 ** (p / 2.0)


def cost32(xa: np.ndarray, xb: np.ndarray, p: int) -> np.ndarray:
    """The ground cost rounded once to float32: RN32(rho^p).

    For p = 2 the integer squared distance is below 2^24 at every grid size
    used here, so it is exact.  For p = 1 it is the correctly rounded float32
    square root of the exact integer squared distance."""
    d2 = sqdist(xa, xb)
    if p == 2:
        return d2.astype(np.float32)
    if p == 1:
        return np.sqrt(d2.astype(np.float32))
    raise ValueError("p must be 1 or 2")


def cmax(N: int, d: int, p: int) -> float:
    """Largest ground cost on the grid, rho(corner, opposite corner)^p."""
    return float(d * (N - 1) ** 2) ** (p / 2.0)
