"""The argmin-window reading of the exact separable stages, on the CPU.

Along one axis the float64 candidates of a line are RN64(a[r] + (r - t)^2).
The stages scan, for a group of targets t0 <= t <= t1, only the sources from
the start of the first block of eight attaining the rounded minimum of t0 to
the end of the last block attaining that of t1, taken over the union of 64
lines; the minimum over that window must equal the minimum over all sources
bit for bit (the per-axis candidates form a Monge matrix and rounding is
monotone).  This checks that claim with numpy on potentials of the shapes the
pipeline and the tests produce: random, lattice-valued (many exact ties),
smooth, linear (ties on every target), with -inf potentials (+inf sources).
No GPU and no library call: the property itself.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth_inputs as si


def windowed_min(A, t0, t1):
    """A[r, line] float64 sources; the rounded minima of targets t0..t1 over
    the window of the union of the lines, as the stages form it."""
    N = A.shape[0]
    r = np.arange(N, dtype=np.float64)[:, None]
    v0 = A + (r - t0) ** 2
    v1 = A + (r - t1) ** 2
    nb = (N + 7) // 8
    lo, hi = N, -1
    for line in range(A.shape[1]):
        b0 = np.full(nb, np.inf)
        b1 = np.full(nb, np.inf)
        for b in range(nb):
            seg0 = v0[8 * b:8 * b + 8, line]
            seg1 = v1[8 * b:8 * b + 8, line]
            seg0 = seg0[~np.isnan(seg0)]
            seg1 = seg1[~np.isnan(seg1)]
            b0[b] = seg0.min() if seg0.size else np.inf
            b1[b] = seg1.min() if seg1.size else np.inf
        m0, m1 = b0.min(), b1.min()
        if np.isfinite(m0):
            lo = min(lo, 8 * int(np.argmax(b0 == m0)))
        if np.isfinite(m1):
            hi = max(hi, min(N - 1, 8 * int(nb - 1 - np.argmax((b1 == m1)[::-1])) + 7))
    out = np.full((t1 - t0 + 1, A.shape[1]), np.inf)
    if lo <= hi:
        for i, t in enumerate(range(t0, t1 + 1)):
            w = A[lo:hi + 1] + (r[lo:hi + 1] - t) ** 2
            out[i] = np.fmin.reduce(w, axis=0, initial=np.inf)
    return out


def full_min(A, t0, t1):
    N = A.shape[0]
    r = np.arange(N, dtype=np.float64)[:, None]
    return np.stack([np.fmin.reduce(A + (r - t) ** 2, axis=0, initial=np.inf) for t in range(t0, t1 + 1)])


def sources(kind, N, L, seed):
    g = si.rng(seed)
    x = np.arange(N, dtype=np.float64)[:, None]
    if kind == "random":
        phi = g.standard_normal((N, L)) * N * N / 4
    elif kind == "lattice":
        phi = np.round(g.standard_normal((N, L)) * N * N / 8 * 64) / 64
    elif kind == "smooth":
        c = g.uniform(0, N, L)
        phi = 0.6 * (x - c) ** 2 + g.uniform(-2, 2, L) * x + 0.01 * g.standard_normal((N, L))
    elif kind == "linear":
        phi = np.broadcast_to(x * 1.0, (N, L)).copy()
    else:   # some -inf potentials and a line of them
        phi = g.standard_normal((N, L)) * N
        phi[g.random((N, L)) < 0.05] = -np.inf
        phi[:, 3] = -np.inf
    a = -phi.astype(np.float32).astype(np.float64)   # sources: the negated float32 potential
    return a


@pytest.mark.parametrize("kind", ["random", "lattice", "smooth", "linear", "neginf"])
@pytest.mark.parametrize("N,T", [(64, 32), (100, 32), (37, 16), (256, 32)])
def test_window_minimum_equals_full_minimum(kind, N, T):
    A = sources(kind, N, 64, 31000 + N + T)
    for t0 in range(0, N, T):
        t1 = min(t0 + T - 1, N - 1)
        got = windowed_min(A, t0, t1)
        ref = full_min(A, t0, t1)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (kind, N, t0)


def test_a_wrong_window_is_caught():
    # a window cut one block short of the boundary scans' bounds misses
    # minimisers on these sources: the property test above would see it
    A = sources("smooth", 64, 64, 31999)
    r = np.arange(64, dtype=np.float64)[:, None]
    ref = full_min(A, 0, 31)
    cut = np.stack([np.fmin.reduce(A[8:] + (r[8:] - t) ** 2, axis=0, initial=np.inf) for t in range(0, 32)])
    assert not np.array_equal(cut, ref)
