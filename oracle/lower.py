"""Dual-upscaling lower bound (Section 3.5, Algorithm 5, lazy c-transform of Section 4).

Given coarse dual potentials f~ on the coarse grid:

1. upscale f~ to the fine grid by multilinear interpolation, f^ = R(f~);
2. g = (f^)^c, i.e. g_j = min_i C_ij - f^_i            (first c-transform)
3. f = g^c,     i.e. f_i = min_j C_ij - g_j            (second c-transform)
4. lower bound = (<f, mu> + <g, nu>)^(1/p).

(f, g) is an admissible pair for C, so <f, mu> + <g, nu> <= L_C(mu, nu)
(the proposition of Section 3.5), for any choice of f^.

Two tracks:

* ``*_o64``: every step in float64 - the mathematical definition.
* ``*_o32``: the float32 reading used by the GPU path.  f^ is rounded once to
  float32; each candidate C_ij - phi_i is one float32 subtraction of the
  float32 cost (exact for p = 2, correctly rounded sqrt for p = 1); the min is
  exact and ties go to the lowest flat index.  The sums <f, mu>, <g, nu> are
  float64.  Because float32 rounding can make (f, g) slightly infeasible, the
  emitted value subtracts a feasibility shift s (``feasibility_shift``), which
  also keeps it at or below the float64 value.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import coords, cost32, cost64


# ----------------------------------------------------------------------------
# Interpolation R of the coarse potential (Section 3.5; multilinear, as in the
# paper's experiments).  Reading: coarse potentials live at the block centres
# k*K + (k-1)/2; fine pixels outside the hull of the centres take the value of
# the nearest edge (clamped, no extrapolation).  The interpolation is the
# nested linear interpolation lerp(a, b, w) = a + w * (b - a), the last axis
# innermost, each operation rounded separately in float64.
# ----------------------------------------------------------------------------

def _axis_weights(N: int, k: int):
    """Per fine coordinate x: (K0, K1, w) with x = centre(K0) + w * k (clamped)."""
    n = N // k
    x = np.arange(N, dtype=np.int64)
    t = 2 * x - (k - 1)          # position relative to centre 0, in units of 1/(2k)
    den = 2 * k
    K0 = np.floor_divide(t, den)
    r = t - den * K0
    w = r.astype(np.float64) / float(den)
    K1 = K0 + 1
    low = t <= 0
    high = K0 >= n - 1
    K0 = np.where(low, 0, np.where(high, n - 1, K0))
    K1 = np.where(low, 0, np.where(high, n - 1, K1))
    w = np.where(low | high, 0.0, w)
    return K0, K1, w


def upscale_potential(ftil: np.ndarray, N: int, d: int, k: int, interp: str = "linear") -> np.ndarray:
    """R(f~) on the fine grid.  interp: "linear" (multilinear, the paper's
    experiments), "nearest" or "cubic" (Section 3.5 allows any interpolation)."""
    if interp == "nearest":
        return upscale_nearest(ftil, N, d, k)
    if interp == "cubic":
        return upscale_cubic(ftil, N, d, k)
    if interp != "linear":
        raise ValueError(f"unknown interpolation {interp!r}")
    n = N // k
    F = np.asarray(ftil, dtype=np.float64).reshape((n,) * d)
    X = coords(N, d)
    K0, K1, W = _axis_weights(N, k)

    def rec(axis, idx):
        if axis == d:
            return F[tuple(idx)]
        xa = X[:, axis]
        lo = rec(axis + 1, idx + [K0[xa]])
        hi = rec(axis + 1, idx + [K1[xa]])
        return lo + W[xa] * (hi - lo)

    return rec(0, [])


def upscale_nearest(ftil: np.ndarray, N: int, d: int, k: int) -> np.ndarray:
    """Nearest-neighbour interpolation: the nearest block centre to a pixel is
    the centre of its own block, so f^_i = f~ of the block containing i."""
    n = N // k
    F = np.asarray(ftil, dtype=np.float64).reshape((n,) * d)
    X = coords(N, d)
    return F[tuple(X[:, a] // k for a in range(d))].copy()


# Cubic reading: separable cubic convolution with the Catmull-Rom kernel (the
# Keys kernel with a = -1/2), through the block centres.  Along one axis the
# pixel sits at coarse position t = (2x - (k-1)) / (2k), clamped to [0, n-1]
# (pixels outside the hull of the centres take the edge value, as for the
# multilinear reading); with i = floor(t) and s = t - i the value is
#   w_{-1} F[i-1] + w_0 F[i] + w_1 F[i+1] + w_2 F[i+2],
#   w_{-1} = (2 s^2 - s^3 - s)/2,  w_0 = (3 s^3 - 5 s^2 + 2)/2,
#   w_1 = (4 s^2 - 3 s^3 + s)/2,   w_2 = (s^3 - s^2)/2,
# taps beyond the edge replaced by the edge value.  Evaluation order (each
# float64 operation rounded separately): s = r / (2k) from the integer
# remainder r; s2 = s*s; s3 = s2*s; each weight as written above, grouped
# as ((a - b) - c) * 0.5 etc. in ``_cubic_weights``; the four taps summed
# left to right; axes nested with the last axis innermost.

def _cubic_weights(s):
    s2 = s * s
    s3 = s2 * s
    wm1 = 0.5 * ((2.0 * s2 - s3) - s)
    w0 = 0.5 * ((3.0 * s3 - 5.0 * s2) + 2.0)
    w1 = 0.5 * ((4.0 * s2 - 3.0 * s3) + s)
    w2 = 0.5 * (s3 - s2)
    return wm1, w0, w1, w2


def _axis_cubic(N: int, k: int):
    """Per fine coordinate x: the four clamped tap indices and their weights."""
    n = N // k
    x = np.arange(N, dtype=np.int64)
    t = 2 * x - (k - 1)
    den = 2 * k
    i = np.floor_divide(t, den)
    r = t - den * i
    low = t <= 0
    high = i >= n - 1
    i = np.where(low, 0, np.where(high, n - 1, i))
    r = np.where(low | high, 0, r)
    s = r.astype(np.float64) / float(den)
    taps = [np.clip(i + o, 0, n - 1) for o in (-1, 0, 1, 2)]
    return taps, _cubic_weights(s)


def upscale_cubic(ftil: np.ndarray, N: int, d: int, k: int) -> np.ndarray:
    n = N // k
    F = np.asarray(ftil, dtype=np.float64).reshape((n,) * d)
    X = coords(N, d)
    taps, W = _axis_cubic(N, k)

    def rec(axis, idx):
        if axis == d:
            return F[tuple(idx)]
        xa = X[:, axis]
        v = [rec(axis + 1, idx + [taps[o][xa]]) for o in range(4)]
        return ((W[0][xa] * v[0] + W[1][xa] * v[1]) + W[2][xa] * v[2]) + W[3][xa] * v[3]

    return rec(0, [])


# ----------------------------------------------------------------------------
# Lazy c-transform psi_j = min_i C_ij - phi_i (Section 4, eq. of the lazy
# c-transform).  The cost is symmetric, so one routine serves both steps.
# ----------------------------------------------------------------------------

def _chunks(P: int):
    step = max(1, (1 << 22) // P)
    for s in range(0, P, step):
        yield s, min(P, s + step)


def ctransform_o64(phi: np.ndarray, N: int, d: int, p: int, targets=None):
    """FP64 c-transform.  Returns (psi, argmin) for all targets (or the given ones)."""
    X = coords(N, d)
    phi = np.asarray(phi, dtype=np.float64)
    tg = np.arange(len(X)) if targets is None else np.asarray(targets)
    psi = np.empty(len(tg))
    arg = np.empty(len(tg), dtype=np.int64)
    for s, e in _chunks(len(X)):
        if s >= len(tg):
            break
        J = tg[s:e]
        t = cost64(X, X[J], p) - phi[:, None]
        arg[s:e] = np.argmin(t, axis=0)
        psi[s:e] = t[arg[s:e], np.arange(len(J))]
    return psi, arg


def ctransform_o32(phi32: np.ndarray, N: int, d: int, p: int, targets=None):
    """FP32-faithful c-transform: min_i RN32(RN32(C_ij) - phi_i), lowest index on ties."""
    X = coords(N, d)
    phi32 = np.asarray(phi32, dtype=np.float32)
    tg = np.arange(len(X)) if targets is None else np.asarray(targets)
    psi = np.empty(len(tg), dtype=np.float32)
    arg = np.empty(len(tg), dtype=np.int64)
    for s, e in _chunks(len(X)):
        if s >= len(tg):
            break
        J = tg[s:e]
        t = cost32(X, X[J], p) - phi32[:, None]       # float32 - float32 -> float32
        assert t.dtype == np.float32
        arg[s:e] = np.argmin(t, axis=0)
        psi[s:e] = t[arg[s:e], np.arange(len(J))]
    return psi, arg


def ctransform_sep_o32(phi32: np.ndarray, N: int, d: int):
    """p = 2 only, float32 reading of the separable evaluation.

    |x - y|^2 is a sum over axes, so min_i |x_i - y|^2 - phi_i is d nested
    one-dimensional minimisations.  Passes run over the last axis first:
        pass 1:  psi_1(.., v) = min_t RN32((t - v)^2 - phi(.., t))
        pass k:  psi_k(.., v) = min_t RN32((t - v)^2 + psi_{k-1}(.., t))
    (the later passes add the previous result).  In exact arithmetic this is
    the c-transform; in float32 every candidate carries one rounding per axis.
    Arg-min: the lowest index of each pass, composed (this is the lowest flat
    index among the pairs attaining the nested float32 minimum)."""
    cur = np.asarray(phi32, dtype=np.float32).reshape((N,) * d)
    t = np.arange(N)
    cost1 = ((t[:, None] - t[None, :]) ** 2).astype(np.float32)   # [source t, target v], exact
    args = []
    for k, axis in enumerate(reversed(range(d))):
        arr = np.moveaxis(cur, axis, -1)                              # (..., N sources)
        if k == 0:
            vals = cost1 - arr[..., :, None]                          # RN32(c - phi)
        else:
            vals = cost1 + arr[..., :, None]                          # RN32(c + psi)
        assert vals.dtype == np.float32
        am = vals.argmin(axis=-2)
        new = np.take_along_axis(vals, am[..., None, :], axis=-2)[..., 0, :]
        cur = np.moveaxis(new, -1, axis)
        args.append((axis, np.moveaxis(am, -1, axis)))
    psi = cur.reshape(-1)
    # compose the arg-mins: the last pass fixes axis 0, then walk back
    tgt = np.indices((N,) * d).reshape(d, -1)                        # target coordinates
    src = tgt.copy()
    for axis, am in reversed(args):
        src[axis] = am[tuple(src)]
    arg = np.ravel_multi_index(tuple(src), (N,) * d)
    return psi, arg.astype(np.int64)


def feasibility_shift_sep(F_hat: float, G: float, Fo: float, N: int, d: int) -> float:
    """Shift for the separable float32 evaluation (p = 2).  Along the arg-min
    path the k-th pass rounds a partial value of size at most |g| + C (C =
    d (N-1)^2 bounds every partial cost), the last one of size |g|:
        |g32 - g64| <= e_g = u (F + d G + (d-1) C)
        |f32 - f64| <= e_f = u (d Fo + (d-1) C) + e_g
    and e_f again bounds the infeasibility; same summation slack as the
    all-pairs shift."""
    u = U32
    C = d * (N - 1) ** 2
    F = F_hat * (1.0 + 2.0 * u)
    e_g = u * (F + d * G + (d - 1) * C)
    e_f = u * (d * Fo + (d - 1) * C) + e_g
    return (e_f + e_g) * (1.0 + 2.0 ** -10) + 2.0 ** -52 * N ** d * (Fo + G)


def lower_bound_sep_o32(mu, nu, ftil, k: int, interp: str = "linear"):
    """Algorithm 5 (p = 2) with the separable float32 c-transforms."""
    d, N = mu.ndim, mu.shape[0]
    fhat32 = upscale_potential(ftil, N, d, k, interp).astype(np.float32)
    g32, ig = ctransform_sep_o32(fhat32, N, d)
    f32, jf = ctransform_sep_o32(g32, N, d)
    S32 = fsum_dot(f32, mu.reshape(-1)) + fsum_dot(g32, nu.reshape(-1))
    s = feasibility_shift_sep(float(np.abs(fhat32).max()), float(np.abs(g32).max()),
                              float(np.abs(f32).max()), N, d)
    S_emit = S32 - s
    return {"fhat32": fhat32, "g32": g32, "f32": f32, "argmin_g": ig, "argmin_f": jf,
            "S32": S32, "shift": s, "S_emit": S_emit,
            "lower": max(S_emit, 0.0) ** 0.5, "clipped": S_emit <= 0.0}


def fsum_dot(x, w) -> float:
    """sum_i x_i * w_i in float64: products rounded once, then an exactly rounded sum."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    return math.fsum((x * w).tolist())


# ----------------------------------------------------------------------------
# Bound assembly
# ----------------------------------------------------------------------------

def lower_bound_o64(mu, nu, ftil, k: int, p: int, interp: str = "linear"):
    """Algorithm 5 in float64: returns f^, g, f, S = <f,mu> + <g,nu>, lower bound."""
    d, N = mu.ndim, mu.shape[0]
    fhat = upscale_potential(ftil, N, d, k, interp)
    g, ig = ctransform_o64(fhat, N, d, p)
    f, jf = ctransform_o64(g, N, d, p)
    S = fsum_dot(f, mu.reshape(-1)) + fsum_dot(g, nu.reshape(-1))
    return {"fhat": fhat, "g": g, "f": f, "argmin_g": ig, "argmin_f": jf,
            "S": S, "lower": max(S, 0.0) ** (1.0 / p)}


U32 = 2.0 ** -24


def feasibility_shift(F_hat: float, G: float, Fo: float, p: int, P: int) -> float:
    """Shift s such that (f32 - s, g32) is admissible for the exact costs and
    <f32 - s, mu> + <g32, nu> <= the float64 value of Algorithm 5.

    Inputs: F_hat = max|f^32|, G = max|g32|, Fo = max|f32|, P = number of
    pixels.  Derivation (first order in u = 2^-24, the rest absorbed by the
    factor 1 + 2^-10): the c-transform is 1-Lipschitz in the sup norm and each
    candidate carries one float32 rounding of a value whose magnitude at the
    arg-min is |g| (resp. |f|), plus the rounding of f^ (u |f^|) and, for p = 1,
    of the cost (u * C with C <= |f| + |g| at the arg-min):
        |g32 - g64| <= e_g = (u + u_p)(G + F)
        |f32 - f64| <= e_f = u Fo + u_p (Fo + G) + e_g
    and the float64 sums of P terms are off by at most P 2^-52 (Fo + G).
    The same e_f bounds the infeasibility f32_i + g32_j - C_ij."""
    u = U32
    up = u if p == 1 else 0.0
    F = F_hat * (1.0 + 2.0 * u)
    e_g = (u + up) * (G + F)
    e_f = u * Fo + up * (Fo + G) + e_g
    return (e_f + e_g) * (1.0 + 2.0 ** -10) + 2.0 ** -52 * P * (Fo + G)


def lower_bound_o32(mu, nu, ftil, k: int, p: int, interp: str = "linear"):
    """Algorithm 5 in the float32 reading, with the float64 sums and shift."""
    d, N = mu.ndim, mu.shape[0]
    P = N ** d
    fhat64 = upscale_potential(ftil, N, d, k, interp)
    fhat32 = fhat64.astype(np.float32)
    g32, ig = ctransform_o32(fhat32, N, d, p)
    f32, jf = ctransform_o32(g32, N, d, p)
    S32 = fsum_dot(f32, mu.reshape(-1)) + fsum_dot(g32, nu.reshape(-1))
    s = feasibility_shift(float(np.abs(fhat32).max()), float(np.abs(g32).max()),
                          float(np.abs(f32).max()), p, P)
    S_emit = S32 - s
    return {"fhat32": fhat32, "g32": g32, "f32": f32, "argmin_g": ig, "argmin_f": jf,
            "S32": S32, "shift": s, "S_emit": S_emit,
            "lower": max(S_emit, 0.0) ** (1.0 / p), "clipped": S_emit <= 0.0}
