"""Primal-upscaling upper bound (Section 3.4, Algorithm 4) and the two other
quantization bounds of Sections 3.2-3.3.

Algorithm 4, given a coupling pi~ of the coarse measures:

1. up-scaled coupling pi^ = pi~ (tensor) K with the uniform kernel
   K = kappa^(-2d) on [kappa]^(2d): pi^_ij = kappa^(-2d) pi~_{k(i) l(j)}
   (Section 3.4 admits any normalised nonnegative kernel; upscale_plan takes
   one, and then IPF no longer converges in one iteration);
2. iterative proportional fitting, starting from b = 1:
       a <- mu / (pi^ b);  b <- nu / (pi^T a);
       mu^ <- a * (pi^ b); nu^ <- b * (pi^T a)
   until ||mu^ - mu||_1 + ||nu - nu^||_1 < xi   (reading: 0/0 := 0);
3. W^ = (sum over supp(pi^) of a_i pi^_ij b_j rho(x_i, x_j)^p)^(1/p);
4. Delta_mu^ = 2^(1-1/p) <w, |mu^ - mu|>^(1/p), Delta_nu^ likewise, with
   w_i = rho(x-bar, x_i)^p and x-bar = mean of the grid (eq. of the weighted
   total variation);
5. upper bound = W^ + Delta_mu^ + Delta_nu^.

The bound holds for any coupling of the coarse measures (the lemma on the
triangle inequality upper bound), so parity tests may feed non-optimal ones.
"""
from __future__ import annotations

import math

import numpy as np

from .coarse import block_of, cbar, centre_cost, cmin, sumpool
from .grid import coords
from .lp import solve_ot


def upscale_plan(rows, cols, vals, N: int, d: int, k: int, kernel=None):
    """Support of pi^ as COO (i, j, value): every coarse entry (K, L) becomes the
    k^d x k^d block X_K x Y_L.

    Section 3.4 upscales the coarse coupling tensor by a Kronecker product with
    a normalised nonnegative kernel tensor on [k]^(2d).  ``kernel`` is that
    tensor as a (k^d, k^d) matrix: entry [s, t] weighs source offset s against
    target offset t, where an offset is the C-order flat index of a pixel's
    position inside its block (which, since block members are listed in
    ascending flat index, is the member's rank).  The fine entry is then
    pi~_KL kernel[s, t].  ``None`` is Algorithm 4's uniform kernel, each fine
    entry worth pi~_KL / k^(2d)."""
    blk = block_of(N, d, k)
    order = np.argsort(blk, kind="stable")
    members = order.reshape(-1, k ** d)          # fine pixels of each block, ascending
    mI = members[np.asarray(rows)]               # (nnz, k^d)
    mJ = members[np.asarray(cols)]
    m = k ** d
    I = np.repeat(mI, m, axis=1).reshape(-1)
    J = np.tile(mJ, (1, m)).reshape(-1)
    if kernel is None:
        V = np.repeat(np.asarray(vals, dtype=np.float64) / float(k) ** (2 * d), m * m)
    else:
        Km = np.asarray(kernel, dtype=np.float64).reshape(m, m)
        V = (np.asarray(vals, dtype=np.float64)[:, None, None] * Km[None, :, :]).reshape(-1)
    return I, J, V


def plan_kernel_gaussian(k: int, d: int, sigma: float) -> np.ndarray:
    """A non-uniform kernel for the coupling upscaling of Section 3.4: weight
    exp(-|s - t|^2 / (2 sigma^2)) between in-block offsets s and t (integer
    offset vectors in [k]^d, C order), normalised to total 1.  It keeps the
    relative position of a pixel inside its block when the coarse plan moves
    the block; sigma -> infinity gives the uniform kernel."""
    offs = np.array([[(s // k ** (d - 1 - a)) % k for a in range(d)] for s in range(k ** d)],
                    dtype=np.float64)
    dist2 = ((offs[:, None, :] - offs[None, :, :]) ** 2).sum(axis=2)
    w = np.exp(-dist2 / (2.0 * sigma * sigma))
    return w / w.sum()


# x86 extended precision (64-bit significand) for the sums of the fitting
# passes; the oracle refuses to run where numpy's long double is narrower.
_EXT = np.longdouble
assert np.finfo(_EXT).nmant >= 63, "the oracle needs an 80-bit long double for its IPF sums"


def _matvec(I, J, V, x, n):
    """(pi^ x)_i = sum over the entries (i, j) of pi^_ij x_j.  Each product is
    rounded to float64; the products are added in extended precision and the
    sum rounded once to float64, so each entry is within about one float64
    rounding of the exact sum of the rounded products, whatever the number of
    terms (up to k^d times a row's coupling entries): the fitted marginals of
    Algorithm 4 then carry only the roundings of the scalings themselves."""
    acc = np.zeros(n, dtype=_EXT)
    np.add.at(acc, I, (V * x[J]).astype(_EXT))
    return acc.astype(np.float64)


def _safe_div(x, y):
    out = np.zeros_like(x)
    np.divide(x, y, out=out, where=y > 0)
    return out


def ipf(mu, nu, I, J, V, xi: float, max_iter: int):
    """Iterative proportional fitting exactly as in Algorithm 4.  Returns
    (a, b, mu_hat, nu_hat, iterations, final L1 residual)."""
    P = len(mu)
    b = np.ones(P)
    a = np.zeros(P)
    mu_hat, nu_hat = np.zeros(P), np.zeros(P)
    err = math.inf
    t = 0
    for t in range(1, max_iter + 1):
        a = _safe_div(mu, _matvec(I, J, V, b, P))
        pta = _matvec(J, I, V, a, P)
        b = _safe_div(nu, pta)
        mu_hat = a * _matvec(I, J, V, b, P)
        nu_hat = b * pta
        err = np.abs(mu_hat - mu).sum() + np.abs(nu - nu_hat).sum()
        if err < xi:
            break
    return a, b, mu_hat, nu_hat, t, float(err)


def tv_weights(N: int, d: int, p: int) -> np.ndarray:
    """w_i = rho(x-bar, x_i)^p with x-bar the mean of the grid, ((N-1)/2,)*d."""
    X = coords(N, d).astype(np.float64)
    r2 = ((X - (N - 1) / 2.0) ** 2).sum(1)
    return r2 if p == 2 else r2 ** (p / 2.0)


def weighted_tv(w, x, y, p: int) -> float:
    """TV_p^w(x, y) = 2^(1-1/p) <w, |x - y|>^(1/p) (eq. of the weighted total variation)."""
    s = math.fsum((w * np.abs(x - y)).tolist())
    return 2.0 ** (1.0 - 1.0 / p) * s ** (1.0 / p)


def plan_cost(I, J, V, a, b, N: int, d: int, p: int) -> float:
    """<pi^_xi, C> summed over supp(pi^) (Section 4, sparse evaluation)."""
    X = coords(N, d)
    diff = X[I] - X[J]
    d2 = (diff * diff).sum(1).astype(np.float64)
    c = d2 if p == 2 else d2 ** (p / 2.0)
    return math.fsum((a[I] * V * b[J] * c).tolist())


def upper_bound_o64(mu, nu, rows, cols, vals, k: int, p: int,
                    xi: float = 1e-12, max_iter: int = 50, kernel=None):
    """Algorithm 4 in float64 from a given coarse coupling (rows, cols, vals);
    ``kernel`` as in upscale_plan (None: the uniform kernel)."""
    d, N = mu.ndim, mu.shape[0]
    muf, nuf = mu.reshape(-1), nu.reshape(-1)
    I, J, V = upscale_plan(rows, cols, vals, N, d, k, kernel)
    a, b, mu_hat, nu_hat, T, err = ipf(muf, nuf, I, J, V, xi, max_iter)
    cost = plan_cost(I, J, V, a, b, N, d, p)
    w = tv_weights(N, d, p)
    d_mu = weighted_tv(w, mu_hat, muf, p)
    d_nu = weighted_tv(w, nuf, nu_hat, p)
    return {"a": a, "b": b, "mu_hat": mu_hat, "nu_hat": nu_hat, "iters": T,
            "residual": err, "plan_cost": cost, "tv_mu": d_mu, "tv_nu": d_nu,
            "upper": max(cost, 0.0) ** (1.0 / p) + d_mu + d_nu}


def weighted_cost_upper(mu, nu, k: int, p: int):
    """Algorithm 3: L_{C-bar}(mu~, nu~)^(1/p) (Section 3.2 theorem: >= W_p)."""
    mt, nt = sumpool(mu, k), sumpool(nu, k)
    *_, obj = solve_ot(mt, nt, cbar(mu, nu, k, p))
    return max(obj, 0.0) ** (1.0 / p)


def min_cost_lower(mu, nu, k: int, p: int):
    """Section 3.3: L_{C^min}(mu~, nu~)^(1/p) <= W_p."""
    d, N = mu.ndim, mu.shape[0]
    mt, nt = sumpool(mu, k), sumpool(nu, k)
    *_, obj = solve_ot(mt, nt, cmin(N, d, k, p))
    return max(obj, 0.0) ** (1.0 / p)


def quantization_coupling_cost(mu, nu, rows, cols, vals, k: int, p: int) -> float:
    """<pi_pi~, C> for the quantization coupling of the lemma in the proof of the
    weighted-cost theorem: pi_pi~(x, y) = pi~_kl mu(x) nu(y) / (mu~_k nu~_l)."""
    d, N = mu.ndim, mu.shape[0]
    mt, nt = sumpool(mu, k), sumpool(nu, k)
    I, J, V = upscale_plan(rows, cols, vals, N, d, k)
    blk = block_of(N, d, k)
    muf, nuf = mu.reshape(-1), nu.reshape(-1)
    scale = V * float(k) ** (2 * d)  # pi~ entry of each fine pair
    den = mt[blk[I]] * nt[blk[J]]
    X = coords(N, d)
    diff = X[I] - X[J]
    d2 = (diff * diff).sum(1).astype(np.float64)
    c = d2 if p == 2 else d2 ** (p / 2.0)
    val = np.zeros_like(c)
    ok = den > 0
    val[ok] = scale[ok] * muf[I[ok]] * nuf[J[ok]] / den[ok] * c[ok]
    return math.fsum(val.tolist())


def coarse_record_lp(mu, nu, k: int, p: int):
    """Exact coarse solve of Algorithms 4-5 on the centre cost C~ (HiGHS):
    returns (rows, cols, vals, f~, g~, objective)."""
    d, N = mu.ndim, mu.shape[0]
    return solve_ot(sumpool(mu, k), sumpool(nu, k), centre_cost(N, d, k, p))
