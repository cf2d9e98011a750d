"""Exact Kantorovich problems and coarse-solution checks (Section 2.1).

L_C(mu, nu) = min_{pi in Pi(mu, nu)} <pi, C>, with the dual
max_{f_i + g_j <= C_ij} <f, mu> + <g, nu>.  The solver here is scipy's HiGHS
LP (the paper uses POT's network simplex; any exact LP solver returns the
same optimal value).
"""
from __future__ import annotations

import numpy as np
import scipy.optimize
import scipy.sparse as sp


def _solve_ot_positive(a, b, C):
    n, m = C.shape
    b = b * (a.sum() / b.sum())
    rows_r = np.repeat(np.arange(n), m)
    cols_r = np.arange(n * m)
    rows_c = n + np.tile(np.arange(m), n)
    keep = rows_c < n + m - 1
    A = sp.csr_matrix(
        (np.ones(n * m + keep.sum()),
         (np.concatenate([rows_r, rows_c[keep]]), np.concatenate([cols_r, cols_r[keep]]))),
        shape=(n + m - 1, n * m))
    beq = np.concatenate([a, b[:-1]])
    res = scipy.optimize.linprog(C.reshape(-1), A_eq=A, b_eq=beq, bounds=(0, None),
                                 method="highs-ds",
                                 options={"primal_feasibility_tolerance": 1e-10,
                                          "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(f"HiGHS failed: {res.message}")
    x = res.x.reshape(n, m)
    y = res.eqlin.marginals
    f = y[:n].copy()
    g = np.concatenate([y[n:], [0.0]])
    r, c = np.nonzero(x > 0)
    return r, c, x[r, c], f, g, float(res.fun)


def solve_ot(a: np.ndarray, b: np.ndarray, C: np.ndarray):
    """Exact OT between a (length n) and b (length m) for cost C (n x m).

    Returns (rows, cols, vals, f, g, obj): the positive entries of an optimal
    plan, optimal dual potentials and the optimal value.

    Points of zero mass carry no mass in any coupling, so they are left out of
    the LP; their potentials are completed by c-transforms of the solved ones
    (f_k = min_l C_kl - g_l, then g_l = min_k C_kl - f_k), which keeps
    f_k + g_l <= C_kl everywhere.  In the reduced LP the last column
    constraint is redundant and is dropped (its potential is fixed to 0); b is
    rescaled to the mass of a so the system is consistent to the last bit.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ia = np.nonzero(a > 0)[0]
    ib = np.nonzero(b > 0)[0]
    r, c, v, fr, gr, obj = _solve_ot_positive(a[ia], b[ib], C[np.ix_(ia, ib)])
    f = np.full(len(a), np.nan)
    g = np.full(len(b), np.nan)
    f[ia] = fr
    g[ib] = gr
    za = np.setdiff1d(np.arange(len(a)), ia)
    zb = np.setdiff1d(np.arange(len(b)), ib)
    if len(za):
        f[za] = (C[np.ix_(za, ib)] - gr[None, :]).min(1)
    if len(zb):
        g[zb] = (C[:, zb] - f[:, None]).min(0)
    return ia[r], ib[c], v, f, g, obj


def wasserstein_exact(mu: np.ndarray, nu: np.ndarray, p: int) -> float:
    """W_p(mu, nu) on the full grid by an exact LP (tiny grids only)."""
    from .grid import coords, cost64
    d, N = mu.ndim, mu.shape[0]
    X = coords(N, d)
    C = cost64(X, X, p)
    *_, obj = solve_ot(mu.reshape(-1), nu.reshape(-1), C)
    return max(obj, 0.0) ** (1.0 / p)


def northwest_corner(a: np.ndarray, b: np.ndarray):
    """A basic feasible coupling of (a, b) (north-west corner rule), as COO.

    Used to build valid (not optimal) coarse couplings for parity tests: the
    primal-upscaling bound holds for any coupling of the coarse measures."""
    a = np.asarray(a, dtype=np.float64).copy()
    b = np.asarray(b, dtype=np.float64) * (a.sum() / np.asarray(b).sum())
    b = b.copy()
    i = j = 0
    rows, cols, vals = [], [], []
    n, m = len(a), len(b)
    while i < n and j < m:
        t = min(a[i], b[j])
        if t > 0:
            rows.append(i)
            cols.append(j)
            vals.append(t)
        a[i] -= t
        b[j] -= t
        if a[i] <= 0 and i < n - 1:
            i += 1
        elif b[j] <= 0:
            j += 1
        else:
            i += 1
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64), np.array(vals)


def certify(rows, cols, vals, f, g, a, b, C):
    """Optimality certificate of a coarse solution (LP duality, Section 2.1).

    Returns the largest violations of primal feasibility (negative entries,
    marginal errors), dual feasibility (f_k + g_l - C_kl) and complementary
    slackness on the plan's support, plus the primal and dual objectives."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    vals = np.asarray(vals, dtype=np.float64)
    n, m = C.shape
    rs = np.bincount(rows, weights=vals, minlength=n)
    cs = np.bincount(cols, weights=vals, minlength=m)
    viol = f[:, None] + g[None, :] - C
    return {
        "min_entry": float(vals.min()) if len(vals) else 0.0,
        "row_err": float(np.abs(rs - a).max()),
        "col_err": float(np.abs(cs - b).max()),
        "dual_viol": float(viol.max()),
        "slack_on_support": float(np.abs(viol[rows, cols]).max()) if len(vals) else 0.0,
        "primal": float((vals * C[rows, cols]).sum()),
        "dual": float(f @ a + g @ b),
        "nnz": int(len(vals)),
    }
