"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: brute force
on tiny inputs, closed forms, textbook or library routines, exact LPs, and the
paper's theorems (bracketing, admissibility, couplings, the total-variation
bound).  None of these tests touches the GPU library.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import synth_inputs as si
from oracle import closed, coarse, grid, lower, lp, upper
from oracle import grad as ograd


def pair(N, d, fam_a, fam_b, seed):
    return si.family(fam_a, N, d, si.rng(seed)), si.family(fam_b, N, d, si.rng(seed + 1))


# ---------------------------------------------------------------- grid / cost

def test_flat_index_is_c_order():
    for N, d in [(5, 2), (4, 3)]:
        X = grid.coords(N, d)
        for i in range(N ** d):
            assert tuple(X[i]) == np.unravel_index(i, (N,) * d)


def test_cost_p2_is_exact_integer_in_float32():
    X = grid.coords(512, 2)[::4099]
    c32 = grid.cost32(X, X, 2).astype(np.int64)
    ref = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(c32, ref) and ref.max() < 2 ** 24


def test_cost_p1_float32_sqrt_equals_rounded_double_sqrt():
    # sqrt rounded to float32 directly equals float32(sqrt in float64): double
    # rounding is innocuous for sqrt when 53 >= 2*24 + 2.
    n = np.arange(0, 2 * 511 ** 2 + 1, dtype=np.int64)
    a = np.sqrt(n.astype(np.float32))
    b = np.sqrt(n.astype(np.float64)).astype(np.float32)
    assert np.array_equal(a, b)


def test_cmax():
    X = grid.coords(7, 3)
    assert grid.cmax(7, 3, 2) == grid.cost64(X, X, 2).max()
    assert grid.cmax(7, 3, 1) == pytest.approx(grid.cost64(X, X, 1).max(), rel=1e-15)


# ---------------------------------------------------------------- coarsening

def test_sumpool_brute_force_and_mass():
    m = si.white_noise(8, 2, si.rng(3))
    k = 4
    out = coarse.sumpool(m, k)
    ref = np.zeros(4)
    for x in range(8):
        for y in range(8):
            ref[(x // k) * 2 + (y // k)] += m[x, y]
    assert np.allclose(out, ref, rtol=16 * 2.0 ** -53, atol=0)  # 16 terms per block
    m3 = si.white_noise(6, 3, si.rng(4))
    assert math.isclose(coarse.sumpool(m3, 3).sum(), 1.0, rel_tol=1e-15)


def test_centres_are_block_means():
    N, d, k = 12, 2, 3
    X = grid.coords(N, d).astype(float)
    blk = coarse.block_of(N, d, k)
    c = coarse.centres(N, d, k)
    for b in range(len(c)):
        assert np.array_equal(c[b], X[blk == b].mean(0))


def test_centre_cost_closed_form():
    N, d, k = 12, 3, 4
    n = N // k
    K = grid.coords(n, d)
    for p in (1, 2):
        ref = (k * k * ((K[:, None] - K[None]) ** 2).sum(-1)) ** (p / 2.0)
        assert np.allclose(coarse.centre_cost(N, d, k, p), ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("N,d,k", [(8, 2, 2), (4, 3, 2)])
@pytest.mark.parametrize("p", [1, 2])
def test_cbar_brute_force(N, d, k, p):
    mu = si.white_noise(N, d, si.rng(10))
    nu = si.gmm(N, d, si.rng(11))
    X = grid.coords(N, d)
    blk = coarse.block_of(N, d, k)
    Q = (N // k) ** d
    S = np.zeros((Q, Q))
    mm, nn = np.zeros(Q), np.zeros(Q)
    muf, nuf = mu.reshape(-1), nu.reshape(-1)
    for i in range(len(X)):
        mm[blk[i]] += muf[i]
        nn[blk[i]] += nuf[i]
        for j in range(len(X)):
            r = math.sqrt(sum((int(X[i, a]) - int(X[j, a])) ** 2 for a in range(d)))
            S[blk[i], blk[j]] += r ** p * muf[i] * nuf[j]
    ref = S / np.outer(mm, nn)
    assert np.allclose(coarse.cbar(mu, nu, k, p), ref, rtol=1e-13, atol=0)


def test_cbar_p2_moment_form():
    # For p = 2 the weighted block cost separates into centroid distance plus
    # the two within-block variances.
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, "grf", "cauchy", 20)
    X = grid.coords(N, d).astype(float)
    blk = coarse.block_of(N, d, k)
    Q = (N // k) ** d

    def moments(m):
        m = m.reshape(-1)
        w = np.bincount(blk, m, Q)
        cen = np.stack([np.bincount(blk, m * X[:, a], Q) for a in range(d)], 1) / w[:, None]
        var = np.bincount(blk, m * ((X - cen[blk]) ** 2).sum(1), Q) / w
        return cen, var

    cm, vm = moments(mu)
    cn, vn = moments(nu)
    ref = ((cm[:, None] - cn[None]) ** 2).sum(-1) + vm[:, None] + vn[None]
    assert np.allclose(coarse.cbar(mu, nu, k, 2), ref, rtol=1e-12, atol=0)


def test_cmin_closed_form():
    N, d, k = 12, 2, 3
    n = N // k
    K = grid.coords(n, d)
    gap = np.maximum(0, k * np.abs(K[:, None] - K[None]) - (k - 1))
    for p in (1, 2):
        ref = ((gap ** 2).sum(-1)) ** (p / 2.0)
        assert np.allclose(coarse.cmin(N, d, k, p), ref, rtol=1e-15, atol=0)


# ---------------------------------------------------------------- LP

def test_lp_matches_assignment_brute_force():
    g = si.rng(30)
    n = 5
    C = g.uniform(0, 10, (n, n))
    a = np.full(n, 1.0 / n)
    r, c, v, f, gg, obj = lp.solve_ot(a, a, C)
    best = min(sum(C[i, s[i]] for i in range(n)) for s in itertools.permutations(range(n))) / n
    assert obj == pytest.approx(best, rel=1e-12)
    cert = lp.certify(r, c, v, f, gg, a, a, C)
    assert cert["dual_viol"] <= 1e-12 and cert["slack_on_support"] <= 1e-12
    assert cert["dual"] == pytest.approx(obj, rel=1e-12)


def test_northwest_corner_is_basic_coupling():
    g = si.rng(31)
    a = g.dirichlet(np.ones(7))
    b = g.dirichlet(np.ones(9))
    r, c, v = lp.northwest_corner(a, b)
    assert len(v) <= 7 + 9 - 1 and v.min() > 0
    assert np.allclose(np.bincount(r, v, 7), a, atol=1e-15)
    assert np.allclose(np.bincount(c, v, 9), b, atol=1e-15)


# ---------------------------------------------------------------- interpolation

def test_upscale_constant_and_centres():
    N, d, k = 15, 2, 3                      # odd k: block centres are pixels
    n = N // k
    ft = si.rng(40).standard_normal(n ** d)
    fh = lower.upscale_potential(ft, N, d, k).reshape(N, N)
    for K in range(n):
        for L in range(n):
            assert fh[k * K + 1, k * L + 1] == ft[K * n + L]
    assert np.all(lower.upscale_potential(np.full(n * n, 2.5), N, d, k) == 2.5)


def test_upscale_matches_np_interp_along_one_axis():
    N, k = 16, 4
    n = N // k
    prof = si.rng(41).standard_normal(n)
    ft = np.repeat(prof, n)                     # varies along axis 0 only
    fh = lower.upscale_potential(ft, N, 2, k).reshape(N, N)
    xc = np.arange(n) * k + (k - 1) / 2
    ref = np.interp(np.arange(N), xc, prof)     # np.interp clamps at both ends
    assert np.allclose(fh[:, 5], ref, rtol=0, atol=1e-14)


def test_upscale_bilinear_of_product_is_product():
    N, k = 16, 4
    n = N // k
    u = si.rng(42).standard_normal(n)
    v = si.rng(43).standard_normal(n)
    ft = np.outer(u, v).reshape(-1)
    fh = lower.upscale_potential(ft, N, 2, k).reshape(N, N)
    xc = np.arange(n) * k + (k - 1) / 2
    ref = np.outer(np.interp(np.arange(N), xc, u), np.interp(np.arange(N), xc, v))
    assert np.allclose(fh, ref, rtol=0, atol=1e-13)


def test_upscale_affine_is_exact_in_3d_interior():
    N, d, k = 8, 3, 2
    c = coarse.centres(N, d, k)
    beta = np.array([0.5, -1.25, 2.0])
    ft = 3.0 + c @ beta
    fh = lower.upscale_potential(ft, N, d, k)
    X = grid.coords(N, d).astype(float)
    inside = np.all((X >= c.min(0)) & (X <= c.max(0)), axis=1)
    assert np.allclose(fh[inside], 3.0 + X[inside] @ beta, rtol=0, atol=1e-13)


def test_upscale_nearest_is_own_block_by_brute_force():
    for N, d, k in [(12, 2, 3), (8, 3, 2), (10, 2, 5)]:
        n = N // k
        ft = si.rng(44).standard_normal(n ** d)
        fh = lower.upscale_potential(ft, N, d, k, "nearest")
        X = grid.coords(N, d)
        C = coarse.centres(N, d, k)
        for i in range(N ** d):
            dist = ((C - X[i]) ** 2).sum(1)
            K = int(np.argmin(dist))                    # nearest centre, unique
            assert np.sum(dist == dist[K]) == 1
            assert fh[i] == ft[K]


def _catmull_rom_hermite(F, t):
    """Independent 1-D form: cubic Hermite segment with tangents (F[i+1] - F[i-1]) / 2,
    edge samples replicated, t clamped to [0, n-1]."""
    n = len(F)
    t = min(max(t, 0.0), n - 1.0)
    i = min(int(math.floor(t)), n - 1)
    s = t - i
    at = lambda j: F[min(max(j, 0), n - 1)]
    m0 = (at(i + 1) - at(i - 1)) / 2.0
    m1 = (at(i + 2) - at(i)) / 2.0
    h00 = 2 * s ** 3 - 3 * s ** 2 + 1
    h10 = s ** 3 - 2 * s ** 2 + s
    h01 = -2 * s ** 3 + 3 * s ** 2
    h11 = s ** 3 - s ** 2
    return h00 * at(i) + h10 * m0 + h01 * at(i + 1) + h11 * m1


def test_upscale_cubic_matches_hermite_form_and_separates():
    N, k = 24, 4
    n = N // k
    u = si.rng(45).standard_normal(n)
    v = si.rng(46).standard_normal(n)
    t = (2 * np.arange(N) - (k - 1)) / (2 * k)
    cu = np.array([_catmull_rom_hermite(u, x) for x in t])
    cv = np.array([_catmull_rom_hermite(v, x) for x in t])
    fh = lower.upscale_potential(np.repeat(u, n), N, 2, k, "cubic").reshape(N, N)
    assert np.allclose(fh[:, 7], cu, rtol=0, atol=1e-13)          # varies along axis 0 only
    fh = lower.upscale_potential(np.outer(u, v).reshape(-1), N, 2, k, "cubic").reshape(N, N)
    assert np.allclose(fh, np.outer(cu, cv), rtol=0, atol=1e-12)  # tensor product


def test_upscale_cubic_interpolates_and_reproduces_quadratics():
    N, d, k = 15, 2, 3                      # odd k: block centres are pixels
    n = N // k
    ft = si.rng(47).standard_normal(n ** d)
    fh = lower.upscale_potential(ft, N, d, k, "cubic").reshape(N, N)
    for K in range(n):
        for L in range(n):
            assert fh[k * K + 1, k * L + 1] == ft[K * n + L]
    const = lower.upscale_potential(np.full(n * n, -7.25), N, d, k, "cubic")
    assert np.allclose(const, -7.25, rtol=4e-16, atol=0)
    # a quadratic in the coarse coordinates is reproduced wherever no tap is clamped
    for N, d, k in [(32, 2, 4), (18, 3, 3)]:
        n = N // k
        Cc = (coarse.centres(N, d, k) - (k - 1) / 2) / k          # coarse coordinates
        q = lambda Z: 0.5 + Z @ np.arange(1.0, d + 1) + 0.25 * (Z ** 2).sum(1) - 0.125 * Z[:, 0] * Z[:, -1]
        fh = lower.upscale_potential(q(Cc), N, d, k, "cubic")
        T = (2 * grid.coords(N, d) - (k - 1)) / (2 * k)
        inside = np.all((T >= 1) & (T <= n - 2), axis=1)
        assert inside.sum() > 0
        assert np.allclose(fh[inside], q(T[inside]), rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("interp", ["nearest", "cubic"])
def test_other_interpolants_keep_the_bound(interp):
    # any interpolation R keeps Algorithm 5 a lower bound (the proposition of
    # Section 3.5): bracketing of the exact LP, and exact admissibility in float32
    N, d, k, p = 8, 2, 2, 2
    mu, nu = pair(N, d, "gmm", "cauchy", 48)
    W = lp.wasserstein_exact(mu, nu, p)
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    L64 = lower.lower_bound_o64(mu, nu, ft, k, p, interp)
    L32 = lower.lower_bound_o32(mu, nu, ft, k, p, interp)
    assert L32["lower"] <= L64["lower"] * (1 + 1e-12) <= W * (1 + 1e-12)
    X = grid.coords(N, d)
    Cm = grid.cost64(X, X, p)
    f = L32["f32"].astype(np.float64) - L32["shift"]
    g = L32["g32"].astype(np.float64)
    assert np.all(f[:, None] + g[None, :] <= Cm)
    Llin = lower.lower_bound_o64(mu, nu, ft, k, p)
    assert L64["lower"] != Llin["lower"]


# ---------------------------------------------------------------- c-transform

@pytest.mark.parametrize("N,d,p", [(4, 2, 2), (4, 2, 1), (3, 3, 2), (3, 3, 1)])
def test_ctransform_brute_force(N, d, p):
    X = grid.coords(N, d)
    P = len(X)
    phi = si.rng(50 + p).standard_normal(P) * 3
    phi32 = phi.astype(np.float32)
    g64, i64 = lower.ctransform_o64(phi, N, d, p)
    g32, i32 = lower.ctransform_o32(phi32, N, d, p)
    for j in range(P):
        vals64, vals32 = [], []
        for i in range(P):
            d2 = sum((int(X[i, a]) - int(X[j, a])) ** 2 for a in range(d))
            c = math.sqrt(d2) if p == 1 else float(d2)
            vals64.append(c - phi[i])
            vals32.append(np.float32(np.float32(c) - phi32[i]))
        assert g64[j] == min(vals64) and i64[j] == int(np.argmin(vals64))
        assert g32[j] == min(vals32) and i32[j] == int(np.argmin(vals32))


def test_ctransform_zero_potential():
    for p in (1, 2):
        g, _ = lower.ctransform_o32(np.zeros(64, np.float32), 8, 2, p)
        assert np.all(g == 0)


def test_ctransform_of_linear_potential_p2():
    # phi_i = -2<x_i, t>: min_x |x - y|^2 + 2<x, t> = 2<y, t> - |t|^2, attained
    # at x = y - t whenever that point is on the grid.
    N, d = 12, 2
    t = np.array([2, -3])
    X = grid.coords(N, d)
    phi = (-2.0 * (X @ t)).astype(np.float32)
    g, arg = lower.ctransform_o32(phi, N, d, 2)
    inside = np.all((X - t >= 0) & (X - t < N), axis=1)
    assert np.array_equal(g[inside], (2.0 * (X[inside] @ t) - t @ t).astype(np.float32))


def test_ctransform_of_distance_potential_p1():
    # phi_i = -|x_i - z|: min_x |x - y| + |x - z| = |y - z| (triangle inequality).
    N, d = 10, 2
    X = grid.coords(N, d)
    z = np.array([3, 7])
    phi = -np.sqrt(((X - z) ** 2).sum(1))
    g, _ = lower.ctransform_o64(phi, N, d, 1)
    assert np.allclose(g, np.sqrt(((X - z) ** 2).sum(1)), rtol=0, atol=1e-12)


def test_ctransform_tie_goes_to_lowest_index():
    N, d = 6, 2
    X = grid.coords(N, d)
    j, i1, i2 = 14, 3, 29
    c = grid.cost32(X, X[[j]], 2)[:, 0]
    phi = np.zeros(N * N, np.float32)
    phi[i1] = c[i1] + 100
    phi[i2] = c[i2] + 100
    g, arg = lower.ctransform_o32(phi, N, d, 2, targets=[j])
    assert g[0] == -100 and arg[0] == i1


def test_double_ctransform_properties():
    N, d, p = 8, 2, 2
    fhat = si.rng(60).standard_normal(N * N) * 20
    g, _ = lower.ctransform_o64(fhat, N, d, p)
    f, _ = lower.ctransform_o64(g, N, d, p)
    assert np.all(f >= fhat - 1e-12)                  # f = fhat^cc >= fhat
    g2, _ = lower.ctransform_o64(f, N, d, p)
    assert np.allclose(g2, g, rtol=0, atol=1e-12)     # f^ccc = f^c


# ---------------------------------------------------------------- lower bound

@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("fams,seed", [(("gmm", "gmm"), 70), (("white_noise", "shapes"), 72),
                                       (("cauchy", "grf"), 74)])
def test_lower_bound_brackets_exact(p, fams, seed):
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, *fams, seed)
    W = lp.wasserstein_exact(mu, nu, p)
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    L64 = lower.lower_bound_o64(mu, nu, ft, k, p)
    L32 = lower.lower_bound_o32(mu, nu, ft, k, p)
    assert L64["lower"] <= W * (1 + 1e-12)
    assert L32["S_emit"] <= L64["S"]
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    assert U["upper"] >= W * (1 - 1e-12)


def test_lower_bound_is_exact_at_k1():
    # k = 1: the coarse problem is the fine one; the optimal dual gives L_C.
    N, d, p = 8, 2, 2
    mu, nu = pair(N, d, "gmm", "grf", 80)
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, 1, p)
    L = lower.lower_bound_o64(mu, nu, ft, 1, p)
    assert L["S"] == pytest.approx(obj, rel=1e-10)
    U = upper.upper_bound_o64(mu, nu, r, c, v, 1, p)
    assert U["plan_cost"] == pytest.approx(obj, rel=1e-12)


@pytest.mark.parametrize("p", [1, 2])
def test_feasibility_shift_gives_admissible_pair(p):
    N, d, k = 16, 2, 4
    for seed in (90, 92):
        mu, nu = pair(N, d, "grf", "cauchy", seed)
        *_, ft, gt, _ = upper.coarse_record_lp(mu, nu, k, p)
        ft = ft + 1e4 * (seed - 91)            # large offsets stress float32 rounding
        L32 = lower.lower_bound_o32(mu, nu, ft, k, p)
        L64 = lower.lower_bound_o64(mu, nu, ft, k, p)
        X = grid.coords(N, d)
        C = grid.cost64(X, X, p)
        f = L32["f32"].astype(np.float64) - L32["shift"]
        g = L32["g32"].astype(np.float64)
        assert (f[:, None] + g[None, :] - C).max() <= 0.0
        # the derived per-transform error bounds hold
        u, up = 2.0 ** -24, (2.0 ** -24 if p == 1 else 0.0)
        F = np.abs(L32["fhat32"]).max() * (1 + 2 * u)
        G = np.abs(L32["g32"]).max()
        Fo = np.abs(L32["f32"]).max()
        e_g = (u + up) * (G + F)
        assert np.abs(L32["g32"] - L64["g"]).max() <= e_g
        assert np.abs(L32["f32"] - L64["f"]).max() <= u * Fo + up * (Fo + G) + e_g
        assert L32["S_emit"] <= L64["S"]


# ---------------------------------------------------------------- upper bound

def test_upper_bound_plan_properties_and_identity():
    N, d, k, p = 16, 2, 4, 2
    mu, nu = pair(N, d, "gmm", "shapes", 100)
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    I, J, V = upper.upscale_plan(r, c, v, N, d, k)
    Q = (N // k) ** d
    assert len(V) <= k ** (2 * d) * (2 * Q - 1)
    assert math.isclose(V.sum(), 1.0, rel_tol=1e-14)
    fitted = U["a"][I] * V * U["b"][J]
    P = N ** d
    assert np.abs(np.bincount(I, fitted, P) - mu.reshape(-1)).sum() < 1e-12
    assert np.abs(np.bincount(J, fitted, P) - nu.reshape(-1)).sum() < 1e-12
    # uniform kernel: the fitted plan is the quantization coupling, whose cost is <pi~, C-bar>
    Cb = coarse.cbar(mu, nu, k, p)
    assert U["plan_cost"] == pytest.approx(float((Cb[r, c] * v).sum()), rel=1e-12)
    assert U["plan_cost"] == pytest.approx(upper.quantization_coupling_cost(mu, nu, r, c, v, k, p), rel=1e-12)
    assert U["iters"] == 1


@pytest.mark.parametrize("p", [1, 2])
def test_tv_terms_bounded_and_upper_bound_valid_when_not_converged(p):
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, "grf", "gmm", 110)
    W = lp.wasserstein_exact(mu, nu, p)
    g = si.rng(111)
    mt = coarse.sumpool(mu, k) * np.exp(0.3 * g.standard_normal(16))
    nt = coarse.sumpool(nu, k)
    r, c, v = lp.northwest_corner(mt / mt.sum(), nt)       # a coupling of the wrong marginals
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p, xi=1e-12, max_iter=1)
    assert U["residual"] > 1e-3 and U["tv_mu"] + U["tv_nu"] > 0
    rad = math.sqrt(d) * (N - 1) / 2.0
    assert U["tv_mu"] + U["tv_nu"] <= 2 ** (2 - 2 / p) * U["residual"] ** (1 / p) * rad
    assert U["upper"] >= W


def test_fitting_matvec_is_within_one_rounding_of_the_exact_sum():
    # The fitting passes' sums (pi^ x) against math.fsum of the same rounded
    # products (the correctly rounded sum): at most one unit in the last place
    # apart, with 1..700 terms per output of mixed magnitudes.
    g = si.rng(9990)
    n = 300
    counts = g.integers(1, 700, size=n)
    I = np.repeat(np.arange(n), counts)
    g.shuffle(I)
    E = len(I)
    J = g.integers(0, 5000, size=E)
    V = g.random(E) * 10.0 ** g.integers(-8, 0, size=E)
    x = g.random(5000) * 10.0 ** g.integers(-3, 3, size=5000)
    mv = upper._matvec(I, J, V, x, n)
    prod = V * x[J]
    for i in range(n):
        ref = math.fsum(prod[I == i].tolist())
        assert abs(mv[i] - ref) <= math.ulp(ref), i


def _dist_to_grid_mean(i, N, d):
    """|x_i - x-bar| for the C-order flat index i, x-bar = ((N-1)/2, ...),
    written out here from the index arithmetic (not through the oracle)."""
    u = np.array(np.unravel_index(int(i), (N,) * d), dtype=np.float64)
    return math.sqrt(float(((u - (N - 1) / 2.0) ** 2).sum()))


@pytest.mark.parametrize("N,d", [(9, 2), (8, 2), (5, 3), (6, 3)])
@pytest.mark.parametrize("p", [1, 2])
def test_tv_of_two_moved_masses_closed_form(N, d, p):
    # Equation of the weighted total variation with the weights of Algorithm 4,
    # w_i = rho(x-bar, x_i)^p: when mu^ - mu = eps (delta_x - delta_y),
    # TV_p^w(mu^, mu) = 2^(1-1/p) (eps (|x - x-bar|^p + |y - x-bar|^p))^(1/p).
    # Weights without the power p, or a missing 2^(1-1/p), change the value.
    g = si.rng(9900 + 10 * N + d + p)
    P = N ** d
    w = upper.tv_weights(N, d, p)
    for _ in range(6):
        i, j = (int(t) for t in g.choice(P, 2, replace=False))
        base = np.floor(g.random(P) * 2 ** 20) / 2 ** 20       # dyadic: the differences below are exact
        eps = float(g.integers(1, 2 ** 20)) / 2 ** 30
        mu_hat = base.copy()
        mu_hat[i] += eps
        mu_hat[j] -= eps
        ri, rj = _dist_to_grid_mean(i, N, d), _dist_to_grid_mean(j, N, d)
        ref = 2.0 ** (1 - 1 / p) * (eps * (ri ** p + rj ** p)) ** (1 / p)
        assert upper.weighted_tv(w, mu_hat, base, p) == pytest.approx(ref, rel=1e-13, abs=0)
        assert upper.weighted_tv(w, base, mu_hat, p) == pytest.approx(ref, rel=1e-13, abs=0)


@pytest.mark.parametrize("N,d", [(7, 2), (5, 3)])
@pytest.mark.parametrize("p", [1, 2])
def test_tv_is_tight_for_diracs_opposite_about_the_grid_mean(N, d, p):
    # Odd N puts x-bar on a pixel.  For y and z = 2 x-bar - y,
    # W_p(delta_y, delta_z) = |y - z| = 2 r and TV_p^w = 2^(1-1/p) (r^p + r^p)^(1/p)
    # = 2 r: the bound W_p <= TV_p^w holds with equality (exact LP on the full
    # grid), which fixes both the power p in the weights and 2^(1-1/p).  For a
    # Dirac at x-bar itself TV_p^w(delta_x, delta_x-bar) = 2^(1-1/p) |x - x-bar|.
    P = N ** d
    g = si.rng(9950 + N + d + p)
    w = upper.tv_weights(N, d, p)
    c = (N - 1) // 2
    for _ in range(3):
        y = g.integers(0, N, size=d)
        if np.all(y == c):
            y[0] = 0
        z = 2 * c - y
        iy, iz = np.ravel_multi_index(tuple(y), (N,) * d), np.ravel_multi_index(tuple(z), (N,) * d)
        my, mz = np.zeros(P), np.zeros(P)
        my[iy] = 1.0
        mz[iz] = 1.0
        r = _dist_to_grid_mean(iy, N, d)
        W = lp.wasserstein_exact(my.reshape((N,) * d), mz.reshape((N,) * d), p)
        tv = upper.weighted_tv(w, my, mz, p)
        assert W == pytest.approx(2 * r, rel=1e-12)
        assert tv == pytest.approx(2 * r, rel=1e-12)
        mc = np.zeros(P)
        mc[np.ravel_multi_index((c,) * d, (N,) * d)] = 1.0
        assert upper.weighted_tv(w, my, mc, p) == pytest.approx(2.0 ** (1 - 1 / p) * r, rel=1e-12)


@pytest.mark.parametrize("N,d", [(8, 2), (4, 3)])
@pytest.mark.parametrize("p", [1, 2])
def test_wasserstein_below_weighted_tv_by_exact_lp(N, d, p):
    # The property behind the equation of the weighted total variation:
    # W_p(mu, nu) <= TV_p^w(mu, nu) for any pair, here by the exact LP.
    w = upper.tv_weights(N, d, p)
    for s, (fa, fb) in enumerate([("grf", "gmm"), ("white_noise", "cauchy"), ("shapes", "grf")]):
        mu, nu = pair(N, d, fa, fb, 9970 + 10 * s + d + p)
        W = lp.wasserstein_exact(mu, nu, p)
        tv = upper.weighted_tv(w, mu.reshape(-1), nu.reshape(-1), p)
        assert W <= tv * (1 + 1e-12)


def test_ordering_of_the_four_bounds():
    N, d, k, p = 16, 2, 4, 2
    mu, nu = pair(N, d, "gmm", "gmm", 120)
    W = lp.wasserstein_exact(mu, nu, p)
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    lo_min = upper.min_cost_lower(mu, nu, k, p)
    up_wc = upper.weighted_cost_upper(mu, nu, k, p)
    up_pu = upper.upper_bound_o64(mu, nu, r, c, v, k, p)["upper"]
    assert lo_min <= W <= up_wc * (1 + 1e-12)
    assert up_wc <= up_pu * (1 + 1e-12)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("p", [1, 2])
def test_closed_forms_match_exact_lp(p):
    N, d = 12, 2
    mu, nu = si.translated_pair(N, d, (2, -3), si.rng(130))
    assert lp.wasserstein_exact(mu, nu, p) == pytest.approx(math.sqrt(13), rel=1e-9)
    a, b = si.axis_constant_pair(N, d, si.rng(131))
    assert lp.wasserstein_exact(a, b, p) == pytest.approx(closed.axis_constant_w(a, b, p), rel=1e-9)
    m1, m2, x, y = si.dirac_pair(N, d, si.rng(132))
    assert lp.wasserstein_exact(m1, m2, p) == pytest.approx(float(np.linalg.norm(x - y)), rel=1e-12)


def test_w1d_against_scipy():
    import scipy.stats
    g = si.rng(140)
    a, b = g.dirichlet(np.ones(30)), g.dirichlet(np.ones(30))
    x = np.arange(30)
    assert closed.w1d(a, b, 1) == pytest.approx(scipy.stats.wasserstein_distance(x, x, a, b), rel=1e-12)


def test_identical_measures():
    N, d, k, p = 16, 2, 4, 2
    mu = si.grf(N, d, si.rng(150))
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, mu, k, p)
    L = lower.lower_bound_o32(mu, mu, ft, k, p)
    assert L["lower"] == 0.0 and L["clipped"]
    U = upper.upper_bound_o64(mu, mu, r, c, v, k, p)
    assert U["upper"] >= 0.0


# ---------------------------------------------------------------- gradients

def _mass_preserving_direction(m, g, block_k=None):
    v = g.uniform(-1, 1, m.shape)
    if block_k is None:
        v -= (m * v).sum() / m.sum()
    else:
        # remove the mu-weighted mean inside every block: block masses unchanged
        d, N = m.ndim, m.shape[0]
        blk = coarse.block_of(N, d, block_k).reshape(m.shape)
        Q = (N // block_k) ** d
        mw = np.bincount(blk.reshape(-1), (m * v).reshape(-1), Q)
        ms = np.bincount(blk.reshape(-1), m.reshape(-1), Q)
        v -= (mw / ms)[blk]
    return v / np.abs(v).max()


def test_lower_bound_gradient_matches_full_pipeline_fd():
    N, d, k, p = 16, 2, 4, 2
    mu, nu = pair(N, d, "gmm", "grf", 160)
    g = si.rng(161)
    _, _, _, ft, _, _ = upper.coarse_record_lp(mu, nu, k, p)
    L = lower.lower_bound_o64(mu, nu, ft, k, p)
    gm, gn = ograd.lower_grad(L["f"], L["g"], L["S"], p)
    v = _mass_preserving_direction(mu, g, block_k=k)
    h = 1e-4

    def full(m):  # re-solves the coarse problem: block masses unchanged -> same solution
        _, _, _, f2, _, _ = upper.coarse_record_lp(m, nu, k, p)
        return lower.lower_bound_o64(m, nu, f2, k, p)["lower"]

    fd = (full(mu * (1 + h * v)) - full(mu * (1 - h * v))) / (2 * h)
    assert fd == pytest.approx(float((gm * (mu * v).reshape(-1)).sum()), rel=1e-6)


@pytest.mark.parametrize("p", [1, 2])
def test_upper_bound_gradient_matches_fd(p):
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, "gmm", "gmm", 170 + p)
    r, c, v, *_ = upper.coarse_record_lp(mu, nu, k, p)
    # a perturbed coupling makes the fitting take several iterations
    v = v * np.exp(0.2 * si.rng(172).standard_normal(len(v)))
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    T = U["iters"]
    assert T >= 2
    gm, gn, val = ograd.upper_grad(mu, nu, r, c, v, k, p, T)
    assert val == pytest.approx(U["plan_cost"] ** (1 / p), rel=1e-12)
    g = si.rng(173)
    h = 1e-4

    def W(m, n):
        U2 = upper.upper_bound_o64(m, n, r, c, v, k, p, xi=-1.0, max_iter=T)
        return U2["plan_cost"] ** (1 / p)

    for _ in range(2):
        vm, vn = _mass_preserving_direction(mu, g), _mass_preserving_direction(nu, g)
        fd = (W(mu * (1 + h * vm), nu * (1 + h * vn)) - W(mu * (1 - h * vm), nu * (1 - h * vn))) / (2 * h)
        an = float((gm * (mu * vm).reshape(-1)).sum() + (gn * (nu * vn).reshape(-1)).sum())
        assert fd == pytest.approx(an, rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------- separable c-transform (p = 2)

@pytest.mark.parametrize("N,d", [(12, 2), (7, 3), (32, 2)])
def test_separable_equals_all_pairs_without_rounding(N, d):
    # integer potentials below 2^20: every float32 operation is exact in both
    # evaluations, so values and arg-mins (lowest flat index) coincide
    phi = si.rng(300 + N).integers(-(2 ** 19), 2 ** 19, N ** d).astype(np.float32)
    phi[::5] = phi[0]                                    # plenty of ties
    g1, a1 = lower.ctransform_sep_o32(phi, N, d)
    g2, a2 = lower.ctransform_o32(phi, N, d, 2)
    assert np.array_equal(g1, g2) and np.array_equal(a1, a2)


def test_separable_brute_force_tiny():
    N, d = 5, 2
    phi = (si.rng(310).standard_normal(N * N) * 7).astype(np.float32)
    g, a = lower.ctransform_sep_o32(phi, N, d)
    P = phi.reshape(N, N)
    for u in range(N):
        for v in range(N):
            h = [min(np.float32(np.float32((t - v) ** 2) - P[s, t]) for t in range(N)) for s in range(N)]
            vals = [np.float32(np.float32((s - u) ** 2) + h[s]) for s in range(N)]
            assert g[u * N + v] == min(vals)
            s_star = int(np.argmin(vals))
            row = [np.float32(np.float32((t - v) ** 2) - P[s_star, t]) for t in range(N)]
            assert a[u * N + v] == s_star * N + int(np.argmin(row))


@pytest.mark.parametrize("N,d", [(16, 2), (8, 3)])
def test_separable_error_bounds_and_feasibility(N, d):
    k = 4 if d == 2 else 2
    mu, nu = pair(N, d, "grf", "cauchy", 320 + N)
    *_, ft, gt, _ = upper.coarse_record_lp(mu, nu, k, 2)
    ft = ft + 3e3                               # offsets stress the rounding
    Ls = lower.lower_bound_sep_o32(mu, nu, ft, k)
    L64 = lower.lower_bound_o64(mu, nu, ft, k, 2)
    u = 2.0 ** -24
    C = d * (N - 1) ** 2
    F = np.abs(Ls["fhat32"]).max() * (1 + 2 * u)
    G = np.abs(Ls["g32"]).max()
    Fo = np.abs(Ls["f32"]).max()
    e_g = u * (F + d * G + (d - 1) * C)
    assert np.abs(Ls["g32"] - L64["g"]).max() <= e_g
    assert np.abs(Ls["f32"] - L64["f"]).max() <= u * (d * Fo + (d - 1) * C) + e_g
    X = grid.coords(N, d)
    Cm = grid.cost64(X, X, 2)
    f = Ls["f32"].astype(np.float64) - Ls["shift"]
    assert (f[:, None] + Ls["g32"].astype(np.float64)[None, :] - Cm).max() <= 0.0
    assert Ls["S_emit"] <= L64["S"]


# ---------------------------------------------------------------- upscaling kernels (Section 3.4)

def _random_coupling(N, d, k, g):
    n = N // k
    mt = g.uniform(0.1, 1.0, n ** d)
    nt = g.uniform(0.1, 1.0, n ** d)
    return lp.northwest_corner(mt / mt.sum(), nt / nt.sum())


def _kron_plan(r, c, v, N, d, k, Km):
    """The upscaled coupling by the paper's definition: the coarse coupling as a
    2d-tensor, Kronecker product with the kernel as a 2d-tensor, reshaped."""
    n = N // k
    Pt = np.zeros((n ** d, n ** d))
    np.add.at(Pt, (np.asarray(r), np.asarray(c)), v)
    big = np.kron(Pt.reshape((n,) * (2 * d)), np.asarray(Km).reshape((k,) * (2 * d)))
    return big.reshape(N ** d, N ** d)


@pytest.mark.parametrize("N,d,k", [(6, 2, 3), (8, 2, 2), (4, 3, 2)])
def test_kernel_upscale_is_the_kronecker_product(N, d, k):
    g = si.rng(600 + N + d)
    r, c, v = _random_coupling(N, d, k, g)
    for Km in (si.random_plan_kernel(k, d, g), si.random_plan_kernel(k, d, g, zero_frac=0.5),
               np.full((k ** d, k ** d), float(k) ** (-2 * d))):
        I, J, V = upper.upscale_plan(r, c, v, N, d, k, Km)
        dense = np.zeros((N ** d, N ** d))
        np.add.at(dense, (I, J), V)
        assert np.allclose(dense, _kron_plan(r, c, v, N, d, k, Km), rtol=1e-15, atol=0)
    I, J, V = upper.upscale_plan(r, c, v, N, d, k)
    dense = np.zeros((N ** d, N ** d))
    np.add.at(dense, (I, J), V)
    assert np.allclose(dense, _kron_plan(r, c, v, N, d, k, np.full((k ** d,) * 2, float(k) ** (-2 * d))),
                       rtol=1e-15, atol=0)


def test_kernel_plan_is_a_coupling_of_block_consistent_marginals():
    # the lemma on normalised kernels: pi^ >= 0 with total 1, and every block of
    # its marginals carries the coarse coupling's marginal
    N, d, k = 12, 2, 3
    g = si.rng(610)
    r, c, v = _random_coupling(N, d, k, g)
    Km = si.random_plan_kernel(k, d, g, zero_frac=0.3)
    I, J, V = upper.upscale_plan(r, c, v, N, d, k, Km)
    assert (V >= 0).all() and math.isclose(V.sum(), 1.0, rel_tol=1e-14)
    blk = coarse.block_of(N, d, k)
    Q = (N // k) ** d
    row = np.bincount(blk[I], V, Q)
    col = np.bincount(blk[J], V, Q)
    assert np.allclose(row, np.bincount(r, v, Q), rtol=1e-13, atol=1e-16)
    assert np.allclose(col, np.bincount(c, v, Q), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("p", [1, 2])
def test_uniform_kernel_given_explicitly_is_algorithm_4(p):
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, "grf", "gmm", 620 + p)
    r, c, v, *_ = upper.coarse_record_lp(mu, nu, k, p)
    v = v * np.exp(0.2 * si.rng(622).standard_normal(len(v)))   # several IPF iterations
    U0 = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    U1 = upper.upper_bound_o64(mu, nu, r, c, v, k, p, kernel=np.full((k ** d,) * 2, float(k) ** (-2 * d)))
    assert U0["iters"] == U1["iters"] and U0["iters"] >= 2
    assert U1["plan_cost"] == pytest.approx(U0["plan_cost"], rel=1e-13)
    assert U1["upper"] == pytest.approx(U0["upper"], rel=1e-12)


def _permuted_translation(N, d, k, shift_blocks, g):
    """mu random on the blocks whose translate by ``shift_blocks`` stays on the
    grid; nu moves pixel (block K, offset s) to (block K + shift, offset
    s + 1 mod k^d).  Returns mu, nu, the pixel map and the block map."""
    n, m = N // k, k ** d
    mu = np.zeros((N,) * d)
    nu = np.zeros((N,) * d)
    sigma = {}
    blocks = {}
    for Kv in itertools.product(range(n), repeat=d):
        Lv = tuple(a + b for a, b in zip(Kv, shift_blocks))
        if not all(0 <= x < n for x in Lv):
            continue
        Kf = int(np.ravel_multi_index(Kv, (n,) * d))
        Lf = int(np.ravel_multi_index(Lv, (n,) * d))
        blocks[Kf] = Lf
        for s in range(m):
            off = np.unravel_index(s, (k,) * d)
            toff = np.unravel_index((s + 1) % m, (k,) * d)
            x = tuple(kk * k + o for kk, o in zip(Kv, off))
            y = tuple(ll * k + o for ll, o in zip(Lv, toff))
            w = g.uniform(0.2, 1.0)
            mu[x] = w
            nu[y] = w
            sigma[np.ravel_multi_index(x, (N,) * d)] = np.ravel_multi_index(y, (N,) * d)
    tot = mu.sum()
    return mu / tot, nu / tot, sigma, blocks


@pytest.mark.parametrize("N,d,k,shift", [(8, 2, 2, (1, 1)), (12, 2, 3, (0, 2)), (4, 3, 2, (1, 0, 1))])
@pytest.mark.parametrize("p", [1, 2])
def test_permutation_kernel_is_exact_on_permuted_translation(N, d, k, shift, p):
    # closed form: with the kernel that sends offset s to offset s + 1 (mod k^d)
    # and the block translation as coarse coupling, the upscaled coupling is the
    # pixel map itself; IPF stops after one iteration and the bound is that
    # map's cost, with no TV correction.  The transposed kernel cannot fit.
    g = si.rng(630 + N + p)
    mu, nu, sigma, blocks = _permuted_translation(N, d, k, shift, g)
    m = k ** d
    Km = np.zeros((m, m))
    Km[np.arange(m), (np.arange(m) + 1) % m] = 1.0 / m
    mt = coarse.sumpool(mu, k)
    rows = np.array(sorted(blocks), dtype=np.int64)
    cols = np.array([blocks[K] for K in rows], dtype=np.int64)
    vals = mt[rows]
    U = upper.upper_bound_o64(mu, nu, rows, cols, vals, k, p, kernel=Km)
    X = grid.coords(N, d)
    muf = mu.reshape(-1)
    cost = 0.0
    for i, j in sigma.items():
        dd = float(((X[i] - X[j]) ** 2).sum())
        cost += muf[i] * (dd if p == 2 else math.sqrt(dd))
    assert U["iters"] == 1
    assert U["plan_cost"] == pytest.approx(cost, rel=1e-13)
    assert U["residual"] < 1e-14
    assert U["upper"] == pytest.approx(cost ** (1.0 / p), rel=1e-6)
    Ut = upper.upper_bound_o64(mu, nu, rows, cols, vals, k, p, kernel=Km.T.copy(), max_iter=5)
    assert Ut["residual"] > 0.1


def test_gaussian_plan_kernel_factorises_over_axes():
    for k, d, sigma in [(4, 2, 1.0), (3, 3, 0.7), (8, 2, 2.5)]:
        Km = upper.plan_kernel_gaussian(k, d, sigma)
        u = np.arange(k, dtype=np.float64)
        g1 = np.exp(-(u[:, None] - u[None, :]) ** 2 / (2 * sigma ** 2))
        ref = g1
        for _ in range(d - 1):
            ref = np.kron(ref, g1)
        assert np.allclose(Km, ref / ref.sum(), rtol=1e-14, atol=0)
        assert math.isclose(Km.sum(), 1.0, rel_tol=1e-14) and np.allclose(Km, Km.T, rtol=0, atol=0)
    assert np.allclose(upper.plan_kernel_gaussian(4, 2, 1e6), 1.0 / 256, rtol=1e-9)


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("which", ["gaussian", "random"])
def test_kernel_upper_bound_brackets_exact(p, which):
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, "gmm", "cauchy", 640 + p)
    W = lp.wasserstein_exact(mu, nu, p)
    r, c, v, *_ = upper.coarse_record_lp(mu, nu, k, p)
    Km = upper.plan_kernel_gaussian(k, d, 1.0) if which == "gaussian" else \
        si.random_plan_kernel(k, d, si.rng(642), zero_frac=0.3)
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p, kernel=Km, max_iter=200)
    assert U["iters"] > 1
    assert U["upper"] >= W * (1 - 1e-12)
    I, J, V = upper.upscale_plan(r, c, v, N, d, k, Km)
    fitted = U["a"][I] * V * U["b"][J]
    P = N ** d
    err = np.abs(np.bincount(I, fitted, P) - mu.reshape(-1)).sum() + \
        np.abs(np.bincount(J, fitted, P) - nu.reshape(-1)).sum()
    assert err == pytest.approx(U["residual"], rel=1e-6, abs=1e-15)


@pytest.mark.parametrize("p", [1, 2])
def test_kernel_upper_bound_gradient_matches_fd(p):
    N, d, k = 8, 2, 2
    mu, nu = pair(N, d, "gmm", "grf", 650 + p)
    r, c, v, *_ = upper.coarse_record_lp(mu, nu, k, p)
    Km = si.random_plan_kernel(k, d, si.rng(652))
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p, kernel=Km, max_iter=6)
    T = U["iters"]
    gm, gn, val = ograd.upper_grad(mu, nu, r, c, v, k, p, T, kernel=Km)
    assert val == pytest.approx(U["plan_cost"] ** (1 / p), rel=1e-12)
    g = si.rng(653)
    h = 1e-4

    def W(m_, n_):
        U2 = upper.upper_bound_o64(m_, n_, r, c, v, k, p, xi=-1.0, max_iter=T, kernel=Km)
        return U2["plan_cost"] ** (1 / p)

    for _ in range(2):
        vm, vn = _mass_preserving_direction(mu, g), _mass_preserving_direction(nu, g)
        fd = (W(mu * (1 + h * vm), nu * (1 + h * vn)) - W(mu * (1 - h * vm), nu * (1 - h * vn))) / (2 * h)
        an = float((gm * (mu * vm).reshape(-1)).sum() + (gn * (nu * vn).reshape(-1)).sum())
        assert fd == pytest.approx(an, rel=1e-6, abs=1e-9)


def _rn32(q):
    """Correctly rounded float32 of an exact rational (ties to even)."""
    from fractions import Fraction
    f = np.float32(float(q))             # within an ulp; fix the last step exactly
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        if not np.isfinite(c):
            continue
        e = abs(Fraction(float(c)) - q)
        even = (int(np.array(c, dtype=np.float32).view(np.uint32)) & 1) == 0
        key = (e, not even)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


@pytest.mark.parametrize("N,d,kind", [(6, 2, "normal"), (5, 3, "normal"), (7, 2, "lattice"), (4, 3, "lattice")])
def test_all_pairs_float32_transform_is_rounded_exact_separable_minimum(N, d, kind):
    # The float32 all-pairs reading min_x RN32(c - phi) equals RN32 of the exact
    # minimum of c - phi (rounding is monotone), and for p = 2 that exact
    # minimum is a nest of per-axis minima: the basis of the exact separable
    # evaluation.  Exact rationals throughout.
    from fractions import Fraction
    r = si.rng(31000 + N + d)
    P = N ** d
    if kind == "normal":
        phi = (r.standard_normal(P) * N * N / 4).astype(np.float32)
    else:
        phi = (r.integers(-64 * N * N, 64 * N * N, P) / 64.0).astype(np.float32)
    ref, _ = lower.ctransform_o32(phi, N, d, 2)
    F = np.array([Fraction(float(v)) for v in phi], dtype=object).reshape((N,) * d)
    # nested exact minima, last axis first: H = min over x_a of (x_a - y_a)^2 + H
    H = -F
    for a in reversed(range(d)):
        sh = list(H.shape)
        out = np.empty(sh, dtype=object)
        for idx in itertools.product(*[range(s) for s in sh]):
            y = idx[a]
            out[idx] = min(Fraction((x - y) ** 2) + H[idx[:a] + (x,) + idx[a + 1:]] for x in range(N))
        H = out
    got = np.array([_rn32(v) for v in H.reshape(-1)], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
