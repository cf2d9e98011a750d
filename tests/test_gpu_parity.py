"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances:
* float32 values and arg-mins of the c-transform, the upscaled potential:
  bit-exact against the oracle's float32 reading;
* float64 sums (lower bound, plan cost, pooled masses, C-bar): relative 1e-9
  or tighter;
* upper bound: the plan-cost part to 1e-9 relative; the total-variation terms
  are square roots (p = 2) of rounding-level sums, so the emitted upper bound
  must lie in [oracle, oracle + the room `ub_tol` derives from the library's
  rounding allowance].
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import coarse, grid, lower, lp, upper
from oracle import grad as ograd

pytestmark = pytest.mark.gpu

qbw = pytest.importorskip("paper_2506_00976_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qbw.load()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device="cuda:0")


def pair(N, d, fa, fb, seed):
    return si.family(fa, N, d, si.rng(seed)), si.family(fb, N, d, si.rng(seed + 1))


def record(mu, nu, k, p):
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    return qbw.Coarse(r, c, v, ft, gt, obj), (r, c, v, ft, gt, obj)


def ub_tol(mu, nu, N, d, p, k, ub, rows, cols, iters):
    """Room above the oracle's upper bound.  Inside each weighted-TV term the
    library adds e u (<w, mu> + T), e bounding the relative error of the fitted
    marginals after `iters` iterations against exact arithmetic, for its own
    iteration (longest coupling row r and column c, pooled block sums s_p additions deep)
    plus a float64 reference's (14 T); allowed here: twice that inside the
    root, on top of 1e-9 relative for the float64 sums."""
    w = upper.tv_weights(N, d, p)
    Mw = max(float(w @ mu.reshape(-1)), float(w @ nu.reshape(-1)))
    r = int(np.bincount(np.asarray(rows)).max())
    c = int(np.bincount(np.asarray(cols)).max())
    m = k ** d
    if k <= 64:   # the pooled block sums' depth (strips of blocks, row groups, the block's columns)
        Wc = min((256 // k) * k, N)
        RG = 256 // Wc
        s_pool = -(-k ** (d - 1) // RG) - 1 + (RG - 1) + (k - 1)
    else:         # lane groups: every g-th pixel, then a butterfly
        g = 64
        s_pool = -(-m // g) - 1 + 6
    T = max(1, int(iters))
    e = 2 * (r + 2) + (2 * T - 1) * (r + c + 2 * s_pool + 6) + 2 + 14 * T
    c1 = 2.0 ** (1 - 1 / p)
    return 1e-9 * ub + 2 * c1 * (2 * e * 2.0 ** -53 * Mw) ** (1 / p)


# ------------------------------------------------------------------ c-transform

CT_CASES = [(32, 2, 2), (32, 2, 1), (16, 3, 2), (16, 3, 1), (24, 2, 2), (20, 2, 1), (15, 2, 2),
            (9, 3, 1), (64, 2, 2)]


@pytest.mark.parametrize("N,d,p", CT_CASES)
def test_ctransform_bit_exact(N, d, p):
    P = N ** d
    phi = (si.rng(7000 + N + p).standard_normal(P) * N * N / 4).astype(np.float32)
    out, arg = qbw.ctransform(dev(phi), N, d, p, want_argmin=True)
    ref, refarg = lower.ctransform_o32(phi, N, d, p)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(arg.cpu().numpy().astype(np.int64), refarg)


# p = 1 costs through the LDS table of each target row (targets per lane R =
# 32, 16, 8, 4; several lanes per row, rows per wave, 2D and 3D), and the
# direct square-root path where the wave does not cover whole rows.  Rows of
# the table come from the context's square-root table where d (N-1)^2 is
# small (up to 128^2 and 32^3 here) and are computed above that (1024^2,
# 2048^2); (16, 16, 2) and (8, 8, 2) give a wave more rows than the grid has.
@pytest.mark.parametrize("R,N,d", [(32, 64, 2), (32, 128, 2), (16, 64, 2), (16, 32, 3), (8, 64, 2), (8, 16, 3),
                                   (4, 32, 2), (4, 8, 3), (16, 48, 2), (32, 1024, 2), (16, 2048, 2),
                                   (16, 16, 2), (8, 8, 2)])
def test_ctransform_p1_tile_sizes_bit_exact(R, N, d, monkeypatch):
    monkeypatch.setenv("QBW_TILE_R", str(R))
    P = N ** d
    phi = (si.rng(7050 + N + R + d).standard_normal(P) * N).astype(np.float32)
    out, arg = qbw.ctransform(dev(phi), N, d, 1, want_argmin=True)
    tg = si.rng(7051).choice(P, min(P, 1500 if P <= 1 << 16 else 160 if P <= 1 << 20 else 64), replace=False)
    ref, refarg = lower.ctransform_o32(phi, N, d, 1, targets=tg)
    assert np.array_equal(out.cpu().numpy()[tg], ref)
    assert np.array_equal(arg.cpu().numpy()[tg].astype(np.int64), refarg)


def test_ctransform_ties_and_constant_potential():
    N, d, p = 16, 2, 2
    phi = np.zeros(N * N, np.float32)           # every target's min is 0 at itself
    out, arg = qbw.ctransform(dev(phi), N, d, p, want_argmin=True)
    assert np.all(out.cpu().numpy() == 0) and np.array_equal(arg.cpu().numpy(), np.arange(N * N))
    phi = np.full(N * N, -3.0, np.float32)
    phi[::7] = 5.0                              # many equal candidates: lowest index wins
    out, arg = qbw.ctransform(dev(phi), N, d, p, want_argmin=True)
    ref, refarg = lower.ctransform_o32(phi, N, d, p)
    assert np.array_equal(out.cpu().numpy(), ref) and np.array_equal(arg.cpu().numpy(), refarg)


# ------------------------------------------------------------------ stages

@pytest.mark.parametrize("N,d,k", [(32, 2, 4), (30, 2, 3), (16, 3, 2), (16, 2, 16), (12, 2, 1), (8, 3, 8)])
def test_upscale_bit_exact(N, d, k):
    n = N // k
    ft = si.rng(7100 + N + k).standard_normal(n ** d) * 100
    out = qbw.upscale_potential(dev(ft), N, d, k)
    ref = lower.upscale_potential(ft, N, d, k).astype(np.float32)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("N,d,k", [(32, 2, 4), (16, 3, 4), (30, 2, 5)])
def test_sumpool(N, d, k):
    m = si.grf(N, d, si.rng(7200 + N))
    out = qbw.sumpool(dev(m), k).cpu().numpy()
    assert np.allclose(out, coarse.sumpool(m, k), rtol=k ** d * 2.0 ** -53, atol=0)


@pytest.mark.parametrize("N,d,k,p", [(16, 2, 4, 2), (16, 2, 4, 1), (8, 3, 2, 2), (8, 3, 2, 1),
                                     (16, 2, 2, 2)])
def test_cbar(N, d, k, p):
    mu, nu = pair(N, d, "shapes", "grf", 7300 + N + p)   # shapes: empty blocks -> C~ fallback
    out = qbw.cbar(dev(mu), dev(nu), k, p).cpu().numpy()
    ref = coarse.cbar(mu, nu, k, p)
    assert np.allclose(out, ref, rtol=1e-11, atol=1e-11 * ref.max())


def test_coarse_cost():
    for p in (1, 2):
        assert np.allclose(qbw.coarse_cost(16, 3, 4, p), coarse.centre_cost(16, 3, 4, p), rtol=1e-15, atol=0)


@pytest.mark.parametrize("N,d,k,p", [(32, 2, 4, 2), (16, 3, 2, 1), (24, 2, 3, 2)])
def test_ipf_plan_cost_tv(N, d, k, p):
    mu, nu = pair(N, d, "gmm", "shapes", 7400 + N)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    a_s, b_s, it, res = qbw.ipf(dev(mu), dev(nu), k, rec)
    P = N ** d
    I, J, V = upper.upscale_plan(r, c, v, N, d, k)
    oa, ob, mh, nh, oit, ores = upper.ipf(mu.reshape(-1), nu.reshape(-1), I, J, V, 1e-12, 50)
    assert it == oit
    assert np.allclose(a_s.cpu().numpy(), oa, rtol=1e-12, atol=0)
    assert np.allclose(b_s.cpu().numpy(), ob, rtol=1e-12, atol=0)
    pc = qbw.plan_cost(a_s, b_s, N, d, k, p, rec)
    assert pc == pytest.approx(upper.plan_cost(I, J, V, oa, ob, N, d, p), rel=1e-12)
    tm, tn = qbw.tv(dev(mu), dev(nu), k, p, rec, a_s, b_s)
    w = upper.tv_weights(N, d, p)
    tol = 2 * 2.0 ** (1 - 1 / p) * (2.0 ** -40 * float(w @ mu.reshape(-1) + w @ nu.reshape(-1))) ** (1 / p)
    assert abs(tm - upper.weighted_tv(w, mh, mu.reshape(-1), p)) <= tol
    assert abs(tn - upper.weighted_tv(w, nu.reshape(-1), nh, p)) <= tol


def test_ipf_not_converged_coupling():
    # a coupling of perturbed marginals: several iterations, non-trivial TV terms
    N, d, k, p = 16, 2, 4, 2
    mu, nu = pair(N, d, "grf", "gmm", 7450)
    mt = coarse.sumpool(mu, k) * np.exp(0.3 * si.rng(7451).standard_normal(16))
    r, c, v = lp.northwest_corner(mt / mt.sum(), coarse.sumpool(nu, k))
    rec = qbw.Coarse(r, c, v, np.zeros(16))
    a_s, b_s, it, res = qbw.ipf(dev(mu), dev(nu), k, rec, max_ipf_iter=3)
    I, J, V = upper.upscale_plan(r, c, v, N, d, k)
    oa, ob, mh, nh, oit, ores = upper.ipf(mu.reshape(-1), nu.reshape(-1), I, J, V, 1e-12, 3)
    assert it == oit == 3
    assert res == pytest.approx(ores, rel=1e-9)
    assert np.allclose(a_s.cpu().numpy(), oa, rtol=1e-12, atol=0)
    tm, tn = qbw.tv(dev(mu), dev(nu), k, p, rec, a_s, b_s)
    w = upper.tv_weights(N, d, p)
    assert tm == pytest.approx(upper.weighted_tv(w, mh, mu.reshape(-1), p), rel=1e-9)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec, max_ipf_iter=3)
    assert out["warn"] & qbw.QBW_WARN_IPF_NOT_CONVERGED
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p, max_iter=3)
    assert U["upper"] <= out["upper"] <= U["upper"] + ub_tol(mu, nu, N, d, p, k, U["upper"], r, c, 3)


# ------------------------------------------------------------------ whole method

BOUND_CASES = [(32, 2, 4, 2, "blobs", "blobs"), (32, 2, 4, 1, "gmm", "grf"), (64, 2, 8, 2, "cauchy", "shapes"),
               (16, 3, 2, 2, "grf", "grf"), (16, 3, 4, 1, "gmm", "white_noise"), (24, 2, 3, 2, "grf", "cauchy")]


@pytest.mark.parametrize("N,d,k,p,fa,fb", BOUND_CASES)
def test_bounds_with_coarse(N, d, k, p, fa, fb):
    mu, nu = pair(N, d, fa, fb, 7500 + N + k + p)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec)
    L32 = lower.lower_bound_o32(mu, nu, ft, k, p)
    L64 = lower.lower_bound_o64(mu, nu, ft, k, p)
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    assert out["lower_S"] == pytest.approx(L32["S_emit"], rel=1e-9)
    assert out["feas_shift"] == pytest.approx(L32["shift"], rel=1e-12)
    assert out["lower"] == pytest.approx(L32["lower"], rel=1e-9)
    assert out["lower"] <= L64["lower"]
    assert out["ipf_iters"] == U["iters"]
    assert out["upper_cost"] == pytest.approx(U["plan_cost"], rel=1e-9)
    assert out["upper_cost"] >= U["plan_cost"]
    assert U["upper"] <= out["upper"] <= U["upper"] + ub_tol(mu, nu, N, d, p, k, U["upper"], r, c, U["iters"])
    assert out["coarse_objective"] == pytest.approx(obj, rel=1e-12)


def test_bounds_potentials_bit_exact():
    N, d, k, p = 32, 2, 4, 2
    mu, nu = pair(N, d, "gmm", "gmm", 7600)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    fhat = qbw.upscale_potential(dev(ft), N, d, k)
    g = qbw.ctransform(fhat, N, d, p)
    f = qbw.ctransform(g, N, d, p)
    L32 = lower.lower_bound_o32(mu, nu, ft, k, p)
    assert np.array_equal(g.cpu().numpy(), L32["g32"]) and np.array_equal(f.cpu().numpy(), L32["f32"])
    L64 = lower.lower_bound_o64(mu, nu, ft, k, p)
    scale = max(np.abs(L64["g"]).max(), 1.0)
    assert np.abs(g.cpu().numpy() - L64["g"]).max() <= 1e-5 * scale


@pytest.mark.parametrize("N,d,k,p", [(16, 2, 4, 2), (16, 2, 4, 1), (8, 3, 2, 2)])
def test_end_to_end_brackets_exact(N, d, k, p):
    mu, nu = pair(N, d, "gmm", "cauchy", 7700 + N + p)
    W = lp.wasserstein_exact(mu, nu, p)
    out = qbw.bounds(dev(mu), dev(nu), k, p)
    *_, obj = upper.coarse_record_lp(mu, nu, k, p)
    assert out["coarse_objective"] == pytest.approx(obj, rel=1e-9)
    assert out["lower"] <= W <= out["upper"]


def test_config1_against_exact_lp():
    import json
    import os
    mu, nu = si.config1_pair()
    gold = os.path.join(os.path.dirname(__file__), "golden", "config1_exact.json")
    if not os.path.exists(gold):
        pytest.skip("golden value not generated")
    W = json.load(open(gold))["exact_W2"]
    out = qbw.bounds(dev(mu), dev(nu), 4, 2)
    assert out["lower"] <= W <= out["upper"]


def test_input_validation():
    N = 16
    mu, nu = pair(N, 2, "grf", "grf", 7800)
    with pytest.raises(qbw.QbwError, match="E_GRID"):
        qbw.bounds(dev(mu), dev(nu), 5, 2)
    bad = mu.copy()
    bad[3, 3] = -1e-3
    with pytest.raises(qbw.QbwError, match="E_MASS"):
        qbw.bounds(dev(bad), dev(nu), 4, 2)
    with pytest.raises(qbw.QbwError, match="E_MASS"):
        qbw.bounds(dev(mu), dev(nu * 1.5), 4, 2)
    nanm = mu.copy()
    nanm[0, 0] = np.nan
    with pytest.raises(qbw.QbwError, match="E_MASS"):
        qbw.bounds(dev(nanm), dev(nu), 4, 2)


# ------------------------------------------------------------------ gradients

@pytest.mark.parametrize("p", [1, 2])
def test_gradients_against_oracle_and_fd(p):
    N, d, k = 16, 2, 4
    mu, nu = pair(N, d, "gmm", "gmm", 7900 + p)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    v2 = v * np.exp(0.2 * si.rng(7902).standard_normal(len(v)))    # several IPF iterations
    rec2 = qbw.Coarse(r, c, v2, ft)
    res, ga, gb, _ = qbw.bounds_with_grads(dev(mu), dev(nu), k, p, coarse=rec2, dlower=0.7, dupper=1.3)
    L32 = lower.lower_bound_o32(mu, nu, ft, k, p)
    lgm, lgn = ograd.lower_grad(L32["f32"], L32["g32"], L32["S_emit"], p)
    U = upper.upper_bound_o64(mu, nu, r, c, v2, k, p)
    ugm, ugn, _ = ograd.upper_grad(mu, nu, r, c, v2, k, p, U["iters"])
    ref_a = 0.7 * lgm + 1.3 * ugm
    ref_b = 0.7 * lgn + 1.3 * ugn
    scale = np.abs(ref_a).max()
    assert np.allclose(ga.cpu().numpy().reshape(-1), ref_a, rtol=1e-9, atol=1e-9 * scale)
    assert np.allclose(gb.cpu().numpy().reshape(-1), ref_b, rtol=1e-9, atol=1e-9 * scale)
    # central differences of the GPU forward (frozen coarse solution), mass preserving
    g = si.rng(7903)
    h = 1e-4
    for _ in range(2):
        vm = g.uniform(-1, 1, mu.shape)
        vm -= (mu * vm).sum() / mu.sum()
        vn = g.uniform(-1, 1, nu.shape)
        vn -= (nu * vn).sum() / nu.sum()

        def F(s):
            o = qbw.bounds(dev(mu * (1 + s * vm)), dev(nu * (1 + s * vn)), k, p, coarse=rec2)
            return 0.7 * o["lower"] + 1.3 * (o["upper_cost"] ** (1 / p))

        fd = (F(h) - F(-h)) / (2 * h)
        an = float((ga.cpu().numpy() * mu * vm).sum() + (gb.cpu().numpy() * nu * vn).sum())
        assert fd == pytest.approx(an, rel=2e-5, abs=1e-7)


# p = 1 on blocks of 36 .. 1024 pixels: plan cost and upper-bound gradient take
# the distance-table kernels (64- and 256-thread work-groups, tables of up to
# 63^2 and 15^3 entries); the oracle sums the pair distances directly.
@pytest.mark.parametrize("N,d,k", [(48, 2, 6), (64, 2, 16), (64, 2, 32), (24, 3, 6), (16, 3, 8), (16, 3, 4)])
def test_p1_distance_table_paths(N, d, k):
    p = 1
    mu, nu = pair(N, d, "grf", "gmm", 7950 + N + k)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    v2 = v * np.exp(0.2 * si.rng(7951).standard_normal(len(v)))    # several IPF iterations
    rec2 = qbw.Coarse(r, c, v2, ft)
    res, ga, gb, _ = qbw.bounds_with_grads(dev(mu), dev(nu), k, p, coarse=rec2, dlower=0.0, dupper=1.0)
    U = upper.upper_bound_o64(mu, nu, r, c, v2, k, p)
    assert res["ipf_iters"] == U["iters"]
    assert res["upper_cost"] == pytest.approx(U["plan_cost"], rel=1e-9)
    assert res["upper_cost"] >= U["plan_cost"]
    assert U["upper"] <= res["upper"] <= U["upper"] + ub_tol(mu, nu, N, d, p, k, U["upper"], r, c, U["iters"])
    ugm, ugn, _ = ograd.upper_grad(mu, nu, r, c, v2, k, p, U["iters"])
    scale = max(np.abs(ugm).max(), np.abs(ugn).max())
    assert np.allclose(ga.cpu().numpy().reshape(-1), ugm, rtol=1e-9, atol=1e-9 * scale)
    assert np.allclose(gb.cpu().numpy().reshape(-1), ugn, rtol=1e-9, atol=1e-9 * scale)


def test_autograd_function():
    N, d, k, p = 16, 2, 4, 2
    mu, nu = pair(N, d, "grf", "gmm", 7950)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    a = dev(mu).requires_grad_(True)
    b = dev(nu).requires_grad_(True)
    lo, up = qbw.wasserstein_bounds(a, b, k, p, coarse=rec)
    (2.0 * lo - up).backward()
    res, ga, gb, _ = qbw.bounds_with_grads(dev(mu), dev(nu), k, p, coarse=rec, dlower=2.0, dupper=-1.0)
    assert torch.equal(a.grad, ga) and torch.equal(b.grad, gb)


def test_fhat_gradient_through_argmins():
    N, d, k, p = 16, 2, 4, 2
    mu, nu = pair(N, d, "grf", "cauchy", 7960)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    res, ga, gb, gf = qbw.bounds_with_grads(dev(mu), dev(nu), k, p, coarse=rec, dlower=1.0, dupper=0.0,
                                            want_fhat_grad=True)
    L32 = lower.lower_bound_o32(mu, nu, ft, k, p)
    s = 0.5 / math.sqrt(L32["S_emit"])
    ref = np.zeros(N * N)
    np.add.at(ref, L32["argmin_g"][L32["argmin_f"]], s * mu.reshape(-1))
    np.add.at(ref, L32["argmin_g"], -s * nu.reshape(-1))
    assert np.allclose(gf.cpu().numpy(), ref, rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------------ batches

def test_batch_matches_single_and_graph_replays():
    jobs, recs, singles = [], [], []
    specs = [(32, 2, 4, 2), (16, 3, 2, 1), (24, 2, 3, 2), (32, 2, 8, 1), (16, 2, 4, 2)]
    for i, (N, d, k, p) in enumerate(specs):
        mu, nu = pair(N, d, "grf", "gmm", 8000 + 2 * i)
        rec, _ = record(mu, nu, k, p)
        a, b = dev(mu), dev(nu)
        jobs.append((a, b, k, p))
        recs.append(rec)
        singles.append(qbw.bounds(a, b, k, p, coarse=rec))
    for graph in (False, True):
        B = qbw.Batch(jobs, coarse=recs, graph=graph, backward=True)
        for rep in range(3):
            for ga, gb in B.grads:
                ga.zero_()
                gb.zero_()
            torch.ones(1000, device="cuda:0").sum().item()   # eager work between replays
            B.run()
            out = B.results()
            for s, o in zip(singles, out):
                for key in ("lower", "upper", "lower_S", "upper_cost", "feas_shift", "ipf_iters"):
                    assert s[key] == o[key], (graph, rep, key)
        # batch gradients equal the single-pair backward
        for (a, b, k, p), rec, (ga, gb) in zip(jobs, recs, B.grads):
            _, sa, sb, _ = qbw.bounds_with_grads(a, b, k, p, coarse=rec)
            assert torch.allclose(ga, sa, rtol=1e-12, atol=0) and torch.allclose(gb, sb, rtol=1e-12, atol=0)


def test_batch_internal_coarse_and_autotune():
    specs = [(32, 2, 4, 2), (16, 3, 4, 1), (32, 2, 8, 2)]
    jobs, refs = [], []
    for i, (N, d, k, p) in enumerate(specs):
        mu, nu = pair(N, d, "cauchy", "grf", 8100 + 2 * i)
        jobs.append((dev(mu), dev(nu), k, p))
        *_, obj = upper.coarse_record_lp(mu, nu, k, p)
        refs.append(obj)
    B = qbw.Batch(jobs, autotune=True)
    B.run()
    for o, obj, (a, b, k, p) in zip(B.results(), refs, jobs):
        assert o["coarse_objective"] == pytest.approx(obj, rel=1e-9)
        assert o["lower"] <= o["upper"]
    for j in range(len(jobs)):
        R, Sp = B.tiling(j)
        assert R in (1, 2, 4, 8, 16) and Sp >= 1


# ------------------------------------------------------------------ full size (256 x 256, k = 8)

@pytest.fixture(scope="module")
def big_records():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "records_256_k8.npz")
    return np.load(path)


@pytest.mark.parametrize("fam", ["grf", "cauchy"])
def test_full_size_sampled_parity(fam, big_records):
    N, d, k, p = 256, 2, 8, 2
    mu, nu = si.config3_pair(N, fam)
    R = big_records
    rec = qbw.Coarse(R[f"{fam}_rows"], R[f"{fam}_cols"], R[f"{fam}_vals"], R[f"{fam}_f"])
    fhat = qbw.upscale_potential(dev(R[f"{fam}_f"]), N, d, k)
    fh_ref = lower.upscale_potential(R[f"{fam}_f"], N, d, k).astype(np.float32)
    assert np.array_equal(fhat.cpu().numpy(), fh_ref)
    g, garg = qbw.ctransform(fhat, N, d, p, want_argmin=True)
    f = qbw.ctransform(g, N, d, p)
    tg = si.rng(8200).choice(N * N, 192, replace=False)
    ref, refarg = lower.ctransform_o32(fh_ref, N, d, p, targets=tg)
    assert np.array_equal(g.cpu().numpy()[tg], ref)
    assert np.array_equal(garg.cpu().numpy()[tg].astype(np.int64), refarg)
    # second transform: f = g^c at sampled targets, for the g the kernel produced
    gn = g.cpu().numpy()
    ref_f, _ = lower.ctransform_o32(gn, N, d, p, targets=tg)
    assert np.array_equal(f.cpu().numpy()[tg], ref_f)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec)
    # the lower bound is the float64 sum of the float32 potentials minus the shift
    S = lower.fsum_dot(f.cpu().numpy(), mu.reshape(-1)) + lower.fsum_dot(gn, nu.reshape(-1))
    assert out["lower_S"] == pytest.approx(S - out["feas_shift"], rel=1e-9)
    assert out["lower"] <= out["upper"]
    assert out["ipf_iters"] == 1
    # uniform kernel + converged fitting: plan cost = <pi~, C-bar>
    Cb = qbw.cbar(dev(mu), dev(nu), k, p).cpu().numpy()
    ident = float((Cb[R[f"{fam}_rows"], R[f"{fam}_cols"]] * R[f"{fam}_vals"]).sum())
    assert out["upper_cost"] == pytest.approx(ident, rel=1e-9)


def test_full_size_translation_closed_form():
    N, d, k, p = 256, 2, 8, 2
    mu, nu = si.translated_pair(N, d, (5, -9), si.rng(8300))
    out = qbw.bounds(dev(mu), dev(nu), k, p)
    W = math.sqrt(5 ** 2 + 9 ** 2)
    assert out["lower"] <= W <= out["upper"]
    assert out["lower"] > 0.9 * W


# ------------------------------------------------------------------ Algorithm 3 and Section 3.3

@pytest.mark.parametrize("N,d,k,p", [(16, 2, 4, 2), (16, 2, 4, 1), (32, 2, 8, 2), (8, 3, 2, 2), (8, 3, 4, 1)])
def test_weighted_cost_and_min_cost_bounds(N, d, k, p):
    mu, nu = pair(N, d, "gmm", "shapes", 9600 + N + k + p)
    ub, uobj = qbw.weighted_cost_upper(dev(mu), dev(nu), k, p)
    lb, lobj = qbw.min_cost_lower(dev(mu), dev(nu), k, p)
    ref_ub = upper.weighted_cost_upper(mu, nu, k, p)
    ref_lb = upper.min_cost_lower(mu, nu, k, p)
    assert ub == pytest.approx(ref_ub, rel=1e-9) and ub >= ref_ub * (1 - 1e-12)
    assert lb == pytest.approx(ref_lb, rel=1e-9) and lb <= ref_lb * (1 + 1e-12)
    if N ** d <= 256:
        W = lp.wasserstein_exact(mu, nu, p)
        assert lb <= W <= ub
    # ordering against the primal-upscaling bound on the same pair
    out = qbw.bounds(dev(mu), dev(nu), k, p)
    assert lb <= out["upper"] and ub <= out["upper"] * (1 + 1e-9)


# ------------------------------------------------------------------ separable c-transform (p = 2)

@pytest.mark.parametrize("N,d", [(32, 2), (16, 3), (24, 2), (15, 2), (9, 3), (70, 2), (256, 2)])
def test_ctransform_separable_bit_exact(N, d):
    phi = (si.rng(9700 + N).standard_normal(N ** d) * N * N / 4).astype(np.float32)
    out, arg = qbw.ctransform_separable(dev(phi), N, d, want_argmin=True)
    ref, refarg = lower.ctransform_sep_o32(phi, N, d)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(arg.cpu().numpy().astype(np.int64), refarg)


@pytest.mark.parametrize("N,d", [(32, 2), (64, 2), (128, 2), (256, 2), (512, 2), (32, 3), (64, 3)])
def test_ctransform_separable_fast_path_bit_exact(N, d):
    # without arg-mins, power-of-two N in [32, 1024] takes the register-window
    # 1-D kernel (R = 4, 8, 16 targets per lane, sources split over lane groups)
    phi = (si.rng(9750 + N + d).standard_normal(N ** d) * N * N / 4).astype(np.float32)
    out = qbw.ctransform_separable(dev(phi), N, d, want_argmin=False)
    ref, _ = lower.ctransform_sep_o32(phi, N, d)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("N,d,k", [(32, 2, 4), (64, 2, 8), (16, 3, 2), (24, 2, 3)])
def test_bounds_separable(N, d, k):
    mu, nu = pair(N, d, "grf", "cauchy", 9800 + N + k)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, 2)
    out = qbw.bounds(dev(mu), dev(nu), k, 2, coarse=rec, separable=True)
    Ls = lower.lower_bound_sep_o32(mu, nu, ft, k)
    L64 = lower.lower_bound_o64(mu, nu, ft, k, 2)
    assert out["lower_S"] == pytest.approx(Ls["S_emit"], rel=1e-9)
    assert out["feas_shift"] == pytest.approx(Ls["shift"], rel=1e-12)
    assert out["lower"] <= L64["lower"]
    allp = qbw.bounds(dev(mu), dev(nu), k, 2, coarse=rec)
    assert out["upper"] == allp["upper"]
    assert abs(out["lower"] - allp["lower"]) <= 1e-3 * allp["lower"]
    res, ga, gb, gf = qbw.bounds_with_grads(dev(mu), dev(nu), k, 2, coarse=rec, dlower=1.0, dupper=0.0,
                                            separable=True, want_fhat_grad=True)
    lgm, lgn = ograd.lower_grad(Ls["f32"], Ls["g32"], Ls["S_emit"], 2)
    scale = np.abs(lgm).max()
    assert np.allclose(ga.cpu().numpy().reshape(-1), lgm, rtol=1e-9, atol=1e-12 * scale)
    s = 0.5 / math.sqrt(Ls["S_emit"])
    ref = np.zeros(N ** d)
    np.add.at(ref, Ls["argmin_g"][Ls["argmin_f"]], s * mu.reshape(-1))
    np.add.at(ref, Ls["argmin_g"], -s * nu.reshape(-1))
    assert np.allclose(gf.cpu().numpy(), ref, rtol=1e-12, atol=1e-15)


def test_batch_separable_mixed_p():
    specs = [(32, 2, 4, 2), (16, 3, 2, 1), (24, 2, 3, 2), (16, 3, 4, 2), (32, 2, 8, 1)]
    jobs, recs = [], []
    for i, (N, d, k, p) in enumerate(specs):
        mu, nu = pair(N, d, "gmm", "grf", 9900 + 2 * i)
        rec, _ = record(mu, nu, k, p)
        jobs.append((dev(mu), dev(nu), k, p))
        recs.append(rec)
    B = qbw.Batch(jobs, coarse=recs, graph=True, backward=True, separable=True)
    B.run()
    out = B.results()
    for (a, b, k, p), rec, o, (ga, gb) in zip(jobs, recs, out, B.grads):
        s, sa, sb, _ = qbw.bounds_with_grads(a, b, k, p, coarse=rec, separable=True)
        for key in ("lower", "upper", "lower_S", "feas_shift", "upper_cost"):
            assert s[key] == o[key], key
        assert torch.allclose(ga, sa, rtol=1e-12, atol=0)


# ------------------------------------------------------------------ degenerate and extreme cases

def test_degenerate_grids_and_measures():
    # k = N: one coarse block (the coarse problem is trivial)
    N, d = 16, 2
    mu, nu = pair(N, d, "gmm", "grf", 10000)
    out = qbw.bounds(dev(mu), dev(nu), N, 2)
    W = lp.wasserstein_exact(mu, nu, 2)
    assert out["lower"] <= W <= out["upper"]
    # k = 1: the coarse problem is the fine one: the lower bound is W up to the shift
    N = 8
    mu, nu = pair(N, d, "gmm", "cauchy", 10002)
    out = qbw.bounds(dev(mu), dev(nu), 1, 2)
    W = lp.wasserstein_exact(mu, nu, 2)
    assert out["lower"] <= W <= out["upper"]
    assert out["lower"] == pytest.approx(W, rel=1e-4)
    assert out["upper"] == pytest.approx(W, rel=1e-4)
    # identical measures: the lower bound clips to 0; the coarse plan is the
    # identity, so the upscaled plan moves mass only inside blocks (each move
    # at most sqrt(d) (k - 1)), and it matches the oracle's upper bound
    m = si.grf(32, 2, si.rng(10004))
    out = qbw.bounds(dev(m), dev(m), 4, 2)
    assert out["lower"] == 0.0 and out["warn"] & qbw.QBW_WARN_LB_CLIPPED
    assert 0.0 < out["upper"] <= math.sqrt(2) * 3
    r, c, v, ft, gt, obj = upper.coarse_record_lp(m, m, 4, 2)
    assert abs(obj) <= 1e-12
    U = upper.upper_bound_o64(m, m, r, c, v, 4, 2)
    assert U["upper"] <= out["upper"] <= U["upper"] + ub_tol(m, m, 32, 2, 2, 4, U["upper"], r, c, U["iters"])
    # Dirac pair: most blocks empty; W = |x - y|
    for p in (1, 2):
        a, b, x, y = si.dirac_pair(32, 2, si.rng(10006 + p))
        out = qbw.bounds(dev(a), dev(b), 4, p)
        W = float(np.linalg.norm(x - y))
        assert out["lower"] <= W * (1 + 1e-12) and W <= out["upper"] * (1 + 1e-12)
    # 3D with k = N and with k = 1
    mu, nu = pair(8, 3, "grf", "gmm", 10010)
    for k in (8, 1):
        out = qbw.bounds(dev(mu), dev(nu), k, 1)
        W = lp.wasserstein_exact(mu, nu, 1)
        assert out["lower"] <= W <= out["upper"]


def test_large_grid_runs():
    # 1024 x 1024 (P = 2^20): the all-pairs transform is 1.1e12 pairs per launch
    N, d, k, p = 1024, 2, 64, 2
    mu, nu = si.translated_pair(N, d, (40, -25), si.rng(10020))
    out = qbw.bounds(dev(mu), dev(nu), k, p, separable=True)
    W = math.sqrt(40 ** 2 + 25 ** 2)
    assert out["lower"] <= W <= out["upper"]
    phi = (si.rng(10021).standard_normal(N * N) * 1e4).astype(np.float32)
    g = qbw.ctransform(dev(phi), N, d, p)
    tg = si.rng(10022).choice(N * N, 8, replace=False)
    ref, _ = lower.ctransform_o32(phi, N, d, p, targets=tg)
    assert np.array_equal(g.cpu().numpy()[tg], ref)


def test_saved_records_reuse_and_outlive_context():
    # repeated forward+backward calls reuse freed device arenas: identical results
    N, d, k, p = 32, 2, 4, 2
    mu, nu = pair(N, d, "gmm", "grf", 10100)
    a, b = dev(mu), dev(nu)
    runs = [qbw.bounds_with_grads(a, b, k, p) for _ in range(3)]
    for res, ga, gb, _ in runs[1:]:
        assert res["lower"] == runs[0][0]["lower"] and res["upper"] == runs[0][0]["upper"]
        assert torch.equal(ga, runs[0][1]) and torch.equal(gb, runs[0][2])
    # a saved record may outlive its context: it is detached, then freed
    import ctypes as C
    from paper_2506_00976_amd import _lib
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.qbw_create(C.byref(h), 0) == 0
    grid = _lib.QbwGrid(d, N, k, p)
    opts = _lib.QbwOpts(1e-12, 50, _lib.QBW_SAVE_FOR_BWD)
    res = _lib.QbwResult()
    saved = C.c_void_p()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.qbw_bounds(h, C.byref(grid), C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                          C.byref(opts), C.byref(res), C.byref(saved), stream) == 0
    assert res.lower == runs[0][0]["lower"]
    lib.qbw_destroy(h)
    lib.qbw_saved_free(saved)


# ------------------------------------------------------------------ other interpolants (Section 3.5)

@pytest.mark.parametrize("interp", ["nearest", "cubic"])
@pytest.mark.parametrize("N,d,k", [(32, 2, 4), (30, 2, 3), (16, 3, 2), (16, 2, 16), (12, 2, 1), (8, 3, 8),
                                   (15, 2, 5), (20, 3, 4)])
def test_upscale_interpolants_bit_exact(interp, N, d, k):
    n = N // k
    ft = si.rng(10200 + N + k).standard_normal(n ** d) * 100
    out = qbw.upscale_potential(dev(ft), N, d, k, interp=interp)
    ref = lower.upscale_potential(ft, N, d, k, interp).astype(np.float32)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("interp", ["nearest", "cubic"])
@pytest.mark.parametrize("N,d,k,p", [(16, 2, 4, 2), (16, 2, 4, 1), (8, 3, 2, 2)])
def test_bounds_with_interpolants(interp, N, d, k, p):
    mu, nu = pair(N, d, "gmm", "grf", 10300 + N + p)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec, interp=interp)
    L = lower.lower_bound_o32(mu, nu, ft, k, p, interp)
    assert out["lower"] == pytest.approx(L["lower"], rel=1e-9)
    assert out["feas_shift"] == pytest.approx(L["shift"], rel=1e-12)
    L64 = lower.lower_bound_o64(mu, nu, ft, k, p, interp)
    assert out["lower"] <= L64["lower"] * (1 + 1e-12)
    W = lp.wasserstein_exact(mu, nu, p)
    assert out["lower"] <= W <= out["upper"]
    # the upper bound does not depend on the interpolation of the potential
    lin = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec)
    assert out["upper"] == lin["upper"]


def test_batch_with_interpolant_matches_single():
    jobs_np = [(16, 2, 4, 2), (16, 2, 4, 1), (8, 3, 2, 2), (24, 2, 3, 2)]
    jobs, recs = [], []
    for i, (N, d, k, p) in enumerate(jobs_np):
        mu, nu = pair(N, d, "grf", "gmm", 10400 + i)
        rec, _ = record(mu, nu, k, p)
        jobs.append((dev(mu), dev(nu), k, p))
        recs.append(rec)
    B = qbw.Batch(jobs, coarse=recs, graph=True, interp="cubic")
    B.run()
    out = B.results()
    for (a, b, k, p), rec, o in zip(jobs, recs, out):
        s = qbw.bounds(a, b, k, p, coarse=rec, interp="cubic")
        assert s["lower"] == o["lower"] and s["upper"] == o["upper"]
    with pytest.raises(qbw.QbwError):
        qbw.upscale_potential(dev(np.zeros(16)), 16, 2, 4, interp="spline")


def test_interpolant_flags_are_exclusive():
    import ctypes as C
    from paper_2506_00976_amd import _lib
    lib = _lib.load()
    mu, nu = pair(16, 2, "grf", "gmm", 10500)
    a, b = dev(mu), dev(nu)
    grid = _lib.QbwGrid(2, 16, 4, 2)
    opts = _lib.QbwOpts(1e-12, 50, _lib.QBW_INTERP_NEAREST | _lib.QBW_INTERP_CUBIC)
    res = _lib.QbwResult()
    rc = lib.qbw_bounds(qbw.context(0).handle, C.byref(grid), C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                        C.byref(opts), C.byref(res), None, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 1   # QBW_E_INVAL
    assert b"exclusive" in lib.qbw_last_error()


def test_ctransform_with_dynamic_tail():
    # 725 is odd, so each lane owns one target: 8213 tiles of 64 targets, more
    # than the persistent grid's 8192 work-groups, so the last items are taken
    # through the work counter after the static round
    N, d, p = 725, 2, 2
    phi = (si.rng(10600).standard_normal(N * N) * 2e4).astype(np.float32)
    out, arg = qbw.ctransform(dev(phi), N, d, p, want_argmin=True)
    P = N * N
    tg = np.concatenate([si.rng(10601).choice(P, 12, replace=False), np.arange(P - 4, P)])
    ref, refarg = lower.ctransform_o32(phi, N, d, p, targets=tg)
    assert np.array_equal(out.cpu().numpy()[tg], ref)
    assert np.array_equal(arg.cpu().numpy()[tg].astype(np.int64), refarg)
