"""Exact separable c-transform (p = 2) against the oracle's all-pairs reading.

The path evaluates min_x RN32(|x - y|^2 - phi(x)) from per-axis minima in
float64, certifies each target against float32 rounding and re-evaluates the
rest with the all-pairs arithmetic over the rows that can hold a tie, so its
values and arg-mins must equal the all-pairs
float32 reading (the oracle's ctransform_o32) bit for bit, whatever the
potential: random, smooth, with exact ties everywhere (linear slope 1), with
near ties, or constant (every minimum exactly 0).
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import grad as ograd
from oracle import lower, upper

pytestmark = pytest.mark.gpu

qbw = pytest.importorskip("paper_2506_00976_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qbw.load()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device="cuda:0")


def coords(N, d):
    return np.stack(np.meshgrid(*[np.arange(N)] * d, indexing="ij"), -1).reshape(-1, d).astype(np.float64)


def potential(kind, N, d, seed):
    """Seeded float32 source potentials of several shapes."""
    r = si.rng(seed)
    X = coords(N, d)
    P = N ** d
    if kind == "normal":
        v = r.standard_normal(P) * N * N / 4
    elif kind == "smooth":
        # concave-up quadratic with a random centre and slope, plus small noise
        c = r.uniform(0, N, d)
        v = 0.6 * ((X - c) ** 2).sum(1) + X @ r.uniform(-2, 2, d) + 0.01 * r.standard_normal(P)
    elif kind == "ties":
        v = X.sum(1)              # slope 1 on every axis: x_a = y_a and y_a + 1 tie exactly
    elif kind == "near_ties":
        v = X.sum(1) * (1.0 + 2.0 ** -20) + 0.5
    elif kind == "zero":
        v = np.zeros(P)
    else:
        raise ValueError(kind)
    return v.astype(np.float32)


EX_CASES = [(32, 2), (16, 3), (24, 2), (15, 2), (64, 2), (9, 3), (7, 2), (2, 2), (20, 3)]


@pytest.mark.parametrize("kind", ["normal", "smooth", "ties", "near_ties", "zero"])
@pytest.mark.parametrize("N,d", EX_CASES)
def test_ctransform_exact_bit_exact(N, d, kind):
    phi = potential(kind, N, d, 12000 + 7 * N + d)
    out, arg, nfb = qbw.ctransform_exact(dev(phi), N, d, want_argmin=True, return_fallback=True)
    ref, refarg = lower.ctransform_o32(phi, N, d, 2)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(arg.cpu().numpy().astype(np.int64), refarg)
    assert 0 <= nfb <= N ** d
    # without arg-mins only the value has to be certified
    out2 = qbw.ctransform_exact(dev(phi), N, d)
    assert np.array_equal(out2.cpu().numpy(), ref)
    if kind == "zero":
        assert nfb == N ** d          # an exact 0 is never certified: all re-evaluated


# targets per lane of the stages: small plans get 2; force 8 and 4 (the
# choice for large batches) on the same grids
@pytest.mark.parametrize("T", [8, 4])
@pytest.mark.parametrize("kind", ["normal", "smooth", "ties"])
@pytest.mark.parametrize("N,d", [(32, 2), (16, 3), (15, 2), (20, 3), (7, 2)])
def test_ctransform_exact_targets_per_lane(N, d, kind, T, monkeypatch):
    monkeypatch.setenv("QBW_XS_T", str(T))
    phi = potential(kind, N, d, 12300 + 7 * N + d + T)
    out, arg = qbw.ctransform_exact(dev(phi), N, d, want_argmin=True)
    ref, refarg = lower.ctransform_o32(phi, N, d, 2)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(arg.cpu().numpy().astype(np.int64), refarg)


def random_case(rng):
    """A seeded random grid and potential: normal at magnitudes 1e-6 .. 1e6,
    integers, multiples of 1/64 (like interpolated integer duals), 30 % exact
    zeros, magnitudes 1e-30 and 1e30, float32 denormals, and exact linear
    slopes in half-integers (ties on every axis)."""
    d = 2 if rng.random() < 0.6 else 3
    N = int(rng.integers(2, 41)) if d == 2 else int(rng.integers(2, 17))
    P = N ** d
    kind = int(rng.integers(0, 8))
    if kind == 0:
        phi = rng.standard_normal(P) * 10.0 ** rng.uniform(-6, 6)
    elif kind == 1:
        phi = rng.integers(-N * N, N * N, P).astype(np.float64)
    elif kind == 2:
        phi = rng.integers(-64 * N * N, 64 * N * N, P) / 64.0
    elif kind == 3:
        phi = rng.standard_normal(P) * N
        phi[rng.random(P) < 0.3] = 0.0
    elif kind == 4:
        phi = rng.standard_normal(P) * 1e-30
    elif kind == 5:
        phi = rng.standard_normal(P) * 1e30
    elif kind == 6:
        phi = rng.standard_normal(P) * 1e-40
    else:
        phi = coords(N, d) @ (2 * rng.integers(-3, 4, d) * 0.5) + rng.integers(0, 3) * 0.25
    return N, d, phi.astype(np.float32)


def test_ctransform_exact_random_sweep(monkeypatch):
    # 120 seeded cases, every targets-per-lane setting, compared bitwise
    # (float32 bit patterns, so signed zeros and denormals count)
    rng = np.random.default_rng(20261202)
    for case in range(120):
        N, d, phi = random_case(rng)
        T = ["2", "4", "8", None, "16"][case % 5]
        if T:
            monkeypatch.setenv("QBW_XS_T", T)
        else:
            monkeypatch.delenv("QBW_XS_T", raising=False)
        out, arg = qbw.ctransform_exact(dev(phi), N, d, want_argmin=True)
        ref, refarg = lower.ctransform_o32(phi, N, d, 2)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32)), (case, N, d)
        assert np.array_equal(arg.cpu().numpy().astype(np.int64), refarg), (case, N, d)
        # values only: the stages track neither index nor runner-up
        out2 = qbw.ctransform_exact(dev(phi), N, d)
        assert np.array_equal(out2.cpu().numpy().view(np.uint32), ref.view(np.uint32)), (case, N, d)


@pytest.mark.parametrize("kind", ["normal", "smooth", "ties", "zero"])
@pytest.mark.parametrize("N,d", [(32, 2), (16, 3), (15, 2), (20, 3), (7, 2), (64, 2)])
def test_ctransform_exact_values_16_targets_per_lane(N, d, kind, monkeypatch):
    # without arg-mins a lane may take 16 targets (large batches)
    monkeypatch.setenv("QBW_XS_T", "16")
    phi = potential(kind, N, d, 12400 + 7 * N + d)
    out = qbw.ctransform_exact(dev(phi), N, d)
    ref, _ = lower.ctransform_o32(phi, N, d, 2)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))


# Two-dimensional value-only stages scan, per item, only the sources between
# the first minimiser of its first target and the last minimiser of its last
# target (the per-axis candidates form a Monge matrix).  Every split of an
# item over 1, 2 or 4 waves (the second phase then takes 16 or 8, 8 or 4, 4 or
# 2 targets per wave), partial target groups and line chunks, and potentials
# of -inf (sources that never attain a minimum; a whole line of them has no
# finite candidate), against the oracle bit for bit.  An item spans one or
# two target groups (QBW_XS_WG, on as many times the waves); QBW_XS_WIN=0
# scans every source.
@pytest.mark.parametrize("mode", ["wg2", "wg1", "full"])
@pytest.mark.parametrize("W", ["1", "2", "4"])
@pytest.mark.parametrize("T", ["8", "16"])
@pytest.mark.parametrize("kind", ["normal", "smooth", "ties", "near_ties", "nonfinite"])
@pytest.mark.parametrize("N", [15, 64, 100])
def test_ctransform_exact_windows(N, kind, T, W, mode, monkeypatch):
    monkeypatch.setenv("QBW_XS_T", T)
    monkeypatch.setenv("QBW_XS_W", W)
    monkeypatch.setenv("QBW_XS_W0", W)
    monkeypatch.setenv("QBW_XS_WIN", "0" if mode == "full" else "1")
    monkeypatch.setenv("QBW_XS_WG", "1" if mode == "wg1" else "2")
    seed = 12800 + N + int(T) + int(W)
    phi = potential("smooth" if kind == "nonfinite" else kind, N, 2, seed)
    if kind == "nonfinite":
        r = si.rng(seed + 1)
        phi = phi.copy()
        phi[r.choice(N * N, N, replace=False)] = -np.inf
        phi.reshape(N, N)[:, int(r.integers(0, N))] = -np.inf   # a line of the first stage
    out = qbw.ctransform_exact(dev(phi), N, 2)
    ref, _ = lower.ctransform_o32(phi, N, 2, 2)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))


# full-size grids on sampled targets (the oracle evaluates them one by one)
@pytest.mark.parametrize("kind", ["normal", "smooth"])
@pytest.mark.parametrize("N,d", [(256, 2), (32, 3), (128, 2)])
def test_ctransform_exact_large_sampled(N, d, kind):
    P = N ** d
    phi = potential(kind, N, d, 12500 + N + d)
    out, arg, nfb = qbw.ctransform_exact(dev(phi), N, d, want_argmin=True, return_fallback=True)
    tg = si.rng(12501).choice(P, 400, replace=False)
    ref, refarg = lower.ctransform_o32(phi, N, d, 2, targets=tg)
    assert np.array_equal(out.cpu().numpy()[tg], ref)
    assert np.array_equal(arg.cpu().numpy()[tg].astype(np.int64), refarg)
    assert nfb <= 0.05 * P, f"{nfb} of {P} targets needed the re-evaluation"


def test_ctransform_exact_matches_all_pairs_kernel_full():
    # every target of a 128^2 smooth potential: oracle on a dense sample, and
    # the all-pairs kernel's own arg-min rule on the rest (both read float32)
    N, d = 128, 2
    phi = potential("smooth", N, d, 12600)
    out, arg = qbw.ctransform_exact(dev(phi), N, d, want_argmin=True)
    tg = np.arange(0, N * N, 7)
    ref, refarg = lower.ctransform_o32(phi, N, d, 2, targets=tg)
    assert np.array_equal(out.cpu().numpy()[tg], ref)
    assert np.array_equal(arg.cpu().numpy()[tg].astype(np.int64), refarg)


def pair(N, d, fa, fb, seed):
    return si.family(fa, N, d, si.rng(seed)), si.family(fb, N, d, si.rng(seed + 1))


def record(mu, nu, k, p):
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    return qbw.Coarse(r, c, v, ft, gt, obj), (r, c, v, ft, gt, obj)


@pytest.mark.parametrize("N,d,k", [(32, 2, 4), (64, 2, 8), (16, 3, 2), (24, 2, 3)])
def test_bounds_exact_separable(N, d, k):
    # the whole lower bound with exact separable transforms is the all-pairs
    # float32 reading: same S, same shift, same arg-mins (f^ gradient)
    mu, nu = pair(N, d, "grf", "cauchy", 12700 + N + k)
    rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, 2)
    out = qbw.bounds(dev(mu), dev(nu), k, 2, coarse=rec, separable="exact")
    L32 = lower.lower_bound_o32(mu, nu, ft, k, 2)
    assert out["lower_S"] == pytest.approx(L32["S_emit"], rel=1e-9)
    assert out["feas_shift"] == pytest.approx(L32["shift"], rel=1e-12)
    assert out["lower"] == pytest.approx(L32["lower"], rel=1e-9)
    res, ga, gb, gf = qbw.bounds_with_grads(dev(mu), dev(nu), k, 2, coarse=rec, dlower=1.0, dupper=0.0,
                                            separable="exact", want_fhat_grad=True)
    lgm, lgn = ograd.lower_grad(L32["f32"], L32["g32"], L32["S_emit"], 2)
    scale = np.abs(lgm).max()
    assert np.allclose(ga.cpu().numpy().reshape(-1), lgm, rtol=1e-9, atol=1e-12 * scale)
    s = 0.5 / math.sqrt(L32["S_emit"])
    ref = np.zeros(N ** d)
    np.add.at(ref, L32["argmin_g"][L32["argmin_f"]], s * mu.reshape(-1))
    np.add.at(ref, L32["argmin_g"], -s * nu.reshape(-1))
    assert np.allclose(gf.cpu().numpy(), ref, rtol=1e-12, atol=1e-15)


def test_batch_exact_separable_mixed_p_graph_replays():
    # p = 1 jobs keep the all-pairs kernel; p = 2 jobs take the exact path;
    # every graph replay (with eager work in between) must give the oracle's S
    specs = [(32, 2, 4, 2), (16, 3, 2, 1), (24, 2, 3, 2), (16, 3, 4, 2), (32, 2, 8, 1)]
    jobs, recs, refs = [], [], []
    for i, (N, d, k, p) in enumerate(specs):
        mu, nu = pair(N, d, "gmm", "grf", 12800 + 2 * i)
        rec, (r, c, v, ft, gt, obj) = record(mu, nu, k, p)
        jobs.append((dev(mu), dev(nu), k, p))
        recs.append(rec)
        refs.append(lower.lower_bound_o32(mu, nu, ft, k, p))
    B = qbw.Batch(jobs, coarse=recs, graph=True, backward=True, separable="exact")
    for rep in range(3):
        B.run()
        out = B.results()
        for o, L32 in zip(out, refs):
            assert o["lower_S"] == pytest.approx(L32["S_emit"], rel=1e-9)
            assert o["feas_shift"] == pytest.approx(L32["shift"], rel=1e-12)
        torch.ones(1000, device="cuda:0").sum().item()   # eager work between replays


def test_exact_and_rounded_separable_are_exclusive():
    mu, nu = pair(16, 2, "grf", "grf", 12900)
    with pytest.raises(ValueError):
        qbw.bounds(dev(mu), dev(nu), 4, 2, separable="both")
