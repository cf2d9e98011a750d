"""Oracle parity at the workloads' own sizes and on the pipeline's own inputs.

* the exact separable c-transform at 256^2 on the potentials the method itself
  produces (interpolated integer duals on a 1/64 lattice, full of exact ties,
  so many targets go through the brute-force re-evaluation): sampled targets
  bit-exact against the oracle's float32 all-pairs reading, values and
  arg-mins, including targets that fail the float64 certification; the whole
  g and f element-wise equal to the all-pairs kernel's;
* the 256^2, k = 8 upper bound against the oracle's, within the derived
  rounding allowance;
* the 128-job uneven batch: one job of every (grid, p) family against the
  oracle, on the coarse solution the batch used: lower bound (whole float32
  transforms where the oracle finishes in seconds, sampled targets and the
  re-summed bound on 128^2 and 32^3), plan cost and upper bound;
* the 64-pair gradient batch: mass-preserving central differences (h = 1e-4)
  of the batched forward on two pairs.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import os

import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import grid as ogrid
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


@pytest.fixture(scope="module")
def big_records():
    return np.load(os.path.join(os.path.dirname(__file__), "golden", "records_256_k8.npz"))


def ub_tol(mu, nu, N, d, p, k, ub, rows, cols, iters):
    """Twice the library's weighted-TV allowance inside the root (fitting error
    bound after `iters` iterations: longest coupling row r, column c, pooled
    sums s_p deep, plus a float64 reference's 14 T), plus 1e-9 relative."""
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


def uncertified_targets(phi32, N, d, cand):
    """Which of the candidate targets the exact separable path cannot certify
    from its float64 minima (so re-evaluates by brute force): the exact minimum
    w1 of c - phi (exact in float64: integer cost minus a float32) lies within
    delta(w) = d 2^-51 (|w| + 2 d (N-1)^2 + 1) of a float32 rounding boundary,
    or the runner-up w2 minus its delta rounds to the same float32."""
    X = ogrid.coords(N, d)
    phi = phi32.astype(np.float64)
    C2 = 2.0 * d * (N - 1) ** 2 + 1.0
    out = np.zeros(len(cand), dtype=bool)
    for s in range(0, len(cand), 64):
        J = cand[s:s + 64]
        t = ogrid.cost64(X, X[J], 2) - phi[:, None]
        i1 = np.argmin(t, axis=0)
        w1 = t[i1, np.arange(len(J))]
        t[i1, np.arange(len(J))] = np.inf
        w2 = t.min(axis=0)
        d1 = d * 2.0 ** -51 * (np.abs(w1) + C2)
        d2 = d * 2.0 ** -51 * (np.abs(w2) + C2)
        psi = (w1).astype(np.float32)
        bad = ((w1 - d1).astype(np.float32) != (w1 + d1).astype(np.float32)) | \
              ((w2 - d2).astype(np.float32) <= psi)
        out[s:s + 64] = bad
    return out


@pytest.mark.parametrize("fam", ["grf", "cauchy"])
def test_exact_separable_on_pipeline_potentials_256(fam, big_records):
    N, d, k, p = 256, 2, 8, 2
    R = big_records
    ft = R[f"{fam}_f"]
    fh_ref = lower.upscale_potential(ft, N, d, k).astype(np.float32)
    fhat = qbw.upscale_potential(dev(ft), N, d, k)
    assert np.array_equal(fhat.cpu().numpy(), fh_ref)
    print(f"exact separable 256^2 {fam}", flush=True)
    g, garg, nfb_g = qbw.ctransform_exact(fhat, N, d, want_argmin=True, return_fallback=True)
    f, farg, nfb_f = qbw.ctransform_exact(g, N, d, want_argmin=True, return_fallback=True)
    assert nfb_g > 0 and nfb_f > 0
    # the whole vectors equal the all-pairs kernel's
    ga, gaa = qbw.ctransform(fhat, N, d, p, want_argmin=True)
    fa, faa = qbw.ctransform(g, N, d, p, want_argmin=True)
    assert torch.equal(g, ga) and torch.equal(garg, gaa)
    assert torch.equal(f, fa) and torch.equal(farg, faa)
    # 400 sampled targets per transform against the oracle: half of them among
    # targets the float64 certification cannot settle
    rng = si.rng(9300 + (fam == "cauchy"))
    for src, val, arg in ((fh_ref, g, garg), (g.cpu().numpy(), f, farg)):
        cand = rng.choice(N * N, 6000, replace=False)
        bad = uncertified_targets(src, N, d, cand)
        assert bad.sum() >= 10, bad.sum()
        tg = np.concatenate([cand[bad][:200], cand[~bad][:200]])
        ref, refarg = lower.ctransform_o32(src, N, d, p, targets=tg)
        assert np.array_equal(val.cpu().numpy()[tg], ref)
        assert np.array_equal(arg.cpu().numpy()[tg].astype(np.int64), refarg)


@pytest.mark.parametrize("fam", ["grf", "cauchy"])
def test_exact_separable_windows_on_pipeline_potentials_256(fam, big_records, monkeypatch):
    # values only at 16 targets per lane: the two-dimensional stages scan
    # argmin windows (items of 64 lines x 32 targets on eight waves, the
    # benchmark's configuration); whole vectors against the all-pairs kernel,
    # sampled targets against the oracle
    monkeypatch.setenv("QBW_XS_T", "16")
    N, d, k, p = 256, 2, 8, 2
    R = big_records
    fh_ref = lower.upscale_potential(R[f"{fam}_f"], N, d, k).astype(np.float32)
    fhat = dev(fh_ref)
    print(f"exact separable windows 256^2 {fam}", flush=True)
    g, nfb_g = qbw.ctransform_exact(fhat, N, d, return_fallback=True)
    f, nfb_f = qbw.ctransform_exact(g, N, d, return_fallback=True)
    assert nfb_g > 0 and nfb_f > 0
    ga = qbw.ctransform(fhat, N, d, p)
    fa = qbw.ctransform(g, N, d, p)
    assert torch.equal(g, ga) and torch.equal(f, fa)
    rng = si.rng(9310 + (fam == "cauchy"))
    for src, val in ((fh_ref, g), (g.cpu().numpy(), f)):
        tg = rng.choice(N * N, 400, replace=False)
        ref, _ = lower.ctransform_o32(src, N, d, p, targets=tg)
        assert np.array_equal(val.cpu().numpy()[tg].view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("fam", ["grf", "cauchy"])
def test_upper_bound_256_against_oracle(fam, big_records):
    N, d, k, p = 256, 2, 8, 2
    R = big_records
    r, c, v, ft = R[f"{fam}_rows"], R[f"{fam}_cols"], R[f"{fam}_vals"], R[f"{fam}_f"]
    mu, nu = si.config3_pair(N, fam)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=qbw.Coarse(r, c, v, ft), separable="exact")
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    print(f"256^2 {fam}: upper {out['upper']!r} oracle {U['upper']!r} "
          f"excess {(out['upper'] - U['upper']) / U['upper']:.3e} relative", flush=True)
    assert out["ipf_iters"] == U["iters"]
    assert out["upper_cost"] >= U["plan_cost"]
    assert out["upper_cost"] == pytest.approx(U["plan_cost"], rel=1e-9)
    assert U["upper"] <= out["upper"] <= U["upper"] + ub_tol(mu, nu, N, d, p, k, U["upper"], r, c, U["iters"])


def test_config5_one_job_per_family_against_oracle():
    jobs_np = si.config5_jobs(128)
    jobs = [(dev(mu), dev(nu), k, p) for (N, d, k, p, mu, nu) in jobs_np]
    pooled = [(qbw.sumpool(a, k).cpu().numpy(), qbw.sumpool(b, k).cpu().numpy(), a.shape[0], a.dim(), k, p)
              for a, b, k, p in jobs]
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        recs = list(ex.map(lambda t: qbw.coarse_solve(*t), pooled))
    B = qbw.Batch(jobs, coarse=recs, backward=True, graph=True, autotune=True)
    B.run()
    out = B.results()
    seen = set()
    for i, (N, d, k, p, mu, nu) in enumerate(jobs_np):
        if (N, d, p) in seen:
            continue
        seen.add((N, d, p))
        rec = recs[i]
        o = out[i]
        print(f"config 5 job {i}: N={N} d={d} k={k} p={p}", flush=True)
        P = N ** d
        if P <= 4096:
            L = lower.lower_bound_o32(mu, nu, rec.f, k, p)
            assert o["lower_S"] == pytest.approx(L["S_emit"], rel=1e-9)
            assert o["lower"] == pytest.approx(L["lower"], rel=1e-9)
            assert o["feas_shift"] == pytest.approx(L["shift"], rel=1e-12)
        else:
            # sampled targets of both transforms, then the bound re-summed
            fh_ref = lower.upscale_potential(rec.f, N, d, k).astype(np.float32)
            fhat = qbw.upscale_potential(dev(rec.f), N, d, k)
            assert np.array_equal(fhat.cpu().numpy(), fh_ref)
            g, garg = qbw.ctransform(fhat, N, d, p, want_argmin=True)
            f = qbw.ctransform(g, N, d, p)
            tg = si.rng(9400 + i).choice(P, 96, replace=False)
            ref, refarg = lower.ctransform_o32(fh_ref, N, d, p, targets=tg)
            assert np.array_equal(g.cpu().numpy()[tg], ref)
            assert np.array_equal(garg.cpu().numpy()[tg].astype(np.int64), refarg)
            gn = g.cpu().numpy()
            ref_f, _ = lower.ctransform_o32(gn, N, d, p, targets=tg)
            assert np.array_equal(f.cpu().numpy()[tg], ref_f)
            fn = f.cpu().numpy()
            S = lower.fsum_dot(fn, mu.reshape(-1)) + lower.fsum_dot(gn, nu.reshape(-1))
            shift = lower.feasibility_shift(float(np.abs(fh_ref).max()), float(np.abs(gn).max()),
                                            float(np.abs(fn).max()), p, P)
            assert o["feas_shift"] == pytest.approx(shift, rel=1e-12)
            assert o["lower_S"] == pytest.approx(S - shift, rel=1e-9)
        U = upper.upper_bound_o64(mu, nu, rec.rows, rec.cols, rec.vals, k, p)
        assert o["ipf_iters"] == U["iters"]
        assert o["upper_cost"] >= U["plan_cost"]
        assert o["upper_cost"] == pytest.approx(U["plan_cost"], rel=1e-9)
        assert U["upper"] <= o["upper"] <= U["upper"] + ub_tol(mu, nu, N, d, p, k, U["upper"], rec.rows,
                                                                 rec.cols, U["iters"])
    assert len(seen) == 10


def _block_preserving(m, k, v):
    """v minus its m-weighted mean over each k x k block: sum_block m v = 0
    for every block, so the pooled masses do not move."""
    N = m.shape[0]
    n = N // k
    mb = m.reshape(n, k, n, k)
    vb = v.reshape(n, k, n, k)
    mean = (mb * vb).sum(axis=(1, 3), keepdims=True) / mb.sum(axis=(1, 3), keepdims=True)
    return (vb - mean).reshape(N, N)


@pytest.mark.parametrize("frozen_T", [False, True])
def test_config4_batched_central_differences(frozen_T):
    # Gradient contract: coarse solution frozen, fitting iterations T frozen.
    # Directions that keep every block's mass leave the pooled masses, hence
    # the coarse problem and T = 1, unchanged; general mass-preserving
    # directions are checked on a batch whose fitting is capped at its
    # forward T (one iteration), so the function differenced is the frozen one.
    pairs = si.config4_pairs(64)
    k, p = 8, 2
    base = [(dev(a), dev(b)) for a, b in pairs]
    jobs = [(a.clone(), b.clone(), k, p) for a, b in base]
    B = qbw.Batch(jobs, backward=True, graph=True, max_ipf_iter=1 if frozen_T else 50)
    for ga, gb in B.grads:
        ga.zero_()
        gb.zero_()
    dl, du = 0.6, 1.4
    B.run(np.full(64, dl), np.full(64, du))
    out0 = B.results()
    assert all(o["ipf_iters"] == 1 for o in out0)
    grads = [(ga.clone(), gb.clone()) for ga, gb in B.grads]
    g = si.rng(9500 + frozen_T)
    h = 1e-4
    for idx in (7, 40):
        mu, nu = pairs[idx]
        for _ in range(2):
            vm = g.uniform(-1, 1, mu.shape)
            vn = g.uniform(-1, 1, nu.shape)
            if frozen_T:
                vm -= (mu * vm).sum() / mu.sum()
                vn -= (nu * vn).sum() / nu.sum()
            else:
                vm = _block_preserving(mu, k, vm)
                vn = _block_preserving(nu, k, vn)

            def F(s):
                # the batch reads its measures through their pointers: rewrite them in place
                jobs[idx][0].copy_(dev(mu * (1 + s * vm)))
                jobs[idx][1].copy_(dev(nu * (1 + s * vn)))
                B.run(np.full(64, 0.0), np.full(64, 0.0))
                o = B.results()[idx]
                assert o["ipf_iters"] == 1
                return dl * o["lower"] + du * (o["upper_cost"] ** (1 / p))

            fd = (F(h) - F(-h)) / (2 * h)
            ga, gb = grads[idx]
            an = float((ga.cpu().numpy() * mu * vm).sum() + (gb.cpu().numpy() * nu * vn).sum())
            print(f"config 4 pair {idx} (T frozen: {frozen_T}): fd {fd!r} analytic {an!r}", flush=True)
            assert fd == pytest.approx(an, rel=2e-5, abs=1e-7)
        jobs[idx][0].copy_(base[idx][0])
        jobs[idx][1].copy_(base[idx][1])
