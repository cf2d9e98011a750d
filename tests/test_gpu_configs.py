"""The workload configurations through the batched path, on the GPU.

* config 2: the 45 pairs of ten 64x64 images (five families), k in {4, 8},
  p in {1, 2}, one batch per (k, p) and one mixed batch;
* config 3: a 512x512 pair (k = 32), c-transform sampled bit-exact;
* config 4: 64 Gaussian-mixture pairs at 64x64, k = 8, forward + backward;
* config 5: 128 uneven jobs (2D and 3D grids, k in {2,4,8}, p in {1,2}) in one
  persistent launch per stage, captured in a hipGraph, forward + backward.
Every batched result is compared with the single-pair path (identical
arithmetic, so bit-for-bit) and, on sampled jobs, with the CPU oracle.
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


KEYS = ("lower", "upper", "lower_S", "upper_cost", "feas_shift", "ipf_iters", "coarse_objective")


def check_against_single(jobs, out, recs=None):
    for i, (jb, o) in enumerate(zip(jobs, out)):
        a, b, k, p = jb[:4]
        s = qbw.bounds(a, b, k, p, coarse=None if recs is None else recs[i])
        for key in KEYS:
            assert s[key] == o[key], (i, key, s[key], o[key])
        assert o["lower"] <= o["upper"]


def test_config2_batches():
    pairs = si.config2_pairs()
    imgs = {}
    for i, j, mu, nu in pairs:
        imgs[i], imgs[j] = mu, nu
    t = {i: dev(m) for i, m in imgs.items()}
    mixed = []
    for k in (4, 8):
        for p in (1, 2):
            jobs = [(t[i], t[j], k, p) for i, j, _, _ in pairs]
            B = qbw.Batch(jobs)
            B.run()
            out = B.results()
            check_against_single(jobs[:6], out[:6])
            assert all(o["lower"] <= o["upper"] for o in out)
            mixed += [jobs[(k + p) % 45], jobs[(3 * k + p) % 45]]
            # oracle on one pair per batch (its own exact coarse solution)
            i, j, mu, nu = pairs[k + p]
            r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
            res = qbw.bounds(dev(mu), dev(nu), k, p, coarse=qbw.Coarse(r, c, v, ft))
            L = lower.lower_bound_o32(mu, nu, ft, k, p)
            assert res["lower"] == pytest.approx(L["lower"], rel=1e-9)
            U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
            assert res["upper_cost"] == pytest.approx(U["plan_cost"], rel=1e-9)
    B = qbw.Batch(mixed, graph=True)
    B.run()
    check_against_single(mixed, B.results())


def test_config3_512_k32_sampled():
    N, d, k, p = 512, 2, 32, 2
    mu, nu = si.config3_pair(N, "cauchy")
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    rec = qbw.Coarse(r, c, v, ft)
    fhat = qbw.upscale_potential(dev(ft), N, d, k)
    fh_ref = lower.upscale_potential(ft, N, d, k).astype(np.float32)
    assert np.array_equal(fhat.cpu().numpy(), fh_ref)
    g, garg = qbw.ctransform(fhat, N, d, p, want_argmin=True)
    tg = si.rng(9500).choice(N * N, 64, replace=False)
    ref, refarg = lower.ctransform_o32(fh_ref, N, d, p, targets=tg)
    assert np.array_equal(g.cpu().numpy()[tg], ref)
    assert np.array_equal(garg.cpu().numpy()[tg].astype(np.int64), refarg)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec)
    assert out["lower"] <= out["upper"]
    assert out["ipf_iters"] >= 1
    # uniform kernel: the fitted plan's cost is <pi~, C-bar> (quantization coupling identity)
    Cb = qbw.cbar(dev(mu), dev(nu), k, p).cpu().numpy()
    assert out["upper_cost"] == pytest.approx(float((Cb[r, c] * v).sum()), rel=1e-8)


def test_config4_batched_gradients():
    pairs = si.config4_pairs(64)
    k, p = 8, 2
    jobs = [(dev(a), dev(b), k, p) for a, b in pairs]
    B = qbw.Batch(jobs, backward=True, graph=True)
    for ga, gb in B.grads:
        ga.zero_()
        gb.zero_()
    dl = np.linspace(0.5, 1.5, 64)
    du = np.linspace(1.5, 0.5, 64)
    B.run(dl, du)
    out = B.results()
    for idx in (0, 17, 63):
        a, b = pairs[idx]
        ga, gb = B.grads[idx]
        res, sa, sb, _ = qbw.bounds_with_grads(jobs[idx][0], jobs[idx][1], k, p, dlower=dl[idx], dupper=du[idx])
        assert res["lower"] == out[idx]["lower"] and res["upper"] == out[idx]["upper"]
        assert torch.allclose(ga, sa, rtol=1e-12, atol=0) and torch.allclose(gb, sb, rtol=1e-12, atol=0)
    # one pair against the oracle gradient on the oracle's own coarse solution
    a, b = pairs[5]
    r, c, v, ft, gt, obj = upper.coarse_record_lp(a, b, k, p)
    res, ga, gb, _ = qbw.bounds_with_grads(dev(a), dev(b), k, p, coarse=qbw.Coarse(r, c, v, ft))
    L = lower.lower_bound_o32(a, b, ft, k, p)
    lgm, lgn = ograd.lower_grad(L["f32"], L["g32"], L["S_emit"], p)
    U = upper.upper_bound_o64(a, b, r, c, v, k, p)
    ugm, ugn, _ = ograd.upper_grad(a, b, r, c, v, k, p, U["iters"])
    ref = lgm + ugm
    assert np.allclose(ga.cpu().numpy().reshape(-1), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_config5_uneven_batch_one_launch():
    import concurrent.futures as cf
    jobs_np = si.config5_jobs(128)
    jobs = [(dev(mu), dev(nu), k, p) for (N, d, k, p, mu, nu) in jobs_np]
    pooled = [(qbw.sumpool(a, k).cpu().numpy(), qbw.sumpool(b, k).cpu().numpy(), a.shape[0], a.dim(), k, p)
              for a, b, k, p in jobs]
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        recs = list(ex.map(lambda t: qbw.coarse_solve(*t), pooled))
    B = qbw.Batch(jobs, coarse=recs, backward=True, graph=True, autotune=True)
    B.run()
    out = B.results()
    for i in range(0, 128, 9):
        a, b, k, p = jobs[i]
        res, sa, sb, _ = qbw.bounds_with_grads(a, b, k, p, coarse=recs[i])
        for key in KEYS:
            assert res[key] == out[i][key], (i, key)
        ga, gb = B.grads[i]
        assert torch.allclose(ga, sa, rtol=1e-12, atol=1e-300) and torch.allclose(gb, sb, rtol=1e-12, atol=1e-300)
    assert all(o["lower"] <= o["upper"] for o in out)
    # a small job against the oracle on the oracle's own coarse solution
    for i, (N, d, k, p, mu, nu) in enumerate(jobs_np):
        if N ** d <= 1024:
            r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
            res = qbw.bounds(jobs[i][0], jobs[i][1], k, p, coarse=qbw.Coarse(r, c, v, ft))
            L = lower.lower_bound_o32(mu, nu, ft, k, p)
            assert res["lower"] == pytest.approx(L["lower"], rel=1e-9)
            break


@pytest.mark.parametrize("N,k", [(256, 16), (256, 32), (512, 16)])
def test_config3_other_pooling_factors(N, k):
    # the remaining (size, k) pairs of the 256^2 / 512^2 configuration: sampled
    # c-transform targets bit-exact on the oracle's coarse potential, the plan
    # cost equal to <pi~, C-bar> (uniform kernel), and bracketing of a translate
    d, p = 2, 2
    mu, nu = si.config3_pair(N, "grf")
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
    rec = qbw.Coarse(r, c, v, ft)
    fh_ref = lower.upscale_potential(ft, N, d, k).astype(np.float32)
    fhat = qbw.upscale_potential(dev(ft), N, d, k)
    assert np.array_equal(fhat.cpu().numpy(), fh_ref)
    g, garg = qbw.ctransform(fhat, N, d, p, want_argmin=True)
    tg = si.rng(9600 + N + k).choice(N * N, 24, replace=False)
    ref, refarg = lower.ctransform_o32(fh_ref, N, d, p, targets=tg)
    assert np.array_equal(g.cpu().numpy()[tg], ref)
    assert np.array_equal(garg.cpu().numpy()[tg].astype(np.int64), refarg)
    out = qbw.bounds(dev(mu), dev(nu), k, p, coarse=rec)
    Cb = qbw.cbar(dev(mu), dev(nu), k, p).cpu().numpy()
    assert out["upper_cost"] == pytest.approx(float((Cb[r, c] * v).sum()), rel=1e-8)
    assert 0.0 <= out["lower"] <= out["upper"]
    a, b = si.translated_pair(N, d, (13, -7), si.rng(9700 + N + k))
    t = qbw.bounds(dev(a), dev(b), k, p)
    W = math.sqrt(13 ** 2 + 7 ** 2)
    assert t["lower"] <= W <= t["upper"]
