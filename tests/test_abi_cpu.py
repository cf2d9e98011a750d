"""CPU checks of the C ABI: the library loads, exports what include/qbw.h
declares, and its host-side parts (network simplex, centre cost, argument
validation) behave.  No device calls."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import synth_inputs as si
from oracle import coarse, lp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qbw.h")


def header_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qbw_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2506_00976_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libqbw.so not built")
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2506_00976_amd import _lib
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(n for n, *_ in _lib.SIGNATURES) == syms


def test_version_and_default_opts(lib):
    assert b"gfx950" in lib.qbw_version()
    o = lib.qbw_default_opts()
    assert o.xi == 1e-12 and o.max_ipf_iter == 50 and o.flags == 0


@pytest.mark.parametrize("N,d,k,p,fa,fb", [
    (16, 2, 4, 2, "gmm", "grf"), (32, 2, 4, 1, "shapes", "cauchy"), (64, 2, 8, 2, "white_noise", "gmm"),
    (8, 3, 2, 2, "grf", "grf"), (16, 3, 4, 1, "gmm", "shapes"), (40, 2, 5, 2, "cauchy", "blobs")])
def test_host_simplex_certified_against_highs(lib, N, d, k, p, fa, fb):
    import paper_2506_00976_amd as qbw
    mu = si.family(fa, N, d, si.rng(9000 + N + p))
    nu = si.family(fb, N, d, si.rng(9001 + N + p))
    mt, nt = coarse.sumpool(mu, k), coarse.sumpool(nu, k)
    rec = qbw.coarse_solve(mt, nt, N, d, k, p)
    Ct = coarse.centre_cost(N, d, k, p)
    *_, obj = lp.solve_ot(mt, nt, Ct)
    cert = lp.certify(rec.rows, rec.cols, rec.vals, rec.f, rec.g, mt, nt, Ct)
    Q = len(mt)
    assert len(rec.vals) <= 2 * Q - 1
    assert cert["min_entry"] > 0
    assert cert["row_err"] <= 1e-15 and cert["col_err"] <= 1e-15
    tol = 0.0 if p == 2 else 1e-9 * Ct.max()
    assert cert["dual_viol"] <= tol and cert["slack_on_support"] <= max(tol, 1e-12 * Ct.max())
    # the certificate (feasible, dual feasible, no slack on the support) proves
    # optimality; HiGHS itself is only converged to its own tolerances
    assert rec.objective == pytest.approx(obj, rel=1e-9)
    assert cert["dual"] == pytest.approx(rec.objective, rel=1e-12)
    # normalised: sum mu~ f~ = 0, to within 1/2 for p = 2 (shift rounded to keep integer duals)
    assert abs(float(rec.f @ mt)) <= (0.5 if p == 2 else 1e-9 * max(1.0, np.abs(rec.f).max()))
    if p == 2:
        assert np.array_equal(rec.f, np.round(rec.f))   # integer costs -> integer duals


def _certified_optimal(rec, mt, nt, Ct, p):
    cert = lp.certify(rec.rows, rec.cols, rec.vals, rec.f, rec.g, mt, nt, Ct)
    assert len(rec.vals) <= 2 * len(mt) - 1
    assert cert["min_entry"] > 0
    assert cert["row_err"] <= 1e-15 and cert["col_err"] <= 1e-15
    tol = 0.0 if p == 2 else 1e-9 * Ct.max()
    assert cert["dual_viol"] <= tol and cert["slack_on_support"] <= max(tol, 1e-12 * Ct.max())
    assert cert["dual"] == pytest.approx(rec.objective, rel=1e-12)


def _dense_start(mt, nt, N, d, k, p):
    import paper_2506_00976_amd as qbw
    os.environ["QBW_COARSE_SOLVER"] = "dense"
    try:
        return qbw.coarse_solve(mt, nt, N, d, k, p)
    finally:
        del os.environ["QBW_COARSE_SOLVER"]


@pytest.mark.parametrize("fam", ["grf", "cauchy"])
def test_multiscale_coarse_solve_q1024_against_highs(lib, fam):
    # 256^2 pairs, k = 8: the multiscale start (the library's default) reaches
    # the optimum HiGHS found for the same pooled masses (stored objective),
    # with an optimality certificate, and the dense start's objective
    import paper_2506_00976_amd as qbw
    N, d, k, p = 256, 2, 8, 2
    mu, nu = si.config3_pair(N, fam)
    mt, nt = coarse.sumpool(mu, k), coarse.sumpool(nu, k)
    rec = qbw.coarse_solve(mt, nt, N, d, k, p)
    golden = np.load(os.path.join(ROOT, "tests", "golden", "records_256_k8.npz"))
    assert rec.objective == pytest.approx(float(golden[f"{fam}_obj"][0]), rel=1e-12)
    _certified_optimal(rec, mt, nt, coarse.centre_cost(N, d, k, p), p)
    assert rec.objective == pytest.approx(_dense_start(mt, nt, N, d, k, p).objective, rel=1e-13)


@pytest.mark.parametrize("N,d,k,p", [(256, 2, 8, 1), (32, 3, 2, 2), (32, 3, 2, 1), (48, 2, 2, 2), (64, 3, 4, 1)])
def test_multiscale_coarse_solve_certified(lib, N, d, k, p):
    # Q = 1024 (p = 1), 4096 (32^3, k = 2), 576 (n = 24: its half level has
    # 144 blocks, solved densely) and 4096 (64^3, k = 4): certificate of
    # optimality and the dense start's objective
    import paper_2506_00976_amd as qbw
    mu = si.family("grf", N, d, si.rng(9200 + N + d + p))
    nu = si.family("cauchy" if d == 2 else "gmm", N, d, si.rng(9201 + N + d + p))
    mt, nt = coarse.sumpool(mu, k), coarse.sumpool(nu, k)
    rec = qbw.coarse_solve(mt, nt, N, d, k, p)
    _certified_optimal(rec, mt, nt, coarse.centre_cost(N, d, k, p), p)
    assert rec.objective == pytest.approx(_dense_start(mt, nt, N, d, k, p).objective, rel=1e-12)


@pytest.mark.parametrize("p", [1, 2])
def test_multiscale_coarse_solve_with_empty_blocks(lib, p):
    # shapes: most blocks carry no mass and are left out of the LP, at both levels
    import paper_2506_00976_amd as qbw
    N, d, k = 128, 2, 4
    mu = si.shapes(N, d, si.rng(9300 + p))
    nu = si.shapes(N, d, si.rng(9301 + p))
    mt, nt = coarse.sumpool(mu, k), coarse.sumpool(nu, k)
    assert (mt == 0).sum() > 100 and (nt == 0).sum() > 100
    rec = qbw.coarse_solve(mt, nt, N, d, k, p)
    Ct = coarse.centre_cost(N, d, k, p)
    *_, obj = lp.solve_ot(mt, nt, Ct)
    assert rec.objective == pytest.approx(obj, rel=1e-9)
    _certified_optimal(rec, mt, nt, Ct, p)


def test_host_simplex_degenerate_and_identical(lib):
    import paper_2506_00976_amd as qbw
    N, d, k, p = 16, 2, 4, 2
    mu = si.grf(N, d, si.rng(9100))
    mt = coarse.sumpool(mu, k)
    rec = qbw.coarse_solve(mt, mt, N, d, k, p)
    assert rec.objective == 0.0
    u = np.full(16, 1 / 16)                  # uniform: massively degenerate
    rec = qbw.coarse_solve(u, u, N, d, k, p)
    assert rec.objective == 0.0
    one = np.zeros(16)
    one[3] = 1.0
    rec = qbw.coarse_solve(one, u, N, d, k, p)
    *_, obj = lp.solve_ot(one, u, coarse.centre_cost(N, d, k, p))
    assert rec.objective == pytest.approx(obj, rel=1e-14)


def test_host_errors(lib):
    import paper_2506_00976_amd as qbw
    with pytest.raises(qbw.QbwError, match="E_GRID"):
        qbw.coarse_solve(np.ones(9) / 9, np.ones(9) / 9, 15, 2, 4, 2)
    with pytest.raises(qbw.QbwError, match="E_GRID"):
        qbw.coarse_solve(np.ones(16) / 16, np.ones(16) / 16, 16, 2, 4, 3)
    with pytest.raises(qbw.QbwError, match="E_MASS"):
        qbw.coarse_solve(np.ones(16) / 16, np.ones(16) / 8, 16, 2, 4, 2)
    bad = np.ones(16) / 16
    bad[0] = -0.1
    with pytest.raises(qbw.QbwError, match="E_MASS"):
        qbw.coarse_solve(bad, np.ones(16) / 16, 16, 2, 4, 2)
    msg = lib.qbw_last_error().decode()
    assert "nonnegative" in msg


def test_coarse_cost_host(lib):
    import paper_2506_00976_amd as qbw
    for p in (1, 2):
        assert np.allclose(qbw.coarse_cost(24, 2, 3, p), coarse.centre_cost(24, 2, 3, p), rtol=1e-15, atol=0)


def test_device_calls_fail_loudly_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    h = C.c_void_p()
    assert lib.qbw_create(C.byref(h), 0) != 0
    import paper_2506_00976_amd as qbw
    with pytest.raises(qbw.QbwError):
        qbw.bounds(torch.zeros(8, 8, dtype=torch.float64), torch.zeros(8, 8, dtype=torch.float64), 2, 2)


def test_gaussian_plan_kernel_host(lib):
    import paper_2506_00976_amd as qbw
    from oracle import upper
    for k, d, sigma in [(4, 2, 1.0), (3, 3, 0.7), (8, 2, 2.5), (2, 3, 5.0)]:
        K = qbw.plan_kernel_gaussian(k, d, sigma)
        assert np.allclose(K, upper.plan_kernel_gaussian(k, d, sigma), rtol=1e-14, atol=0)
    assert np.allclose(qbw.plan_kernel_gaussian(4, 2, float("inf")), 1.0 / 256, rtol=1e-15, atol=0)
    with pytest.raises(qbw.QbwError):
        qbw.plan_kernel_gaussian(4, 2, 0.0)
    with pytest.raises(qbw.QbwError):
        qbw.plan_kernel_gaussian(32, 3, 1.0)     # k^d = 32768 offsets
