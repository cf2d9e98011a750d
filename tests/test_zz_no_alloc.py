"""The allocation-free c-transform entry point, qbw_ctransform_noalloc, called
through the C ABI and compared bit for bit (values and arg-mins) with
qbw_ctransform on the same seeded potentials: two calls in a row on one
device, the second with a smaller grid, so the second runs on scratch that the
first left behind."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu

qbw = pytest.importorskip("paper_2506_00976_amd")
from paper_2506_00976_amd._lib import QbwGrid  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qbw.load()


def _potential(N, d, seed):
    g = si.rng(seed)
    # a smooth part plus noise, with exact ties from a coarse lattice
    x = g.normal(size=(N,) * d) * 3.0 + np.round(g.normal(size=(N,) * d) * 8.0) / 4.0
    return torch.tensor(x.astype(np.float32).reshape(-1), device="cuda:0")


def _noalloc(N, d, p, src, dst, arg):
    grid = QbwGrid(d, N, 1, p)
    return qbw.load().qbw_ctransform_noalloc(
        qbw.context(0).handle, C.byref(grid), C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
        C.c_void_p(arg.data_ptr()) if arg is not None else None,
        C.c_void_p(torch.cuda.current_stream().cuda_stream))


# (first call, second smaller call): 2D and 3D, p = 1 and 2, ragged tiles
SEQUENCES = [
    [(256, 2, 2), (40, 2, 2)],
    [(128, 2, 1), (24, 2, 1)],
    [(32, 3, 2), (9, 3, 1)],
    [(64, 2, 1), (15, 2, 2)],
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=lambda s: "-".join(f"{N}^{d}p{p}" for N, d, p in s))
def test_noalloc_equals_ctransform_two_calls(seq):
    for i, (N, d, p) in enumerate(seq):
        print(f"noalloc case N={N} d={d} p={p} call={i}", flush=True)
        src = _potential(N, d, 5100 + 10 * N + d + p)
        ref, refarg = qbw.ctransform(src, N, d, p, want_argmin=True)
        dst = torch.full_like(src, float("nan"))
        arg = torch.full(src.shape, -7, dtype=torch.int32, device=src.device)
        assert _noalloc(N, d, p, src, dst, arg) == 0, qbw.load().qbw_last_error()
        assert torch.equal(dst, ref)
        assert torch.equal(arg, refarg)
        # without arg-mins
        dst2 = torch.full_like(src, float("nan"))
        assert _noalloc(N, d, p, src, dst2, None) == 0, qbw.load().qbw_last_error()
        assert torch.equal(dst2, ref)
        # the Python binding's wrapper of the same entry point
        out, oarg = qbw.ctransform_noalloc(src, N, d, p, argmin=torch.empty_like(arg))
        assert torch.equal(out, ref) and torch.equal(oarg, refarg)


def test_noalloc_rejects_grids_beyond_its_scratch():
    # 2900^2 pixels need more than the 64 MiB scratch even at one source split;
    # the host rejects the call before any launch, so the buffers stay untouched
    N, d, p = 2896, 2, 2
    src = torch.zeros(N * N, dtype=torch.float32, device="cuda:0")
    dst = torch.full_like(src, 3.0)
    rc = _noalloc(N, d, p, src, dst, None)
    assert rc != 0
    msg = qbw.load().qbw_last_error().decode()
    assert "scratch" in msg
    assert bool((dst == 3.0).all())
    # a call after the rejected one still works
    src = _potential(48, 2, 5300)
    ref = qbw.ctransform(src, 48, 2, 2)
    out = torch.empty_like(src)
    assert _noalloc(48, 2, 2, src, out, None) == 0
    assert torch.equal(out, ref)
