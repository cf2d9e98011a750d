"""The Python binding and the C ABI at their edges: buffers of the wrong size
are refused before any launch, and batch runs issued back to back without a
synchronisation keep their own upstream gradients."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import upper

pytestmark = pytest.mark.gpu

qbw = pytest.importorskip("paper_2506_00976_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qbw.load()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device="cuda:0")


def test_short_buffers_are_refused():
    N, d = 32, 2
    short = torch.zeros(N * N - 1, dtype=torch.float32, device="cuda:0")
    for fn in (lambda: qbw.ctransform(short, N, d, 2), lambda: qbw.ctransform_separable(short, N, d),
               lambda: qbw.ctransform_exact(short, N, d), lambda: qbw.ctransform_noalloc(short, N, d, 2)):
        with pytest.raises(qbw.QbwError):
            fn()
    a = torch.full((N, N), 1.0 / (N * N), dtype=torch.float64, device="cuda:0")
    b = torch.full((N // 2, N // 2), 4.0 / (N * N), dtype=torch.float64, device="cuda:0")
    with pytest.raises(qbw.QbwError):
        qbw.bounds(a, b, 4, 2)
    with pytest.raises(qbw.QbwError):
        qbw.upscale_potential(torch.zeros(63, dtype=torch.float64, device="cuda:0"), N, d, 4)
    with pytest.raises(qbw.QbwError):   # a gradient buffer of another size
        qbw.Batch([(a, a, 4, 2, torch.zeros(N * N - 2, dtype=torch.float64, device="cuda:0"),
                    torch.zeros_like(a))], backward=True)
    with pytest.raises(qbw.QbwError):   # a non-contiguous gradient buffer would be written as a copy
        qbw.Batch([(a, a, 4, 2, torch.zeros(N, 2 * N, dtype=torch.float64, device="cuda:0")[:, ::2],
                    torch.zeros_like(a))], backward=True)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_runs_back_to_back_keep_their_upstream_gradients(graph):
    # two runs with different (dlower, dupper) and no synchronisation between
    # them accumulate exactly the sum of the two single-pair gradients
    specs = [(64, 2, 8, 2), (32, 2, 4, 1), (16, 3, 4, 2)]
    jobs, recs = [], []
    for i, (N, d, k, p) in enumerate(specs):
        mu = si.family("grf", N, d, si.rng(9100 + 2 * i))
        nu = si.family("gmm", N, d, si.rng(9101 + 2 * i))
        r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, k, p)
        jobs.append((dev(mu), dev(nu), k, p))
        recs.append(qbw.Coarse(r, c, v, ft, gt, obj))
    B = qbw.Batch(jobs, coarse=recs, backward=True, graph=graph)
    for ga, gb in B.grads:
        ga.zero_()
        gb.zero_()
    dl1, du1 = np.array([0.25, 2.0, -1.0]), np.array([3.0, 0.5, 1.5])
    dl2, du2 = np.array([1.75, -0.5, 4.0]), np.array([-2.0, 1.25, 0.125])
    torch.cuda.synchronize()
    B.run(dl1, du1)
    B.run(dl2, du2)          # no synchronisation in between
    torch.cuda.synchronize()
    for j, ((a, b, k, p), rec, (ga, gb)) in enumerate(zip(jobs, recs, B.grads)):
        _, sa1, sb1, _ = qbw.bounds_with_grads(a, b, k, p, coarse=rec, dlower=dl1[j], dupper=du1[j])
        _, sa2, sb2, _ = qbw.bounds_with_grads(a, b, k, p, coarse=rec, dlower=dl2[j], dupper=du2[j])
        ea, eb = sa1 + sa2, sb1 + sb2
        assert torch.allclose(ga, ea, rtol=1e-12, atol=1e-14 * float(ea.abs().max())), j
        assert torch.allclose(gb, eb, rtol=1e-12, atol=1e-14 * float(eb.abs().max())), j
