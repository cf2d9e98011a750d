#!/usr/bin/env python
"""Benchmark: bound pairs per second at 256x256, k = 8, p = 2 (lower + upper
bound), batched forward + backward, on one MI355X.

One step = one pass of the whole fine-grid path over a batch of B pairs:
pooling, potential upscaling, both c-transforms, lower-bound sums and shift,
IPF, plan cost, TV terms, finalisation, and the backward kernels of both
bounds, replayed as one hipGraph.  The c-transforms run as exact separable
minima (the same float32 values and arg-mins as the all-pairs kernel, which
is timed beside them on the same batch; --all-pairs swaps the two).  The coarse Kantorovich problems are solved
once before the timed region by the host network simplex (all host cores);
their cost is reported separately as the end-to-end rate.

Prints ONE JSON line (stdout); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 vector peak of MI355X: 157.3 TFLOP/s = 256 CUs x 128 FMA lanes/clk x 2 flop x 2.4 GHz,
# i.e. 78.6 T VALU lane-operations/s (measured: all-VGPR v_sub_f32 issues at ~100 lanes/clk/CU).
PEAK_LANE_OPS = 256 * 128 * 2.4e9
INSTR_PER_PAIR = 1.5               # minimum per (source, target) pair: one v_sub_f32 + half a v_min3_f32
PEAK_PAIRS = PEAK_LANE_OPS / INSTR_PER_PAIR
# FP64 vector peak: 78.6 TFLOP/s counts an FMA as two, i.e. 256 CUs x 64 lanes/clk x 2.4 GHz
# = 39.3 T float64 lane-operations/s.  Per (source, target) candidate an exact separable
# stage needs at least a v_add_f64 and a v_min_f64 (the best value); with arg-mins also
# v_cmp_lt_f64 + v_cndmask_b32 (the index) and v_max_f64 + v_min_f64 (the runner-up).  The
# timed batch asks for no arg-mins (the gradients in a and b are f and g themselves).
# The value-only two-dimensional stages scan argmin windows (the per-axis candidates
# are Monge): per item, its two boundary targets over every source, its other targets
# over the window between their minimisers.  The candidate count stays the separable
# evaluation's (P N per stage, every source for every target), so against this peak
# the fraction is the rate relative to evaluating all of them at full issue rate.
PEAK_F64_LANE_OPS = 256 * 64 * 2.4e9
XS_INSTR_PER_CAND = 2
XS_INSTR_PER_CAND_ARGMIN = 6
PEAK_XS = PEAK_F64_LANE_OPS / XS_INSTR_PER_CAND


# The paper's own figures (Section 5, NVIDIA L40 GPU + AMD EPYC 9654 CPU, JAX
# for the bounds, an exact network-simplex solver for the reference), as
# percentages, each pair [kappa = 2, kappa = 4]: relative errors against the
# exact distance (accuracy table, DOTmark classes at 128x128) and computation
# time relative to the exact solver (DOTmark time table; 3D cryo-EM time
# table at 32^3).  Other hardware, other data: context, not a target.
PAPER_CONTEXT = {
    "hardware": "NVIDIA L40 GPU + AMD EPYC 9654 CPU; bounds in JAX, exact OT by network simplex (Section 5)",
    "units": "percent; each entry [kappa=2, kappa=4]",
    "relative_error_dotmark_128": {
        "dual_upscaling_lower": {"classic": {"p1": [0.3, 0.7], "p2": [0.7, 2.4]},
                                 "microscopy": {"p1": [0.4, 0.9], "p2": [0.2, 0.7]},
                                 "shapes": {"p1": [0.5, 1.0], "p2": [0.9, 1.7]}},
        "primal_upscaling_upper": {"classic": {"p1": [9.6, 23.0], "p2": [2.2, 8.8]},
                                   "microscopy": {"p1": [2.4, 6.5], "p2": [0.7, 2.7]},
                                   "shapes": {"p1": [3.2, 7.8], "p2": [1.4, 3.6]}},
        "weighted_cost_upper": {"classic": {"p1": [3.1, 11.0], "p2": [1.6, 7.9]},
                                "microscopy": {"p1": [0.9, 3.4], "p2": [0.5, 2.2]},
                                "shapes": {"p1": [1.1, 3.6], "p2": [1.2, 3.2]}},
        "min_cost_lower": {"classic": {"p1": [10.0, 27.0], "p2": [13.0, 33.0]},
                           "microscopy": {"p1": [6.2, 17.0], "p2": [5.5, 16.0]},
                           "shapes": {"p1": [7.3, 20.0], "p2": [7.7, 20.0]}}},
    "relative_time_dotmark": {
        "dual_upscaling_lower": {"classic": {"p1": [4.9, 0.2], "p2": [6.1, 0.3]},
                                 "microscopy": {"p1": [14.4, 2.2], "p2": [15.6, 2.0]},
                                 "shapes": {"p1": [7.8, 1.5], "p2": [7.4, 1.2]}},
        "primal_upscaling_upper": {"classic": {"p1": [5.0, 0.3], "p2": [6.1, 0.3]},
                                   "microscopy": {"p1": [20.7, 6.6], "p2": [17.4, 3.0]},
                                   "shapes": {"p1": [15.1, 10.8], "p2": [9.6, 4.2]}},
        "weighted_cost_upper": {"classic": {"p1": [4.4, 0.3], "p2": [6.1, 0.4]},
                                "microscopy": {"p1": [16.7, 2.3], "p2": [15.4, 1.9]},
                                "shapes": {"p1": [10.2, 1.9], "p2": [7.9, 1.5]}}},
    "relative_time_cryoem_32cubed": {
        "dual_upscaling_lower": {"p1": [0.55, 0.33], "p2": [0.19, 0.04]},
        "primal_upscaling_upper": {"p1": [1.09, 27.23], "p2": [0.30, 0.16]},
        "weighted_cost_upper": {"p1": [0.22, 0.12], "p2": [0.22, 0.06]},
        "min_cost_lower": {"p1": [0.20, 0.11], "p2": [0.21, 0.04]}},
    "absolute_throughput": None,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)

def settle(batch, seconds=0.1):
    """Run `batch` untimed for about `seconds`: after the host-side phases
    the GPU's clocks are still ramping, and the first milliseconds of steps
    run a few per cent slower than the steady state."""
    import torch
    t = time.perf_counter()
    while time.perf_counter() - t < seconds:
        for _ in range(8):
            batch.run()
        torch.cuda.synchronize()


def kernel_source_hash() -> str:
    """Hash of the code that decides what one c-transform launch does: the
    device helpers and the c-transform section of kernels.hip, the shared
    header, the host planner (item table, splits) and the build flags, with
    comments and blank space removed.  Edits to comments or to other kernels
    do not invalidate counters taken on the same c-transform code."""
    import re
    csrc = os.path.join(ROOT, "paper_2506_00976_amd", "csrc")

    def norm(text):
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        return " ".join(text.split())

    with open(os.path.join(csrc, "kernels.hip")) as fh:
        src = fh.read()
    mark = "// ------------------------------------------------------------------ "
    helpers = src[:src.index(mark + "pooling")]
    ct = src[src.index(mark + "c-transform\n"):src.index(mark + "separable c-transform")]
    launch = src[src.index("int ctransform_waves_per_cu()"):src.index("int launch_merge(")]
    parts = [helpers, ct, launch]
    for name in ("qbw_internal.h", "api.cpp"):
        with open(os.path.join(csrc, name)) as fh:
            parts.append(fh.read())
    with open(os.path.join(ROOT, "paper_2506_00976_amd", "build.py")) as fh:
        parts.append(fh.read())
    return hashlib.sha256("\n".join(norm(x) for x in parts).encode()).hexdigest()[:16]


def xs_source_hash() -> str:
    """The same for the exact separable c-transform: the device helpers, its
    section of kernels.hip and its launchers, the shared header, the host
    planner and the build flags."""
    import re
    csrc = os.path.join(ROOT, "paper_2506_00976_amd", "csrc")

    def norm(text):
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        return " ".join(text.split())

    with open(os.path.join(csrc, "kernels.hip")) as fh:
        src = fh.read()
    mark = "// ------------------------------------------------------------------ "
    helpers = src[:src.index(mark + "pooling")]
    xs = src[src.index(mark + "exact separable c-transform"):src.index(mark + "separable c-transform (p = 2)")]
    launch = src[src.index("int launch_xs_squares("):src.index("int launch_sep_argmin(")]
    parts = [helpers, xs, launch]
    for name in ("qbw_internal.h", "api.cpp"):
        with open(os.path.join(csrc, name)) as fh:
            parts.append(fh.read())
    with open(os.path.join(ROOT, "paper_2506_00976_amd", "build.py")) as fh:
        parts.append(fh.read())
    return hashlib.sha256("\n".join(norm(x) for x in parts).encode()).hexdigest()[:16]


def read_traffic(kernel: str = "xs_stage"):
    """HBM bytes per launch of the kernel ("xs_stage" or "ctransform") from
    the committed counter summary, only if it was taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_256_k8.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    want = xs_source_hash() if kernel == "xs_stage" else kernel_source_hash()
    if d.get("kernel_source_sha256_16") != want:
        return None
    return d.get("bytes_per_launch")


def make_inputs(batch: int, N: int = 256):
    import synth_inputs as si
    pairs = []
    for i in range(batch):
        fam = "grf" if i % 2 == 0 else "cauchy"
        pairs.append(si.config3_pair(N, fam, idx=i // 2))
    return pairs


def cpu_baseline(N: int, k: int, p: int, budget_s: float = 10.0):
    """The oracle as it stands, on a bounded sample of one 256x256 pair: as many
    targets of the float32 c-transform as fit in about `budget_s` seconds
    (extrapolated to all 2 N^2 targets of the two transforms) plus the full
    upper bound and its gradient; the lower-bound gradient is f, g themselves."""
    import synth_inputs as si
    from oracle import grad as og
    from oracle import lower, upper
    mu, nu = si.config3_pair(N, "grf")
    R = np.load(os.path.join(ROOT, "tests", "golden", "records_256_k8.npz"))
    r, c, v, ft = R["grf_rows"], R["grf_cols"], R["grf_vals"], R["grf_f"]
    P = N * N
    t0 = time.perf_counter()
    fh = lower.upscale_potential(ft, N, 2, k).astype(np.float32)
    order = np.random.Generator(np.random.PCG64(0)).permutation(P)
    done = 0
    while done < P and time.perf_counter() - t0 < budget_s:
        lower.ctransform_o32(fh, N, 2, p, targets=order[done:done + 128])
        done += 128
    t_ct = time.perf_counter() - t0
    t1 = time.perf_counter()
    U = upper.upper_bound_o64(mu, nu, r, c, v, k, p)
    og.upper_grad(mu, nu, r, c, v, k, p, U["iters"])
    t_ub = time.perf_counter() - t1
    per_pair = t_ct / done * 2 * P + t_ub
    return {"value": 1.0 / per_pair, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"one 256x256 GRF pair, k=8: {done} random targets of the float32 c-transform "
                      f"(scaled to the 2 x {P} targets of both transforms) + the full upper bound and "
                      f"its gradient; {t_ct + t_ub:.1f} s measured, {per_pair:.1f} s per bound pair",
            "seconds_measured": t_ct + t_ub, "seconds_upper": t_ub}


def _oracle_targets_worker(fh, N, p, targets, budget_s):
    """One process of the all-cores oracle timing: float32 c-transform targets,
    128 at a time, until the budget is spent.  Returns (targets done, seconds)."""
    from oracle import lower
    t0 = time.perf_counter()
    done = 0
    while done < len(targets) and time.perf_counter() - t0 < budget_s:
        lower.ctransform_o32(fh, N, 2, p, targets=targets[done:done + 128])
        done += 128
    return done, time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_all_cores(N: int, k: int, p: int, budget_s: float = 10.0):
    """The same oracle c-transform sample on every host core (up to 16 worker
    processes, each on its own random targets); the upper bound's share is
    taken from the single-core run.  Workers are spawned processes that never
    touch the GPU."""
    import multiprocessing as mp
    import concurrent.futures as cf
    import synth_inputs as si
    from oracle import lower
    R = np.load(os.path.join(ROOT, "tests", "golden", "records_256_k8.npz"))
    fh = lower.upscale_potential(R["grf_f"], N, 2, k).astype(np.float32)
    P = N * N
    workers = min(os.cpu_count() or 1, 16)
    order = np.random.Generator(np.random.PCG64(1)).permutation(P)
    slices = np.array_split(order, workers)
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_oracle_targets_worker, [fh] * workers, [N] * workers, [p] * workers, slices,
                          [budget_s] * workers))
    done = sum(d for d, _ in out)
    secs = max(t for _, t in out)
    rate = done / secs   # targets per second over all workers
    return {"targets_per_s": rate, "cores": workers, "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "targets_done": done, "seconds": secs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the 128-job uneven batch (its coarse solves take seconds of host time)")
    ap.add_argument("--profile", action="store_true",
                    help="only the timed steps (for rocprofv3 runs)")
    ap.add_argument("--eager", action="store_true",
                    help="launch the kernels one by one on the stream (the default)")
    ap.add_argument("--graph", action="store_true",
                    help="replay a captured hipGraph per step instead")
    ap.add_argument("--all-pairs", action="store_true",
                    help="time the all-pairs c-transform path instead of the exact separable one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain device copy of 1 GiB (calibrates FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the method's "
              "fine-grid path runs on a single MI355X here (the pairs of a batch are independent, so "
              "a batch would be split over GPUs, one process each).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2506_00976_amd as qbw

    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8, "copies": 3}))
        return

    N, d, k, p = 256, 2, 8, 2
    B = args.batch
    dev = torch.device("cuda:0")
    qbw.load()
    log(f"[bench] generating {B} pairs at {N}x{N}")
    pairs = make_inputs(B, N)
    A = [torch.tensor(a, device=dev) for a, _ in pairs]
    Bm = [torch.tensor(b, device=dev) for _, b in pairs]
    torch.cuda.synchronize()

    # ---- coarse solutions: pool on the device, host network simplex on all cores
    t0 = time.perf_counter()
    mts = [qbw.sumpool(a, k).cpu().numpy() for a in A]
    nts = [qbw.sumpool(b, k).cpu().numpy() for b in Bm]
    t_pool = time.perf_counter() - t0
    workers = min(os.cpu_count() or 1, 16)

    def solve_all(dense: bool):
        if dense:
            os.environ["QBW_COARSE_SOLVER"] = "dense"
        try:
            t = time.perf_counter()
            with cf.ThreadPoolExecutor(max_workers=workers) as ex:
                rs = list(ex.map(lambda t: qbw.coarse_solve(t[0], t[1], N, d, k, p), zip(mts, nts)))
            return rs, time.perf_counter() - t
        finally:
            os.environ.pop("QBW_COARSE_SOLVER", None)

    # the library's multiscale start against pricing every block pair from the
    # first pivot, on the same pooled masses, each the best of two rounds
    runs = {False: [], True: []}
    for _ in range(2):
        for dense in (True, False):
            runs[dense].append(solve_all(dense))
    recs = runs[False][-1][0]
    recs_d = runs[True][-1][0]
    t_solve = min(t for _, t in runs[False])
    t_coarse_dense = min(t for _, t in runs[True])
    t_coarse = t_pool + t_solve
    same_obj = all(abs(x.objective - y.objective) <= 1e-12 * abs(y.objective) for x, y in zip(recs, recs_d))
    log(f"[bench] coarse: pooling + transfer {t_pool:.3f} s, solves {t_solve:.3f} s (multiscale start), "
        f"{t_coarse_dense:.3f} s (dense start) for {B} pairs on {workers} threads; same objectives: {same_obj}")

    grads = [(torch.zeros_like(a), torch.zeros_like(b)) for a, b in zip(A, Bm)]
    jobs = [(a, b, k, p, ga, gb) for (a, b), (ga, gb) in zip(zip(A, Bm), grads)]
    # p = 2 c-transforms: exact separable (the all-pairs float32 values and
    # arg-mins from per-axis float64 minima), or the all-pairs kernel itself
    mode = False if args.all_pairs else "exact"
    # Steps launch their kernels on the stream: the coarse launch's stream
    # joins the batch's with a stream event, which costs less than the
    # cross-queue dependency of a replayed graph's parallel branch (both are
    # timed; the other mode is reported beside the value)
    use_graph = args.graph and not args.eager
    batch = qbw.Batch(jobs, coarse=recs, backward=True, graph=use_graph, separable=mode)
    if not args.profile:
        settle(batch)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} {'graph' if use_graph else 'stream'} steps (batch {B}, fwd+bwd)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = B / (ms_step / 1e3)
    res = batch.results()
    if args.profile:
        print(json.dumps({"profile_run": True, "ms_per_step": ms_step}))
        return
    log(f"[bench] {ms_step:.3f} ms/step -> {value:.1f} pairs/s")
    # the other launch mode on the same work
    ob_mode = qbw.Batch(jobs, coarse=recs, backward=True, graph=not use_graph, separable=mode)
    settle(ob_mode)
    for _ in range(args.warmup):
        ob_mode.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ob_mode.run()
    torch.cuda.synchronize()
    ms_other_mode = (time.perf_counter() - t0) * 1e3 / args.steps
    same_mode = all(x[key] == y[key] for x, y in zip(ob_mode.results(), res) for key in ("lower", "upper"))
    del ob_mode
    launch_modes = {"stream": ms_other_mode if use_graph else ms_step,
                    "hipgraph": ms_step if use_graph else ms_other_mode, "bounds_identical": same_mode}
    log(f"[bench] ms/step by launch mode: stream {launch_modes['stream']:.3f}, hipGraph {launch_modes['hipgraph']:.3f}")

    # ---- the library's own end-to-end path: a batch built from the fine
    # measures alone (one pooling launch and one transfer for all pairs, host
    # network simplex on all cores, upload, plan), then one eager step
    def e2e_once():
        torch.cuda.synchronize()
        t = time.perf_counter()
        eb = qbw.Batch(jobs, coarse=None, backward=True, graph=False, separable=mode)
        t_create = time.perf_counter() - t
        eb.run()
        r = eb.results()
        return t_create, time.perf_counter() - t, r
    e2e = [e2e_once() for _ in range(5)]
    t_create = min(x[0] for x in e2e)
    t_e2e = min(x[1] for x in e2e)
    same_e2e = all(x[key] == y[key] for x, y in zip(e2e[-1][2], res) for key in ("lower", "upper"))
    log(f"[bench] library end-to-end: batch creation {t_create:.3f} s, with one step {t_e2e:.3f} s "
        f"-> {B / t_e2e:.1f} pairs/s; bounds as with the pre-solved coarse records: {same_e2e}")

    # ---- the dominant kernel, timed live with HIP events on its stream
    def kernel_timing(sep_mode):
        eager = qbw.Batch(jobs, coarse=recs, backward=True, graph=False, separable=sep_mode)
        settle(eager)
        eager.set_timing(True)
        for _ in range(max(3, args.steps // 2)):
            eager.run()
        mean, n = eager.ctransform_time()
        eager.set_timing(False)
        return mean, n, eager.ctransform_pairs()

    def roofline(sep_mode, mean, evals):
        ach = evals / (mean / 1e3)
        if sep_mode == "exact":
            return {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_XS / 1e12, "unit": "Tcand/s",
                    "frac": ach / PEAK_XS, "traffic": read_traffic("xs_stage"), "kernel": "k_xs_stage",
                    "work": "separable candidates, P N per stage launch; the kernel itself evaluates the two "
                            "boundary targets of each item over every source and the rest over argmin windows",
                    "mean_launch_ms": mean, "candidates_per_launch": evals}
        return {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_PAIRS / 1e12, "unit": "Tpair/s",
                "frac": ach / PEAK_PAIRS, "traffic": read_traffic("ctransform"), "kernel": "k_ctransform",
                "mean_launch_ms": mean, "pairs_per_launch": evals}

    mean_ms, launches, evals = kernel_timing(mode)
    roof = roofline(mode, mean_ms, evals)
    log(f"[bench] {roof['kernel']}: {launches} launches, mean {mean_ms:.3f} ms, "
        f"{roof['achieved']:.2f} {roof['unit']} ({roof['frac']:.1%} of {roof['peak']:.2f})")

    # ---- the other c-transform path on the same batch
    other = "exact" if mode is False else False
    ob = qbw.Batch(jobs, coarse=recs, backward=True, graph=True, separable=other)
    settle(ob)
    for _ in range(args.warmup):
        ob.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nrep_o = args.steps if other == "exact" else max(3, args.steps // 4)
    for _ in range(nrep_o):
        ob.run()
    torch.cuda.synchronize()
    ms_other = (time.perf_counter() - t0) * 1e3 / nrep_o
    rother = ob.results()
    del ob
    same = all(x[key] == y[key] for x, y in zip(rother, res) for key in ("lower", "upper", "lower_S", "feas_shift"))
    m_o, n_o, e_o = kernel_timing(other)
    roof_other = roofline(other, m_o, e_o)
    log(f"[bench] {'exact separable' if other else 'all-pairs'}: {ms_other:.3f} ms/step -> "
        f"{B / (ms_other / 1e3):.1f} pairs/s; {roof_other['kernel']} {roof_other['achieved']:.2f} "
        f"{roof_other['unit']} ({roof_other['frac']:.1%}); bounds identical: {same}")

    # ---- plain single-pair path (one pair per call, no graph, same accuracy)
    nplain = min(8, B)
    for i in range(2):
        qbw.bounds(A[i], Bm[i], k, p, coarse=recs[i], separable=mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nplain):
        qbw.bounds(A[i], Bm[i], k, p, coarse=recs[i], separable=mode)
    torch.cuda.synchronize()
    plain_fwd = nplain / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    for i in range(nplain):
        qbw.bounds_with_grads(A[i], Bm[i], k, p, coarse=recs[i], separable=mode)
    torch.cuda.synchronize()
    plain_fb = nplain / (time.perf_counter() - t0)
    log(f"[bench] plain: fwd {plain_fwd:.1f} pairs/s, fwd+bwd {plain_fb:.1f} pairs/s")

    # ---- the same batch with the separable p = 2 c-transforms (QBW_SEPARABLE)
    sep = qbw.Batch(jobs, coarse=recs, backward=True, graph=True, separable=True)
    settle(sep)
    for _ in range(args.warmup):
        sep.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sep.run()
    torch.cuda.synchronize()
    ms_sep = (time.perf_counter() - t0) * 1e3 / args.steps
    rsep = sep.results()
    log(f"[bench] separable: {ms_sep:.3f} ms/step -> {B / (ms_sep / 1e3):.1f} pairs/s")

    # ---- uneven batch: 128 jobs over 2D/3D grids, k in {2,4,8}, p in {1,2},
    # one persistent launch per stage in a hipGraph, autotuned tiling
    uneven = None
    if not args.no_uneven:
        import synth_inputs as si
        jobs5 = si.config5_jobs(128)
        J5 = [(torch.tensor(mu, device=dev), torch.tensor(nu, device=dev), kk, pp)
              for (_, _, kk, pp, mu, nu) in jobs5]
        t0 = time.perf_counter()
        pooled = [(qbw.sumpool(a, kk).cpu().numpy(), qbw.sumpool(b, kk).cpu().numpy(), a.shape[0], a.dim(), kk, pp)
                  for a, b, kk, pp in J5]
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            recs5 = list(ex.map(lambda t: qbw.coarse_solve(*t), pooled))
        t_c5 = time.perf_counter() - t0
        log(f"[bench] uneven batch: coarse solves {t_c5:.1f} s for {len(J5)} jobs on {workers} threads")
        b5 = qbw.Batch(J5, coarse=recs5, backward=True, graph=True, autotune=True)
        settle(b5)
        for _ in range(args.warmup):
            b5.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b5.run()
        torch.cuda.synchronize()
        ms5 = (time.perf_counter() - t0) * 1e3 / args.steps
        ev5 = qbw.Batch(J5, coarse=recs5, backward=True, graph=False, autotune=True)   # same tiling as b5
        settle(ev5)
        ev5.set_timing(True)
        for _ in range(3):
            ev5.run()
        m5, _ = ev5.ctransform_time()
        pairs5 = ev5.ctransform_pairs()
        log(f"[bench] uneven batch: {ms5:.3f} ms/step -> {len(J5) / (ms5 / 1e3):.1f} jobs/s; "
            f"c-transform {pairs5 / (m5 / 1e3) / 1e12:.2f} Tpair/s")
        r5 = b5.results()
        del b5, ev5
        # the same jobs with the p = 2 c-transforms on the exact separable path
        # (p = 1 jobs keep the autotuned all-pairs kernel)
        x5 = qbw.Batch(J5, coarse=recs5, backward=True, graph=True, autotune=True, separable="exact")
        settle(x5)
        for _ in range(args.warmup):
            x5.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x5.run()
        torch.cuda.synchronize()
        ms5x = (time.perf_counter() - t0) * 1e3 / args.steps
        same5 = all(x[key] == y[key] for x, y in zip(x5.results(), r5) for key in ("lower", "upper", "lower_S"))
        del x5
        log(f"[bench] uneven batch, exact separable p = 2: {ms5x:.3f} ms/step -> {len(J5) / (ms5x / 1e3):.1f} jobs/s; "
            f"bounds identical: {same5}")
        uneven = {"jobs": len(J5), "jobs_per_s": len(J5) / (ms5 / 1e3), "ms_per_step": ms5,
                  "workload": "128 jobs: 32^2, 64^2, 128^2, 16^3, 32^3 grids x k in {2,4,8} x p in {1,2}, "
                              "GRF measures, forward+backward, hipGraph, autotuned all-pairs c-transforms; coarse pre-solved",
                  "ctransform_Tpair_per_s": pairs5 / (m5 / 1e3) / 1e12,
                  "ctransform_ms_per_launch": m5, "coarse_seconds": t_c5,
                  "exact_separable_p2": {"jobs_per_s": len(J5) / (ms5x / 1e3), "ms_per_step": ms5x,
                                         "bounds_identical": same5}}

    # ---- upper bound with a non-uniform coupling-upscaling kernel (Gaussian,
    # sigma = 1 pixel) on the first pair: the fitting runs on fine vectors
    K = qbw.plan_kernel_gaussian(k, d, 1.0)
    kub = qbw.upper_kernel(A[0], Bm[0], k, p, K, coarse=recs[0], max_ipf_iter=50)
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        kub = qbw.upper_kernel(A[0], Bm[0], k, p, K, coarse=recs[0], max_ipf_iter=50)
    ms_kub = (time.perf_counter() - t0) * 1e3 / reps
    log(f"[bench] upper bound, Gaussian kernel: {ms_kub:.2f} ms per bound, {kub['ipf_iters']} fitting "
        f"iterations; upper {kub['upper']:.6f} (uniform kernel {res[0]['upper']:.6f})")
    upper_kernel = {"ms_per_bound": ms_kub, "ipf_iters": kub["ipf_iters"],
                    "ms_per_ipf_iter": ms_kub / max(1, kub["ipf_iters"]),
                    "upper": kub["upper"], "upper_uniform_kernel": res[0]["upper"],
                    "ipf_residual": kub["ipf_residual"],
                    "workload": "first pair of the batch (256x256, k=8, p=2), Gaussian kernel sigma=1 px, "
                                "at most 50 fitting iterations, coarse pre-solved, synchronous call"}

    # ---- batch-size sweep: the same workload at 8 and 128 pairs per step
    # (32 is the timed value above); each batch repeats the 32 pairs' measures
    sweep = {str(B): value}
    for Bs in (8, 128):
        idx = [i % B for i in range(Bs)]
        js = [(A[i], Bm[i], k, p, torch.zeros_like(A[i]), torch.zeros_like(Bm[i])) for i in idx]
        bs = qbw.Batch(js, coarse=[recs[i] for i in idx], backward=True, graph=use_graph, separable=mode)
        for _ in range(args.warmup):
            bs.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nrep = max(3, args.steps * 32 // Bs)
        for _ in range(nrep):
            bs.run()
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1e3 / nrep
        sweep[str(Bs)] = Bs / (ms_b / 1e3)
        del bs
    log("[bench] batch sizes: " + ", ".join(f"{kb} pairs -> {v:.1f} pairs/s" for kb, v in sorted(sweep.items(), key=lambda x: int(x[0]))))

    # consistency of the timed results with the single-pair path
    ref = qbw.bounds(A[0], Bm[0], k, p, coarse=recs[0], separable=mode)
    assert ref["lower"] == res[0]["lower"] and ref["upper"] == res[0]["upper"], (ref, res[0])

    out = {
        "metric": "bound pairs/sec at 256^2 k=8 (lower+upper), batched fwd+bwd",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mode else "f32",
        "data": "synthetic",
        "config": {"workload": f"batch of {B} pairs of 256x256 measures (GRF and Cauchy families), "
                               "k=8, p=2, forward+backward of both bounds, coarse solutions pre-solved",
                   "N": N, "d": d, "k": k, "p": p, "batch": B,
                   "precision": ("float32 c-transform results (the all-pairs reading) from float64 stage minima, "
                                 "float64 sums/IPF/plan cost" if mode else
                                 "float32 c-transforms, float64 sums/IPF/plan cost"),
                   "c_transform": ("exact separable: the all-pairs float32 values and arg-mins from "
                                   "per-axis float64 minima, certified per target" if mode else
                                   "all-pairs (lazy) kernel"),
                   "launch": "hipGraph replay per step" if use_graph else "kernels launched on the stream per step"},
        "launch_modes_ms_per_step": launch_modes,
        "roofline": roof,
        "roofline_note": ("the c-transform roofline is that of the timed path's kernel, "
                          + ("k_xs_stage (exact separable stages); the all-pairs k_ctransform is reported "
                             "beside it under all_pairs" if mode else "k_ctransform (all-pairs)")),
        ("all_pairs" if mode else "exact_separable"): {
            "pairs_per_s": B / (ms_other / 1e3), "ms_per_step": ms_other,
            "bounds_identical": same, "roofline": roof_other},
        "plain": {"fwd_pairs_per_s": plain_fwd, "fwd_bwd_pairs_per_s": plain_fb,
                  "batched_over_plain_fwd_bwd": value / plain_fb},
        "separable_p2": {"pairs_per_s": B / (ms_sep / 1e3), "ms_per_step": ms_sep,
                         "note": "same batch, c-transforms as d nested 1-D transforms (O(N^3) here); "
                                 "float32 rounding once per axis, larger derived shift",
                         "lower_sample": rsep[0]["lower"], "upper_sample": rsep[0]["upper"]},
        "end_to_end": {"coarse_seconds": t_coarse, "host_threads": workers,
                       "coarse_solver": "host network simplex, multiscale start (half-resolution problem "
                                        "solved first, its support's children priced first, optimality "
                                        "checked over every block pair)",
                       "coarse_pool_seconds": t_pool, "coarse_solve_seconds": t_solve,
                       "coarse_solve_seconds_dense_start": t_coarse_dense, "same_objectives": same_obj,
                       "pairs_per_s_sequential": B / (t_coarse + ms_step / 1e3),
                       "pairs_per_s_pipelined": B / max(t_coarse, ms_step / 1e3),
                       "library_batch_creation_seconds": t_create,
                       "library_creation_and_step_seconds": t_e2e,
                       "library_pairs_per_s": B / t_e2e,
                       "library_pairs_per_s_pipelined": B / max(t_create, ms_step / 1e3),
                       "library_bounds_identical": same_e2e,
                       "note": ("pairs_per_s_* time the per-pair sumpool calls and the host solves "
                                "separately; library_* time the batch built from the fine measures "
                                "alone (one pooling launch for every pair, solves on "
                                "QBW_HOST_THREADS or all cores); pipelined: the coarse work of the "
                                "next batch overlapping the device step of this one")},
        "bounds_sample": {"lower": res[0]["lower"], "upper": res[0]["upper"]},
    }
    out["paper_context"] = PAPER_CONTEXT
    if uneven is not None:
        out["uneven_batch"] = uneven
    out["upper_kernel"] = upper_kernel
    out["batch_sizes_pairs_per_s"] = sweep
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(N, k, p)
        log(f"[bench] cpu oracle: {out['cpu_baseline']['value']:.3e} pairs/s")
        allc = cpu_baseline_all_cores(N, k, p)
        one = out["cpu_baseline"]
        # per pair on all cores: the c-transform part scaled by the measured
        # all-core target rate, the upper-bound part as on one core
        t_ub = one["seconds_upper"]
        per_pair = 2 * N * N / allc["targets_per_s"] + t_ub
        out["cpu_baseline_all_cores"] = {
            "value": 1.0 / per_pair, "unit": "pairs/s", "cores": allc["cores"], "kind": "oracle",
            "cpu_model": allc["cpu_model"], "cpu_count": allc["cpu_count"],
            "sample": f"{allc['targets_done']} random targets of the float32 c-transform on {allc['cores']} "
                      f"processes in {allc['seconds']:.1f} s, scaled to both transforms, plus the "
                      f"single-core upper bound and gradient ({t_ub:.1f} s)"}
        log(f"[bench] cpu oracle, {allc['cores']} cores ({allc['cpu_model']}): "
            f"{out['cpu_baseline_all_cores']['value']:.3e} pairs/s")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
