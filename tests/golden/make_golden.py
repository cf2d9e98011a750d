"""Writes the stored expected values under tests/golden/ (calls only the oracle).

* config1_exact.json - exact W_2 of the 32x32 blob pair (1024 x 1024 full LP,
  HiGHS), the pair's coarse solution value at k=4, and the oracle's bounds.
* records_256_k8.npz  - exact coarse solutions (k=8, p=2, centre cost) of the
  256x256 GRF and Cauchy pairs, solved by the oracle's LP, so GPU parity at the
  benchmark size can start from an optimal coarse solution.

Run:  python tests/golden/make_golden.py [config1] [records]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth_inputs as si  # noqa: E402
from oracle import lower, lp, upper  # noqa: E402


def config1():
    mu, nu = si.config1_pair()
    t = time.time()
    W = lp.wasserstein_exact(mu, nu, 2)
    t_lp = time.time() - t
    r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, 4, 2)
    lb = lower.lower_bound_o64(mu, nu, ft, 4, 2)["lower"]
    ub = upper.upper_bound_o64(mu, nu, r, c, v, 4, 2)["upper"]
    out = {"what": "config 1: 32x32 blobs, k=4, p=2",
           "exact_W2": W, "coarse_objective": obj, "oracle_lower": lb, "oracle_upper": ub,
           "lp_seconds": t_lp}
    with open(os.path.join(HERE, "config1_exact.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


def records():
    arrs = {}
    for fam in ("grf", "cauchy"):
        mu, nu = si.config3_pair(256, fam)
        t = time.time()
        r, c, v, ft, gt, obj = upper.coarse_record_lp(mu, nu, 8, 2)
        print(fam, "coarse LP", time.time() - t, "s, nnz", len(v), "obj", obj, flush=True)
        arrs[f"{fam}_rows"] = r.astype(np.int32)
        arrs[f"{fam}_cols"] = c.astype(np.int32)
        arrs[f"{fam}_vals"] = v
        arrs[f"{fam}_f"] = ft
        arrs[f"{fam}_g"] = gt
        arrs[f"{fam}_obj"] = np.array([obj])
    np.savez_compressed(os.path.join(HERE, "records_256_k8.npz"), **arrs)


if __name__ == "__main__":
    what = sys.argv[1:] or ["config1", "records"]
    if "config1" in what:
        config1()
    if "records" in what:
        records()
