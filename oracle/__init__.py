"""CPU oracle for quantization-based bounds on the Wasserstein metric.

TEST INFRASTRUCTURE ONLY.  This package restates, in plain and slow numpy /
scipy / PyTorch-CPU code, what the method of "Quantization-based Bounds on the
Wasserstein Metric" (Bobrutsky & Moscovich) computes:

* ``grid``    - the regular grid [N]^d, the flat index convention and the
                ground cost rho(x, y)^p (Section 2.1)
* ``coarse``  - SumPool / AvgPool coarsening (Section 2.2), the centre cost
                C~, the marginally weighted cost C-bar (Section 3.2, eq. of the
                marginally weighted cost) and the locally minimal cost C^min
                (Section 3.3)
* ``lp``      - exact Kantorovich solves (HiGHS), a north-west-corner
                coupling and an optimality certificate for coarse solutions
* ``lower``   - dual-upscaling lower bound (Section 3.5, Algorithm 5) in FP64
                and its FP32-faithful twin
* ``upper``   - primal-upscaling upper bound (Section 3.4, Algorithm 4),
                weighted-cost upper bound (Algorithm 3), min-cost lower bound
* ``grad``    - gradients of both bounds with the coarse solution frozen
* ``closed``  - closed forms used as pins (1-D quantile formula, translation)

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library and must never
be reached from the library's own code path.
"""
from . import grid, coarse, lp, lower, upper, closed  # noqa: F401

__all__ = ["grid", "coarse", "lp", "lower", "upper", "closed"]
