"""Selection-gap bookkeeping for support parity.

TEST INFRASTRUCTURE: imported only by tests.

A GPU correlation within a relative tolerance tol of the FP64 correlation (in
the infinity norm, ||h_gpu - h|| <= tol ||h||_inf) picks the same index as the
oracle whenever the oracle's relative identification gap
(|h|_(1) - |h|_(2)) / ||h||_inf exceeds 2 tol.  An instance is certified at a
precision if every iteration's gap is at least 2.5 tol; certified instances
must then reproduce the oracle's support exactly.
"""
from __future__ import annotations

import numpy as np

TOL = {"fp64": 1e-12, "fp32": 1e-5}
DELTA = {k: 2.5 * v for k, v in TOL.items()}

__all__ = ["TOL", "DELTA", "certified", "min_gap"]


def min_gap(result) -> float:
    g = result.gaps()
    return float(np.min(g)) if g.size else float("inf")


def certified(result, precision: str) -> bool:
    return min_gap(result) >= DELTA[precision]
