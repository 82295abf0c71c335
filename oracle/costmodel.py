"""Flop model of Table I and the worked numbers of Sec. IV.

TEST INFRASTRUCTURE: imported only by tests and the benchmark's CPU leg.

Convention of Sec. III-B: one complex multiplication = 6 flops, one complex
addition = 2 flops.  Per OMP iteration t (Table I):

* Fourier, conventional: one N-point FFT, 5 N log2 N flops at every t;
  proposed: 5 N log2 N at t = 1, then 6 N (t - 1) (the conjugate-symmetry
  count of Sec. III-B: (N/2)(t-1) complex multiplications, 2 (N/2)(t-1) real
  additions and N (t-1) complex additions).
* Hadamard, conventional: one N-point FHT, N log2 N complex additions =
  2 N log2 N flops; proposed: 2 N log2 N at t = 1, then about N (t-1)
  complex additions = 2 N (t-1).

The "excessive point" of Sec. IV is the last iteration at which the proposed
count does not exceed the conventional one; the proposed CoSaMP spends K
taps at every iteration after the first.
"""
from __future__ import annotations

import math

__all__ = ["conventional_flops", "proposed_flops", "relative", "excessive_point",
           "cosamp_relative", "omp_totals"]


def _log2(N: int) -> int:
    n = int(round(math.log2(N)))
    if 1 << n != N:
        raise ValueError("N must be a power of two")
    return n


def conventional_flops(cls: str, N: int, t: int) -> int:
    n = _log2(N)
    return 5 * N * n if cls == "F" else 2 * N * n


def proposed_flops(cls: str, N: int, t: int) -> int:
    if t <= 1:
        return conventional_flops(cls, N, t)
    return 6 * N * (t - 1) if cls == "F" else 2 * N * (t - 1)


def relative(cls: str, N: int, t: int) -> float:
    return proposed_flops(cls, N, t) / conventional_flops(cls, N, t)


def excessive_point(cls: str, N: int, t_max: int = 1 << 20) -> int:
    """Largest t with proposed <= conventional (the iteration after it is the
    first where the conventional correlation is cheaper)."""
    t = 1
    while t + 1 <= t_max and proposed_flops(cls, N, t + 1) <= conventional_flops(cls, N, t + 1):
        t += 1
    return t


def cosamp_relative(cls: str, N: int, K: int) -> float:
    """Proposed / conventional CoSaMP correlation cost at an iteration t > 1
    (K taps of the kernel vector against one N-point transform)."""
    per_tap = 6 * N if cls == "F" else 2 * N
    return per_tap * K / conventional_flops(cls, N, 2)


def omp_totals(cls: str, N: int, K: int) -> dict:
    """Total correlation flops over K OMP iterations: conventional, proposed,
    and the adaptive strategy (proposed up to the excessive point)."""
    conv = sum(conventional_flops(cls, N, t) for t in range(1, K + 1))
    prop = sum(proposed_flops(cls, N, t) for t in range(1, K + 1))
    hyb = sum(min(proposed_flops(cls, N, t), conventional_flops(cls, N, t))
              for t in range(1, K + 1))
    return {"conventional": conv, "proposed": prop, "adaptive": hyb}
