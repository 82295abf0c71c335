"""Seeded synthetic inputs for sparse-recovery problems y = Phi x + eta.

This module only draws random numbers: the row set Omega, the support and the
nonzero values of x, and a raw (unscaled) noise vector.  It holds none of the
recovery method's arithmetic -- forming y = Phi x and scaling the noise to a
target SNR are done by whoever consumes the draw (the CPU oracle in tests, the
library's own forward operator in the benchmark).

Every draw uses ``numpy.random.Generator(PCG64(seed))`` and takes its numbers
in a fixed order: Omega (M of N rows without replacement, sorted), the support
(K of N columns without replacement), the K values, then the M noise samples.

Problem classes: ``"H"`` partial Hadamard (real), ``"F"`` partial Fourier
(complex).  Value laws:

* ``"gauss"``   real N(0, 1)
* ``"cgauss"``  complex CN(0, 1) = (a + i b) / sqrt(2), a, b ~ N(0, 1)
* ``"pm_u12"``  +-U(1, 2) with a random sign
* ``"int"``     small nonzero integers in [-4, 4] (exactly representable data)

Noise is drawn as N(0, I) (class H) or CN(0, I) (class F) and returned raw,
together with the requested SNR in dB (``None`` = noiseless).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Instance", "draw_instance", "draw_config", "draw_batch", "draw_stream",
    "CONFIGS",
]


@dataclass
class Instance:
    cls: str                 # "H" or "F"
    N: int
    M: int
    K: int
    omega: np.ndarray        # int64[M], strictly increasing, in [0, N)
    support: np.ndarray      # int64[K], distinct, in [0, N) (draw order)
    values: np.ndarray       # float64[K] or complex128[K]
    noise: Optional[np.ndarray]  # raw noise draw, length M, or None
    snr_db: Optional[float]
    seed: int = 0
    extra: dict = field(default_factory=dict)

    def x_dense(self) -> np.ndarray:
        """The N-vector x with the drawn values at the drawn support."""
        dt = np.complex128 if self.cls == "F" else np.float64
        x = np.zeros(self.N, dtype=dt)
        x[self.support] = self.values
        return x


def _values(rng: np.random.Generator, law: str, K: int) -> np.ndarray:
    if law == "gauss":
        return rng.standard_normal(K)
    if law == "cgauss":
        a = rng.standard_normal(K)
        b = rng.standard_normal(K)
        return (a + 1j * b) / np.sqrt(2.0)
    if law == "pm_u12":
        mag = rng.uniform(1.0, 2.0, K)
        sgn = rng.choice(np.array([-1.0, 1.0]), K)
        return mag * sgn
    if law == "int":
        v = rng.integers(1, 5, K).astype(np.float64)
        sgn = rng.choice(np.array([-1.0, 1.0]), K)
        return v * sgn
    raise ValueError(f"unknown value law {law!r}")


def draw_instance(cls: str, N: int, M: int, K: int, law: str,
                  snr_db: Optional[float], seed) -> Instance:
    """Draw one instance; ``seed`` may be an int or a list of ints."""
    if cls not in ("H", "F"):
        raise ValueError("cls must be 'H' or 'F'")
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = np.sort(rng.choice(N, M, replace=False)).astype(np.int64)
    support = rng.choice(N, K, replace=False).astype(np.int64)
    values = _values(rng, law, K)
    if cls == "F" and not np.iscomplexobj(values):
        values = values.astype(np.complex128)
    noise = None
    if snr_db is not None:
        if cls == "F":
            a = rng.standard_normal(M)
            b = rng.standard_normal(M)
            noise = (a + 1j * b) / np.sqrt(2.0)
        else:
            noise = rng.standard_normal(M)
    s = seed if isinstance(seed, int) else int(np.asarray(seed).ravel()[0])
    return Instance(cls, N, M, K, omega, support, values, noise, snr_db, s)


# The five workloads, by name.  Each entry: class, N, M, K, value law, SNR,
# correlation precision, algorithms/methods, number of instances, seed base.
CONFIGS = {
    "hadamard_n1024": dict(cls="H", N=1 << 10, M=256, K=16, law="gauss",
                           snr_db=None, precision="fp64", count=64, seed=1000),
    "fourier_n65536": dict(cls="F", N=1 << 16, M=1 << 14, K=256, law="cgauss",
                           snr_db=30.0, precision="fp32", count=8, seed=2000),
    "hadamard_n1m": dict(cls="H", N=1 << 20, M=1 << 17, K=1024, law="pm_u12",
                         snr_db=None, precision="fp32", count=4, seed=3000),
}


def draw_config(name: str, index: int) -> Instance:
    """Instance ``index`` of a named single-instance workload."""
    c = CONFIGS[name]
    return draw_instance(c["cls"], c["N"], c["M"], c["K"], c["law"],
                         c["snr_db"], c["seed"] + index)


def draw_batch(count: int = 4096, seed: int = 4000,
               logn_range=(10, 14), snr_db: float = 40.0) -> List[Instance]:
    """The uneven batch: instance i is Fourier if i is even else Hadamard,
    N = 2**U{logn_range}, M = N/4, K ~ U{8 .. M/8}, N(0,1) / CN(0,1) values.
    Descriptors come from a master generator; each instance then draws from
    its own generator seeded with (seed, i)."""
    master = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        logn = int(master.integers(logn_range[0], logn_range[1] + 1))
        N = 1 << logn
        M = N // 4
        K = int(master.integers(8, M // 8 + 1))
        cls = "F" if i % 2 == 0 else "H"
        law = "cgauss" if cls == "F" else "gauss"
        out.append(draw_instance(cls, N, M, K, law, snr_db, [seed, i]))
    return out


def draw_stream(count: int, seed: int = 5000, rate_hz: float = 20000.0,
                logn_range=(12, 18), snr_db: float = 30.0):
    """A Poisson request stream: returns (arrival_times_s, instances).
    Inter-arrival ~ Exp(1/rate); class ~ Bernoulli(1/2); log2 N ~ U{logn_range};
    M ~ U{N/8 .. N/4}; K ~ U{16 .. M/16}."""
    master = np.random.Generator(np.random.PCG64(seed))
    gaps = master.exponential(1.0 / rate_hz, count)
    arrivals = np.cumsum(gaps)
    out = []
    for i in range(count):
        cls = "F" if master.integers(0, 2) == 1 else "H"
        logn = int(master.integers(logn_range[0], logn_range[1] + 1))
        N = 1 << logn
        M = int(master.integers(N // 8, N // 4 + 1))
        K = int(master.integers(16, M // 16 + 1))
        law = "cgauss" if cls == "F" else "gauss"
        out.append(draw_instance(cls, N, M, K, law, snr_db, [seed, i]))
    return arrivals, out
