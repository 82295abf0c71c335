"""The measurement model y = Phi x + eta of eq. (CSbasic).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The paper names noise but no SNR convention.  Reading used here: the raw
noise draw g is scaled per instance so that the SNR holds exactly,
eta = g * (||Phi x|| / ||g||) * 10^(-SNR/20); no noise when SNR is None.
"""
from __future__ import annotations

import numpy as np

from .unitary import make_operator

__all__ = ["measure", "clean_measure"]


def clean_measure(cls: str, N: int, omega, x, tier: str = "auto") -> np.ndarray:
    """Phi x (noiseless)."""
    op = make_operator(cls, N, omega, tier)
    return op.forward(np.asarray(x))


def measure(cls: str, N: int, omega, x, noise=None, snr_db=None,
            tier: str = "auto") -> np.ndarray:
    """y = Phi x + eta with eta scaled to ``snr_db`` (see module doc)."""
    y = clean_measure(cls, N, omega, x, tier)
    if snr_db is None or noise is None:
        return y
    g = np.asarray(noise)
    scale = np.linalg.norm(y) / np.linalg.norm(g) * 10.0 ** (-snr_db / 20.0)
    return y + g * scale


def instance_measure(inst, tier: str = "auto") -> np.ndarray:
    """y for an ``instancegen.Instance``."""
    return measure(inst.cls, inst.N, inst.omega, inst.x_dense(), inst.noise,
                   inst.snr_db, tier)
