"""The paper's fast correlation, Sec. II and Sec. III-A (FP64).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

* Correlation kernel vector (defined right after eq. (kernelsum)):
  c = U^H S_Omega^T S_Omega U e_1; with 0-based indexing e_1 is e_0 and U e_0
  is the constant column 1/sqrt(N), so c = Phi^H (column 0 of Phi).
* P_lambda = U^H D_lambda U with D_lambda = sqrt(N) diag(u_lambda) is a
  permutation (Thm 2-1).  Sec. III-B says it is a cyclic shift for the
  Fourier class and composes from log2(N) stored permutations for the
  Hadamard class; with the sign/order conventions of ``unitary`` these are
  (P_lambda v)(j) = v((j - lambda) mod N) and (P_lambda v)(j) = v(j XOR lambda).
* Fast correlation, eq. (kernelsum): h_t = h_0 - sum_tau x_t(tau) P_{Lambda_t(tau)} c,
  with h_0 = Phi^H y; eq. (kernelsumOMP) is its OMP form.
"""
from __future__ import annotations

import numpy as np

from .unitary import make_operator, sensing_matrix

__all__ = ["kernel_vector", "permutation_matrix", "permute", "fast_correlation"]


def kernel_vector(cls: str, N: int, omega, tier: str = "auto") -> np.ndarray:
    """c = U^H S_Omega^T S_Omega U e_0."""
    op = make_operator(cls, N, omega, tier)
    col0 = op.columns([0])[:, 0]          # S_Omega U e_0
    return op.adjoint(col0)               # U^H S_Omega^T (.)


def permutation_matrix(cls: str, N: int, lam: int) -> np.ndarray:
    """U^H D_lambda U formed densely (small N only; Thm 2-1)."""
    U = sensing_matrix(cls, N, np.arange(N))
    D = np.sqrt(N) * np.diag(U[:, lam])
    return U.conj().T @ D @ U


def permute(cls: str, N: int, lam: int, v) -> np.ndarray:
    """P_lambda v as the index map of Sec. III-B."""
    v = np.asarray(v)
    j = np.arange(N, dtype=np.int64)
    if cls == "F":
        return v[(j - int(lam)) % N]
    return v[j ^ int(lam)]


def fast_correlation(cls: str, N: int, h0, c, lams, xs) -> np.ndarray:
    """h = h_0 - sum_tau x(tau) P_{lambda_tau} c, eq. (kernelsum)."""
    h = np.array(h0, dtype=np.complex128 if cls == "F" else np.float64, copy=True)
    for lam, xv in zip(np.asarray(lams, dtype=np.int64), np.asarray(xs)):
        h -= xv * permute(cls, N, int(lam), c)
    return h
