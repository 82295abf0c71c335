"""The two partial unitary classes of the paper, written out plainly (FP64).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Sec. I defines the sensing matrix as M rows, indexed by Omega, of an N x N
matrix: Phi = S_Omega U.  Sec. I (the two constraints) requires every entry
of U to have magnitude 1/sqrt(N) and the scaled columns to be closed under the
elementwise product; the Fourier and Hadamard matrices are the two classes
named.  The paper fixes neither the DFT sign nor the Hadamard ordering and
indexes from 1 with the constant column first; this oracle indexes from 0
(column 0 is the constant column) and uses

* Fourier:  U[k, n] = exp(-2 pi i ((k n) mod N) / N) / sqrt(N)
* Hadamard: U[k, n] = (-1)^popcount(k AND n) / sqrt(N)   (Sylvester order,
  N a power of two)

Two tiers compute the same maps:

* dense tier: the rows of Phi are formed entry by entry from the formulas
  above and the correlation of Algorithm 1.1 step 2 is the matrix product
  Phi^H r -- the plain definition;
* transform tier (sizes where a dense Phi does not fit): the correlation is
  one N-point transform of the zero-filled residual (the FFT route of
  Sec. III-B for Fourier, the FHT route for Hadamard), using numpy's FFT and
  a plain radix-2 Walsh-Hadamard transform.
"""
from __future__ import annotations

import numpy as np

__all__ = ["popcount", "fourier_rows", "hadamard_rows", "sensing_matrix",
           "columns", "wht", "adjoint_transform", "forward_transform",
           "Operator", "DenseOperator", "TransformOperator", "make_operator"]


def popcount(a: np.ndarray) -> np.ndarray:
    """Number of set bits of each non-negative int64 entry (bit by bit, up
    to the highest bit any entry has)."""
    a = np.asarray(a, dtype=np.int64)
    out = np.zeros(a.shape, dtype=np.int64)
    nbits = int(a.max()).bit_length() if a.size else 0
    for b in range(nbits):
        out += (a >> b) & 1
    return out


def _check_n(N: int) -> None:
    if N < 1 or (N & (N - 1)) != 0:
        raise ValueError("N must be a power of two")


def fourier_rows(N: int, rows) -> np.ndarray:
    """Rows ``rows`` of the unitary DFT matrix, entry by entry."""
    k = np.asarray(rows, dtype=np.int64)
    n = np.arange(N, dtype=np.int64)
    p = np.multiply.outer(k, n) % N          # reduce the phase in integers
    return np.exp(-2j * np.pi * p / N) / np.sqrt(N)


def hadamard_rows(N: int, rows) -> np.ndarray:
    """Rows ``rows`` of the Sylvester-ordered unitary Hadamard matrix."""
    _check_n(N)
    k = np.asarray(rows, dtype=np.int64)
    n = np.arange(N, dtype=np.int64)
    parity = popcount(np.bitwise_and.outer(k, n)) & 1
    return np.where(parity == 0, 1.0, -1.0) / np.sqrt(N)


def sensing_matrix(cls: str, N: int, omega) -> np.ndarray:
    """Dense Phi = S_Omega U (M x N)."""
    if cls == "F":
        return fourier_rows(N, omega)
    if cls == "H":
        return hadamard_rows(N, omega)
    raise ValueError("cls must be 'H' or 'F'")


def columns(cls: str, N: int, omega, idx) -> np.ndarray:
    """Columns ``idx`` of Phi (M x len(idx)), entry by entry."""
    k = np.asarray(omega, dtype=np.int64)
    j = np.asarray(idx, dtype=np.int64)
    if cls == "F":
        p = np.multiply.outer(k, j) % N
        return np.exp(-2j * np.pi * p / N) / np.sqrt(N)
    parity = popcount(np.bitwise_and.outer(k, j)) & 1
    return np.where(parity == 0, 1.0, -1.0) / np.sqrt(N)


def wht(v: np.ndarray) -> np.ndarray:
    """Unnormalised natural-order Walsh-Hadamard transform, radix-2 stages:
    out[j] = sum_k (-1)^popcount(j AND k) v[k]."""
    v = np.array(v, copy=True)
    N = v.shape[0]
    _check_n(N)
    h = 1
    while h < N:
        w = v.reshape(-1, 2, h)
        a = w[:, 0, :].copy()
        b = w[:, 1, :].copy()
        w[:, 0, :] = a + b
        w[:, 1, :] = a - b
        v = w.reshape(N)
        h *= 2
    return v


def adjoint_transform(cls: str, N: int, omega, r) -> np.ndarray:
    """h = Phi^H r = U^H S_Omega^T r by one N-point transform of the
    zero-filled r (Sec. III-B: FFT for Fourier, FHT for Hadamard)."""
    r = np.asarray(r)
    if cls == "F":
        z = np.zeros(N, dtype=np.complex128)
        z[np.asarray(omega)] = r
        # numpy's ifft carries 1/N and the + sign: sqrt(N) ifft = U^H z.
        return np.sqrt(N) * np.fft.ifft(z)
    z = np.zeros(N, dtype=np.float64 if not np.iscomplexobj(r) else np.complex128)
    z[np.asarray(omega)] = r
    return wht(z) / np.sqrt(N)


def forward_transform(cls: str, N: int, omega, s) -> np.ndarray:
    """Phi s = S_Omega U s by one N-point transform."""
    s = np.asarray(s)
    if cls == "F":
        return (np.fft.fft(s) / np.sqrt(N))[np.asarray(omega)]
    return (wht(s) / np.sqrt(N))[np.asarray(omega)]


class Operator:
    """What an MPA needs from Phi: the correlation Phi^H r, the product
    Phi s, and explicit selected columns for least squares."""

    def __init__(self, cls: str, N: int, omega):
        _check_n(N)
        self.cls = cls
        self.N = int(N)
        self.omega = np.asarray(omega, dtype=np.int64)
        self.M = int(self.omega.shape[0])
        self.dtype = np.complex128 if cls == "F" else np.float64

    def adjoint(self, r):
        raise NotImplementedError

    def forward(self, s):
        raise NotImplementedError

    def columns(self, idx) -> np.ndarray:
        return columns(self.cls, self.N, self.omega, idx)


class DenseOperator(Operator):
    """Phi formed explicitly; correlation is the plain matrix product."""

    def __init__(self, cls, N, omega):
        super().__init__(cls, N, omega)
        self.Phi = sensing_matrix(cls, N, self.omega)

    def adjoint(self, r):
        return self.Phi.conj().T @ np.asarray(r)

    def forward(self, s):
        return self.Phi @ np.asarray(s)

    def columns(self, idx):
        return self.Phi[:, np.asarray(idx, dtype=np.int64)]


class TransformOperator(Operator):
    """Phi applied through N-point transforms (large N)."""

    def adjoint(self, r):
        h = adjoint_transform(self.cls, self.N, self.omega, r)
        return h if self.cls == "F" else np.real(h)

    def forward(self, s):
        return forward_transform(self.cls, self.N, self.omega, s)


DENSE_LIMIT = 1 << 26   # M*N entries above which the dense tier is not used


def make_operator(cls: str, N: int, omega, tier: str = "auto") -> Operator:
    omega = np.asarray(omega, dtype=np.int64)
    if tier == "dense" or (tier == "auto" and omega.shape[0] * N <= DENSE_LIMIT):
        return DenseOperator(cls, N, omega)
    return TransformOperator(cls, N, omega)
