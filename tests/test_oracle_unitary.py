"""Pins for oracle.unitary: the two unitary classes and the correlation
Phi^H r, checked against textbook facts and independent library routines."""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import unitary as un

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _full(cls, N):
    return un.sensing_matrix(cls, N, np.arange(N))


@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("N", [2, 4, 8, 32, 64])
def test_unitary(cls, N):
    U = _full(cls, N)
    assert np.allclose(U.conj().T @ U, np.eye(N), atol=1e-13)


@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("N", [4, 16, 64])
def test_paper_constraints(cls, N):
    """Sec. I: |U_kn| = 1/sqrt(N), and {sqrt(N) u_n} closed under the
    elementwise product; column 0 is the constant column."""
    U = _full(cls, N)
    assert np.allclose(np.abs(U), 1 / np.sqrt(N), atol=1e-15)
    S = np.sqrt(N) * U
    assert np.allclose(S[:, 0], 1.0)
    for a in range(N):
        for b in range(N):
            prod = S[:, a] * S[:, b]
            d = np.max(np.abs(S - prod[:, None]), axis=0)
            assert np.min(d) < 1e-9


def test_dft4_golden():
    rows = []
    for line in open(os.path.join(GOLD, "dft4.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [float(t) for t in line.split()]
        rows.append([complex(v[2 * i], v[2 * i + 1]) for i in range(4)])
    G = np.array(rows) / 2.0
    assert np.allclose(un.fourier_rows(4, np.arange(4)), G, atol=1e-15)


@pytest.mark.parametrize("N", [2, 8, 64, 256])
def test_fourier_matches_numpy_fft(N):
    """Columns of the numpy FFT of the identity are the DFT matrix."""
    ref = np.fft.fft(np.eye(N), axis=0) / np.sqrt(N)
    assert np.allclose(_full("F", N), ref, atol=1e-12)


@pytest.mark.parametrize("N", [2, 4, 16, 128])
def test_hadamard_matches_scipy_sylvester(N):
    assert np.array_equal(_full("H", N) * np.sqrt(N), scipy.linalg.hadamard(N))


@pytest.mark.parametrize("N", [2, 16, 64])
def test_hadamard_square_is_n_identity(N):
    H = np.round(_full("H", N) * np.sqrt(N))
    assert np.array_equal(H @ H, N * np.eye(N))


def test_wht_matches_hadamard_product():
    rng = np.random.default_rng(1)
    for N in (1, 2, 8, 256):
        v = rng.standard_normal(N)
        H = scipy.linalg.hadamard(N) if N > 1 else np.ones((1, 1))
        assert np.allclose(un.wht(v), H @ v, atol=1e-12)


@pytest.mark.parametrize("cls", ["F", "H"])
def test_transform_tier_equals_dense(cls):
    rng = np.random.default_rng(7)
    for N, M in [(16, 5), (256, 64), (1024, 300)]:
        omega = np.sort(rng.choice(N, M, replace=False))
        r = rng.standard_normal(M) + (1j * rng.standard_normal(M) if cls == "F" else 0)
        d = un.DenseOperator(cls, N, omega).adjoint(r)
        t = un.TransformOperator(cls, N, omega).adjoint(r)
        assert np.max(np.abs(d - t)) <= 1e-12 * np.max(np.abs(d))
        s = rng.standard_normal(N) + (1j * rng.standard_normal(N) if cls == "F" else 0)
        fd = un.DenseOperator(cls, N, omega).forward(s)
        ft = un.TransformOperator(cls, N, omega).forward(s)
        assert np.max(np.abs(fd - ft)) <= 1e-12 * np.max(np.abs(fd))


@pytest.mark.parametrize("cls", ["F", "H"])
def test_parseval(cls):
    """U unitary and r zero-filled: ||Phi^H r|| = ||r||."""
    rng = np.random.default_rng(3)
    N, M = 4096, 1000
    omega = np.sort(rng.choice(N, M, replace=False))
    r = rng.standard_normal(M) + (1j * rng.standard_normal(M) if cls == "F" else 0)
    h = un.TransformOperator(cls, N, omega).adjoint(r)
    assert abs(np.linalg.norm(h) - np.linalg.norm(r)) <= 1e-12 * np.linalg.norm(r)


def test_correlation_single_row_closed_form():
    """With Omega = {k} and r = 1 the correlation is conj of row k of U:
    Fourier h(j) = exp(+2 pi i k j / N)/sqrt(N) = (cos, sin)(2 pi k j / N)/sqrt(N)."""
    N, k = 64, 5
    h = un.DenseOperator("F", N, [k]).adjoint(np.array([1.0 + 0j]))
    j = np.arange(N)
    ang = 2 * np.pi * k * j / N
    assert np.allclose(h, (np.cos(ang) + 1j * np.sin(ang)) / 8.0, atol=1e-15)


def test_columns_match_dense():
    rng = np.random.default_rng(5)
    for cls in ("F", "H"):
        N = 128
        omega = np.sort(rng.choice(N, 40, replace=False))
        idx = rng.choice(N, 7, replace=False)
        P = un.sensing_matrix(cls, N, omega)
        assert np.allclose(un.columns(cls, N, omega, idx), P[:, idx], atol=0)


def test_hadamard_integer_exactness():
    """For N = 4^m, sqrt(N) is a power of two: integer r gives exactly
    representable correlations (the bit-exact pin of the GPU tests)."""
    rng = np.random.default_rng(11)
    N, M = 1024, 256
    omega = np.sort(rng.choice(N, M, replace=False))
    r = rng.integers(-8, 9, M).astype(np.float64)
    h = un.TransformOperator("H", N, omega).adjoint(r)
    assert np.array_equal(h * 32.0, np.round(h * 32.0))
    hd = un.DenseOperator("H", N, omega).adjoint(r)
    assert np.array_equal(h, hd)
