"""The index algebra behind the fused residual kernel, checked in plain numpy
against the direct forward transform of a sparse vector (no GPU, no oracle):
for rows k = c + N1 m,

  Fourier:  sum_lam x_lam e^{-2 pi i lam k / N}
            = sum_{l < N2} A(c, l) e^{-2 pi i l m / N2},
            A(c, l) = sum_{lam = l mod N2} x_lam e^{-2 pi i lam c / N};
  Hadamard: sum_lam x_lam (-1)^popcount(lam & k)
            = sum_{l < N2} A(c, l) (-1)^popcount(l & m),
            A(c, l) = sum_{lam >> log2 N1 = l} x_lam (-1)^popcount(lam & c),

with N1 = 2^ceil(log2 N / 2), N2 = N / N1, for even and odd log2 N."""
import numpy as np
import pytest


def _popc(a):
    return bin(int(a)).count("1")


@pytest.mark.parametrize("logn", [8, 9, 10, 11])
def test_fourier_bucket_decomposition(logn):
    rng = np.random.default_rng(logn)
    N = 1 << logn
    n2 = logn // 2
    n1 = logn - n2
    N1, N2 = 1 << n1, 1 << n2
    lam = rng.choice(N, 29, replace=False)
    x = rng.standard_normal(29) + 1j * rng.standard_normal(29)
    direct = np.exp(-2j * np.pi * np.outer(np.arange(N), lam) / N) @ x
    X = np.zeros(N, complex)
    for c in range(N1):
        A = np.zeros(N2, complex)
        for lv, xv in zip(lam, x):
            A[lv % N2] += xv * np.exp(-2j * np.pi * lv * c / N)
        m = np.arange(N2)
        X[c + N1 * m] = np.exp(-2j * np.pi * np.outer(m, np.arange(N2)) / N2) @ A
    assert np.max(np.abs(X - direct)) < 1e-10 * np.max(np.abs(direct))


@pytest.mark.parametrize("logn", [8, 9, 10])
def test_hadamard_bucket_decomposition(logn):
    rng = np.random.default_rng(100 + logn)
    N = 1 << logn
    n2 = logn // 2
    n1 = logn - n2
    N1, N2 = 1 << n1, 1 << n2
    lam = rng.choice(N, 23, replace=False)
    x = rng.integers(-4, 5, 23).astype(float)
    direct = np.array([sum(xv * (-1) ** _popc(lv & k) for lv, xv in zip(lam, x))
                       for k in range(N)])
    X = np.zeros(N)
    for c in range(N1):
        A = np.zeros(N2)
        for lv, xv in zip(lam, x):
            A[lv >> n1] += xv * (-1) ** _popc(lv & (N1 - 1) & c)
        for m in range(N2):
            X[c + N1 * m] = sum(A[l] * (-1) ** _popc(l & m) for l in range(N2))
    assert np.array_equal(X, direct)   # integers: exact
