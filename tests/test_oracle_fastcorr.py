"""Pins for oracle.fastcorr: Thm 2-1, the shift/XOR form of P_lambda, the
kernel vector's invariants and closed forms, and the fast identity."""
import numpy as np
import pytest

import oracle
from oracle import fastcorr as fc
from oracle import unitary as un


@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("N", [4, 8, 32])
def test_theorem_2_1_permutation(cls, N):
    """U^H D_lambda U is a 0/1 matrix with one 1 per row and column, and it
    acts as the index map used by the fast path (cyclic shift / XOR)."""
    rng = np.random.default_rng(N)
    for lam in range(N):
        P = fc.permutation_matrix(cls, N, lam)
        R = np.round(P.real)
        assert np.max(np.abs(P - R)) < 1e-12
        assert set(np.unique(R)) <= {0.0, 1.0}
        assert np.array_equal(R.sum(0), np.ones(N)) and np.array_equal(R.sum(1), np.ones(N))
        v = rng.standard_normal(N)
        assert np.allclose(P @ v, fc.permute(cls, N, lam, v), atol=1e-12)


def test_shift_direction_fourier():
    """(P_lambda v)(j) = v(j - lambda): e_0 moves to e_lambda."""
    N = 16
    e0 = np.zeros(N)
    e0[0] = 1
    for lam in (1, 5, 15):
        out = fc.permute("F", N, lam, e0)
        assert out[lam] == 1 and out.sum() == 1


def test_hadamard_permutations_compose():
    """Sec. III-B: any P_lambda is a product of the log2 N single-bit ones."""
    N = 64
    rng = np.random.default_rng(2)
    v = rng.standard_normal(N)
    for lam in (0, 1, 37, 63):
        w = v.copy()
        for b in range(6):
            if lam >> b & 1:
                w = fc.permute("H", N, 1 << b, w)
        assert np.array_equal(w, fc.permute("H", N, lam, v))


def _omega(N, M, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, M, replace=False))


@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("N,M", [(64, 20), (1024, 256), (4096, 1024)])
def test_kernel_vector_invariants(cls, N, M):
    for seed in range(3):
        om = _omega(N, M, seed)
        c = fc.kernel_vector(cls, N, om)
        assert abs(c[0] - M / N) < 1e-14                      # ||phi_j||^2
        assert abs(np.vdot(c, c).real - M / N) < 1e-13        # ||c||^2
        assert abs(np.sum(c) - (1.0 if 0 in om else 0.0)) < 1e-11
        if cls == "F":
            j = np.arange(N)
            assert np.allclose(c[(-j) % N], np.conj(c), atol=1e-14)
        else:
            Nc = c * N
            assert np.allclose(Nc, np.round(Nc), atol=1e-9)
            assert np.max(np.abs(Nc)) <= M


@pytest.mark.parametrize("cls", ["F", "H"])
def test_kernel_vector_subgroup_closed_form(cls):
    """Omega a subgroup: Hadamard {0..M-1}, Fourier (N/M){0..M-1} give
    c(j) = (M/N) [j mod M == 0] / [j mod (N/M)...]: checked by definition of
    the character sums (geometric / product sums)."""
    N, M = 256, 16
    if cls == "H":
        om = np.arange(M)
        c = fc.kernel_vector(cls, N, om)
        want = np.where(np.arange(N) % M == 0, M / N, 0.0)
    else:
        om = (N // M) * np.arange(M)
        c = fc.kernel_vector(cls, N, om)
        want = np.where(np.arange(N) % M == 0, M / N, 0.0)
    assert np.allclose(c, want, atol=1e-14)


@pytest.mark.parametrize("cls", ["F", "H"])
def test_gram_column_is_shifted_kernel(cls):
    """(Phi^H Phi)[:, lambda] = P_lambda c for every lambda."""
    N, M = 64, 24
    om = _omega(N, M, 9)
    Phi = un.sensing_matrix(cls, N, om)
    G = Phi.conj().T @ Phi
    c = fc.kernel_vector(cls, N, om, "dense")
    for lam in range(N):
        assert np.allclose(G[:, lam], fc.permute(cls, N, lam, c), atol=1e-14)


@pytest.mark.parametrize("cls", ["F", "H"])
def test_fast_identity_equals_dense(cls):
    """eq. (corr_com)/(kernelsum): h_0 - sum x P c = Phi^H (y - Phi S^T x)."""
    rng = np.random.default_rng(4)
    N, M, t = 128, 40, 9
    om = _omega(N, M, 4)
    Phi = un.sensing_matrix(cls, N, om)
    y = rng.standard_normal(M) + (1j * rng.standard_normal(M) if cls == "F" else 0)
    lam = rng.choice(N, t, replace=False)
    xv = rng.standard_normal(t) + (1j * rng.standard_normal(t) if cls == "F" else 0)
    s = np.zeros(N, dtype=complex)
    s[lam] = xv
    want = Phi.conj().T @ (y - Phi @ s)
    h0 = Phi.conj().T @ y
    c = fc.kernel_vector(cls, N, om)
    got = fc.fast_correlation(cls, N, h0, c, lam, xv)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_fast_identity_hadamard_integer_exact():
    """Hadamard, N = 4^m: N c is an integer, so integer taps on an integer
    h_0 give an exact result equal to the dense product."""
    rng = np.random.default_rng(6)
    N, M = 256, 64
    om = _omega(N, M, 6)
    Phi = un.sensing_matrix("H", N, om)
    y = rng.integers(-5, 6, M).astype(float)
    lam = rng.choice(N, 5, replace=False)
    xv = rng.integers(-3, 4, 5).astype(float)
    s = np.zeros(N)
    s[lam] = xv
    want = Phi.T @ (y - Phi @ s)
    got = fc.fast_correlation("H", N, Phi.T @ y, fc.kernel_vector("H", N, om), lam, xv)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("cls", ["F", "H"])
def test_fast_equals_conventional_along_omp(cls):
    """Sec. III-A: the fast OMP is the same algorithm -- h agrees to FP64
    rounding at every iteration and the supports are identical."""
    import instancegen
    inst = instancegen.draw_instance(cls, 2048, 512, 40,
                                     "cgauss" if cls == "F" else "gauss", 30.0, 77)
    y = oracle.problem.instance_measure(inst)
    op = oracle.make_operator(cls, inst.N, inst.omega, "transform")
    a = oracle.omp(op, y, inst.K, "conventional", keep_h=True)
    b = oracle.omp(op, y, inst.K, "fast", keep_h=True)
    assert np.array_equal(a.support, b.support)
    for ha, hb in zip(a.h, b.h):
        assert np.max(np.abs(ha - hb)) <= 1e-12 * np.max(np.abs(ha))
