"""Pins for oracle.mpa: OMP (Algorithm 1.1) and the SP/CoSaMP readings,
checked against exact recovery, closed-form trajectories, brute force and
least-squares optimality conditions."""
import itertools

import numpy as np
import pytest

import instancegen
import oracle
from oracle import unitary as un


def _inst(cls, N, M, K, law, snr, seed):
    inst = instancegen.draw_instance(cls, N, M, K, law, snr, seed)
    y = oracle.problem.instance_measure(inst)
    return inst, y


@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("method", ["conventional", "fast"])
def test_omp_exact_noiseless_recovery(cls, method):
    for seed in range(4):
        inst, y = _inst(cls, 1024, 256, 12, "cgauss" if cls == "F" else "gauss", None, 100 + seed)
        op = oracle.make_operator(cls, inst.N, inst.omega)
        r = oracle.omp(op, y, inst.K, method)
        xh = np.zeros(inst.N, dtype=complex)
        xh[r.support] = r.x
        x = inst.x_dense()
        assert np.linalg.norm(xh - x) <= 1e-12 * np.linalg.norm(x)
        assert set(r.support) == set(inst.support)


@pytest.mark.parametrize("cls", ["F", "H"])
def test_omp_full_rows_selects_by_magnitude(cls):
    """M = N: Phi is unitary, so h_0 = x and each iteration picks the largest
    remaining |x|; x_hat = x exactly after K steps."""
    N, K = 64, 6
    rng = np.random.default_rng(8)
    supp = rng.choice(N, K, replace=False)
    mags = np.array([6.0, 5.0, 4.0, 3.0, 2.0, 1.0])
    x = np.zeros(N, dtype=complex if cls == "F" else float)
    x[supp] = mags * (np.exp(1j * rng.uniform(0, 6, K)) if cls == "F" else rng.choice([-1, 1], K))
    y = oracle.measure(cls, N, np.arange(N), x)
    r = oracle.omp(oracle.make_operator(cls, N, np.arange(N)), y, K)
    assert list(r.support) == list(supp)
    assert np.allclose(r.x, x[supp], atol=1e-13)


def test_omp_matches_bruteforce_l0():
    """Tiny N: when OMP reaches a zero residual its support is the unique
    K-subset that explains y exactly (exhaustive search)."""
    hits = 0
    for seed in range(30):
        cls = "H" if seed % 2 else "F"
        inst, y = _inst(cls, 16, 8, 2, "gauss" if cls == "H" else "cgauss", None, 500 + seed)
        op = oracle.make_operator(cls, 16, inst.omega)
        r = oracle.omp(op, y, 2)
        exact = []
        for S in itertools.combinations(range(16), 2):
            A = op.columns(list(S))
            xs = np.linalg.lstsq(A, y, rcond=None)[0]
            if np.linalg.norm(y - A @ xs) <= 1e-10 * np.linalg.norm(y):
                exact.append(set(S))
        if r.res_norm <= 1e-10 * np.linalg.norm(y):
            assert exact == [set(r.support)]
            hits += 1
    assert hits >= 10


@pytest.mark.parametrize("cls", ["F", "H"])
def test_omp_residual_orthogonal_and_norm_identity(cls):
    inst, y = _inst(cls, 2048, 512, 30, "cgauss" if cls == "F" else "gauss", 20.0, 42)
    op = oracle.make_operator(cls, inst.N, inst.omega)
    r = oracle.omp(op, y, inst.K)
    A = op.columns(r.support)
    res = y - A @ r.x
    assert np.linalg.norm(A.conj().T @ res) <= 1e-12 * np.linalg.norm(y)
    b = A.conj().T @ y
    lhs = np.linalg.norm(res) ** 2
    rhs = np.linalg.norm(y) ** 2 - np.real(np.vdot(b, r.x))
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(y) ** 2


def test_argmax_ties_lowest_index():
    """Integer Hadamard data with exact ties: the lowest index wins."""
    h = np.array([0.0, 3.0, -3.0, 1.0, 3.0, -2.0])
    assert oracle.argmax_excluding(h, [])[0] == 1
    assert oracle.argmax_excluding(h, [1])[0] == 2
    assert oracle.argmax_excluding(h, [1, 2])[0] == 4
    hc = np.array([0.5j, 1 + 1j, 1 - 1j, -1 + 1j])
    assert oracle.argmax_excluding(hc, [])[0] == 1
    assert oracle.argmax_excluding(hc, [1])[0] == 2


def test_topk_ties_and_exclusion():
    a = np.array([1.0, 5.0, 5.0, 2.0, 5.0, 0.0])
    assert list(oracle.topk(a, 2)) == [1, 2]
    assert list(oracle.topk(a, 3, excluded=[2])) == [1, 4, 3]


@pytest.mark.parametrize("alg", ["sp", "cosamp"])
@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("method", ["conventional", "fast"])
def test_set_algorithms_noiseless_recovery(alg, cls, method):
    f = getattr(oracle, alg)
    for seed in range(3):
        inst, y = _inst(cls, 1024, 256, 10, "cgauss" if cls == "F" else "pm_u12", None, 300 + seed)
        op = oracle.make_operator(cls, inst.N, inst.omega)
        r = f(op, y, inst.K, method)
        assert list(r.support) == sorted(inst.support)
        x = inst.x_dense()
        assert np.allclose(r.x, x[r.support], atol=1e-12)


@pytest.mark.parametrize("alg", ["sp", "cosamp"])
@pytest.mark.parametrize("cls", ["F", "H"])
def test_set_algorithms_full_rows_one_pass(alg, cls):
    """M = N: the first proxy already equals x, so the true support is found
    at the first selection and the loop stops at its first check."""
    N, K = 64, 5
    rng = np.random.default_rng(12)
    supp = rng.choice(N, K, replace=False)
    x = np.zeros(N, dtype=complex if cls == "F" else float)
    x[supp] = rng.uniform(1, 2, K) * rng.choice([-1, 1], K)
    y = oracle.measure(cls, N, np.arange(N), x)
    r = getattr(oracle, alg)(oracle.make_operator(cls, N, np.arange(N)), y, K)
    assert list(r.support) == sorted(supp)
    assert r.iterations == 1
    assert np.allclose(r.x, x[r.support], atol=1e-13)


def test_sp_cosamp_fast_equals_conventional():
    for alg in ("sp", "cosamp"):
        for cls in ("F", "H"):
            inst, y = _inst(cls, 2048, 400, 25, "cgauss" if cls == "F" else "gauss", 25.0, 900)
            op = oracle.make_operator(cls, inst.N, inst.omega, "transform")
            a = getattr(oracle, alg)(op, y, inst.K, "conventional")
            b = getattr(oracle, alg)(op, y, inst.K, "fast")
            assert np.array_equal(a.support, b.support)
            assert np.allclose(a.x, b.x, atol=1e-12 * np.linalg.norm(a.x))


def test_measure_snr_exact():
    inst = instancegen.draw_instance("F", 512, 128, 8, "cgauss", 30.0, 1)
    y = oracle.problem.instance_measure(inst)
    clean = oracle.problem.clean_measure("F", 512, inst.omega, inst.x_dense())
    snr = 20 * np.log10(np.linalg.norm(clean) / np.linalg.norm(y - clean))
    assert abs(snr - 30.0) < 1e-9


@pytest.mark.parametrize("cls", ["F", "H"])
@pytest.mark.parametrize("method", ["conventional", "fast"])
def test_omp_residual_rule_stops_at_the_true_sparsity(cls, method):
    """Noiseless K0-sparse x with OMP asked for 3 K0 selections: after the K0
    planted columns the residual is 0 up to rounding, so the residual rule
    (||r|| <= res_tol ||y||) ends the solve there with x exact; without the
    rule OMP makes all 3 K0 selections."""
    K0 = 8
    inst, y = _inst(cls, 512, 160, K0, "pm_u12", None, 130)
    op = oracle.make_operator(cls, inst.N, inst.omega)
    r = oracle.omp(op, y, 3 * K0, method, res_tol=1e-9)
    assert r.iterations == K0
    assert set(r.support) == set(inst.support)
    assert np.allclose(r.x, inst.x_dense()[r.support], rtol=0, atol=1e-12)
    assert r.res_norm <= 1e-9 * np.linalg.norm(y)
    full = oracle.omp(op, y, 3 * K0, method)
    assert full.iterations == 3 * K0
    assert list(full.support[:K0]) == list(r.support)


def test_omp_residual_rule_threshold_sides():
    """The rule compares the residual after each selection with res_tol ||y||:
    M = N (unitary Phi) and x with magnitudes 8, 4, 2, 1 on four columns, so
    after t selections ||r||^2 is the sum of the remaining squared magnitudes
    (closed form).  A tolerance just above that ratio at t = 2 stops at 2, one
    just below it at 3."""
    N = 32
    om = np.arange(N, dtype=np.int32)
    op = un.make_operator("H", N, om, "dense")
    x = np.zeros(N)
    x[[3, 9, 17, 30]] = [8.0, -4.0, 2.0, 1.0]
    y = op.forward(x)
    ratio2 = np.sqrt(2.0 ** 2 + 1.0) / np.sqrt(64 + 16 + 4 + 1)
    assert oracle.omp(op, y, 4, res_tol=ratio2 * (1 + 1e-9)).iterations == 2
    assert oracle.omp(op, y, 4, res_tol=ratio2 * (1 - 1e-9)).iterations == 3


@pytest.mark.parametrize("alg", ["sp", "cosamp"])
def test_set_pursuit_residual_rule(alg):
    """M = N: the first fit is already exact, so with the residual rule SP
    ends before its loop (0 iterations) and CoSaMP after its first; both
    return the planted support and x."""
    N, K = 64, 5
    om = np.arange(N, dtype=np.int32)
    op = un.make_operator("F", N, om, "dense")
    rng = np.random.default_rng(31)
    supp = np.sort(rng.choice(N, K, replace=False))
    x = np.zeros(N, dtype=complex)
    x[supp] = 1.5 + rng.standard_normal(K) + 1j * rng.standard_normal(K)
    y = op.forward(x)
    r = getattr(oracle, alg)(op, y, K, res_tol=1e-10)
    assert r.iterations == (0 if alg == "sp" else 1)
    assert list(r.support) == list(supp)
    assert np.allclose(r.x, x[supp], rtol=0, atol=1e-12)
