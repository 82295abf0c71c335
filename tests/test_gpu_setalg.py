"""SP and CoSaMP on the GPU against the FP64 oracle's readings of them, and
exact recovery at the full N = 2^20 partial-Hadamard size."""
import numpy as np
import pytest

import instancegen
import oracle
from tests.gpu_util import lib, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


CASES = [
    ("H", 1024, 256, 10, "pm_u12", None),
    ("F", 1024, 256, 10, "cgauss", 40.0),
    ("H", 4096, 1024, 40, "gauss", 40.0),
    ("F", 16384, 4096, 100, "cgauss", 30.0),
    ("H", 65536, 16384, 256, "pm_u12", None),
]
_REF = {}


def _ref(alg, case, seed):
    key = (alg, case, seed)
    if key not in _REF:
        cls, N, M, K, law, snr = case
        inst = instancegen.draw_instance(cls, N, M, K, law, snr, seed)
        y = oracle.problem.instance_measure(inst, tier="transform")
        op = oracle.make_operator(cls, N, inst.omega, "transform")
        _REF[key] = (inst, y, getattr(oracle, alg)(op, y, K))
    return _REF[key]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["conventional", "fast"])
@pytest.mark.parametrize("alg", ["sp", "cosamp"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}-{c[3]}")
def test_set_algorithm_parity(fc, case, alg, method, precision):
    inst, y, ref = _ref(alg, case, 9100)
    res = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y), algorithm=alg,
                   method=method, precision=precision)
    sup = to_np(res.support)
    x = to_np(res.x)
    assert res.stats.status_detail == 0
    assert list(sup) == list(ref.support)
    assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("alg", ["sp", "cosamp"])
def test_set_algorithm_full_rows(fc, alg):
    """M = N: the first selection is the true support."""
    N, K = 256, 12
    rng = np.random.default_rng(5)
    supp = rng.choice(N, K, replace=False)
    x = np.zeros(N)
    x[supp] = rng.uniform(1, 2, K) * rng.choice([-1, 1], K)
    om = np.arange(N)
    y = oracle.measure("H", N, om, x)
    res = fc.solve("H", N, N, K, om, to_dev(y), algorithm=alg)
    assert list(to_np(res.support)) == sorted(supp)
    assert res.stats.iterations == 1
    assert np.allclose(to_np(res.x), x[sorted(supp)], atol=1e-12)


@pytest.mark.parametrize("method", ["conventional", "fast"])
@pytest.mark.parametrize("alg", ["sp", "cosamp"])
def test_full_size_hadamard_exact_recovery(fc, alg, method):
    """Partial Hadamard N = 2^20, M = 2^17, K = 1024, +-U(1,2), noiseless,
    FP32 correlation: the recovered support and values are the planted ones
    (a property that holds at any size, checked without the oracle)."""
    import torch
    inst = instancegen.draw_config("hadamard_n1m", 0)
    xd = torch.from_numpy(inst.x_dense()).cuda()
    y = fc.measure("H", inst.N, inst.omega, xd)
    res = fc.solve("H", inst.N, inst.M, inst.K, inst.omega, y, algorithm=alg, method=method,
                   precision="fp32")
    sup = to_np(res.support)
    assert list(sup) == sorted(inst.support)
    x = to_np(res.x)
    want = inst.x_dense()[sup]
    assert np.linalg.norm(x - want) <= 1e-10 * np.linalg.norm(want)


@pytest.mark.parametrize("alg", ["sp", "cosamp"])
def test_set_pursuit_res_tol_and_select_time(fc, alg):
    """SP / CoSaMP with res_tol: the loop stops where the oracle's does, with
    the same support and x; FCMP_FLAG_PHASE_TIMES reports the top-K time."""
    inst = instancegen.draw_instance("H", 4096, 1024, 20, "pm_u12", None, 7400)
    y = oracle.problem.instance_measure(inst, tier="transform")
    op = oracle.make_operator("H", 4096, inst.omega)
    ref = getattr(oracle, alg)(op, y, 20, res_tol=1e-6)
    res = fc.solve("H", 4096, 1024, 20, inst.omega, to_dev(y), algorithm=alg, precision="fp64",
                   res_tol=1e-6, flags=fc.FLAG_PHASE_TIMES)
    assert res.stats.iterations == ref.iterations
    assert list(to_np(res.support)) == list(ref.support)
    assert np.linalg.norm(to_np(res.x) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    assert res.stats.ms_select > 0 and np.isnan(res.stats.min_gap)
