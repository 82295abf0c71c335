"""Edge cases of the hot path on the GPU against the FP64 oracle: the largest
transform sizes the library accepts (Fourier N = 2^22, Hadamard N = 2^24,
ragged M), and degenerate OMP shapes (N = 2, M = N, K = 1, and K = 2 where the
only conventional correlation has one tap)."""
import numpy as np
import pytest

import instancegen
import oracle
from oracle import certify
from tests.gpu_util import inf_rel, lib, omega, rand_vec, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


_MAX = {}


def _max_case(cls, logn):
    if (cls, logn) not in _MAX:
        N = 1 << logn
        M = N // 8 + 5
        rng = np.random.default_rng(logn)
        om = omega(rng, N, M)
        r = rand_vec(rng, M, cls == "F")
        _MAX[(cls, logn)] = (N, om, r)
    return _MAX[(cls, logn)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cls,logn", [("F", 22), ("H", 24)])
def test_correlate_largest_sizes(fc, cls, logn, precision):
    N, om, r = _max_case(cls, logn)
    if precision == "fp32":
        r = r.astype(np.complex64 if cls == "F" else np.float32)
    rd = to_dev(r)
    h, sel = fc.correlate(cls, N, om, rd, precision)
    rin = to_np(rd).astype(np.complex128 if cls == "F" else np.float64)
    want = oracle.unitary.TransformOperator(cls, N, om).adjoint(rin)
    assert inf_rel(to_np(h), want) <= TOL[precision]
    idx, _key = fc.decode_sel(sel)
    a = np.abs(want)
    assert a[idx] >= a.max() * (1 - 2 * TOL[precision])


EDGE = [
    # cls, N, M, K, law, snr
    ("H", 2, 2, 1, "gauss", None),
    ("F", 2, 2, 1, "cgauss", None),
    ("H", 1024, 1024, 16, "gauss", None),      # M = N: Phi is the whole unitary matrix
    ("F", 4096, 4096, 20, "cgauss", 30.0),
    ("F", 65536, 16384, 1, "cgauss", 30.0),    # only h_0 and one least-squares step
    ("F", 65536, 16384, 2, "cgauss", 30.0),    # one conventional correlation, one tap
    ("H", 65536, 8192, 2, "gauss", 30.0),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["conventional", "fast"])
@pytest.mark.parametrize("case", EDGE, ids=lambda c: f"{c[0]}{c[1]}-M{c[2]}-K{c[3]}")
def test_omp_degenerate_shapes(fc, case, method, precision):
    cls, N, M, K, law, snr = case
    inst = instancegen.draw_instance(cls, N, M, K, law, snr, 9100 + N + K)
    y = oracle.problem.instance_measure(inst, tier="transform")
    ref = oracle.omp(oracle.make_operator(cls, N, inst.omega, "transform"), y, K)
    res = fc.solve(cls, N, M, K, inst.omega, to_dev(y), method=method, precision=precision)
    assert res.stats.status_detail == 0
    assert res.stats.iterations == K
    # every case's seed was chosen so the oracle's gaps certify it at both
    # precisions (smallest gap 2.9e-3 over the list), so each one is checked
    assert certify.certified(ref, precision)
    assert list(to_np(res.support)) == list(ref.support)
    assert np.linalg.norm(to_np(res.x) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
