"""GPU OMP solves (Algorithm 1.1) against the FP64 oracle: supports must match
exactly on instances whose identification gaps are certified at the
correlation precision, and x must agree to 1e-10 relative."""
import numpy as np
import pytest

import instancegen
import oracle
from oracle import certify
from tests.gpu_util import lib, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [
    # cls, N, M, K, law, snr
    ("H", 1024, 256, 16, "gauss", None),
    ("F", 1024, 256, 16, "cgauss", 30.0),
    ("H", 4096, 1000, 37, "gauss", 40.0),
    ("F", 16384, 4096, 40, "cgauss", 30.0),
    ("H", 65536, 8192, 60, "pm_u12", None),
    ("F", 65536, 16384, 64, "cgauss", 30.0),
    ("H", 131072, 16384, 48, "gauss", 30.0),
    ("F", 131072, 32768, 48, "cgauss", 30.0),
]
METHODS = ["conventional", "fast", "adaptive"]


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


_REF = {}


def _reference(case, seed):
    key = (case, seed)
    if key not in _REF:
        cls, N, M, K, law, snr = case
        inst = instancegen.draw_instance(cls, N, M, K, law, snr, seed)
        y = oracle.problem.instance_measure(inst, tier="transform")
        op = oracle.make_operator(cls, N, inst.omega)
        ref = oracle.omp(op, y, K)
        _REF[key] = (inst, y, ref)
    return _REF[key]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}-{c[3]}")
def test_omp_parity(fc, case, method, precision):
    checked = 0
    for seed in range(3):
        inst, y, ref = _reference(case, 7000 + seed)
        if not certify.certified(ref, precision):
            continue
        res = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y),
                       method=method, precision=precision)
        sup = to_np(res.support)
        x = to_np(res.x)
        assert res.stats.status_detail == 0
        assert res.stats.iterations == inst.K
        assert list(sup) == list(ref.support)
        assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
        # the library reports ||r|| from the normal equations, ||y||^2 - ||z||^2,
        # whose absolute accuracy is eps ||y||^2 on the squared norm
        assert abs(res.stats.res_norm ** 2 - ref.res_norm ** 2) <= 1e-12 * np.linalg.norm(y) ** 2
        checked += 1
    assert checked >= 1


LONG_CASES = [
    ("F", 32768, 4096, 100, "cgauss", 30.0),    # odd log2 N: separate output grouping
    ("H", 65536, 8192, 100, "pm_u12", None),    # Hadamard: contiguous output groups
    ("F", 16384, 4096, 150, "cgauss", 30.0),
]


@pytest.mark.parametrize("resid", ["fused", "transform", "direct"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", LONG_CASES, ids=lambda c: f"{c[0]}{c[1]}-{c[3]}")
def test_omp_long_support_residual_paths(fc, case, precision, resid, monkeypatch):
    """Supports long enough for the split least-squares update (t > 64); the
    residual is fused into the correlation's first pass (the default where
    the correlation takes two passes), or forced through the separate forward
    transform or the direct sum."""
    if resid == "fused":
        monkeypatch.delenv("FCMP_RESID_RATIO", raising=False)
    else:
        monkeypatch.setenv("FCMP_RESID_RATIO", "0" if resid == "transform" else "1e30")
    checked = 0
    for seed in range(2):
        inst, y, ref = _reference(case, 7100 + seed)
        if not certify.certified(ref, precision):
            continue
        res = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y),
                       method="conventional", precision=precision)
        assert list(to_np(res.support)) == list(ref.support)
        assert np.linalg.norm(to_np(res.x) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("cls", ["H", "F"])
def test_omp_more_taps_than_one_staged_chunk(fc, cls):
    """K = 300: the fused residual stages its taps in chunks of 256, so the
    last iterations take two chunks.  N = 65536, M = 16384, noiseless
    +-U(1,2) values (seed 7100, certified at FP64 but not at FP32), FP64
    correlation: the support matches the oracle's selection order and x
    agrees to 1e-10."""
    inst, y, ref = _reference((cls, 65536, 16384, 300, "pm_u12", None), 7100)
    assert certify.certified(ref, "fp64")
    res = fc.solve(cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y), precision="fp64")
    assert list(to_np(res.support)) == list(ref.support)
    assert np.linalg.norm(to_np(res.x) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [CASES[0], CASES[3], CASES[5]], ids=lambda c: f"{c[0]}{c[1]}")
def test_min_gap_matches_oracle(fc, case, precision):
    """stats.min_gap is the smallest relative identification gap of the solve.
    The oracle normalises by the largest |h| over all columns, the library by
    the winner's |h|; selected columns have |h| = 0 in exact arithmetic, so the
    two agree up to the correlation error (a few tol)."""
    for method in ("conventional", "fast"):
        inst, y, ref = _reference(case, 7000)
        res = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y), method=method,
                       precision=precision)
        assert abs(res.stats.min_gap - certify.min_gap(ref)) <= 3 * TOL[precision] + 1e-12


@pytest.mark.parametrize("method", ["conventional", "fast"])
@pytest.mark.parametrize("cls,N,M", [("H", 1024, 256), ("F", 65536, 16384)])
def test_res_tol_stops_with_the_oracle(fc, cls, N, M, method):
    """Noiseless K0-sparse x, OMP asked for 3 K0 selections with
    res_tol = 1e-6: the library stops where the oracle does (after the K0
    planted columns), with the same selection order and x.  The persistent
    batch kernel (N = 1024 through fcmp_batch_solve) stops the same way."""
    K0 = 12
    inst = instancegen.draw_instance(cls, N, M, K0, "pm_u12", None, 7300)
    y = oracle.problem.instance_measure(inst, tier="transform")
    ref = oracle.omp(oracle.make_operator(cls, N, inst.omega), y, 3 * K0, res_tol=1e-6)
    assert ref.iterations == K0
    res = fc.solve(cls, N, M, 3 * K0, inst.omega, to_dev(y), method=method, precision="fp64",
                   res_tol=1e-6)
    assert res.stats.iterations == K0
    sup = to_np(res.support)
    assert list(sup[:K0]) == list(ref.support) and np.all(sup[K0:] == -1)
    assert np.linalg.norm(to_np(res.x)[:K0] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    assert res.stats.res_norm <= 1e-6 * np.linalg.norm(y)
    if N <= 4096:
        sups, xs, st = fc.batch_solve([(cls, N, M, 3 * K0, inst.omega)], [to_dev(y)],
                                      method=method, precision="fp64", res_tol=1e-6)
        assert st[0].iterations == K0
        assert list(to_np(sups[0])[:K0]) == list(ref.support)


def test_phase_times_per_solve(fc):
    """FCMP_FLAG_PHASE_TIMES: the solve reports its own phase times, which
    are positive where the phase ran and together stay within the solve's
    device time."""
    inst, y, ref = _reference(CASES[5], 7000)
    res = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y), precision="fp32",
                   flags=fc.FLAG_PHASE_TIMES)
    s = res.stats
    assert s.ms_corr > 0 and s.ms_ls > 0 and s.ms_select == 0
    assert s.ms_corr + s.ms_ls + s.ms_resid <= 1.05 * s.ms_total
    plain = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y), precision="fp32")
    assert plain.stats.ms_corr == 0 and plain.stats.ms_ls == 0
    assert list(to_np(plain.support)) == list(to_np(res.support))
