"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times: a sampled instance against the stored oracle solve (the
oracle needs about a minute per instance at this size, so it is solved once by
tests/golden/make_fullsize.py), and size-independent properties elsewhere
(exact noiseless recovery; an instance solved in a batch or a serving wave is
bit-identical to the same instance solved alone)."""
import json
import os

import numpy as np
import pytest

import instancegen
import oracle
from oracle import certify
from tests.gpu_util import lib, to_dev, to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "omp_fourier_n65536_m16384_k256_seed2000.json")
UNEVEN = os.path.join(os.path.dirname(__file__), "golden",
                      "uneven_batch4096_seed4000_n16384.json")
N, M, K = 65536, 16384, 256
BATCH = 256          # the benchmark's lockstep plan


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


@pytest.mark.parametrize("method", ["conventional", "adaptive"])
def test_fourier_65536_lockstep_plan_256(fc, method):
    """The benchmark's plan: 256 instances (seeds 2000..2255), complex64/FP32
    correlation.  Instance 0 reproduces the stored oracle solve (support
    exactly: its gaps are certified at FP32; x to 1e-10); instances 0 and 255
    solved alone give bit-identical results; every instance runs K steps."""
    import torch
    ref = json.load(open(GOLDEN))
    assert ref["certified"]["fp32"]
    insts = [instancegen.draw_instance("F", N, M, K, "cgauss", 30.0, 2000 + i) for i in range(BATCH)]
    ys = torch.stack([to_dev(oracle.problem.instance_measure(i, tier="transform")) for i in insts])
    plan = fc.Plan("F", N, M, K, [i.omega for i in insts], precision="fp32", method=method)
    sup, x, stats = plan.solve(ys, method=method, stats=True)
    sup, x = to_np(sup).copy(), to_np(x).copy()
    assert all(s.status_detail == 0 and s.iterations == K for s in stats)
    assert list(sup[0]) == ref["support"]
    xr = np.array(ref["x_re"]) + 1j * np.array(ref["x_im"])
    assert np.linalg.norm(x[0] - xr) <= 1e-10 * np.linalg.norm(xr)
    for b in (0, BATCH - 1):
        alone = fc.solve("F", N, M, K, insts[b].omega, ys[b], method=method, precision="fp32")
        assert np.array_equal(to_np(alone.support), sup[b])
        assert np.array_equal(to_np(alone.x), x[b])
    plan.close()


HADAMARD = os.path.join(os.path.dirname(__file__), "golden",
                        "hadamard_n1m_m131072_k1024_seed3000.json")


def _xh(e):
    return np.array(e["x"]["re"]) + (1j * np.array(e["x"]["im"]) if "im" in e["x"] else 0.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["conventional", "adaptive"])
def test_hadamard_1m_omp_against_stored_oracle(fc, method, precision):
    """Partial Hadamard N = 2^20, M = 2^17, K = 1024, +-U(1,2) values,
    noiseless, against the stored FP64 oracle solve.  Its gaps are certified
    at FP64 (smallest 4.7e-7), so the FP64 correlation must reproduce the
    selection order exactly.  At FP32, 12 of the 1024 selections have gaps
    below 2.5 tol (the first at iteration 26; two planted columns of nearly
    equal magnitude), so the order must match up to that iteration and the
    final set must be the oracle's.  x agrees to 1e-10 (FP64 least squares).
    (The fast method alone would gather (t - 1) N kernel entries per
    iteration, about 2 TB over the solve; the adaptive method runs it up to
    its switch iteration.)"""
    ref = json.load(open(HADAMARD))
    omp = ref["omp"]
    inst = instancegen.draw_config("hadamard_n1m", 0)
    y = oracle.problem.instance_measure(inst, tier="transform")
    res = fc.solve("H", inst.N, inst.M, inst.K, inst.omega, to_dev(y), method=method,
                   precision=precision)
    assert res.stats.iterations == inst.K
    sup = to_np(res.support)
    x = to_np(res.x)
    xr = _xh(omp)
    gaps = np.array(omp["gaps"])
    if precision == "fp64":
        assert omp["certified"]["fp64"]
        assert list(sup) == omp["support"]
        assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
    else:
        first = int(np.argmax(gaps < 2.5e-5))
        assert first == 26
        assert list(sup[:first]) == omp["support"][:first]
        assert sorted(sup) == sorted(omp["support"])
        o1, o2 = np.argsort(sup), np.argsort(omp["support"])
        assert np.linalg.norm(x[o1] - xr[o2]) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["conventional", "fast"])
@pytest.mark.parametrize("alg", ["sp", "cosamp"])
def test_hadamard_1m_set_pursuits_against_stored_oracle(fc, alg, method, precision):
    """SP and CoSaMP on the same instance: the final support (ascending) and
    x match the stored oracle solves."""
    ref = json.load(open(HADAMARD))[alg]
    inst = instancegen.draw_config("hadamard_n1m", 0)
    y = oracle.problem.instance_measure(inst, tier="transform")
    res = fc.solve("H", inst.N, inst.M, inst.K, inst.omega, to_dev(y), algorithm=alg,
                   method=method, precision=precision)
    assert list(to_np(res.support)) == ref["support"]
    xr = _xh(ref)
    assert np.linalg.norm(to_np(res.x) - xr) <= 1e-10 * np.linalg.norm(xr)


def test_uneven_4096_batch_plan(fc):
    """The benchmark's 4096-instance uneven batch as one graph-captured batch
    plan: ten sampled instances against the oracle (N <= 4096, certified at
    FP32), six N = 2^14 instances against stored oracle solves, two against
    the same instance solved alone on the same one-workgroup-per-instance
    path."""
    insts = instancegen.draw_batch(4096, 4000)
    ys = [to_dev(oracle.problem.instance_measure(i, tier="transform")) for i in insts]
    bp = fc.BatchPlan([(i.cls, i.N, i.M, i.K, i.omega) for i in insts], precision="fp32")
    sup, x, st = bp.solve(ys, stats=True)
    assert all(st[k].status_detail == 0 and st[k].iterations == insts[k].K for k in range(len(insts)))
    rng = np.random.default_rng(77)
    small = [k for k in range(len(insts)) if insts[k].N <= 4096]
    checked = 0
    for k in rng.choice(small, 10, replace=False):
        inst = insts[k]
        ref = oracle.omp(oracle.make_operator(inst.cls, inst.N, inst.omega),
                         to_np(ys[k]), inst.K)
        if certify.certified(ref, "fp32"):
            assert list(to_np(sup[k])) == list(ref.support), k
            assert np.linalg.norm(to_np(x[k]) - ref.x) <= 1e-10 * np.linalg.norm(ref.x), k
            checked += 1
    assert checked >= 5
    # the largest size of the batch (N = 2^14, the persistent kernel's largest
    # tile): the stored oracle solves of three Fourier and three Hadamard
    # instances, certified at FP32 (selection order exactly, x to 1e-10)
    gold = json.load(open(UNEVEN))
    assert len(gold["instances"]) == 6
    for e in gold["instances"]:
        k = e["index"]
        assert insts[k].N == 16384 and insts[k].cls == e["cls"]
        assert list(to_np(sup[k])) == e["support"], k
        xr = np.array(e["x"]["re"]) + (1j * np.array(e["x"]["im"]) if "im" in e["x"] else 0.0)
        assert np.linalg.norm(to_np(x[k]) - xr) <= 1e-10 * np.linalg.norm(xr), k
    for k in (1, 4094):
        i = insts[k]
        s1, x1, _ = fc.batch_solve([(i.cls, i.N, i.M, i.K, i.omega)], [ys[k]], precision="fp32")
        assert np.array_equal(to_np(s1[0]), to_np(sup[k]))
        assert np.array_equal(to_np(x1[0]), to_np(x[k]))
    bp.close()


def test_serving_stream_full_sizes_mix_equals_alone(fc):
    """The first twelve requests of the benchmark's Poisson stream (N up to
    2^18, K up to 2763): each result served in a mixed wave equals the same
    request served alone, bit for bit."""
    _arr, insts = instancegen.draw_stream(12, seed=5000)
    ys = [oracle.problem.instance_measure(i, tier="transform") for i in insts]
    srv = fc.Server(16 << 30)
    tickets = [srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32")
               for i, y in zip(insts, ys)]
    srv.drain(100000)
    mixed = [srv.poll(t) for t in tickets]
    srv.close()
    assert all(r["stats"].iterations == i.K for r, i in zip(mixed, insts))
    srv = fc.Server(16 << 30, n_streams=1)
    for k, (i, y) in enumerate(zip(insts, ys)):
        t = srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32")
        srv.drain(100000)
        alone = srv.poll(t)
        assert np.array_equal(alone["support"], mixed[k]["support"]), k
        assert np.array_equal(alone["x"], mixed[k]["x"]), k
    srv.close()
