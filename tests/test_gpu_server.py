"""The continuous-batching server: a request served in a mixed stream gives
bit-for-bit the result it gives when served alone, certified requests match
the oracle, and admission respects a small device pool."""
import numpy as np
import pytest

import instancegen
import oracle
from oracle import certify
from tests.gpu_util import lib

pytestmark = pytest.mark.gpu

_STREAM = {}


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


def _stream(count=24, seed=5100, logn=(11, 16)):
    key = (count, seed, logn)
    if key not in _STREAM:
        _arr, insts = instancegen.draw_stream(count, seed=seed, logn_range=logn)
        ys = [oracle.problem.instance_measure(i, tier="transform") for i in insts]
        _STREAM[key] = (insts, ys)
    return _STREAM[key]


def _serve(fc, insts, ys, **cfg):
    srv = fc.Server(cfg.pop("pool_bytes", 2 << 30), **cfg)
    tickets = [srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32")
               for i, y in zip(insts, ys)]
    srv.drain(300000)
    out = [srv.poll(t) for t in tickets]
    info = srv.info()
    srv.close()
    return out, info


def test_server_mix_equals_alone_and_oracle(fc):
    insts, ys = _stream()
    mixed, info = _serve(fc, insts, ys)
    assert info["submitted"] == info["completed"] == len(insts)
    assert info["queued"] == 0 and info["inflight"] == 0
    srv = fc.Server(2 << 30, n_streams=1)
    checked = 0
    for k, (inst, y) in enumerate(zip(insts, ys)):
        t = srv.submit(inst.cls, inst.N, inst.M, inst.K, inst.omega, y, precision="fp32")
        srv.drain(120000)
        alone = srv.poll(t)
        assert np.array_equal(alone["support"], mixed[k]["support"]), k
        assert np.array_equal(alone["x"], mixed[k]["x"]), k
        assert mixed[k]["stats"].iterations == inst.K
        tm = mixed[k]["times"]
        assert tm[0] <= tm[1] <= tm[2]
        if inst.N <= 4096:
            ref = oracle.omp(oracle.make_operator(inst.cls, inst.N, inst.omega), y, inst.K)
            if certify.certified(ref, "fp32"):
                assert list(mixed[k]["support"]) == list(ref.support)
                assert np.linalg.norm(mixed[k]["x"] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
                checked += 1
    srv.close()
    assert checked >= 3


def test_server_small_pool_admission(fc):
    """A pool that holds little more than the largest request: requests are
    admitted as room frees up, all complete, the pool is never overcommitted,
    and the results equal the roomy run's."""
    insts, ys = _stream()
    feet = [fc.server_footprint(i.cls, i.N, i.M, i.K, i.omega, precision="fp32") for i in insts]
    pool = int(max(feet) * 1.25) + (1 << 20)
    small, info = _serve(fc, insts, ys, pool_bytes=pool, max_slots=8)
    roomy, _ = _serve(fc, insts, ys)
    assert info["completed"] == len(insts)
    assert 0 < info["pool_peak"] <= pool
    assert info["waves"] > 1
    for a, b in zip(small, roomy):
        assert np.array_equal(a["support"], b["support"])
        assert np.array_equal(a["x"], b["x"])


def test_server_ticket_collected_once(fc):
    insts, ys = _stream()
    srv = fc.Server(1 << 30)
    i, y = insts[0], ys[0]
    t = srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32")
    srv.drain(60000)
    assert srv.poll(t) is not None
    srv._shapes[t] = (i.cls, i.K)
    with pytest.raises(fc.FcmpError, match="unknown ticket"):
        srv.poll(t)
    srv.close()
