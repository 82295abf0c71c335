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


def test_server_rejects_invalid_requests_without_disturbing_others(fc):
    """Invalid requests fail at submit (host validation); the valid ones
    around them complete exactly as they do alone."""
    insts, ys = _stream()
    srv = fc.Server(1 << 30)
    good = []
    for k, (i, y) in enumerate(zip(insts[:6], ys[:6])):
        good.append(srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32"))
        if k == 2:
            with pytest.raises(fc.FcmpError, match="K must be"):
                srv.submit(i.cls, i.N, i.M, i.M, i.omega, y, precision="fp32")
            bad_om = np.array(i.omega[::-1])
            with pytest.raises(fc.FcmpError, match="strictly increasing"):
                srv.submit(i.cls, i.N, i.M, i.K, bad_om, y, precision="fp32")
    srv.drain(120000)
    got = [srv.poll(t) for t in good]
    info = srv.info()
    srv.close()
    assert info["submitted"] == info["completed"] == 6
    alone, _ = _serve(fc, insts[:6], ys[:6], n_streams=1)
    for a, b in zip(got, alone):
        assert np.array_equal(a["support"], b["support"])
        assert np.array_equal(a["x"], b["x"])


def test_server_queue_full_is_busy(fc):
    """One request slot and two queue places: while a long solve holds the
    slot, the fourth submission is refused with FCMP_E_BUSY."""
    big = instancegen.draw_instance("F", 1 << 18, 1 << 15, 1500, "cgauss", 30.0, 5200)
    small = instancegen.draw_instance("H", 8192, 1600, 80, "gauss", 30.0, 5201)
    yb = oracle.problem.instance_measure(big, tier="transform")
    ysm = oracle.problem.instance_measure(small, tier="transform")
    srv = fc.Server(4 << 30, max_slots=1, max_pending=2, n_streams=2)
    t1 = srv.submit(big.cls, big.N, big.M, big.K, big.omega, yb, precision="fp32")
    import time
    t0 = time.time()
    while srv.info()["inflight"] < 1 and time.time() - t0 < 30:   # t1 holds the slot
        time.sleep(0.001)
    assert srv.info()["inflight"] == 1
    t2 = srv.submit(small.cls, small.N, small.M, small.K, small.omega, ysm, precision="fp32")
    t3 = srv.submit(small.cls, small.N, small.M, small.K, small.omega, ysm, precision="fp32")
    with pytest.raises(fc.FcmpError) as e:
        srv.submit(small.cls, small.N, small.M, small.K, small.omega, ysm, precision="fp32")
    assert e.value.code == fc.E_BUSY
    srv.drain(300000)
    assert all(srv.poll(t) is not None for t in (t1, t2, t3))
    srv.close()
