"""Launch-schedule autotuning: plans built under any schedule (transform
tile, transform threads, fused first-pass threads), set by hand or chosen by
the tuner, give bit for bit the results of the default schedule."""
import os

import numpy as np
import pytest

import instancegen
import oracle
from tests.gpu_util import lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


def _batch(cls, N, M, K, B, seed):
    import torch
    insts = [instancegen.draw_instance(cls, N, M, K, "cgauss" if cls == "F" else "gauss", 30.0,
                                       seed + b) for b in range(B)]
    ys = torch.stack([torch.from_numpy(oracle.problem.instance_measure(i, tier="transform"))
                      for i in insts]).to("cuda")
    return insts, ys


def _solve(fc, cls, N, M, K, insts, ys):
    P = fc.Plan(cls, N, M, K, [i.omega for i in insts], precision="fp32")
    sup, x, _ = P.solve(ys)
    return sup.cpu().numpy().copy(), x.cpu().numpy().copy()


CASES = [
    # (class, N, M, K, batch, schedules (tile, threads, rthreads))
    ("F", 1 << 16, 16384, 64, 8, [(512, 64, 0), (4096, 128, 0), (8192, 256, 0)]),
    ("H", 1 << 20, 32768, 48, 4, [(256, 128, 64), (2048, 64, 256), (8192, 256, 128)]),
    ("F", 1 << 19, 40000, 40, 1, [(1024, 64, 128), (4096, 256, 64)]),
    ("H", 1 << 18, 30000, 40, 2, [(512, 64, 0), (8192, 128, 0)]),
    ("F", 1 << 12, 1000, 30, 3, [(256, 64, 0), (2048, 128, 0)]),
]


@pytest.mark.parametrize("cls,N,M,K,B,scheds", CASES)
def test_schedules_bit_identical(fc, cls, N, M, K, B, scheds):
    print("schedules:", cls, N, M, K, B, flush=True)
    insts, ys = _batch(cls, N, M, K, B, 7600 + N % 97)
    assert not fc.schedule_get(cls, N, "fp32", B)["tuned"]
    sup0, x0 = _solve(fc, cls, N, M, K, insts, ys)
    try:
        for tile, th, rt in scheds:
            fc.schedule_set(cls, N, "fp32", B, tile, th, rt)
            g = fc.schedule_get(cls, N, "fp32", B)
            assert g["tuned"] and g["threads"] == th
            sup, x = _solve(fc, cls, N, M, K, insts, ys)
            assert np.array_equal(sup, sup0), (tile, th, rt)
            assert np.array_equal(x, x0), (tile, th, rt)
    finally:
        fc.schedule_set(cls, N, "fp32", B, drop=True)
    assert not fc.schedule_get(cls, N, "fp32", B)["tuned"]


def test_schedule_tune_records_cache_and_keeps_results(fc, tmp_path):
    cls, N, M, K, B = "F", 1 << 16, 16384, 48, 8
    insts, ys = _batch(cls, N, M, K, B, 7700)
    sup0, x0 = _solve(fc, cls, N, M, K, insts, ys)
    cache = str(tmp_path / "tune.txt")
    try:
        r = fc.schedule_tune(cls, N, M, "fp32", batch=B, cache_path=cache)
        assert r["ms_best"] > 0 and r["ms_best"] <= r["ms_default"] * 1.0001
        g = fc.schedule_get(cls, N, "fp32", B)
        assert g["tuned"]
        sup, x = _solve(fc, cls, N, M, K, insts, ys)
        assert np.array_equal(sup, sup0) and np.array_equal(x, x0)
        lines = [l for l in open(cache).read().splitlines() if l.startswith("sched ")]
        assert len(lines) == 1 and lines[0].split()[2:5] == [str(fc.CLASS[cls]), str(N),
                                                             str(fc.PREC["fp32"])]
        # a dropped entry comes back from the cache file, with no measuring
        fc.schedule_set(cls, N, "fp32", B, drop=True)
        assert not fc.schedule_get(cls, N, "fp32", B)["tuned"]
        fc.autotune_load(cache)
        assert fc.schedule_get(cls, N, "fp32", B)["tuned"]
        r2 = fc.schedule_tune(cls, N, M, "fp32", batch=B, cache_path=cache)
        assert (r2["tile"], r2["threads"], r2["rthreads"]) == (r["tile"], r["threads"], r["rthreads"])
        assert len([l for l in open(cache).read().splitlines() if l.startswith("sched ")]) == 1
    finally:
        fc.schedule_set(cls, N, "fp32", B, drop=True)
