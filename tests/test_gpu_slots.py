"""Slot groups of the server (iteration-granular admission): requests that
join a running group between iterations, at different iterations of their
own solves, give bit for bit the result of solving them alone, and the
(class, N, Omega) table cache and slot-resident tables are reused."""
import time

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


def _alone(fc, inst, y):
    import torch
    yd = torch.from_numpy(np.asarray(y)).to("cuda")
    r = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, yd, precision="fp32")
    return r.support.cpu().numpy(), r.x.cpu().numpy()


# (class, N, M, K, law, seed): one Fourier and one Hadamard group, K from 1
# to past the one-workgroup update (t > 64), so slots at mixed iterations run
# both update kernels in one step
SHAPES = [("F", 1 << 15, 6000, 300, "cgauss", 7301), ("F", 1 << 15, 5000, 40, "cgauss", 7302),
          ("F", 1 << 15, 7000, 1, "cgauss", 7303), ("F", 1 << 15, 5500, 120, "pm_u12", 7304),
          ("H", 1 << 16, 12000, 500, "gauss", 7305), ("H", 1 << 16, 9000, 70, "gauss", 7306),
          ("F", 1 << 15, 4000, 64, "cgauss", 7307), ("H", 1 << 16, 10000, 65, "gauss", 7308),
          ("F", 1 << 15, 6500, 200, "cgauss", 7309), ("H", 1 << 16, 8000, 2, "gauss", 7310)]


def _insts(shapes):
    out = []
    for cls, N, M, K, law, seed in shapes:
        i = instancegen.draw_instance(cls, N, M, K, law, 30.0, seed)
        out.append((i, oracle.problem.instance_measure(i, tier="transform")))
    return out


def test_slot_joins_mid_solve_equal_alone(fc):
    data = _insts(SHAPES)
    print("slot joins: staggered submissions", flush=True)
    srv = fc.Server(8 << 30)
    tickets = []
    for k, (i, y) in enumerate(data):
        tickets.append(srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32"))
        time.sleep(0.004 * (k % 3))   # later requests join running groups
    srv.drain(300000)
    got = [srv.poll(t) for t in tickets]
    info = srv.info()
    srv.close()
    assert info["completed"] == len(data)
    assert info["slot_joins"] == len(data)
    assert info["groups"] >= 2 and info["slot_steps"] > 0
    for (i, y), g in zip(data, got):
        sup, x = _alone(fc, i, y)
        assert np.array_equal(g["support"], sup), (i.cls, i.N, i.M, i.K)
        assert np.array_equal(g["x"], x), (i.cls, i.N, i.M, i.K)
        assert g["stats"].iterations == i.K
        assert g["stats"].status_detail == 0


def test_slot_groups_equal_waves(fc):
    """The same stream with slot groups disabled (lockstep waves only)."""
    data = _insts(SHAPES[:6])
    res = []
    for groups in (0, -1):
        srv = fc.Server(8 << 30, max_groups=groups)
        ts = [srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32") for i, y in data]
        srv.drain(300000)
        res.append([srv.poll(t) for t in ts])
        info = srv.info()
        srv.close()
        assert info["slot_joins"] == (len(data) if groups == 0 else 0)
    for a, b in zip(*res):
        assert np.array_equal(a["support"], b["support"])
        assert np.array_equal(a["x"], b["x"])


def test_fixed_omega_stream_reuses_tables(fc):
    """Requests sharing one Omega (class, N): tables are built at most once
    per preparing thread, then found in the cache, and joins reuse the slot's
    device tables or copy another slot's; results equal solving alone."""
    base = instancegen.draw_instance("F", 1 << 16, 12000, 150, "cgauss", 30.0, 7400)
    data = []
    for k in range(12):
        K = 40 + 13 * k
        i = instancegen.draw_instance("F", 1 << 16, 12000, K, "cgauss", 30.0, 7401 + k)
        i.omega = base.omega
        data.append((i, oracle.problem.instance_measure(i, tier="transform")))
    srv = fc.Server(8 << 30, n_streams=1)
    tickets = []
    for i, y in data:
        tickets.append(srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32"))
        time.sleep(0.002)
    srv.drain(300000)
    got = [srv.poll(t) for t in tickets]
    info = srv.info()
    srv.close()
    assert info["tables_built"] + info["tables_cached"] == len(data)
    assert 1 <= info["tables_built"] <= 2
    assert info["tables_resident"] + info["tables_copied"] >= 1
    for (i, y), g in zip(data, got):
        sup, x = _alone(fc, i, y)
        assert np.array_equal(g["support"], sup)
        assert np.array_equal(g["x"], x)


def test_slot_capacities_and_group_cycling(fc):
    """One group at a time (max_groups = 1): requests of other shapes wait for
    the running group to drain and leave; a request beyond a group's
    capacities (M above N/4, K above N/64) gets a group of its own; K = 1
    joins finish at once.  Every result equals solving alone."""
    shapes = [("F", 1 << 15, 6000, 200, "cgauss", 7501), ("H", 1 << 16, 9000, 50, "gauss", 7502),
              ("F", 1 << 15, 12000, 700, "cgauss", 7503),   # M > N/4, K > N/64
              ("F", 1 << 15, 5000, 1, "cgauss", 7504), ("H", 1 << 16, 16000, 1100, "gauss", 7505),
              ("F", 1 << 15, 7000, 90, "cgauss", 7506)]
    data = _insts(shapes)
    srv = fc.Server(4 << 30, max_groups=1, n_streams=2)
    ts = [srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32") for i, y in data]
    srv.drain(300000)
    got = [srv.poll(t) for t in ts]
    info = srv.info()
    srv.close()
    assert info["completed"] == len(data) and info["slot_joins"] == len(data)
    assert info["groups"] >= 3
    for (i, y), g in zip(data, got):
        sup, x = _alone(fc, i, y)
        assert np.array_equal(g["support"], sup), (i.cls, i.N, i.M, i.K)
        assert np.array_equal(g["x"], x)


def test_slot_server_close_with_running_groups(fc):
    """Closing the server while groups run: running requests finish, queued
    ones are dropped, and nothing hangs."""
    data = _insts(SHAPES[:4])
    srv = fc.Server(4 << 30)
    for i, y in data:
        srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, precision="fp32")
    time.sleep(0.01)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 120


def test_slot_groups_beside_waves(fc):
    """Slot-group requests (conventional OMP) served together with wave
    requests (adaptive and fast OMP, SP, CoSaMP, and small problems on the
    persistent kernel): every result equals the same request solved alone."""
    import torch
    reqs = []
    for k, (cls, N, M, K, law, seed) in enumerate(SHAPES[:5]):
        reqs.append((cls, N, M, K, law, seed, "omp", "conventional"))
    reqs += [("F", 1 << 15, 6000, 120, "cgauss", 7601, "omp", "adaptive"),
             ("H", 1 << 16, 9000, 80, "gauss", 7602, "omp", "fast"),
             ("F", 1 << 15, 4000, 40, "cgauss", 7603, "sp", "conventional"),
             ("H", 1 << 16, 6000, 30, "gauss", 7604, "cosamp", "fast"),
             ("F", 4096, 1000, 30, "cgauss", 7605, "omp", "conventional")]
    data = []
    for cls, N, M, K, law, seed, alg, meth in reqs:
        i = instancegen.draw_instance(cls, N, M, K, law, 30.0, seed)
        data.append((i, oracle.problem.instance_measure(i, tier="transform"), alg, meth))
    srv = fc.Server(8 << 30)
    ts = [srv.submit(i.cls, i.N, i.M, i.K, i.omega, y, algorithm=alg, method=meth, precision="fp32")
          for i, y, alg, meth in data]
    srv.drain(300000)
    got = [srv.poll(t) for t in ts]
    info = srv.info()
    srv.close()
    assert info["completed"] == len(data)
    assert info["slot_joins"] == 5 and info["waves"] >= 2
    for (i, y, alg, meth), g in zip(data, got):
        yd = torch.from_numpy(np.asarray(y)).to("cuda")
        r = fc.solve(i.cls, i.N, i.M, i.K, i.omega, yd, algorithm=alg, method=meth, precision="fp32")
        sup, x = r.support.cpu().numpy(), r.x.cpu().numpy()
        if alg == "omp":
            assert np.array_equal(g["support"], sup), (alg, meth, i.N)
            assert np.array_equal(g["x"], x), (alg, meth, i.N)
        else:   # set pursuits: the support as a set, x aligned with it
            assert np.array_equal(np.sort(g["support"]), np.sort(sup)), (alg, meth, i.N)
            assert np.allclose(g["x"][np.argsort(g["support"])], x[np.argsort(sup)], rtol=0,
                               atol=1e-12 * np.abs(x).max())
