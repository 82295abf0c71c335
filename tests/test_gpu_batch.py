"""Lockstep plans and mixed batches: every instance must match the oracle on
certified instances, and each result must be bit-identical to the same
instance solved alone."""
import numpy as np
import pytest

import instancegen
import oracle
from oracle import certify
from tests.gpu_util import lib, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


def _insts(cls, N, M, K, law, snr, n, base):
    out = []
    for i in range(n):
        inst = instancegen.draw_instance(cls, N, M, K, law, snr, base + i)
        y = oracle.problem.instance_measure(inst, tier="transform")
        out.append((inst, y))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["conventional", "fast", "adaptive"])
@pytest.mark.parametrize("shape", [("H", 4096, 1000, 37, "gauss", 40.0),
                                   ("F", 16384, 4096, 40, "cgauss", 30.0)],
                         ids=["H4096", "F16384"])
def test_plan_lockstep_matches_alone_and_oracle(fc, shape, method, precision):
    import torch
    cls, N, M, K, law, snr = shape
    data = _insts(cls, N, M, K, law, snr, 5, 8100)
    plan = fc.Plan(cls, N, M, K, [d[0].omega for d in data], precision=precision, method=method)
    ys = torch.stack([to_dev(d[1]) for d in data])
    sup, x, stats = plan.solve(ys, method=method, stats=True)
    sup = to_np(sup)
    x = to_np(x)
    for b, (inst, y) in enumerate(data):
        alone = fc.solve(cls, N, M, K, inst.omega, to_dev(y), method=method, precision=precision)
        assert np.array_equal(to_np(alone.support), sup[b])
        assert np.array_equal(to_np(alone.x), x[b])
        ref = oracle.omp(oracle.make_operator(cls, N, inst.omega), y, K)
        if certify.certified(ref, precision):
            assert list(sup[b]) == list(ref.support)
            assert np.linalg.norm(x[b] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
        assert stats[b].iterations == K


def test_plan_reuse_and_kernel_recompute(fc):
    """A plan solves several right-hand sides; recomputing the kernel vector
    inside the solve gives bit-identical results."""
    import torch
    data = _insts("F", 4096, 1024, 20, "cgauss", 30.0, 3, 8200)
    plan = fc.Plan("F", 4096, 1024, 20, [d[0].omega for d in data], precision="fp32")
    ys = torch.stack([to_dev(d[1]) for d in data])
    s1, x1, _ = plan.solve(ys)
    s1, x1 = to_np(s1).copy(), to_np(x1).copy()
    s2, x2, _ = plan.solve(ys, flags=fc.FLAG_RECOMPUTE_KERNEL)
    assert np.array_equal(s1, to_np(s2)) and np.array_equal(x1, to_np(x2))
    s3, x3, _ = plan.solve(ys * 2.0)
    assert np.array_equal(s1, to_np(s3))
    assert np.allclose(to_np(x3), 2 * x1, rtol=1e-12, atol=0)


def test_mixed_batch_solve(fc):
    shapes = [("H", 1024, 256, 16, "gauss", None), ("F", 2048, 512, 20, "cgauss", 30.0),
              ("H", 1024, 256, 16, "gauss", None), ("F", 65536, 8192, 30, "cgauss", 30.0)]
    probs, ys, refs = [], [], []
    for i, (cls, N, M, K, law, snr) in enumerate(shapes):
        inst = instancegen.draw_instance(cls, N, M, K, law, snr, 8300 + i)
        y = oracle.problem.instance_measure(inst, tier="transform")
        probs.append((cls, N, M, K, inst.omega))
        ys.append(to_dev(y))
        refs.append(oracle.omp(oracle.make_operator(cls, N, inst.omega), y, K))
    sups, xs, stats = fc.batch_solve(probs, ys)
    for i, ref in enumerate(refs):
        if certify.certified(ref, "fp64"):
            assert list(to_np(sups[i])) == list(ref.support)
            assert np.linalg.norm(to_np(xs[i]) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
        assert stats[i].iterations == probs[i][3]


_UNEVEN = {}


def _uneven(count, seed, logn=(10, 13), snr=40.0):
    key = (count, seed, logn, snr)
    if key not in _UNEVEN:
        insts = instancegen.draw_batch(count, seed, logn_range=logn, snr_db=snr)
        ys = [oracle.problem.instance_measure(i, tier="transform") for i in insts]
        refs = [oracle.omp(oracle.make_operator(i.cls, i.N, i.omega), y, i.K)
                for i, y in zip(insts, ys)]
        _UNEVEN[key] = (insts, ys, refs)
    return _UNEVEN[key]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["conventional", "fast", "adaptive"])
def test_persistent_batch_matches_oracle_and_alone(fc, method, precision):
    """The persistent one-workgroup-per-instance path: every instance agrees
    with the oracle (certified instances) and is bit-identical when solved
    alone."""
    insts, ys, refs = _uneven(24, 8400)
    probs = [(i.cls, i.N, i.M, i.K, i.omega) for i in insts]
    sups, xs, stats = fc.batch_solve(probs, [to_dev(y) for y in ys], method=method,
                                     precision=precision)
    checked = 0
    for k, (inst, y, ref) in enumerate(zip(insts, ys, refs)):
        assert stats[k].iterations == inst.K
        if certify.certified(ref, precision):
            assert list(to_np(sups[k])) == list(ref.support)
            assert np.linalg.norm(to_np(xs[k]) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
            checked += 1
    assert checked >= 12
    for k in (0, 5, 17):
        s1, x1, _ = fc.batch_solve([probs[k]], [to_dev(ys[k])], method=method, precision=precision)
        assert np.array_equal(to_np(s1[0]), to_np(sups[k]))
        assert np.array_equal(to_np(x1[0]), to_np(xs[k]))


def test_persistent_and_lockstep_agree(fc):
    insts, ys, _ = _uneven(10, 8500)
    probs = [(i.cls, i.N, i.M, i.K, i.omega) for i in insts]
    yd = [to_dev(y) for y in ys]
    a = fc.batch_solve(probs, yd, precision="fp64")
    b = fc.batch_solve(probs, yd, precision="fp64", flags=fc.FLAG_NO_PERSISTENT)
    for k in range(len(insts)):
        assert np.array_equal(to_np(a[0][k]), to_np(b[0][k]))
        assert np.allclose(to_np(a[1][k]), to_np(b[1][k]), rtol=0, atol=1e-12 * np.abs(to_np(b[1][k])).max())


@pytest.mark.parametrize("method", ["conventional", "adaptive"])
def test_batch_plan_graph_replays_match_eager(fc, method):
    """A batch plan replays one captured graph: persistent part plus two
    lockstep plans (N = 2^16 is beyond one workgroup's LDS).  Every replay,
    with eager work and synchronisations in between and with right-hand
    sides changing between replays, is bit-identical to the eager one-shot
    batch solve."""
    import torch
    insts, ys, _ = _uneven(12, 8600)
    big = [instancegen.draw_instance("F", 65536, 8192, 24, "cgauss", 30.0, 8650 + i)
           for i in range(2)]
    big.append(instancegen.draw_instance("H", 65536, 8192, 24, "gauss", 30.0, 8660))
    allin = list(insts) + big
    ya = list(ys) + [oracle.problem.instance_measure(i, tier="transform") for i in big]
    rng = np.random.default_rng(8670)
    yb = []
    for inst in allin:
        x = np.zeros(inst.N, dtype=complex if inst.cls == "F" else float)
        sup = rng.choice(inst.N, inst.K, replace=False)
        x[sup] = rng.standard_normal(inst.K)
        yb.append(oracle.measure(inst.cls, inst.N, inst.omega, x))
    probs = [(i.cls, i.N, i.M, i.K, i.omega) for i in allin]
    bp = fc.BatchPlan(probs, method=method, precision="fp32")
    for rep, yset in enumerate([ya, yb, ya]):
        yd = [to_dev(y) for y in yset]
        s, x, st = bp.solve(yd, stats=True)
        got_s = [to_np(t).copy() for t in s]
        got_x = [to_np(t).copy() for t in x]
        torch.cuda.synchronize()
        ref_s, ref_x, ref_st = fc.batch_solve(probs, yd, method=method, precision="fp32")
        torch.cuda.synchronize()
        for k in range(len(allin)):
            assert np.array_equal(got_s[k], to_np(ref_s[k])), (rep, k)
            assert np.array_equal(got_x[k], to_np(ref_x[k])), (rep, k)
            assert st[k].iterations == ref_st[k].iterations == allin[k].K
    bp.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lockstep_plan_with_mixed_m_and_k(fc, precision, monkeypatch):
    """One lockstep plan over problems of one class and N with different M
    and K: every problem stops after its own K selections and equals its
    solve alone bit for bit; with the residual switch pulled in, instances
    take the direct and the transform residual in the same iterations."""
    monkeypatch.setenv("FCMP_RESID_RATIO", "0.5")
    shapes = [(4096, 90), (1500, 80), (3000, 40), (2000, 100)]
    insts = [instancegen.draw_instance("F", 16384, M, K, "cgauss", 30.0, 8700 + i)
             for i, (M, K) in enumerate(shapes)]
    ys = [oracle.problem.instance_measure(i, tier="transform") for i in insts]
    probs = [(i.cls, i.N, i.M, i.K, i.omega) for i in insts]
    sups, xs, stats = fc.batch_solve(probs, [to_dev(y) for y in ys], precision=precision,
                                     flags=fc.FLAG_NO_PERSISTENT)
    for k, (inst, y) in enumerate(zip(insts, ys)):
        assert stats[k].iterations == inst.K
        alone = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y),
                         precision=precision)
        assert np.array_equal(to_np(alone.support), to_np(sups[k])), k
        assert np.array_equal(to_np(alone.x), to_np(xs[k])), k
        ref = oracle.omp(oracle.make_operator(inst.cls, inst.N, inst.omega), y, inst.K)
        if certify.certified(ref, precision):
            assert list(to_np(sups[k])) == list(ref.support)
            assert np.linalg.norm(to_np(xs[k]) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [("F", 32768, "cgauss", [(8192, 120), (3000, 70), (6000, 30), (4096, 90)]),
                                  ("H", 65536, "gauss", [(8192, 100), (5000, 70), (7000, 40)])],
                         ids=["F32768", "H65536"])
def test_fused_residual_plan_with_mixed_m_and_k(fc, case, precision, monkeypatch):
    """The residual fused into the correlation's first pass, in one lockstep
    plan whose problems have different M and K: problems that are done stop
    while the others continue (their tap order is no longer maintained), and
    every problem equals its solve alone bit for bit and the oracle on
    certified instances."""
    monkeypatch.delenv("FCMP_RESID_RATIO", raising=False)
    cls, N, law, shapes = case
    insts = [instancegen.draw_instance(cls, N, M, K, law, 30.0, 8750 + i)
             for i, (M, K) in enumerate(shapes)]
    ys = [oracle.problem.instance_measure(i, tier="transform") for i in insts]
    probs = [(i.cls, i.N, i.M, i.K, i.omega) for i in insts]
    sups, xs, stats = fc.batch_solve(probs, [to_dev(y) for y in ys], precision=precision,
                                     flags=fc.FLAG_NO_PERSISTENT)
    checked = 0
    for k, (inst, y) in enumerate(zip(insts, ys)):
        assert stats[k].iterations == inst.K
        alone = fc.solve(inst.cls, inst.N, inst.M, inst.K, inst.omega, to_dev(y),
                         precision=precision)
        assert np.array_equal(to_np(alone.support), to_np(sups[k])), k
        assert np.array_equal(to_np(alone.x), to_np(xs[k])), k
        ref = oracle.omp(oracle.make_operator(inst.cls, inst.N, inst.omega, "transform"), y, inst.K)
        if certify.certified(ref, precision):
            assert list(to_np(sups[k])) == list(ref.support)
            assert np.linalg.norm(to_np(xs[k]) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
            checked += 1
    assert checked >= 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fast_correlation_half_kernel_vector(fc, precision):
    """Fast correlation gathering only c(0..N/2), with c(m) = conj(c(N - m))
    above N/2: the oracle's support on certified instances and x to 1e-10,
    and x within rounding of the full-table solve; the flag leaves the
    Hadamard class unchanged bit for bit."""
    import torch
    data = _insts("F", 65536, 8192, 60, "cgauss", 30.0, 3, 8950)
    plan = fc.Plan("F", 65536, 8192, 60, [d[0].omega for d in data], precision=precision,
                   method="fast")
    ys = torch.stack([to_dev(d[1]) for d in data])
    s_full, x_full, _ = plan.solve(ys, method="fast")
    s_full, x_full = to_np(s_full).copy(), to_np(x_full).copy()
    s_half, x_half, st = plan.solve(ys, method="fast", flags=fc.FLAG_HALF_KERNEL, stats=True)
    s_half, x_half = to_np(s_half), to_np(x_half)
    checked = 0
    for b, (inst, y) in enumerate(data):
        assert st[b].iterations == 60
        ref = oracle.omp(oracle.make_operator("F", 65536, inst.omega, "transform"), y, 60)
        if certify.certified(ref, precision):
            assert list(s_half[b]) == list(ref.support)
            assert np.linalg.norm(x_half[b] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
            checked += 1
        if list(s_half[b]) == list(s_full[b]):
            assert np.linalg.norm(x_half[b] - x_full[b]) <= 1e-12 * np.linalg.norm(x_full[b])
    assert checked >= 1
    hd = _insts("H", 4096, 1000, 37, "gauss", 40.0, 2, 8960)
    hplan = fc.Plan("H", 4096, 1000, 37, [d[0].omega for d in hd], precision=precision,
                    method="fast")
    hy = torch.stack([to_dev(d[1]) for d in hd])
    a, ax, _ = hplan.solve(hy, method="fast")
    a, ax = to_np(a).copy(), to_np(ax).copy()
    b2, bx, _ = hplan.solve(hy, method="fast", flags=fc.FLAG_HALF_KERNEL)
    assert np.array_equal(a, to_np(b2)) and np.array_equal(ax, to_np(bx))


def test_autotuned_adaptive_switch(fc, tmp_path):
    """The autotuner records a measured switch iteration; adaptive solves with
    switch_t = 0 then use it, bit for bit as when it is passed explicitly, and
    a cache file written by one call short-cuts the next."""
    cache = str(tmp_path / "tune.txt")
    t = fc.autotune("F", 16384, 4096, "fp32", batch=4, cache_path=cache)
    assert 1 <= t <= 8 * (2 + (5 * 14) // 6) + 8
    assert fc.adaptive_switch("F", 16384, "fp32") == (t, True)
    assert open(cache).read().split() == ["1", "16384", "1", str(t)]
    assert fc.autotune("F", 16384, 4096, "fp32", batch=4, cache_path=cache) == t
    data = _insts("F", 16384, 4096, 40, "cgauss", 30.0, 2, 8800)
    plan = fc.Plan("F", 16384, 4096, 40, [d[0].omega for d in data], precision="fp32",
                   method="adaptive")
    import torch
    ys = torch.stack([to_dev(d[1]) for d in data])
    s1, x1, _ = plan.solve(ys, method="adaptive")
    s1, x1 = to_np(s1).copy(), to_np(x1).copy()
    s2, x2, _ = plan.solve(ys, method="adaptive", switch_t=t)
    assert np.array_equal(s1, to_np(s2)) and np.array_equal(x1, to_np(x2))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["fast", "adaptive"])
def test_hadamard_integer_kernel_bit_identical(fc, method, precision):
    """Hadamard plans with M < 2^15 gather the kernel vector's integers N c as
    int16; since (N c)/N is exact, the solve equals the floating-point gather
    bit for bit (and the oracle on certified instances)."""
    import torch
    data = _insts("H", 4096, 1000, 37, "gauss", 40.0, 3, 8900)
    plan = fc.Plan("H", 4096, 1000, 37, [d[0].omega for d in data], precision=precision,
                   method=method)
    ys = torch.stack([to_dev(d[1]) for d in data])
    s1, x1, _ = plan.solve(ys, method=method)
    s1, x1 = to_np(s1).copy(), to_np(x1).copy()
    s2, x2, _ = plan.solve(ys, method=method, flags=fc.FLAG_FLOAT_KERNEL)
    assert np.array_equal(s1, to_np(s2)) and np.array_equal(x1, to_np(x2))
    for b, (inst, y) in enumerate(data):
        ref = oracle.omp(oracle.make_operator("H", 4096, inst.omega), y, 37)
        if certify.certified(ref, precision):
            assert list(s1[b]) == list(ref.support)


def test_fused_residual_choice_independent_of_plan_size(fc):
    """Whether the residual is fused into the correlation's first pass
    depends on (class, N, precision) only: complex128 Fourier N = 2^20 (the
    non-register fused kernel) solved in a plan of 34 instances and alone
    gives bit-identical supports and x."""
    import torch
    N, M, K = 1 << 20, 1 << 17, 6
    data = _insts("F", N, M, K, "cgauss", 30.0, 34, 8500)
    plan = fc.Plan("F", N, M, K, [d[0].omega for d in data], precision="fp64")
    ys = torch.stack([to_dev(d[1]) for d in data])
    sup, x, _ = plan.solve(ys)
    sup, x = to_np(sup).copy(), to_np(x).copy()
    plan.close()
    for b in (0, 33):
        inst, y = data[b]
        alone = fc.solve("F", N, M, K, inst.omega, to_dev(y), precision="fp64")
        assert np.array_equal(to_np(alone.support), sup[b])
        assert np.array_equal(to_np(alone.x), x[b])


@pytest.mark.parametrize("cls", ["F", "H"])
def test_split_update_batch_of_eight_matches_alone(fc, cls):
    """A lockstep batch whose size is a multiple of 8 runs the split
    least-squares update (t > 64) on the XCD-grouped grid; every instance
    still equals its solve alone bit for bit (same rows per workgroup, same
    sum order), and the oracle on certified instances."""
    import torch
    N, M, K = 8192, 2048, 100
    law = "cgauss" if cls == "F" else "gauss"
    data = _insts(cls, N, M, K, law, 30.0, 16, 8700)
    plan = fc.Plan(cls, N, M, K, [d[0].omega for d in data], precision="fp32")
    ys = torch.stack([to_dev(d[1]) for d in data])
    sup, x, stats = plan.solve(ys, stats=True)
    sup, x = to_np(sup).copy(), to_np(x).copy()
    plan.close()
    for b, (inst, y) in enumerate(data):
        alone = fc.solve(cls, N, M, K, inst.omega, to_dev(y), precision="fp32")
        assert np.array_equal(to_np(alone.support), sup[b]), b
        assert np.array_equal(to_np(alone.x), x[b]), b
        assert stats[b].iterations == K
    checked = 0
    for b in (0, 9):
        inst, y = data[b]
        ref = oracle.omp(oracle.make_operator(cls, N, inst.omega), y, K)
        if certify.certified(ref, "fp32"):
            assert list(sup[b]) == list(ref.support)
            assert np.linalg.norm(x[b] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
            checked += 1
    assert checked >= 1
