"""GPU parity of the single steps of the hot path against the FP64 oracle:
kernel vector (A1), conventional correlation with fused identification
(A3 + A5), fast correlation (A4 + A5) and the forward operator."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import inf_rel, lib, omega, rand_vec, to_dev, to_np

pytestmark = pytest.mark.gpu

# (N, M): single-workgroup sizes, two-pass sizes, ragged M
SIZES = [(2, 1), (16, 5), (1024, 256), (4096, 1000), (16384, 4096), (65536, 16384),
         (1 << 18, 1 << 15)]
TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


def _cplx(cls):
    return cls == "F"


@pytest.mark.parametrize("cls", ["H", "F"])
@pytest.mark.parametrize("N,M", SIZES)
def test_kernel_vector(fc, cls, N, M):
    rng = np.random.default_rng(N + M)
    om = omega(rng, N, M)
    want = oracle.kernel_vector(cls, N, om, "transform")
    c64, cp = fc.kernel_vector(cls, N, om, "fp32")
    c64 = to_np(c64)
    cp = to_np(cp)
    assert inf_rel(c64, want) <= TOL["fp64"]
    assert inf_rel(cp, want) <= 1e-6
    if cls == "H":
        # N c is an integer: the FP64 result is exact
        assert np.array_equal(c64 * N, np.round(want * N))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cls", ["H", "F"])
@pytest.mark.parametrize("N,M", SIZES)
def test_correlate(fc, cls, N, M, precision):
    rng = np.random.default_rng(3 * N + M)
    om = omega(rng, N, M)
    r = rand_vec(rng, M, _cplx(cls))
    want = oracle.unitary.TransformOperator(cls, N, om).adjoint(r)
    rd = to_dev(r.astype(np.complex64 if (_cplx(cls) and precision == "fp32") else
                         np.float32 if precision == "fp32" else r.dtype))
    h, sel = fc.correlate(cls, N, om, rd, precision)
    h = to_np(h)
    # the oracle sees the same (rounded) input the GPU saw
    rin = to_np(rd).astype(np.complex128 if _cplx(cls) else np.float64)
    want = oracle.unitary.TransformOperator(cls, N, om).adjoint(rin)
    assert inf_rel(h, want) <= TOL[precision]
    idx, key = fc.decode_sel(sel)
    a = np.abs(want) ** 2
    order = np.argsort(-a, kind="stable")
    gap = (np.sqrt(a[order[0]]) - np.sqrt(a[order[1]])) / np.sqrt(a[order[0]]) if N > 1 else 1
    if gap >= 2.5 * TOL[precision]:
        assert idx == order[0]
    else:
        assert np.sqrt(a[idx]) >= np.sqrt(a[order[0]]) * (1 - 2 * TOL[precision])


@pytest.mark.parametrize("N", [1024, 65536, 1 << 20])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_correlate_hadamard_integer_bitexact(fc, N, precision):
    """N = 4^m: integer residuals give exactly representable correlations, so
    the GPU must match the oracle bit for bit."""
    rng = np.random.default_rng(N)
    M = N // 8
    om = omega(rng, N, M)
    r = rng.integers(-6, 7, M).astype(np.float64)
    want = oracle.unitary.TransformOperator("H", N, om).adjoint(r)
    rd = to_dev(r.astype(np.float32) if precision == "fp32" else r)
    h, sel = fc.correlate("H", N, om, rd, precision)
    assert np.array_equal(to_np(h).astype(np.float64), want)


def test_correlate_ties_lowest_index(fc):
    """A single nonzero residual entry: every |h(j)| is equal, so the lowest
    eligible index wins; the exclusion bitmap removes columns."""
    import torch
    N, M = 1024, 64
    rng = np.random.default_rng(1)
    om = omega(rng, N, M)
    r = np.zeros(M)
    r[7] = 3.0
    h, sel = fc.correlate("H", N, om, to_dev(r))
    assert fc.decode_sel(sel)[0] == 0
    excl = np.zeros(N // 32, dtype=np.uint32)
    excl[0] = 0x1F          # columns 0..4 excluded
    ex = torch.from_numpy(excl.view(np.int32)).cuda()
    h, sel = fc.correlate("H", N, om, to_dev(r), excl=ex)
    assert fc.decode_sel(sel)[0] == 5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cls", ["H", "F"])
@pytest.mark.parametrize("N,M,T", [(64, 20, 3), (1024, 256, 15), (65536, 16384, 255),
                                   (1 << 20, 1 << 17, 40)])
def test_fast_correlate(fc, cls, N, M, T, precision):
    rng = np.random.default_rng(N + T)
    om = omega(rng, N, M)
    y = rand_vec(rng, M, _cplx(cls))
    op = oracle.unitary.TransformOperator(cls, N, om)
    h0 = op.adjoint(y)
    c = oracle.kernel_vector(cls, N, om, "transform")
    lam = rng.choice(N, T, replace=False).astype(np.int32)
    xt = rand_vec(rng, T, _cplx(cls)) * 0.3
    cp_np = c.astype(np.complex64 if _cplx(cls) else np.float32) if precision == "fp32" else c
    want = oracle.fast_correlation(cls, N, h0, cp_np.astype(c.dtype), lam, xt)
    h, sel = fc.fast_correlate(cls, N, to_dev(h0), to_dev(cp_np), to_dev(lam), to_dev(xt),
                               precision)
    h = to_np(h)
    # FP64 accumulation of the same rounded kernel vector: FP64-level agreement
    assert inf_rel(h, want) <= TOL["fp64"] * max(1, T)
    # against the exact kernel vector the FP32 storage error stays in tolerance
    exact = oracle.fast_correlation(cls, N, h0, c, lam, xt)
    assert inf_rel(h, exact) <= TOL[precision]
    idx, _ = fc.decode_sel(sel)
    a = np.abs(want) ** 2
    assert idx == int(np.argmax(a))


def test_fast_correlate_hadamard_integer_bitexact(fc):
    N, M, T = 4096, 1024, 50
    rng = np.random.default_rng(9)
    om = omega(rng, N, M)
    y = rng.integers(-5, 6, M).astype(np.float64)
    op = oracle.unitary.TransformOperator("H", N, om)
    h0 = op.adjoint(y)
    c = oracle.kernel_vector("H", N, om, "transform")
    lam = rng.choice(N, T, replace=False).astype(np.int32)
    xt = rng.integers(-3, 4, T).astype(np.float64)
    want = oracle.fast_correlation("H", N, h0, c, lam, xt)
    for prec, cp in (("fp64", c), ("fp32", c.astype(np.float32))):
        h, _ = fc.fast_correlate("H", N, to_dev(h0), to_dev(cp), to_dev(lam), to_dev(xt), prec)
        assert np.array_equal(to_np(h), want)


@pytest.mark.parametrize("cls", ["H", "F"])
@pytest.mark.parametrize("N,M", [(16, 5), (1024, 256), (65536, 16384)])
def test_measure(fc, cls, N, M):
    rng = np.random.default_rng(N)
    om = omega(rng, N, M)
    x = rand_vec(rng, N, _cplx(cls))
    want = oracle.unitary.TransformOperator(cls, N, om).forward(x)
    y = to_np(fc.measure(cls, N, om, to_dev(x)))
    assert inf_rel(y, want) <= TOL["fp64"]
    g = rand_vec(rng, M, _cplx(cls))
    yn = to_np(fc.measure(cls, N, om, to_dev(x), to_dev(g), 30.0))
    wn = oracle.measure(cls, N, om, x, g, 30.0, tier="transform")
    assert inf_rel(yn, wn) <= TOL["fp64"]


def _topk_case(N, K, seed):
    """|v|^2 with many exact ties straddling the K-th position: integer
    values with a few distinct magnitudes, and an exclusion set."""
    rng = np.random.default_rng(seed)
    v = rng.integers(-6, 7, N).astype(np.float64)
    # a block of exact ties around the K-th largest magnitude
    order = np.argsort(-np.abs(v), kind="stable")
    kth = abs(v[order[K - 1]])
    tie = rng.choice(N, 4 * K, replace=False)
    v[tie[: 2 * K]] = kth * rng.choice([-1.0, 1.0], 2 * K)
    excl = np.sort(rng.choice(N, N // 64, replace=False))
    return v, excl


@pytest.mark.parametrize("K", [2048, 3072])
@pytest.mark.parametrize("cls,precision", [("H", "fp32"), ("H", "fp64"), ("F", "fp32")])
def test_topk_full_size_with_ties(fc, K, cls, precision):
    """The set pursuits' top-K at N = 2^20 (K = 2K and 3K of the N = 2^20,
    K = 1024 workload) with exact ties at the K-th key and an exclusion
    bitmap: the index set equals the oracle's (ties to the lowest index)."""
    N = 1 << 20
    v, excl = _topk_case(N, K, 40 + K)
    if cls == "F":
        # |v|^2 of (a + ib) with integer parts: ties in magnitude across phases
        v = v.astype(np.complex128) * np.where(np.arange(N) % 3 == 0, 1.0, 1j)
    vd = to_dev(v.astype({("H", "fp32"): np.float32, ("H", "fp64"): np.float64,
                          ("F", "fp32"): np.complex64}[(cls, precision)]))
    bm = np.zeros((N + 31) // 32, dtype=np.uint32)
    np.bitwise_or.at(bm, excl >> 5, (np.uint32(1) << (excl & 31).astype(np.uint32)))
    out = to_np(fc.topk(cls, vd, K, precision, excl=to_dev(bm)))
    want = np.sort(oracle.topk(np.abs(v) ** 2, K, excluded=excl))
    assert np.array_equal(out, want)
    # without exclusions too
    out = to_np(fc.topk(cls, vd, K, precision))
    assert np.array_equal(out, np.sort(oracle.topk(np.abs(v) ** 2, K)))


def test_topk_fewer_eligible_than_k(fc):
    """Every entry but five excluded: the five eligible indices, then -1."""
    N, K = 4096, 8
    v = np.arange(N, dtype=np.float64)
    keep = np.array([7, 100, 2000, 2001, 4095])
    bm = np.full((N + 31) // 32, 0xFFFFFFFF, dtype=np.uint32)
    for j in keep:
        bm[j >> 5] &= ~np.uint32(1 << (j & 31))
    out = to_np(fc.topk("H", to_dev(v), K, "fp64", excl=to_dev(bm)))
    assert list(out) == list(keep) + [-1, -1, -1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cls", ["H", "F"])
@pytest.mark.parametrize("N", [1 << 15, 1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20])
def test_correlate_identification_only(fc, cls, N, precision):
    """The correlation whose outputs are only identified (the register-resident
    second pass, rows of 256, 512 or 1024): the fused argmax, with an exclusion
    bitmap that removes the oracle's top columns, picks the oracle's argmax
    over the remaining columns when its gap is certified, else a column within
    tolerance of it."""
    import torch
    rng = np.random.default_rng(N + 17)
    M = N // 4 + 3
    om = omega(rng, N, M)
    r = rand_vec(rng, M, _cplx(cls))
    rd = to_dev(r.astype(np.complex64 if (_cplx(cls) and precision == "fp32") else
                         np.float32 if precision == "fp32" else r.dtype))
    rin = to_np(rd).astype(np.complex128 if _cplx(cls) else np.float64)
    want = oracle.unitary.TransformOperator(cls, N, om).adjoint(rin)
    a = np.abs(want) ** 2
    top = np.argsort(-a, kind="stable")[:5]
    excl = np.zeros(N // 32, dtype=np.uint32)
    for j in top[:3]:
        excl[j >> 5] |= np.uint32(1 << (j & 31))
    ex = torch.from_numpy(excl.view(np.int32)).cuda()
    for e, skip in ((None, 0), (ex, 3)):
        h, sel = fc.correlate(cls, N, om, rd, precision, excl=e, want_h=False)
        assert h is None
        idx, key = fc.decode_sel(sel)
        best, second = top[skip], top[skip + 1]
        gap = (np.sqrt(a[best]) - np.sqrt(a[second])) / np.sqrt(a[top[0]])
        if gap >= 2.5 * TOL[precision]:
            assert idx == best
        else:
            assert idx not in top[:skip]
            assert np.sqrt(a[idx]) >= np.sqrt(a[best]) - 2 * TOL[precision] * np.sqrt(a[top[0]])
        assert abs(np.sqrt(key) - np.sqrt(a[idx])) <= TOL[precision] * np.sqrt(a[top[0]])


def test_corr_curve(fc):
    """fcmp_corr_curve: positive device times at every iteration; the fast
    correlation's cost grows with the tap count while the conventional one's
    does not (its residual taps are summed per column, a small share)."""
    ts = [2, 16, 128]
    fast, conv = fc.corr_curve("F", 16384, 4096, ts, precision="fp32", batch=4)
    assert all(f > 0 for f in fast) and all(c > 0 for c in conv)
    assert fast[2] > fast[0]
    assert conv[2] < 4 * conv[0]
