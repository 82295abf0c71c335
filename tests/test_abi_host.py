"""C-ABI checks that need no GPU: every declared symbol is exported, and
host-side validation rejects bad problems before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcmp.h")


@pytest.fixture(scope="module")
def fc():
    import paper_1205_4139_amd as fc
    return fc


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fcmp_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported(fc):
    names = declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(fc.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_status(fc):
    assert fc.lib.fcmp_abi_version() == 3
    assert fc.lib.fcmp_status_str(0) == b"ok"
    assert fc.lib.fcmp_status_str(-2) == b"workspace too small"


def _q(fc, cls="F", N=1024, M=256, K=16, omega=None, **opt):
    om = (np.arange(M) * (N // max(M, 1))) if omega is None else omega
    return fc.query_workspace(cls, N, M, K, om, **opt)


def test_query_workspace_sizes(fc):
    a = _q(fc)
    b = _q(fc, K=32)
    c = _q(fc, precision="fp32")
    assert a > 0 and b > a and c > 0
    big = _q(fc, N=1 << 20, M=1 << 17, K=1024, cls="H")
    assert big > 1 << 24


@pytest.mark.parametrize("kw,msg", [
    (dict(N=1000, M=250), "power of two"),
    (dict(N=1 << 25, M=256), "power of two"),
    (dict(cls="F", N=1 << 23, M=256), "Fourier N"),
    (dict(K=256), "K must be"),
    (dict(K=0), "K must be"),
    (dict(M=0, K=1), "M must be"),
    (dict(omega=np.array([3, 2] + list(range(10, 264)))), "strictly increasing"),
    (dict(omega=np.arange(256) + 900), "out of"),
    (dict(method="bogus"), "corr_method"),
])
def test_validation_errors(fc, kw, msg):
    with pytest.raises(fc.FcmpError) as ei:
        if kw.get("method") == "bogus":
            kw = dict(kw, method=7)
        _q(fc, **kw)
    assert ei.value.code == fc.E_INVALID
    assert msg in str(ei.value)


def test_solve_rejects_null_pointers_without_device(fc):
    p, om = fc.make_problem("H", 1024, 256, 16, np.arange(256) * 4)
    o = fc.make_options()
    rc = fc.lib.fcmp_solve(ctypes.byref(p), ctypes.byref(o), None, None, 0, None, None, None, None)
    assert rc == fc.E_INVALID
    assert b"NULL" in fc.lib.fcmp_last_error()


def test_plan_shape_rules(fc):
    """OMP plans take one class and N with per-problem M and K; SP plans need
    one (M, K); different N is always rejected."""
    probs = (fc.Problem * 2)()
    oms = [np.arange(256, dtype=np.int32) * 4, np.arange(128, dtype=np.int32) * 8]

    def fill(N2=1024, K2=16):
        for i, (M, om, N, K) in enumerate(zip((256, 128), oms, (1024, N2), (16, K2))):
            probs[i] = fc.Problem(0, 0, N, M, K, om.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    n = ctypes.c_size_t(0)
    fill(K2=20)
    o = fc.make_options()
    assert fc.lib.fcmp_plan_query_workspace(2, probs, ctypes.byref(o), ctypes.byref(n)) == 0
    mixed = n.value
    o_sp = fc.make_options("sp")
    rc = fc.lib.fcmp_plan_query_workspace(2, probs, ctypes.byref(o_sp), ctypes.byref(n))
    assert rc == fc.E_INVALID and b"share M and K" in fc.lib.fcmp_last_error()
    fill(N2=2048)
    rc = fc.lib.fcmp_plan_query_workspace(2, probs, ctypes.byref(o), ctypes.byref(n))
    assert rc == fc.E_INVALID and b"class and N" in fc.lib.fcmp_last_error()
    fill(K2=20)
    rc = fc.lib.fcmp_batch_query_workspace(2, probs, ctypes.byref(o), ctypes.byref(n))
    assert rc == 0 and n.value > 0
    assert mixed > 0


def test_options_validation(fc):
    with pytest.raises(fc.FcmpError):
        _q(fc, precision=5)
    p, om = fc.make_problem("H", 1024, 256, 16, np.arange(256) * 4)
    o = fc.make_options()
    o.flags = 64   # no such flag
    n = ctypes.c_size_t(0)
    assert fc.lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)) == fc.E_INVALID
    # the conjugate-symmetric pairing: Fourier and N <= 8192 only
    o.flags = fc.FLAG_CONJ_PAIR
    with pytest.raises(fc.FcmpError, match="CONJ_PAIR"):
        fc._check(fc.lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)))
    pf, omf = fc.make_problem("F", 8192, 2048, 16, np.arange(2048) * 4)
    assert fc.lib.fcmp_query_workspace(ctypes.byref(pf), ctypes.byref(o), ctypes.byref(n)) == 0
    pg, omg = fc.make_problem("F", 16384, 2048, 16, np.arange(2048) * 8)
    assert fc.lib.fcmp_query_workspace(ctypes.byref(pg), ctypes.byref(o), ctypes.byref(n)) == fc.E_INVALID


def test_server_footprint_host_only(fc):
    """Admission footprint: at least y + support + x plus the h_0 and kernel
    vectors, grows with K, on either path."""
    om = np.arange(256) * 4
    floor = 256 * 16 + 16 * (4 + 16) + 2 * 1024 * 16
    small = fc.server_footprint("F", 1024, 256, 16, om)
    assert small >= floor
    assert fc.server_footprint("F", 1024, 256, 32, om) > small
    lock = fc.server_footprint("F", 1024, 256, 16, om, flags=fc.FLAG_NO_PERSISTENT)
    assert lock >= floor
    big = fc.server_footprint("H", 1 << 18, 1 << 16, 4096, np.arange(1 << 16) * 4)
    assert big > 4096 * 4097 // 2 * 8   # the packed FP64 inverse factor
    with pytest.raises(fc.FcmpError, match="K must be"):
        fc.server_footprint("F", 1024, 256, 256, om)


def test_batch_plan_query_host_only(fc):
    oms = [(np.arange(256) * 4).astype(np.int32), (np.arange(512) * 2).astype(np.int32)]
    probs = [("F", 1024, 256, 16, oms[0]), ("H", 1024, 512, 40, oms[1])]
    arr = (fc.Problem * 2)()
    for i, (cls, N, M, K, om) in enumerate(probs):
        arr[i] = fc.Problem(fc.CLASS[cls], 0, N, M, K,
                            om.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    o = fc.make_options()
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert fc.lib.fcmp_batch_query_workspace(2, arr, ctypes.byref(o), ctypes.byref(a)) == 0
    assert fc.lib.fcmp_batch_plan_query_workspace(2, arr, ctypes.byref(o), ctypes.byref(b)) == 0
    assert b.value >= a.value > 0


def test_server_create_rejects_missing_pool(fc):
    h = ctypes.c_void_p(0)
    assert fc.lib.fcmp_server_create(ctypes.byref(h), None, 1 << 20, None) == -1
    assert b"pool" in fc.lib.fcmp_last_error()


def test_adaptive_switch_model_and_cache(fc, tmp_path):
    """Untuned switch iterations follow Table I's flop model; a cache file
    loads tuned entries (a size no other test uses)."""
    t, tuned = fc.adaptive_switch("F", 65536, "fp32")
    assert not tuned and t == 2 + (5 * 16) // 6
    t, tuned = fc.adaptive_switch("H", 1 << 20, "fp64")
    assert not tuned and t == 1 + 20
    path = tmp_path / "switch.txt"
    path.write_text("1 2097152 1 9\n0 2097152 0 23\nbogus line\n")
    fc.autotune_load(path)
    assert fc.adaptive_switch("F", 1 << 21, "fp32") == (9, True)
    assert fc.adaptive_switch("H", 1 << 21, "fp64") == (23, True)
    (tmp_path / "empty.txt").write_text("")
    with pytest.raises(fc.FcmpError, match="no valid entries"):
        fc.autotune_load(tmp_path / "empty.txt")
    with pytest.raises(fc.FcmpError, match="power of two"):
        fc.adaptive_switch("F", 1000, "fp32")


def _struct_fields(name):
    """Member names of a typedef struct in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            out += [v.strip().lstrip("*") for v in decl.split(None, 1)[1].split(",")]
    return out


def test_stats_layout_matches_header(fc):
    """fcmp_stats: the binding's field order is the header's, and its size is
    what the C layout gives (int32 x 2, double x 2, float x 4, double)."""
    assert [f[0] for f in fc.Stats._fields_] == _struct_fields("fcmp_stats")
    assert ctypes.sizeof(fc.Stats) == 48
    assert fc.Stats.min_gap.offset == 16 and fc.Stats.ms_total.offset == 40
    assert [f[0] for f in fc.Options._fields_] == _struct_fields("fcmp_options")


@pytest.mark.parametrize("tol,ok", [(0.0, True), (0.3, True), (1e-12, True), (-1e-3, False),
                                    (1.0, False), (float("nan"), False)])
def test_res_tol_validation(fc, tol, ok):
    p, om = fc.make_problem("H", 1024, 256, 16, np.arange(256) * 4)
    o = fc.make_options(res_tol=tol)
    n = ctypes.c_size_t(0)
    rc = fc.lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n))
    if ok:
        assert rc == 0 and n.value > 0
    else:
        assert rc == fc.E_INVALID and b"res_tol" in fc.lib.fcmp_last_error()


def test_phase_times_flag_accepted(fc):
    p, om = fc.make_problem("H", 1024, 256, 16, np.arange(256) * 4)
    n = ctypes.c_size_t(0)
    o = fc.make_options(flags=fc.FLAG_PHASE_TIMES)
    assert fc.lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)) == 0
    o = fc.make_options(flags=64)
    assert fc.lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)) == fc.E_INVALID


def test_schedule_host_only(fc, tmp_path):
    """Launch schedules: the defaults a plan shape uses, argument checks, and
    cache lines of both kinds loading (no device: an entry recorded for
    another device's architecture is never used)."""
    g = fc.schedule_get("F", 1 << 16, "fp32", 256)
    assert g == {"tile": 2048, "threads": 256, "rthreads": 0, "tuned": False}
    g = fc.schedule_get("H", 1 << 20, "fp32", 8)
    assert g["tile"] == 1024 and g["rthreads"] in (64, 128, 256) and not g["tuned"]
    assert fc.schedule_get("H", 1 << 18, "fp32", 8)["rthreads"] == 0   # register-resident pass
    for bad in ((3000, 0, 0), (512, 96, 0), (512, 0, 512), (16384, 0, 0)):
        with pytest.raises(fc.FcmpError, match="tile must be"):
            fc.schedule_set("F", 1 << 16, "fp32", 8, *bad)
    nb = ctypes.c_size_t(0)
    assert fc.lib.fcmp_schedule_query_workspace(fc.CLASS["F"], 1 << 16, 16384, fc.PREC["fp32"], 8,
                                                ctypes.byref(nb)) == 0
    assert nb.value > 8 * 16384 * 16
    assert fc.lib.fcmp_schedule_query_workspace(fc.CLASS["F"], 1 << 16, 8, fc.PREC["fp32"], 8,
                                                ctypes.byref(nb)) == fc.E_INVALID
    p = tmp_path / "cache.txt"
    p.write_text("sched gfx-none 1 65536 1 4 1024 128 0\n1 8388608 1 7\nbogus line\n")
    fc.autotune_load(str(p))
    assert not fc.schedule_get("F", 1 << 16, "fp32", 256)["tuned"]


def test_slot_group_footprint_capacities(fc):
    """OMP with the fused conventional correlation is admitted as a one-slot
    group at capacities (M up to N/4, N/2 or N; K up to max(256, N/64) or the
    next power of two), so the footprint is flat inside a capacity and steps
    at its edges; other requests keep their wave footprint, growing with K."""
    N = 1 << 16
    om = np.arange(16384) * 4
    f = {K: fc.server_footprint("F", N, 16384, K, om, precision="fp32") for K in (100, 1000, 1024,
                                                                                    1025, 2000)}
    assert f[100] == f[1000] == f[1024] < f[1025] == f[2000]
    # the packed FP64 complex inverse factor of one slot at K capacity 2048
    assert f[2000] - f[1024] >= (2048 * 2049 - 1024 * 1025) // 2 * 16
    om2 = np.arange(20000) * 3   # M above N/4: the N/2 capacity
    assert fc.server_footprint("F", N, 20000, 100, om2, precision="fp32") > f[100]
    # adaptive requests run in waves: the footprint follows K itself
    a1 = fc.server_footprint("F", N, 16384, 100, om, method="adaptive", precision="fp32")
    a2 = fc.server_footprint("F", N, 16384, 1000, om, method="adaptive", precision="fp32")
    assert a1 < a2 < f[1000]
