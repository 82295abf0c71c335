"""Python binding of libfcmp.so (fast correlation for matching pursuit on MI355X).

Argument marshalling only: every step of the recovery runs in the library's
HIP kernels.  Device buffers are torch tensors on the current HIP device;
work is enqueued on ``torch.cuda.current_stream()``.  There is no CPU
fallback: importing the binding fails when the library has not been built
(``python -m paper_1205_4139_amd.build``).

Value types on the device:
  Hadamard class: float64 (y, x, h_0, kernel vector), float32 in FP32 mode;
  Fourier class : complex128, complex64 in FP32 mode.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FCMP_LIBRARY selects another build of the same library (the host-sanitizer
# builds of paper_1205_4139_amd/build.py); there is no fallback when it is absent.
LIB_PATH = os.environ.get("FCMP_LIBRARY") or os.path.join(_HERE, "libfcmp.so")

HADAMARD, FOURIER = 0, 1
OMP, SP, COSAMP = 0, 1, 2
CONVENTIONAL, FAST, ADAPTIVE = 0, 1, 2
FP64, FP32 = 0, 1

E_OK, E_INVALID, E_WORKSPACE, E_DEVICE, E_BUSY, E_NUMERIC, E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6

CLASS = {"H": HADAMARD, "F": FOURIER, HADAMARD: HADAMARD, FOURIER: FOURIER}
METHOD = {"conventional": CONVENTIONAL, "fast": FAST, "adaptive": ADAPTIVE}
ALGO = {"omp": OMP, "sp": SP, "cosamp": COSAMP}
PREC = {"fp64": FP64, "fp32": FP32}


class FcmpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fcmp error {code}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("matrix_class", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("N", ctypes.c_int64), ("M", ctypes.c_int64), ("K", ctypes.c_int64),
                ("omega", ctypes.POINTER(ctypes.c_int32))]


class Options(ctypes.Structure):
    _fields_ = [("algorithm", ctypes.c_int32), ("corr_method", ctypes.c_int32),
                ("corr_precision", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("switch_t", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("res_tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status_detail", ctypes.c_int32),
                ("res_norm", ctypes.c_double), ("min_gap", ctypes.c_double),
                ("ms_corr", ctypes.c_float), ("ms_select", ctypes.c_float),
                ("ms_ls", ctypes.c_float), ("ms_resid", ctypes.c_float),
                ("ms_total", ctypes.c_double)]


NPHASE = 8
PHASES = ["kernel", "h0", "corr", "fast", "resid", "ls", "other", "select"]
FLAG_RECOMPUTE_KERNEL = 1
FLAG_PHASE_TIMES = 16
FLAG_CONJ_PAIR = 32


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("max_pending", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("max_wave", ctypes.c_int32),
                ("max_groups", ctypes.c_int32)]


class Times(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("inflight", ctypes.c_int64),
                ("waves", ctypes.c_int64), ("pool_peak", ctypes.c_int64),
                ("groups", ctypes.c_int64), ("slot_joins", ctypes.c_int64),
                ("slot_steps", ctypes.c_int64), ("tables_built", ctypes.c_int64),
                ("tables_cached", ctypes.c_int64), ("tables_resident", ctypes.c_int64),
                ("tables_copied", ctypes.c_int64)]


class Schedule(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("threads", ctypes.c_int32), ("rthreads", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NPHASE), ("launches", ctypes.c_int64 * NPHASE)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run: python -m paper_1205_4139_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P, O = ctypes.POINTER(Problem), ctypes.POINTER(Options)
    sigs = {
        "fcmp_abi_version": ([], ctypes.c_int),
        "fcmp_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "fcmp_last_error": ([], ctypes.c_char_p),
        "fcmp_query_workspace": ([P, O, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_solve": ([P, O, vp, vp, sz, vp, vp, ctypes.POINTER(Stats), vp], ctypes.c_int),
        "fcmp_solve_noalloc": ([P, O, vp, vp, vp, ctypes.POINTER(Stats), vp], ctypes.c_int),
        "fcmp_batch_query_workspace": ([i64, P, O, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_batch_solve": ([i64, P, O, ctypes.POINTER(vp), vp, sz, ctypes.POINTER(vp),
                              ctypes.POINTER(vp), ctypes.POINTER(Stats), vp], ctypes.c_int),
        "fcmp_batch_plan_query_workspace": ([i64, P, O, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_batch_plan_create": ([ctypes.POINTER(vp), i64, P, O, vp, sz, vp], ctypes.c_int),
        "fcmp_batch_plan_solve": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(Stats), vp], ctypes.c_int),
        "fcmp_batch_plan_destroy": ([vp], ctypes.c_int),
        "fcmp_plan_query_workspace": ([i64, P, O, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_autotune_query_workspace": ([i32, i64, i64, i32, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_autotune": ([i32, i64, i64, i32, i32, ctypes.c_char_p, vp, sz,
                           ctypes.POINTER(i32), vp], ctypes.c_int),
        "fcmp_autotune_load": ([ctypes.c_char_p], ctypes.c_int),
        "fcmp_schedule_query_workspace": ([i32, i64, i64, i32, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_schedule_tune": ([i32, i64, i64, i32, i32, ctypes.c_char_p, vp, sz,
                                ctypes.POINTER(Schedule), ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), vp], ctypes.c_int),
        "fcmp_schedule_set": ([i32, i64, i32, i32, ctypes.POINTER(Schedule)], ctypes.c_int),
        "fcmp_schedule_get": ([i32, i64, i32, i32, ctypes.POINTER(Schedule),
                               ctypes.POINTER(i32)], ctypes.c_int),
        "fcmp_corr_curve_query_workspace": ([i32, i64, i64, i32, i32, i32, ctypes.POINTER(sz)],
                                            ctypes.c_int),
        "fcmp_corr_curve": ([i32, i64, i64, i32, i32, ctypes.c_uint32, ctypes.POINTER(i32), i32, vp, sz,
                             ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), vp],
                            ctypes.c_int),
        "fcmp_adaptive_switch": ([i32, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
                                 ctypes.c_int),
        "fcmp_server_footprint": ([P, O, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_server_create": ([ctypes.POINTER(vp), vp, sz, ctypes.POINTER(ServerConfig)],
                               ctypes.c_int),
        "fcmp_server_submit": ([vp, P, O, vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "fcmp_server_poll": ([vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(Stats),
                             ctypes.POINTER(Times), ctypes.POINTER(i32)], ctypes.c_int),
        "fcmp_server_drain": ([vp, dbl], ctypes.c_int),
        "fcmp_server_get_info": ([vp, ctypes.POINTER(ServerInfo)], ctypes.c_int),
        "fcmp_server_destroy": ([vp], ctypes.c_int),
        "fcmp_plan_create": ([ctypes.POINTER(vp), i64, P, O, vp, sz, vp], ctypes.c_int),
        "fcmp_plan_solve": ([vp, O, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                             ctypes.POINTER(Stats), vp], ctypes.c_int),
        "fcmp_plan_destroy": ([vp], ctypes.c_int),
        "fcmp_profile_enable": ([ctypes.c_int], ctypes.c_int),
        "fcmp_profile_read": ([ctypes.POINTER(Profile), ctypes.c_int], ctypes.c_int),
        "fcmp_kernel_vector_workspace": ([P, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_kernel_vector": ([P, i32, vp, vp, vp, sz, vp], ctypes.c_int),
        "fcmp_correlate_workspace": ([P, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_correlate": ([P, i32, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "fcmp_fast_correlate_workspace": ([P, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_fast_correlate": ([P, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "fcmp_topk_workspace": ([i64, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_topk": ([i32, i32, vp, i64, vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "fcmp_measure_workspace": ([P, ctypes.POINTER(sz)], ctypes.c_int),
        "fcmp_measure": ([P, vp, vp, dbl, vp, vp, sz, vp], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(rc: int):
    if rc != 0:
        raise FcmpError(rc, lib.fcmp_last_error().decode())
    return rc


def make_problem(cls, N: int, M: int, K: int, omega) -> tuple:
    """(Problem struct, keep-alive omega array)."""
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.int32))
    p = Problem(CLASS[cls], 0, int(N), int(M), int(K),
                om.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return p, om


def make_options(algorithm="omp", method="conventional", precision="fp64",
                 max_iter=0, switch_t=0, flags=0, res_tol=0.0) -> Options:
    return Options(ALGO.get(algorithm, algorithm), METHOD.get(method, method),
                   PREC.get(precision, precision), int(max_iter), int(switch_t), int(flags),
                   float(res_tol))


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dtype(cls, precision="fp64"):
    torch = _torch()
    f = CLASS[cls] == FOURIER
    if PREC.get(precision, precision) == FP32:
        return torch.complex64 if f else torch.float32
    return torch.complex128 if f else torch.float64


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class SolveResult:
    support: "object"      # int32 tensor [K]
    x: "object"            # float64 / complex128 tensor [K]
    stats: Optional[Stats]


def query_workspace(cls, N, M, K, omega, algorithm="omp", method="conventional",
                    precision="fp64", switch_t=0) -> int:
    p, _om = make_problem(cls, N, M, K, omega)
    o = make_options(algorithm, method, precision, switch_t=switch_t)
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)))
    return n.value


def solve(cls, N, M, K, omega, y, algorithm="omp", method="conventional", precision="fp64",
          switch_t=0, max_iter=0, stats=True, workspace=None, flags=0,
          res_tol=0.0) -> SolveResult:
    torch = _torch()
    p, _om = make_problem(cls, N, M, K, omega)
    o = make_options(algorithm, method, precision, max_iter, switch_t, flags, res_tol)
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)))
    dev = y.device
    ws = workspace if workspace is not None and workspace.numel() >= n.value else _workspace(n.value, dev)
    sup = torch.empty(int(K), dtype=torch.int32, device=dev)
    x = torch.empty(int(K), dtype=_dtype(cls), device=dev)
    st = Stats() if stats else None
    _check(lib.fcmp_solve(ctypes.byref(p), ctypes.byref(o), _ptr(y), _ptr(ws), ws.numel(),
                          _ptr(sup), _ptr(x), ctypes.byref(st) if st is not None else None,
                          _stream()))
    return SolveResult(sup, x, st)


def solve_noalloc(cls, N, M, K, omega, y, algorithm="omp", method="conventional",
                  precision="fp64", switch_t=0, max_iter=0, stats=True) -> SolveResult:
    """fcmp_solve_noalloc: the solve's workspace is the library's static
    device scratch (no workspace argument, no device allocation inside)."""
    torch = _torch()
    p, _om = make_problem(cls, N, M, K, omega)
    o = make_options(algorithm, method, precision, max_iter, switch_t)
    dev = y.device
    sup = torch.empty(int(K), dtype=torch.int32, device=dev)
    x = torch.empty(int(K), dtype=_dtype(cls), device=dev)
    st = Stats() if stats else None
    _check(lib.fcmp_solve_noalloc(ctypes.byref(p), ctypes.byref(o), _ptr(y), _ptr(sup), _ptr(x),
                                  ctypes.byref(st) if st is not None else None, _stream()))
    return SolveResult(sup, x, st)


def kernel_vector(cls, N, omega, precision="fp64", device="cuda"):
    torch = _torch()
    p, _om = make_problem(cls, N, len(omega), 1, omega)
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_kernel_vector_workspace(ctypes.byref(p), ctypes.byref(n)))
    ws = _workspace(n.value, device)
    c64 = torch.empty(int(N), dtype=_dtype(cls), device=device)
    cp = torch.empty(int(N), dtype=_dtype(cls, precision), device=device)
    _check(lib.fcmp_kernel_vector(ctypes.byref(p), PREC[precision], _ptr(c64), _ptr(cp),
                                  _ptr(ws), ws.numel(), _stream()))
    return c64, cp


def _sel_tensor(device):
    torch = _torch()
    return torch.zeros(3, dtype=torch.float64, device=device)   # {key, index, runner-up key}


def decode_sel(sel) -> tuple:
    """(index, |h|^2) from the selection record {key, index, runner-up key}."""
    a = sel.detach().cpu().numpy()
    key = float(a[0])
    idx = int(a[1:2].view(np.int64)[0])
    return idx, key


def correlate(cls, N, omega, r, precision="fp64", excl=None, want_h=True):
    """h = Phi^H r (conventional, one transform) and the fused selection."""
    torch = _torch()
    p, _om = make_problem(cls, N, len(omega), 1, omega)
    pr = PREC[precision]
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_correlate_workspace(ctypes.byref(p), pr, ctypes.byref(n)))
    ws = _workspace(n.value, r.device)
    h = torch.empty(int(N), dtype=_dtype(cls, precision), device=r.device) if want_h else None
    sel = _sel_tensor(r.device)
    _check(lib.fcmp_correlate(ctypes.byref(p), pr, _ptr(r), _ptr(h), _ptr(excl), _ptr(sel),
                              _ptr(ws), ws.numel(), _stream()))
    return h, sel


def fast_correlate(cls, N, h0, cp, lam, xt, precision="fp64", excl=None, want_h=True):
    """h = h0 - sum x P_lam c (eq. (kernelsum)) and the fused selection."""
    torch = _torch()
    p, _om = make_problem(cls, N, 1, 1, [0])
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_fast_correlate_workspace(ctypes.byref(p), ctypes.byref(n)))
    ws = _workspace(n.value, h0.device)
    h = torch.empty(int(N), dtype=_dtype(cls), device=h0.device) if want_h else None
    sel = _sel_tensor(h0.device)
    nt = 0 if lam is None else int(lam.numel())
    _check(lib.fcmp_fast_correlate(ctypes.byref(p), PREC[precision], _ptr(h0), _ptr(cp),
                                   _ptr(lam), _ptr(xt), nt, _ptr(h), _ptr(excl), _ptr(sel),
                                   _ptr(ws), ws.numel(), _stream()))
    return h, sel


def topk(cls, v, K, precision="fp64", excl=None):
    """The K indices of largest |v|^2 (ties to the lowest index, excluded
    bits skipped), ascending; -1 in slots past the last eligible index."""
    torch = _torch()
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_topk_workspace(int(v.numel()), ctypes.byref(n)))
    ws = _workspace(n.value, v.device)
    out = torch.empty(int(K), dtype=torch.int32, device=v.device)
    _check(lib.fcmp_topk(CLASS[cls], PREC[precision], _ptr(v), int(v.numel()), _ptr(excl), int(K),
                         _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def measure(cls, N, omega, x, noise=None, snr_db=None):
    """y = Phi x (+ noise scaled to snr_db)."""
    torch = _torch()
    p, _om = make_problem(cls, N, len(omega), 1, omega)
    n = ctypes.c_size_t(0)
    _check(lib.fcmp_measure_workspace(ctypes.byref(p), ctypes.byref(n)))
    ws = _workspace(n.value, x.device)
    y = torch.empty(len(omega), dtype=_dtype(cls), device=x.device)
    use_noise = noise is not None and snr_db is not None
    _check(lib.fcmp_measure(ctypes.byref(p), _ptr(x), _ptr(noise) if use_noise else None,
                            float(snr_db) if use_noise else 0.0, _ptr(y), _ptr(ws), ws.numel(),
                            _stream()))
    return y


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))()
    for i, v in enumerate(ptrs):
        arr[i] = v
    return arr


class Plan:
    """n problems of one shape (class, N, M, K), each with its own Omega,
    solved in lockstep; the kernel vectors are computed once at creation."""

    def __init__(self, cls, N, M, K, omegas, algorithm="omp", method="conventional",
                 precision="fp64", switch_t=0, max_iter=0, device="cuda"):
        torch = _torch()
        self.cls, self.N, self.M, self.K = cls, int(N), int(M), int(K)
        self.n = len(omegas)
        self._oms = [np.ascontiguousarray(np.asarray(o, dtype=np.int32)) for o in omegas]
        self._probs = (Problem * self.n)()
        for i, om in enumerate(self._oms):
            self._probs[i] = Problem(CLASS[cls], 0, self.N, self.M, self.K,
                                     om.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self.opt = make_options(algorithm, method, precision, max_iter, switch_t)
        self.algorithm, self.precision = algorithm, precision
        n = ctypes.c_size_t(0)
        _check(lib.fcmp_plan_query_workspace(self.n, self._probs, ctypes.byref(self.opt),
                                             ctypes.byref(n)))
        self.ws_bytes = n.value
        self.ws = _workspace(n.value, device)
        self._h = ctypes.c_void_p(0)
        _check(lib.fcmp_plan_create(ctypes.byref(self._h), self.n, self._probs,
                                    ctypes.byref(self.opt), _ptr(self.ws), self.ws.numel(),
                                    _stream()))
        self.device = device
        self.support = torch.empty((self.n, self.K), dtype=torch.int32, device=device)
        self.x = torch.empty((self.n, self.K), dtype=_dtype(cls), device=device)

    def solve(self, ys, method=None, switch_t=0, flags=0, stats=False, res_tol=0.0):
        """ys: tensor [n, M] (or list of n tensors).  Returns (support [n, K],
        x [n, K], stats list or None); outputs are overwritten by the next solve."""
        o = make_options(self.algorithm, method or METHOD_NAME[self.opt.corr_method],
                         self.precision, self.opt.max_iter, switch_t, flags, res_tol)
        if hasattr(ys, "dim") and ys.dim() == 2:
            yp = [ys.data_ptr() + i * ys.stride(0) * ys.element_size() for i in range(self.n)]
        else:
            yp = [t.data_ptr() for t in ys]
        sp = [self.support.data_ptr() + i * self.K * 4 for i in range(self.n)]
        xe = self.x.element_size()
        xp = [self.x.data_ptr() + i * self.K * xe for i in range(self.n)]
        st = (Stats * self.n)() if stats else None
        _check(lib.fcmp_plan_solve(self._h, ctypes.byref(o), _ptr_array(yp), _ptr_array(sp),
                                   _ptr_array(xp), st, _stream()))
        return self.support, self.x, (list(st) if stats else None)

    def close(self):
        if self._h:
            lib.fcmp_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


METHOD_NAME = {CONVENTIONAL: "conventional", FAST: "fast", ADAPTIVE: "adaptive"}


def profile_enable(on=True):
    _check(lib.fcmp_profile_enable(1 if on else 0))


def profile_read(reset=True) -> dict:
    pr = Profile()
    _check(lib.fcmp_profile_read(ctypes.byref(pr), 1 if reset else 0))
    return {name: (pr.ms[i], int(pr.launches[i])) for i, name in enumerate(PHASES)}


FLAG_NO_PERSISTENT = 2
FLAG_FLOAT_KERNEL = 4
FLAG_HALF_KERNEL = 8


def batch_solve(problems, ys, algorithm="omp", method="conventional", precision="fp64",
                switch_t=0, device="cuda", flags=0, stats=True, res_tol=0.0):
    """Mixed-shape batch.  problems: list of (cls, N, M, K, omega); ys: list of
    device tensors.  Returns (supports, xs, stats) as lists."""
    torch = _torch()
    n = len(problems)
    oms = [np.ascontiguousarray(np.asarray(p[4], dtype=np.int32)) for p in problems]
    probs = (Problem * n)()
    for i, (cls, N, M, K, _o) in enumerate(problems):
        probs[i] = Problem(CLASS[cls], 0, int(N), int(M), int(K),
                           oms[i].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    o = make_options(algorithm, method, precision, 0, switch_t, flags, res_tol)
    nb = ctypes.c_size_t(0)
    _check(lib.fcmp_batch_query_workspace(n, probs, ctypes.byref(o), ctypes.byref(nb)))
    ws = _workspace(nb.value, device)
    sups = [torch.empty(int(p[3]), dtype=torch.int32, device=device) for p in problems]
    xs = [torch.empty(int(p[3]), dtype=_dtype(p[0]), device=device) for p in problems]
    st = (Stats * n)() if stats else None
    _check(lib.fcmp_batch_solve(n, probs, ctypes.byref(o), _ptr_array([y.data_ptr() for y in ys]),
                                _ptr(ws), ws.numel(), _ptr_array([t.data_ptr() for t in sups]),
                                _ptr_array([t.data_ptr() for t in xs]), st, _stream()))
    return sups, xs, (list(st) if stats else None)


class BatchPlan:
    """A fixed set of uneven problems, list of (cls, N, M, K, omega): tables and
    kernel vectors built once; each solve replays one captured device graph
    (OMP).  Outputs are lists of device tensors, overwritten by the next solve."""

    def __init__(self, problems, algorithm="omp", method="conventional", precision="fp64",
                 switch_t=0, flags=0, device="cuda"):
        torch = _torch()
        self.n = len(problems)
        self.problems = problems
        self._oms = [np.ascontiguousarray(np.asarray(p[4], dtype=np.int32)) for p in problems]
        self._probs = (Problem * self.n)()
        for i, (cls, N, M, K, _o) in enumerate(problems):
            self._probs[i] = Problem(CLASS[cls], 0, int(N), int(M), int(K),
                                     self._oms[i].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self.opt = make_options(algorithm, method, precision, 0, switch_t, flags)
        nb = ctypes.c_size_t(0)
        _check(lib.fcmp_batch_plan_query_workspace(self.n, self._probs, ctypes.byref(self.opt),
                                                   ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = _workspace(nb.value, device)
        self._h = ctypes.c_void_p(0)
        _check(lib.fcmp_batch_plan_create(ctypes.byref(self._h), self.n, self._probs,
                                          ctypes.byref(self.opt), _ptr(self.ws), self.ws.numel(),
                                          _stream()))
        self.support = [torch.empty(int(p[3]), dtype=torch.int32, device=device) for p in problems]
        self.x = [torch.empty(int(p[3]), dtype=_dtype(p[0]), device=device) for p in problems]
        self._sp = _ptr_array([t.data_ptr() for t in self.support])
        self._xp = _ptr_array([t.data_ptr() for t in self.x])

    def solve(self, ys, stats=False):
        st = (Stats * self.n)() if stats else None
        _check(lib.fcmp_batch_plan_solve(self._h, _ptr_array([y.data_ptr() for y in ys]),
                                         self._sp, self._xp, st, _stream()))
        return self.support, self.x, (list(st) if stats else None)

    def close(self):
        if self._h:
            lib.fcmp_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_footprint(cls, N, M, K, omega, algorithm="omp", method="conventional",
                     precision="fp64", switch_t=0, flags=0) -> int:
    """Device pool bytes one request occupies when admitted alone (host-only)."""
    prob, _keep = make_problem(cls, N, M, K, omega)
    o = make_options(algorithm, method, precision, 0, switch_t, flags)
    nb = ctypes.c_size_t(0)
    _check(lib.fcmp_server_footprint(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(nb)))
    return nb.value


class Server:
    """Continuous-batching solver service over a device pool of pool_bytes.
    submit() takes host arrays and returns a ticket; poll() returns None while
    the request runs, else a dict with support, x, stats and times."""

    def __init__(self, pool_bytes, max_slots=0, max_pending=0, n_streams=0, max_wave=0,
                 max_groups=0, device="cuda"):
        self.pool = _workspace(int(pool_bytes), device)
        cfg = ServerConfig(max_slots, max_pending, n_streams, max_wave, max_groups)
        self._h = ctypes.c_void_p(0)
        _check(lib.fcmp_server_create(ctypes.byref(self._h), _ptr(self.pool), self.pool.numel(),
                                      ctypes.byref(cfg)))
        self._shapes = {}

    def submit(self, cls, N, M, K, omega, y, algorithm="omp", method="conventional",
               precision="fp64", switch_t=0, flags=0) -> int:
        prob, _keep = make_problem(cls, N, M, K, omega)
        o = make_options(algorithm, method, precision, 0, switch_t, flags)
        yh = np.ascontiguousarray(np.asarray(y, dtype=np.complex128 if cls == "F" else np.float64))
        if yh.shape != (int(M),):
            raise ValueError("y must hold M values")
        t = ctypes.c_uint64(0)
        _check(lib.fcmp_server_submit(self._h, ctypes.byref(prob), ctypes.byref(o),
                                      yh.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)))
        self._shapes[t.value] = (cls, int(K))
        return t.value

    def poll(self, ticket):
        cls, K = self._shapes[ticket]
        sup = np.empty(K, dtype=np.int32)
        x = np.empty(K, dtype=np.complex128 if cls == "F" else np.float64)
        st, tm, done = Stats(), Times(), ctypes.c_int32(0)
        rc = lib.fcmp_server_poll(self._h, ticket, sup.ctypes.data_as(ctypes.c_void_p),
                                  x.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                                  ctypes.byref(tm), ctypes.byref(done))
        if rc == 0 and not done.value:
            return None
        del self._shapes[ticket]
        _check(rc)
        return {"support": sup, "x": x, "stats": st,
                "times": (tm.t_submit, tm.t_launch, tm.t_done)}

    def drain(self, timeout_ms=0.0):
        _check(lib.fcmp_server_drain(self._h, float(timeout_ms)))

    def info(self) -> dict:
        i = ServerInfo()
        _check(lib.fcmp_server_get_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _t in ServerInfo._fields_}

    def close(self):
        if self._h:
            lib.fcmp_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(cls, N, M, precision="fp32", batch=8, cache_path=None, device="cuda") -> int:
    """Measures the adaptive switch iteration for (class, N, precision) on the
    device and records it for later adaptive solves; returns it."""
    nb = ctypes.c_size_t(0)
    _check(lib.fcmp_autotune_query_workspace(CLASS[cls], int(N), int(M), PREC[precision],
                                             int(batch), ctypes.byref(nb)))
    ws = _workspace(nb.value, device)
    t = ctypes.c_int32(0)
    _check(lib.fcmp_autotune(CLASS[cls], int(N), int(M), PREC[precision], int(batch),
                             cache_path.encode() if cache_path else None, _ptr(ws), ws.numel(),
                             ctypes.byref(t), _stream()))
    return t.value


def corr_curve(cls, N, M, ts, precision="fp32", batch=1, device="cuda", flags=0):
    """Per-iteration device time (ms per launch sequence over the batch) of
    the fast and the conventional correlation at each iteration t in ts
    (flags: the fast correlation's kernel-vector variant)."""
    ts = [int(t) for t in ts]
    nb = ctypes.c_size_t(0)
    _check(lib.fcmp_corr_curve_query_workspace(CLASS[cls], int(N), int(M), PREC[precision],
                                               int(batch), max(ts), ctypes.byref(nb)))
    ws = _workspace(nb.value, device)
    ta = (ctypes.c_int32 * len(ts))(*ts)
    fa = (ctypes.c_float * len(ts))()
    ca = (ctypes.c_float * len(ts))()
    _check(lib.fcmp_corr_curve(CLASS[cls], int(N), int(M), PREC[precision], int(batch),
                               int(flags), ta,
                               len(ts), _ptr(ws), ws.numel(), fa, ca, _stream()))
    return list(fa), list(ca)


def schedule_tune(cls, N, M, precision="fp32", batch=8, cache_path=None, device="cuda") -> dict:
    """Times launch schedules (transform tile, thread counts) for a lockstep
    plan of `batch` problems (class, N, M) and records the fastest for plans
    of that shape; returns it with the default's and its timed cost."""
    nb = ctypes.c_size_t(0)
    _check(lib.fcmp_schedule_query_workspace(CLASS[cls], int(N), int(M), PREC[precision],
                                             int(batch), ctypes.byref(nb)))
    ws = _workspace(nb.value, device)
    best, a, b = Schedule(), ctypes.c_float(0), ctypes.c_float(0)
    _check(lib.fcmp_schedule_tune(CLASS[cls], int(N), int(M), PREC[precision], int(batch),
                                  cache_path.encode() if cache_path else None, _ptr(ws),
                                  ws.numel(), ctypes.byref(best), ctypes.byref(a), ctypes.byref(b),
                                  _stream()))
    return {"tile": best.tile, "threads": best.threads, "rthreads": best.rthreads,
            "ms_default": a.value, "ms_best": b.value}


def schedule_set(cls, N, precision="fp32", batch=1, tile=0, threads=0, rthreads=0, drop=False):
    """Sets (or drops) the schedule plans of (class, N, precision, batch
    bucket) use on the current device."""
    s = Schedule(int(tile), int(threads), int(rthreads))
    _check(lib.fcmp_schedule_set(CLASS[cls], int(N), PREC[precision], int(batch),
                                 None if drop else ctypes.byref(s)))


def schedule_get(cls, N, precision="fp32", batch=1) -> dict:
    """The schedule a plan of `batch` problems of (class, N, precision) uses."""
    s, tuned = Schedule(), ctypes.c_int32(0)
    _check(lib.fcmp_schedule_get(CLASS[cls], int(N), PREC[precision], int(batch), ctypes.byref(s),
                                 ctypes.byref(tuned)))
    return {"tile": s.tile, "threads": s.threads, "rthreads": s.rthreads, "tuned": bool(tuned.value)}


def autotune_load(cache_path) -> None:
    _check(lib.fcmp_autotune_load(str(cache_path).encode()))


def adaptive_switch(cls, N, precision="fp32") -> tuple:
    """(switch iteration used by adaptive solves with switch_t = 0, tuned?)."""
    t, tuned = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib.fcmp_adaptive_switch(CLASS[cls], int(N), PREC[precision], ctypes.byref(t),
                                    ctypes.byref(tuned)))
    return t.value, bool(tuned.value)
