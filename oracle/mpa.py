"""Matching pursuit algorithms in FP64 (plain, slow, step by step).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

OMP follows Algorithm 1.1 (Sec. I): correlation h_{t-1} = Phi^H r_{t-1}
(step 2), identification by the largest |h| (step 3), augmenting the support
(step 4), least squares on the selected columns (steps 5-6) and the residual
update (step 7).  With ``method="fast"`` step 2 is replaced by eq.
(kernelsumOMP): h_0 at t = 1, else h_0 - sum_tau x_{t-1}(tau) P_{lambda_tau} c
(Sec. III-A), which the paper states gives the identical algorithm.

Readings where the paper is silent (each listed in the design notes):
* identification compares |h|^2 over the columns not yet selected; ties go
  to the lowest index; if that maximum is exactly 0 the loop stops early;
* halting: OMP runs exactly K iterations, or (optional residual rule,
  Algorithm 1.1 step 8 leaves the criterion open) stops after the first
  iteration whose residual satisfies ||r|| <= res_tol ||y||;
* least squares uses LAPACK lstsq on the explicit selected columns.

SP and CoSaMP are only cited by the paper (Sec. I, Sec. IV); the loops below
are this project's reading of them, so their halting and pruning details are
"parity unpinned" by the paper.  Their correlation step is the same call
(conventional, or fast with the current K-support as taps).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .unitary import Operator, make_operator
from .fastcorr import kernel_vector, fast_correlation

__all__ = ["argmax_excluding", "topk", "lstsq", "omp", "sp", "cosamp",
           "OmpResult", "SetResult"]


def _mag2(h: np.ndarray) -> np.ndarray:
    h = np.asarray(h)
    if np.iscomplexobj(h):
        return h.real * h.real + h.imag * h.imag
    return h * h


def argmax_excluding(h, excluded) -> tuple:
    """(index, |h|^2 at it, runner-up |h|^2) over j not in ``excluded``;
    lowest index on ties (numpy's argmax returns the first maximum)."""
    a = _mag2(h).copy()
    ex = np.asarray(list(excluded), dtype=np.int64)
    if ex.size:
        a[ex] = -np.inf
    j = int(np.argmax(a))
    top = a[j]
    a2 = a.copy()
    a2[j] = -np.inf
    second = float(np.max(a2)) if a2.size > 1 else -np.inf
    return j, float(top), second


def topk(a, k: int, excluded=()) -> np.ndarray:
    """Indices of the k largest entries of a (real, >= 0), largest first,
    ties to the lowest index; ``excluded`` indices never chosen."""
    a = np.asarray(a, dtype=np.float64).copy()
    ex = np.asarray(list(excluded), dtype=np.int64)
    if ex.size:
        a[ex] = -np.inf
    order = np.argsort(-a, kind="stable")
    return order[:k].astype(np.int64)


def lstsq(A: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.linalg.lstsq(A, y, rcond=None)[0]


@dataclass
class OmpResult:
    support: np.ndarray                   # selection order
    x: np.ndarray                         # aligned with support
    iterations: int
    res_norm: float
    top: List[float] = field(default_factory=list)      # |h|^2 of the pick
    second: List[float] = field(default_factory=list)   # runner-up |h|^2
    hmax: List[float] = field(default_factory=list)     # max |h|^2 over all j
    h: Optional[list] = None                            # h per iteration
    xs: Optional[list] = None                           # x per iteration

    def gaps(self) -> np.ndarray:
        """Relative identification gap per iteration on the |h| scale:
        (|h|_(1) - |h|_(2)) / ||h||_inf."""
        t = np.sqrt(np.maximum(self.top, 0.0))
        s = np.sqrt(np.maximum(self.second, 0.0))
        m = np.sqrt(np.maximum(self.hmax, 0.0))
        return (t - s) / m


def omp(op: Operator, y, K: int, method: str = "conventional",
        keep_h: bool = False, c=None, res_tol: float = 0.0) -> OmpResult:
    """Algorithm 1.1 for exactly K iterations (early stop if max |h| = 0, or,
    with res_tol > 0, once ||r|| <= res_tol ||y||)."""
    y = np.asarray(y)
    N = op.N
    r = y.copy()                                       # step 1
    lam: List[int] = []
    x = np.zeros(0, dtype=op.dtype)
    res = OmpResult(np.zeros(0, np.int64), x, 0, float(np.linalg.norm(y)))
    hs, xs = [], []
    h0 = None
    if method == "fast":
        if c is None:
            c = kernel_vector(op.cls, N, op.omega, "dense" if hasattr(op, "Phi") else "transform")
        h0 = op.adjoint(y)                             # h_0 = Phi^H r_0
    Phi_all = None                                     # columns of Phi at Lambda
    for t in range(1, K + 1):
        if method == "fast":                           # eq. (kernelsumOMP)
            h = h0 if t == 1 else fast_correlation(op.cls, N, h0, c, lam, x)
        else:
            h = op.adjoint(r)                          # step 2
        j, top, second = argmax_excluding(h, lam)      # step 3
        if top <= 0.0:
            break
        res.top.append(top)
        res.second.append(second)
        res.hmax.append(float(np.max(_mag2(h))))
        if keep_h:
            hs.append(np.array(h))
        lam.append(j)                                  # step 4
        # step 5: Phi_t = Phi S_{Lambda_t}^T, the previous columns with the
        # new one appended (Lambda_t in selection order)
        if Phi_all is None:
            Phi_all = np.empty((op.M, K), dtype=op.dtype)
        Phi_all[:, t - 1] = op.columns([j])[:, 0]
        Phi_t = Phi_all[:, :t]
        x = lstsq(Phi_t, y)                            # step 6
        r = y - Phi_t @ x                              # step 7
        if keep_h:
            xs.append(x.copy())
        if res_tol > 0.0 and np.linalg.norm(r) <= res_tol * np.linalg.norm(y):
            break                                      # step 8 (residual rule)
    res.support = np.asarray(lam, dtype=np.int64)
    res.x = x
    res.iterations = len(lam)
    res.res_norm = float(np.linalg.norm(r))
    if keep_h:
        res.h = hs
        res.xs = xs
    return res


@dataclass
class SetResult:
    support: np.ndarray        # ascending
    x: np.ndarray              # aligned with support
    iterations: int
    res_norm: float
    supports: list = field(default_factory=list)   # pruned K-support per iteration


def _correlate(op: Operator, method: str, r, h0, c, taps_idx, taps_val):
    if method == "fast":
        return fast_correlation(op.cls, op.N, h0, c, taps_idx, taps_val)
    return op.adjoint(r)


def _sorted_pair(idx, val):
    order = np.argsort(idx)
    return np.asarray(idx)[order], np.asarray(val)[order]


def sp(op: Operator, y, K: int, method: str = "conventional",
       max_iter: int = 50, c=None, res_tol: float = 0.0) -> SetResult:
    """Subspace pursuit (reading): start from the K largest |h_0|; each
    iteration merges the K largest |Phi^H r| outside T, fits on the 2K merged
    columns, keeps the K largest |x|, refits, and stops when the support
    repeats or the residual stops shrinking (keeping the previous one), or,
    with res_tol > 0, before an iteration once ||r|| <= res_tol ||y||."""
    y = np.asarray(y)
    h0 = op.adjoint(y)
    if method == "fast" and c is None:
        c = kernel_vector(op.cls, op.N, op.omega, "dense" if hasattr(op, "Phi") else "transform")
    T = np.sort(topk(_mag2(h0), K))
    x = lstsq(op.columns(T), y)
    r = y - op.columns(T) @ x
    rn = np.linalg.norm(r)
    out = SetResult(T, x, 0, float(rn), [T.copy()])
    it = 0
    ny = np.linalg.norm(y)
    while it < max_iter and not (res_tol > 0.0 and rn <= res_tol * ny):
        it += 1
        h = _correlate(op, method, r, h0, c, T, x)
        extra = topk(_mag2(h), K, excluded=T)
        Tt = np.sort(np.concatenate([T, extra]))
        xt = lstsq(op.columns(Tt), y)
        keep = topk(_mag2(xt), K)
        Tn = np.sort(Tt[keep])
        xn = lstsq(op.columns(Tn), y)
        rnew = y - op.columns(Tn) @ xn
        rnn = np.linalg.norm(rnew)
        if np.array_equal(Tn, T):
            T, x, r, rn = Tn, xn, rnew, rnn
            out.supports.append(T.copy())
            break
        if rnn >= rn:
            break
        T, x, r, rn = Tn, xn, rnew, rnn
        out.supports.append(T.copy())
    out.support, out.x = T, x
    out.iterations = it
    out.res_norm = float(rn)
    return out


def cosamp(op: Operator, y, K: int, method: str = "conventional",
           max_iter: int = 50, c=None, res_tol: float = 0.0) -> SetResult:
    """CoSaMP (reading): proxy Phi^H v, merge its 2K largest with the current
    support, fit on the merged columns, prune to the K largest (no refit in
    the loop), update v = y - Phi a; stop when the support repeats, when
    ||v|| <= 1e-12 ||y|| (or <= res_tol ||y|| with res_tol > 0), or after
    max_iter; finally refit on the support."""
    y = np.asarray(y)
    ny = np.linalg.norm(y)
    h0 = op.adjoint(y)
    if method == "fast" and c is None:
        c = kernel_vector(op.cls, op.N, op.omega, "dense" if hasattr(op, "Phi") else "transform")
    S = np.zeros(0, dtype=np.int64)          # supp(a), ascending
    a = np.zeros(0, dtype=op.dtype)          # values on S
    v = y.copy()
    out = SetResult(S, a, 0, float(ny), [])
    it = 0
    while it < max_iter:
        it += 1
        u = h0 if S.size == 0 else _correlate(op, method, v, h0, c, S, a)
        big = topk(_mag2(u), 2 * K)
        T = np.union1d(big, S)
        b = lstsq(op.columns(T), y)
        keep = topk(_mag2(b), K)
        Sn, an = _sorted_pair(T[keep], b[keep])
        v = y - op.columns(Sn) @ an
        changed = not np.array_equal(Sn, S)
        S, a = Sn, an
        out.supports.append(S.copy())
        vn = np.linalg.norm(v)
        if not changed or vn <= 1e-12 * ny or (res_tol > 0.0 and vn <= res_tol * ny):
            break
    x = lstsq(op.columns(S), y)
    out.support, out.x = S, x
    out.iterations = it
    out.res_norm = float(np.linalg.norm(y - op.columns(S) @ x))
    return out


def omp_from_instance(inst, y, method="conventional", tier="auto", **kw):
    op = make_operator(inst.cls, inst.N, inst.omega, tier)
    return omp(op, y, inst.K, method, **kw)
