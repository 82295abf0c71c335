"""Writes the stored oracle solves used by the full-size GPU parity tests.
Calls only the oracle and the seeded input generator; y comes from the
oracle's own forward transform.

* ``fourier``  partial Fourier N = 65536, M = 16384, K = 256, CN(0,1) values,
  30 dB, seed 2000: the FP64 OMP of Algorithm 1.1 (selection order, x,
  certification flags of the selection gaps).
* ``hadamard`` partial Hadamard N = 2^20, M = 2^17, K = 1024, +-U(1,2)
  values, noiseless, seed 3000: OMP (selection order, x, per-iteration
  gaps), SP and CoSaMP (final supports, x, iteration counts).  The OMP solve
  takes tens of minutes on a few cores (1024 least-squares fits on up to
  131072 x 1024 explicit columns).
* ``uneven``   the 4096-instance uneven batch (seed 4000): the first three
  Fourier and the first three Hadamard instances with N = 2^14 whose OMP
  gaps are certified at FP32 (how many were tried is recorded too).

    python tests/golden/make_fullsize.py [fourier|hadamard|uneven ...]
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))

import instancegen  # noqa: E402
import oracle  # noqa: E402
from oracle import certify  # noqa: E402

HERE = os.path.dirname(__file__)
FOURIER = os.path.join(HERE, "omp_fourier_n65536_m16384_k256_seed2000.json")
HADAMARD = os.path.join(HERE, "hadamard_n1m_m131072_k1024_seed3000.json")
UNEVEN = os.path.join(HERE, "uneven_batch4096_seed4000_n16384.json")


def _cplx(v):
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return {"re": [float(a) for a in v.real], "im": [float(a) for a in v.imag]}
    return {"re": [float(a) for a in v]}


def _dump(path, doc):
    with open(path, "w") as f:
        json.dump(doc, f, indent=0)
    print(path, flush=True)


def fourier():
    seed = 2000
    inst = instancegen.draw_instance("F", 65536, 16384, 256, "cgauss", 30.0, seed)
    y = oracle.problem.instance_measure(inst, tier="transform")
    op = oracle.make_operator("F", 65536, inst.omega, "transform")
    ref = oracle.omp(op, y, 256)
    doc = {
        "workload": "F N=65536 M=16384 K=256 cgauss 30 dB",
        "seed": seed,
        "support": [int(v) for v in ref.support],
        "x_re": [float(v) for v in ref.x.real],
        "x_im": [float(v) for v in ref.x.imag],
        "res_norm": float(ref.res_norm),
        "min_gap": certify.min_gap(ref),
        "certified": {p: bool(certify.certified(ref, p)) for p in ("fp32", "fp64")},
    }
    _dump(FOURIER, doc)


def hadamard():
    inst = instancegen.draw_config("hadamard_n1m", 0)
    y = oracle.problem.instance_measure(inst, tier="transform")
    op = oracle.make_operator("H", inst.N, inst.omega, "transform")
    doc = {"workload": "H N=1048576 M=131072 K=1024 pm_u12 noiseless",
           "config": "hadamard_n1m", "index": 0, "seed": inst.seed}
    t0 = time.time()
    ref = oracle.omp(op, y, inst.K)
    doc["omp"] = {
        "support": [int(v) for v in ref.support],
        "x": _cplx(ref.x),
        "res_norm": float(ref.res_norm),
        "gaps": [float(g) for g in ref.gaps()],
        "min_gap": certify.min_gap(ref),
        "certified": {p: bool(certify.certified(ref, p)) for p in ("fp32", "fp64")},
        "seconds": round(time.time() - t0, 1),
    }
    print("omp", doc["omp"]["min_gap"], doc["omp"]["certified"], doc["omp"]["seconds"], flush=True)
    for alg in ("sp", "cosamp"):
        t0 = time.time()
        r = getattr(oracle, alg)(op, y, inst.K)
        doc[alg] = {
            "support": [int(v) for v in r.support],
            "x": _cplx(r.x),
            "iterations": int(r.iterations),
            "res_norm": float(r.res_norm),
            "seconds": round(time.time() - t0, 1),
        }
        print(alg, r.iterations, doc[alg]["seconds"], flush=True)
    _dump(HADAMARD, doc)


def uneven():
    insts = instancegen.draw_batch(4096, 4000)
    picked = {"F": [], "H": []}
    tried = {"F": 0, "H": 0}
    for i, inst in enumerate(insts):
        if inst.N != 1 << 14 or len(picked[inst.cls]) >= 3:
            continue
        tried[inst.cls] += 1
        y = oracle.problem.instance_measure(inst, tier="transform")
        op = oracle.make_operator(inst.cls, inst.N, inst.omega, "transform")
        ref = oracle.omp(op, y, inst.K)
        if not certify.certified(ref, "fp32"):
            continue
        picked[inst.cls].append({
            "index": i, "cls": inst.cls, "N": inst.N, "M": inst.M, "K": inst.K,
            "support": [int(v) for v in ref.support],
            "x": _cplx(ref.x),
            "min_gap": certify.min_gap(ref),
        })
        print(inst.cls, i, inst.K, certify.min_gap(ref), flush=True)
        if all(len(v) >= 3 for v in picked.values()):
            break
    doc = {"workload": "uneven batch of 4096, seed 4000, N = 2^14 instances certified at FP32",
           "tried": tried, "instances": picked["F"] + picked["H"]}
    _dump(UNEVEN, doc)


if __name__ == "__main__":
    which = sys.argv[1:] or ["fourier", "hadamard", "uneven"]
    for w in which:
        {"fourier": fourier, "hadamard": hadamard, "uneven": uneven}[w]()
