"""Writes the stored oracle solve of the full-size Fourier workload
(N = 65536, M = 16384, K = 256, CN(0,1) values, 30 dB, seed 2000) used by the
full-size GPU parity test: y from the oracle's own forward transform, the FP64
OMP of Algorithm 1.1, and the certification flags of the selection gaps.
Calls only the oracle and the seeded input generator.

    python tests/golden/make_fullsize.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))

import instancegen  # noqa: E402
import oracle  # noqa: E402
from oracle import certify  # noqa: E402

SEED = 2000
OUT = os.path.join(os.path.dirname(__file__), "omp_fourier_n65536_m16384_k256_seed2000.json")


def main():
    inst = instancegen.draw_instance("F", 65536, 16384, 256, "cgauss", 30.0, SEED)
    y = oracle.problem.instance_measure(inst, tier="transform")
    op = oracle.make_operator("F", 65536, inst.omega, "transform")
    ref = oracle.omp(op, y, 256)
    doc = {
        "workload": "F N=65536 M=16384 K=256 cgauss 30 dB",
        "seed": SEED,
        "support": [int(v) for v in ref.support],
        "x_re": [float(v) for v in ref.x.real],
        "x_im": [float(v) for v in ref.x.imag],
        "res_norm": float(ref.res_norm),
        "min_gap": certify.min_gap(ref),
        "certified": {p: bool(certify.certified(ref, p)) for p in ("fp32", "fp64")},
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(OUT, doc["certified"])


if __name__ == "__main__":
    main()
