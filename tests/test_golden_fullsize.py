"""The stored oracle solve of the full-size Fourier workload, pinned to the
planted signal it was drawn from (not to the oracle itself): at 30 dB with
M / K = 64 the support is recovered in full, and x is the planted values up
to the noise."""
import json
import os

import numpy as np

import instancegen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "omp_fourier_n65536_m16384_k256_seed2000.json")


def test_stored_fullsize_solve_matches_planted_signal():
    ref = json.load(open(GOLDEN))
    inst = instancegen.draw_instance("F", 65536, 16384, 256, "cgauss", 30.0, ref["seed"])
    sup = np.array(ref["support"])
    assert len(sup) == 256 and len(set(sup.tolist())) == 256
    assert set(sup.tolist()) == set(inst.support.tolist())
    x = np.array(ref["x_re"]) + 1j * np.array(ref["x_im"])
    want = inst.x_dense()[sup]
    # noise energy is 1e-3 of the signal's; the LS error is a fraction K/M of it
    assert np.linalg.norm(x - want) <= 0.01 * np.linalg.norm(want)
    assert ref["certified"]["fp32"] and ref["certified"]["fp64"]
    assert ref["min_gap"] >= 2.5e-5


UNEVEN = os.path.join(os.path.dirname(__file__), "golden",
                      "uneven_batch4096_seed4000_n16384.json")


def test_stored_uneven_batch_solves_match_planted_signals():
    """The six stored N = 2^14 solves of the uneven batch (40 dB): each holds
    K distinct columns, at least 97% of them planted ones, and x on them is
    the planted values to within 1% (N(0,1) values: the smallest planted
    coefficients sit near the noise and may be swapped for another column)."""
    ref = json.load(open(UNEVEN))
    insts = instancegen.draw_batch(4096, 4000)
    assert len(ref["instances"]) == 6
    assert sorted(e["cls"] for e in ref["instances"]) == ["F"] * 3 + ["H"] * 3
    for e in ref["instances"]:
        inst = insts[e["index"]]
        assert (e["cls"], e["N"], e["M"], e["K"]) == (inst.cls, inst.N, inst.M, inst.K) and inst.N == 16384
        sup = np.array(e["support"])
        assert len(sup) == inst.K and len(set(sup.tolist())) == inst.K
        assert len(set(sup.tolist()) & set(inst.support.tolist())) >= 0.97 * inst.K
        x = np.array(e["x"]["re"]) + (1j * np.array(e["x"]["im"]) if "im" in e["x"] else 0.0)
        want = inst.x_dense()[sup]
        assert np.linalg.norm(x - want) <= 0.01 * np.linalg.norm(want)
        assert e["min_gap"] >= 2.5e-5
