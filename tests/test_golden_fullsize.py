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


HADAMARD = os.path.join(os.path.dirname(__file__), "golden",
                        "hadamard_n1m_m131072_k1024_seed3000.json")


def test_stored_hadamard_1m_solves_match_planted_signal():
    """The stored oracle solves of partial Hadamard N = 2^20, M = 2^17,
    K = 1024 (noiseless, +-U(1,2) values): OMP, SP and CoSaMP each return the
    planted support with the planted values (noiseless exact recovery), and
    the OMP gaps are certified at FP64."""
    ref = json.load(open(HADAMARD))
    inst = instancegen.draw_config("hadamard_n1m", ref["index"])
    assert inst.seed == ref["seed"] and inst.N == 1 << 20 and inst.K == 1024
    want_set = sorted(inst.support.tolist())
    for alg in ("omp", "sp", "cosamp"):
        e = ref[alg]
        sup = np.array(e["support"])
        assert sorted(sup.tolist()) == want_set
        x = np.array(e["x"]["re"])
        assert np.max(np.abs(x - inst.x_dense()[sup])) <= 1e-10
    assert ref["sp"]["support"] == want_set and ref["cosamp"]["support"] == want_set
    g = np.array(ref["omp"]["gaps"])
    assert len(g) == 1024 and np.all(g > 0)
    assert ref["omp"]["certified"]["fp64"] and not ref["omp"]["certified"]["fp32"]
    assert abs(ref["omp"]["min_gap"] - g.min()) == 0.0
