"""The conjugate-symmetric pairing of the fast correlation (FCMP_FLAG_CONJ_PAIR,
partial Fourier, N <= 8192): OMP, adaptive OMP and the set pursuits with the
paired kernel against the FP64 oracle, and against the unpaired half-table
fast correlation it must agree with to rounding."""
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


# (N, M, K, law, snr, seed): a ragged tap count past one staged chunk (K > 256)
# at the largest N, the smallest sizes, and a K = 1 solve (no taps at all)
CASES = [(8192, 2048, 300, "cgauss", 30.0, 7801), (4096, 1024, 60, "cgauss", 40.0, 7802),
         (1024, 256, 24, "pm_u12", None, 7803), (64, 24, 5, "cgauss", None, 7804),
         (2048, 512, 1, "cgauss", 30.0, 7805)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"F{c[0]}-{c[2]}")
def test_paired_omp_matches_oracle_and_half_table(fc, case, precision):
    N, M, K, law, snr, seed = case
    print("pairing:", case, precision, flush=True)
    inst = instancegen.draw_instance("F", N, M, K, law, snr, seed)
    y = oracle.problem.instance_measure(inst, tier="transform")
    op = oracle.make_operator("F", N, inst.omega, "transform")
    ref = oracle.omp(op, y, K)
    yd = to_dev(y)
    pair = fc.solve("F", N, M, K, inst.omega, yd, method="fast", precision=precision,
                    flags=fc.FLAG_CONJ_PAIR)
    half = fc.solve("F", N, M, K, inst.omega, yd, method="fast", precision=precision,
                    flags=fc.FLAG_HALF_KERNEL)
    assert pair.stats.status_detail == 0 and pair.stats.iterations == K
    xs = to_np(pair.x)
    if certify.certified(ref, precision):
        assert list(to_np(pair.support)) == list(ref.support)
        assert np.linalg.norm(xs - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    # the same selections as the unpaired half-table kernel, x to rounding
    assert list(to_np(pair.support)) == list(to_np(half.support))
    xh = to_np(half.x)
    assert np.linalg.norm(xs - xh) <= 1e-12 * np.linalg.norm(xh)


def test_paired_counts_checked(fc):
    """Enough of the cases above are certified for the oracle check to bite."""
    n = 0
    for N, M, K, law, snr, seed in CASES:
        inst = instancegen.draw_instance("F", N, M, K, law, snr, seed)
        y = oracle.problem.instance_measure(inst, tier="transform")
        ref = oracle.omp(oracle.make_operator("F", N, inst.omega, "transform"), y, K)
        n += certify.certified(ref, "fp32")
    assert n >= 3


def test_paired_adaptive_and_batch(fc):
    """Adaptive OMP (fast up to the switch, then conventional) in a lockstep
    plan of three instances, paired against unpaired."""
    import torch
    N, M, K = 8192, 2000, 120
    insts = [instancegen.draw_instance("F", N, M, K, "cgauss", 30.0, 7810 + b) for b in range(3)]
    ys = torch.stack([torch.from_numpy(oracle.problem.instance_measure(i, tier="transform"))
                      for i in insts]).to("cuda")
    P = fc.Plan("F", N, M, K, [i.omega for i in insts], precision="fp32", method="adaptive")
    s1, x1, _ = P.solve(ys, method="adaptive", switch_t=40, flags=fc.FLAG_CONJ_PAIR)
    s1, x1 = s1.cpu().numpy().copy(), x1.cpu().numpy().copy()
    s2, x2, _ = P.solve(ys, method="adaptive", switch_t=40, flags=fc.FLAG_HALF_KERNEL)
    s2, x2 = s2.cpu().numpy(), x2.cpu().numpy()
    assert np.array_equal(s1, s2)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)


@pytest.mark.parametrize("alg", ["sp", "cosamp"])
def test_paired_set_pursuits(fc, alg):
    N, M, K = 4096, 1024, 40
    inst = instancegen.draw_instance("F", N, M, K, "cgauss", 40.0, 7820)
    y = oracle.problem.instance_measure(inst, tier="transform")
    ref = getattr(oracle, alg)(oracle.make_operator("F", N, inst.omega, "transform"), y, K)
    res = fc.solve("F", N, M, K, inst.omega, to_dev(y), algorithm=alg, method="fast",
                   precision="fp32", flags=fc.FLAG_CONJ_PAIR)
    assert list(to_np(res.support)) == list(ref.support)
    assert np.linalg.norm(to_np(res.x) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
