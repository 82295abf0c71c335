"""fcmp_solve_noalloc (workspace in the library's static device scratch)
against fcmp_solve (caller workspace) through the C ABI: two calls in a row,
the second on a smaller problem, each bit-identical to fcmp_solve on the
same input; plus the host-side refusal of a problem larger than the
scratch."""
import numpy as np
import pytest

import instancegen
import oracle
from tests.gpu_util import lib, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib()


CALLS = [
    # two calls in a row, the second smaller; both take two-pass transforms
    # with the fused residual (N = 2^16) or the one-workgroup path (N = 2^12)
    [("F", 65536, 16384, 64, "cgauss", 30.0, "fp32", "conventional"),
     ("F", 4096, 1024, 20, "cgauss", 30.0, "fp32", "conventional")],
    [("H", 1 << 18, 1 << 15, 128, "pm_u12", None, "fp32", "adaptive"),
     ("H", 1024, 256, 16, "gauss", None, "fp64", "fast")],
]


@pytest.mark.parametrize("seq", CALLS, ids=["F65536-then-F4096", "H262144-then-H1024"])
def test_noalloc_matches_solve(fc, seq):
    for k, (cls, N, M, K, law, snr, prec, method) in enumerate(seq):
        inst = instancegen.draw_instance(cls, N, M, K, law, snr, 7700 + k)
        y = to_dev(oracle.problem.instance_measure(inst, tier="transform"))
        want = fc.solve(cls, N, M, K, inst.omega, y, method=method, precision=prec)
        got = fc.solve_noalloc(cls, N, M, K, inst.omega, y, method=method, precision=prec)
        assert got.stats.status_detail == 0 and got.stats.iterations == K
        assert np.array_equal(to_np(got.support), to_np(want.support)), (k, cls, N)
        assert np.array_equal(to_np(got.x), to_np(want.x)), (k, cls, N)
        assert got.stats.iterations == want.stats.iterations
        assert got.stats.res_norm == want.stats.res_norm


def test_noalloc_refuses_problem_above_scratch(fc):
    """SP at N = 2^20, K = 1024 needs 76 MiB of workspace: refused on the
    host with FCMP_E_WORKSPACE before any device work."""
    import torch
    N, M, K = 1 << 20, 1 << 17, 1024
    om = np.arange(M) * (N // M)
    y = torch.zeros(M, dtype=torch.float64, device="cuda")
    with pytest.raises(fc.FcmpError) as ei:
        fc.solve_noalloc("H", N, M, K, om, y, algorithm="sp", precision="fp32")
    assert ei.value.code == fc.E_WORKSPACE
