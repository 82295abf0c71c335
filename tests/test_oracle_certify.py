"""Pins for the selection-gap bookkeeping (oracle.certify, OmpResult.gaps).

The certification argument: if every entry of a computed correlation is
within tol * ||h||_inf of the exact one, the identification of Algorithm 1.1
step 3 cannot change while the winner leads the runner-up by more than
2 tol * ||h||_inf on the |h| scale.  The pins below fix what that gap is --
measured on |h| (not |h|^2), normalised by the largest |h| over ALL columns
(selected ones included, since the tolerance is stated on the whole vector),
with the runner-up taken over the columns not yet selected -- and where the
acceptance threshold 2.5 tol sits, using values known in closed form.
"""
import numpy as np
import pytest

import oracle
from oracle import certify
from oracle.mpa import OmpResult


def _result(top_abs, second_abs, hmax_abs):
    """An OmpResult whose per-iteration bookkeeping holds the given |h|
    values (stored, like the oracle stores them, as squares)."""
    r = OmpResult(np.zeros(0, np.int64), np.zeros(0), len(top_abs), 0.0)
    r.top = [a * a for a in top_abs]
    r.second = [a * a for a in second_abs]
    r.hmax = [a * a for a in hmax_abs]
    return r


def test_gap_closed_form_on_magnitude_scale():
    # |h|: winner 4, runner-up 3, largest entry 5 (at a selected column).
    # On |h|: (4 - 3) / 5 = 0.2.  On |h|^2 it would be 7/25 = 0.28, and
    # normalised by the winner (4 - 3) / 4 = 0.25: both slips fail here.
    g = _result([4.0], [3.0], [5.0]).gaps()
    assert g.shape == (1,)
    assert g[0] == pytest.approx(0.2, rel=1e-15)


def test_gap_uses_largest_entry_even_when_already_selected():
    # Iteration 2: the largest |h| (1.0) sits at an already-selected column,
    # the remaining winner has 0.9 and the runner-up 0.8: gap 0.1, not 0.1/0.9.
    r = _result([2.0, 0.9], [1.0, 0.8], [2.0, 1.0])
    g = r.gaps()
    assert g[0] == pytest.approx(0.5, rel=1e-15)
    assert g[1] == pytest.approx(0.1, rel=1e-14)
    assert certify.min_gap(r) == pytest.approx(0.1, rel=1e-14)


def test_exact_tie_gives_zero_and_is_never_certified():
    r = _result([3.0, 2.0], [2.0, 2.0], [3.0, 2.0])
    assert certify.min_gap(r) == 0.0
    assert not certify.certified(r, "fp64")
    assert not certify.certified(r, "fp32")


def test_no_iterations_is_vacuously_certified():
    r = _result([], [], [])
    assert certify.min_gap(r) == float("inf")
    assert certify.certified(r, "fp32")


@pytest.mark.parametrize("precision, tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_threshold_is_two_and_a_half_tolerances(precision, tol):
    # With winner 1 and largest entry 1 the gap is 1 - runner-up exactly
    # (up to one rounding of the runner-up's square and square root).
    assert certify.TOL[precision] == tol
    assert certify.DELTA[precision] == pytest.approx(2.5 * tol, rel=1e-15)
    above = _result([1.0], [1.0 - 2.6 * tol], [1.0])
    below = _result([1.0], [1.0 - 2.4 * tol], [1.0])
    assert certify.certified(above, precision)
    assert not certify.certified(below, precision)
    # the smallest gap over the iterations decides
    mixed = _result([1.0, 1.0, 1.0], [0.5, 1.0 - 2.4 * tol, 0.25], [1.0, 1.0, 1.0])
    assert not certify.certified(mixed, precision)
    assert certify.min_gap(mixed) == pytest.approx(2.4 * tol, rel=1e-3)


@pytest.mark.parametrize("cls", ["F", "H"])
def test_omp_records_gaps_of_the_full_rows_trajectory(cls):
    """M = N (Phi unitary, c = e_0): h_0 = x, and after t exact least-squares
    steps h is x with the selected entries removed, so iteration t picks the
    t-th largest |x| with the (t+1)-th as runner-up (0 after the last nonzero)
    and the largest remaining |h| equal to the winner.  With |x| = 8, 4, 2, 1
    the gaps are 1/2, 1/2, 1/2 and 1 in closed form."""
    N = 32
    supp = np.array([5, 17, 2, 30])
    mags = np.array([8.0, 4.0, 2.0, 1.0])
    rng = np.random.default_rng(3)
    x = np.zeros(N, dtype=complex if cls == "F" else float)
    x[supp] = mags * (np.exp(1j * rng.uniform(0, 6, 4)) if cls == "F" else np.array([1, -1, -1, 1]))
    y = oracle.measure(cls, N, np.arange(N), x)
    r = oracle.omp(oracle.make_operator(cls, N, np.arange(N)), y, 4)
    assert list(r.support) == list(supp)
    np.testing.assert_allclose(r.gaps(), [0.5, 0.5, 0.5, 1.0], atol=1e-13)
    np.testing.assert_allclose(np.sqrt(r.top), mags, rtol=1e-13)
    np.testing.assert_allclose(np.sqrt(r.second), [4.0, 2.0, 1.0, 0.0], atol=1e-13)
    assert certify.min_gap(r) == pytest.approx(0.5, abs=1e-13)
    assert certify.certified(r, "fp64") and certify.certified(r, "fp32")


def test_omp_tie_in_trajectory_is_not_certified():
    """M = N with two equal magnitudes: the iteration that meets the tie has
    gap 0 (lowest index wins), so the instance is not certified."""
    N = 16
    x = np.zeros(N)
    x[[3, 9, 12]] = [5.0, -3.0, 3.0]
    y = oracle.measure("H", N, np.arange(N), x)
    r = oracle.omp(oracle.make_operator("H", N, np.arange(N)), y, 3)
    assert list(r.support) == [3, 9, 12]
    g = r.gaps()
    assert g[0] == pytest.approx(0.4, abs=1e-14)
    assert g[1] == pytest.approx(0.0, abs=1e-14)
    assert not certify.certified(r, "fp32")
