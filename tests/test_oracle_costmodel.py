"""Pins for oracle.costmodel against the numbers the paper prints."""
import json
import os

import pytest

from oracle import costmodel as cm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_table1_samples():
    for s in GOLD["table1"]["samples"]:
        assert cm.conventional_flops(s["cls"], s["N"], s["t"]) == s["conventional"]
        assert cm.proposed_flops(s["cls"], s["N"], s["t"]) == s["proposed"]


def test_fourier_excessive_point():
    g = GOLD["fourier_excessive_point"]
    t = cm.excessive_point("F", g["N"])
    assert t == g["excessive_t"]
    assert cm.proposed_flops("F", g["N"], g["first_conventional_t"]) > \
        cm.conventional_flops("F", g["N"], g["first_conventional_t"])


def test_cosamp_ratio():
    g = GOLD["cosamp_ratio"]
    assert round(100 * cm.cosamp_relative("F", g["N"], g["K"])) == g["percent"]


def test_first_iteration_equal():
    for cls in ("F", "H"):
        for N in (1024, 65536):
            assert cm.relative(cls, N, 1) == 1.0


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        cm.conventional_flops("F", 1000, 1)
