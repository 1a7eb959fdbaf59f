"""Amortization model of dynamic tuning: the oracle and the library's
functions against the paper's worked examples (tests/golden/amortization.json)
and against each other."""
import json
import math
import os

import pytest

from oracle import tuning

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "amortization.json")))


@pytest.mark.parametrize("case", GOLD["invocations"])
def test_oracle_invocations_worked_example(case):
    n = tuning.invocations(case["rp"], case["s"], case["t_avg"], case["t_well"])
    assert n == pytest.approx(case["n"], rel=1e-12)
    # the reading of Eq. 3 used here gives back rp at that n
    assert tuning.relative_performance(n, case["s"], case["t_avg"], case["t_well"]) == pytest.approx(case["rp"])


@pytest.mark.parametrize("case", GOLD["steps"])
def test_oracle_steps_worked_example(case):
    s = tuning.steps(case["r"], case["p"])
    assert math.ceil(s) == case["s"]
    assert 229.0 < s < 229.2


def test_oracle_model_properties():
    # no tuning cost when every kernel is as fast as the good one
    assert tuning.invocations(0.9, 50, 5.0, 5.0) == 0.0
    # a near-certain search needs more steps than a likely one
    assert tuning.steps(0.05, 0.99) > tuning.steps(0.05, 0.9) > tuning.steps(0.05, 0.5)
    # rp rises toward 1 with more invocations
    rps = [tuning.relative_performance(n, 50, 10.0, 4.0) for n in (100, 1000, 10000)]
    assert rps[0] < rps[1] < rps[2] < 1.0
    with pytest.raises(ValueError):
        tuning.invocations(1.0, 1, 1, 1)


@pytest.fixture(scope="module")
def recon():
    from paper_1910_08498_amd import recon as r
    r.load_library()
    return r


def test_library_model_matches_oracle_and_paper(recon):
    for case in GOLD["invocations"]:
        n = recon.recon_tune_invocations(case["rp"], case["s"], case["t_avg"], case["t_well"])
        assert n == pytest.approx(case["n"], rel=1e-12)
    for case in GOLD["steps"]:
        assert math.ceil(recon.recon_tune_steps(case["r"], case["p"])) == case["s"]
    for args in [(0.95, 37, 9.0, 2.0), (0.5, 3, 1.5, 1.0)]:
        assert recon.recon_tune_invocations(*args) == pytest.approx(tuning.invocations(*args), rel=1e-14)
    for args in [(0.2, 0.9), (0.001, 0.5)]:
        assert recon.recon_tune_steps(*args) == pytest.approx(tuning.steps(*args), rel=1e-14)
    with pytest.raises(recon.ReconError):
        recon.recon_tune_invocations(1.0, 1, 1, 1)
    with pytest.raises(recon.ReconError):
        recon.recon_tune_steps(0.0, 0.5)
