"""The per-iteration time model (host logic): the work of each task per
iteration against closed forms, Tab. 2's printed ratios to first order, and
the weighted-neighbour predictor on synthetic timings."""
import math

import pytest

from paper_2301_03166_amd import timemodel as tm


@pytest.mark.parametrize("kind,total", [("chol", 1.0 / 3.0), ("lu", 2.0 / 3.0), ("qr", 4.0 / 3.0)])
def test_work_sums_to_the_decomposition_flops(kind, total):
    """PD + PU + TMU over all iterations = the textbook operation count
    (n^3/3, 2n^3/3, 4n^3/3) up to terms of relative order b / n."""
    n, b = 8192, 64
    s = sum(tm.work(kind, op, n, b, k) for op in ("pd", "pu", "tmu") for k in range(tm.iterations(n, b)))
    assert abs(s / n ** 3 - total) <= 2.0 * b / n


def test_work_closed_forms_small():
    n, b = 10, 4  # iterations: panels of 4, 4, 2
    assert tm.shape(n, b, 2) == (2, 2, 0)
    assert tm.work("lu", "tmu", n, b, 0) == 2 * 6 * 6 * 4
    assert tm.work("lu", "pu", n, b, 1) == 4 * 4 * 2
    assert tm.work("lu", "pd", n, b, 2) == 2 * 2 * 2 - 8 / 3
    assert tm.work("chol", "tmu", n, b, 1) == 2 * 2 * 4
    assert tm.work("qr", "tmu", n, b, 0) == 4 * 10 * 6 * 4 + 2 * 16 * 6
    assert tm.work("lu", "tmu", n, b, 2) == 0.0 and tm.work("lu", "verify", n, b, 2) == 0.0


@pytest.mark.parametrize("kind,op", [("lu", "tmu"), ("lu", "pu"), ("qr", "tmu")])
def test_consecutive_ratios_match_table2_to_first_order(kind, op):
    """r_{k,k+1} from the flop counts against Tab. 2's printed ratio: the
    difference is of second order in b / (n - k b)."""
    n, b = 32768, 512
    for k in range(0, tm.iterations(n, b) - 3):
        x = b / (n - k * b - b)
        ours = tm.ratio(kind, op, n, b, k, k + 1)
        paper = tm.table2_ratio(kind, op, n, b, k)
        assert abs(ours - paper) <= 4.0 * x * x, (k, ours, paper)
    # and the first-order term itself is not trivially small
    assert 1.0 - tm.ratio(kind, op, n, b, 0, 1) > 0.9 * b / n


def test_garbled_entries_are_not_used():
    assert tm.table2_ratio("chol", "tmu", 1000, 100, 1) is None
    assert tm.table2_ratio("lu", "pd", 1000, 100, 1) is None
    assert tm.table2_ratio("qr", "pd", 1000, 100, 1) is None


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
@pytest.mark.parametrize("op", ["pd", "tmu", "verify"])
def test_constant_efficiency_is_predicted_exactly(kind, op):
    """Times proportional to the work (one efficiency throughout): both
    predictors reproduce every iteration exactly."""
    n, b = 4096, 256
    N = tm.iterations(n, b)
    ts = [3e-9 * tm.work(kind, op, n, b, k) for k in range(N)]
    for k in range(1, N):
        if ts[k] == 0:
            continue
        for pred in (tm.predict_neighbours, tm.predict_first):
            assert math.isclose(pred(ts, kind, op, n, b, k), ts[k], rel_tol=1e-12)


def test_neighbour_weights_and_short_history():
    n, b = 2048, 256
    ts = [1.0] * tm.iterations(n, b)
    assert sum(tm.WEIGHTS) == 1.0 and len(tm.WEIGHTS) == 4
    assert tm.predict_neighbours(ts, "lu", "tmu", n, b, 0) is None
    # k = 1: only iteration 0, weight rescaled to 1
    assert math.isclose(tm.predict_neighbours(ts, "lu", "tmu", n, b, 1), tm.ratio("lu", "tmu", n, b, 0, 1))
    # k = 5: the weighted sum of the four neighbours' scaled times
    k = 5
    want = sum(w * tm.ratio("lu", "tmu", n, b, k - i, k) for i, w in enumerate(tm.WEIGHTS, start=1))
    assert math.isclose(tm.predict_neighbours(ts, "lu", "tmu", n, b, k), want)


def test_neighbours_track_a_drifting_efficiency():
    """The reason for the enhanced predictor: when the efficiency changes
    over the factorization (smaller trailing matrices run below peak), the
    neighbours follow it and the first iteration does not."""
    n, b = 32768, 512
    N = tm.iterations(n, b)
    ts = []
    for k in range(N):
        w = tm.work("lu", "tmu", n, b, k)
        t = n - (k + 1) * b
        eff = 1.0 / (1.0 + 2000.0 / max(t, 1))  # efficiency falls as the update shrinks
        ts.append(w / eff * 1e-12)
    e_nb = tm.prediction_error(ts, "lu", "tmu", n, b, tm.predict_neighbours)
    e_first = tm.prediction_error(ts, "lu", "tmu", n, b, tm.predict_first)
    assert e_nb < 0.05 and e_first > 3 * e_nb


def test_slack_formula():
    pred = {"pd": [2.0], "pu": [0.5], "tmu": [5.0], "carry": [0.25], "verify": [0.75]}
    assert tm.slack(pred, 0) == 5.0 + 0.5 + 0.25 + 0.75 - 2.0


def test_validate_on_synthetic_profile():
    n, b = 4096, 512
    N = tm.iterations(n, b)
    prof = {op: [1e-9 * tm.work("qr", op, n, b, k) for k in range(N)] for op in tm.OPS}
    v = tm.validate(prof, "qr", n, b, floor=0.0)
    assert set(v) == {"pd", "tmu", "carry", "verify"}
    for op, r in v.items():
        assert r["neighbours_p4"] < 1e-12 and r["first_iteration"] < 1e-12
