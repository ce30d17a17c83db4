"""Host helpers of the search drivers."""
import pytest

from paper_2204_09131_amd.search import overlap_accuracy


def test_overlap_accuracy():
    ref = [(0, 64), (100, 64), (300, 64)]
    assert overlap_accuracy(ref, [(50, 10), (310, 10)]) == pytest.approx(2 / 3)
    assert overlap_accuracy(ref, [(50, 64)]) == pytest.approx(2 / 3)  # one window overlapping two
    assert overlap_accuracy(ref, []) == 0.0
    assert overlap_accuracy([], [(0, 1)]) == 1.0
    assert overlap_accuracy(ref, [(64, 36)]) == 0.0  # touching is not overlapping
    assert overlap_accuracy(ref, ref) == 1.0


def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "selection_scores.json")) as f:
        return json.load(f)


def test_efficiency_scores_by_hand():
    from paper_2204_09131_amd.search import efficiency_scores
    # runtimes 1 s and 3 s -> 0.25 / 0.75; 6 large TD and 2 small BU windows -> 0.75 / 0.25
    td, bu = efficiency_scores(1.0, 3.0, 6, 2, 0.5)
    assert td == pytest.approx(0.5 / 0.25 + 0.5 * 0.75) and bu == pytest.approx(0.5 / 0.75 + 0.5 * 0.25)
    assert efficiency_scores(2.0, 2.0, 0, 0, 0.3) == pytest.approx((0.6, 0.6))


def test_efficiency_scores_against_the_papers_table():
    """Every printed score pair obeys what the score definition forces at
    alpha = 0.5: with t~_TD + t~_BU = 1 and n~_L + n~_S = 1 the two scores sum
    to 0.5 (1/t + 1/(1-t)) + 0.5 >= 2.5.  For (Wind Speed, Rotor Speed) the
    alpha = 0.5 pair fixes t~_TD and n~_L; the definition then reproduces the
    scores the text gives for alpha = 0.2 within the rounding of the table."""
    from paper_2204_09131_amd.search import efficiency_scores
    g = _golden()
    for name, (td, bu) in g["alpha_0_5"].items():
        assert td + bu >= 2.5 - 0.015, name
    td5, bu5 = g["alpha_0_5"]["Wind Speed, Rotor Speed"]
    # 1/t + n = 2 td5 and 1/(1-t) + (1-n) = 2 bu5  =>  1/t + 1/(1-t) = 2 (td5 + bu5) - 1
    s = 2 * (td5 + bu5) - 1
    t = 0.5 + (0.25 - 1 / s) ** 0.5          # the root that keeps n inside [0, 1]
    n = 2 * td5 - 1 / t
    assert 0 <= n <= 1
    # runtimes and counts in these proportions give back the alpha = 0.5 pair ...
    got5 = efficiency_scores(t, 1 - t, round(n * 1000), round((1 - n) * 1000), 0.5)
    assert got5 == pytest.approx((td5, bu5), abs=2e-3)
    # ... and the alpha = 0.2 pair of the text
    td2, bu2 = g["wind_speed_rotor_speed_alpha_0_2"]
    got2 = efficiency_scores(t, 1 - t, round(n * 1000), round((1 - n) * 1000), 0.2)
    assert got2 == pytest.approx((td2, bu2), abs=0.03)
