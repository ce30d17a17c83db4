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
