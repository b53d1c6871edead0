"""Selection rule of the tile autotuner (host logic, no GPU)."""
import math

import pytest

from paper_1602_02313_amd.autotune import TIE, pick


def test_fastest_wins_outside_the_tie_band():
    assert pick([10.0, 9.0, 12.0]) == 1


def test_ties_go_to_the_lower_index():
    assert pick([10.0, 10.0 * (1 + TIE / 2), 9.95]) == 0
    assert pick([10.5, 10.0, 10.0 * (1 - TIE / 4)]) == 1


def test_unavailable_variants_are_skipped():
    assert pick([math.inf, 7.0, math.inf, 6.0]) == 3
    with pytest.raises(RuntimeError):
        pick([math.inf, math.inf])
