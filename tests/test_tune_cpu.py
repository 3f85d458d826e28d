"""Tuner host logic: the choice among timed candidates."""
from paper_1405_1020_amd import tune


def test_pick_fastest_beyond_the_tie_margin():
    assert tune.pick([("a", 10.0), ("b", 9.0), ("c", 9.5)]) == ("b", 9.0)


def test_pick_earlier_on_near_ties():
    # within 2 % of the fastest the earlier candidate wins, so that runs
    # whose timings differ by noise install the same shape
    assert tune.pick([("a", 10.0), ("b", 9.85), ("c", 9.8)]) == ("b", 9.85)
    assert tune.pick([("a", 1.0), ("b", 0.99)]) == ("a", 1.0)
    assert tune.pick([("only", 3.0)]) == ("only", 3.0)
