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


def test_candidates_cover_registers_and_column_form():
    from paper_1405_1020_amd import binding as B

    def hists(r, L):
        return {(v.hist, v.waves) for v in tune.candidates(r, L)}
    # histograms in registers: radius <= 7, at most 16 levels
    for r, L in [(0, 1), (1, 8), (3, 16), (7, 9)]:
        assert (B.HIST_REGS, 1) in hists(r, L)
    for r, L in [(8, 8), (3, 17), (15, 64)]:
        assert (B.HIST_REGS, 1) not in hists(r, L)
    # the column layout's radius <= 15 form from radius 3, up to 64 levels
    for r, L in [(3, 8), (5, 64), (15, 20)]:
        assert (B.HIST_COLUMN, 4) in hists(r, L)
    for r, L in [(2, 20), (5, 65)]:
        assert (B.HIST_COLUMN, 4) not in hists(r, L)
    assert (B.HIST_COLUMN, 1) in hists(16, 20)
    # the count-word column form with two or four wavefronts up to radius 31
    for r, L in [(16, 8), (31, 64)]:
        assert {(B.HIST_COLUMN, 2), (B.HIST_COLUMN, 4), (B.HIST_COLUMN, 1)} <= hists(r, L)
    for r, L in [(32, 20), (20, 65)]:
        assert (B.HIST_COLUMN, 4) not in hists(r, L)
