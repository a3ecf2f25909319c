"""Pins for the oracle's cycle schedules (Alg. 4-6, Table 1)."""
from fractions import Fraction

import pytest

import oracle as O


def totals(cycle, L, T):
    return O.level_iteration_totals(O.schedule(cycle, L, T), L)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("k", [1, 3, 10, 25])
def test_table1_nested_iteration(L, k):
    # Table 1: budget T = 4k fine iterations -> 3k iterations at every
    # non-coarsest level and 4k at the coarsest.
    T = 4 * k * 4 ** (L - 1)      # makes every share an integer
    kk = T // 4
    want = [3 * kk] * (L - 1) + [4 * kk]
    assert totals(O.NI, L, T) == want


@pytest.mark.parametrize("L", [2, 3, 4])
@pytest.mark.parametrize("T", [64, 256, 1000, 4096])
def test_vcycle_spends_the_same_per_level_as_nested_iteration(L, T):
    # Section 4.3.2: three quarters of the time at the current level, as for NI.
    assert totals(O.VC, L, T) == totals(O.NI, L, T)


def test_time_column_of_table1():
    # time per level = iterations * 4^-d : 3T/4, 3T/16, ..., T/4^(L-1)
    L, T = 4, 4 ** 5
    t = totals(O.NI, L, T)
    time = [Fraction(c, 4 ** d) for d, c in enumerate(t)]
    assert time == [Fraction(3 * T, 4 ** (d + 1)) for d in range(L - 1)] + [Fraction(T, 4 ** (L - 1))]
    assert sum(time) == T


def test_small_config_example():
    # 16x16 -> 8x8, NI with T = 200: 200 coarse iterations, then 150 fine.
    assert O.schedule(O.NI, 2, 200) == [("restrict", 0, 0), ("run", 1, 200),
                                         ("prolong", 0, 0), ("run", 0, 150)]


@pytest.mark.parametrize("T", [16, 64, 160, 4096])
def test_fmg_two_levels(T):
    # FMG(2, T): 9T/16 iterations at the fine level and 7T/4 at the coarse one.
    assert totals(O.FMG, 2, T) == [9 * T // 16, 7 * T // 4]


def test_vcycle_order():
    s = O.schedule(O.VC, 3, 64)
    assert s == [("run", 0, 16), ("restrict", 0, 0), ("run", 1, 16), ("restrict", 1, 0),
                 ("run", 2, 64), ("prolong", 1, 0), ("run", 1, 32), ("prolong", 0, 0),
                 ("run", 0, 32)]


def test_fmg_order():
    s = O.schedule(O.FMG, 2, 16)
    assert s == [("restrict", 0, 0), ("run", 1, 16), ("prolong", 0, 0),
                 ("run", 0, 3), ("restrict", 0, 0), ("run", 1, 12), ("prolong", 0, 0),
                 ("run", 0, 6)]


@pytest.mark.parametrize("cycle", [O.NI, O.VC, O.FMG])
@pytest.mark.parametrize("L", [1, 2, 3, 4])
@pytest.mark.parametrize("T", [0, 1, 7, 40, 123, 1000])
def test_schedule_is_well_formed(cycle, L, T):
    depth = 0
    fe = Fraction(0)
    for kind, d, c in O.schedule(cycle, L, T):
        if kind == "restrict":
            assert d == depth
            depth += 1
        elif kind == "prolong":
            assert d == depth - 1
            depth -= 1
        else:
            assert d == depth and c > 0
            fe += Fraction(c, 4 ** d)
        assert 0 <= depth < L
    assert depth == 0
    assert fe <= T          # floors never exceed the budget


def test_single_level_is_plain_run():
    for cyc in (O.NI, O.VC, O.FMG):
        assert O.schedule(cyc, 1, 37) == [("run", 0, 37)]


# ------------------------------------------------------------------ W-cycle

@pytest.mark.parametrize("levels", [2, 3, 4, 5])
@pytest.mark.parametrize("T", [64, 256, 4096])
def test_w_cycle_keeps_the_table1_totals(levels, T):
    # reading R13: the V-cycle's split, so every level gets the Table 1 totals
    # (3T/4 iterations at each non-coarsest level, T at the coarsest) when
    # every run's budget is a whole number of iterations (T a multiple of
    # 2^(levels+1); smaller budgets lose iterations to the floor of each run)
    st = O.schedule(O.WC, levels, T)
    tot = O.level_iteration_totals(st, levels)
    assert tot == O.level_iteration_totals(O.schedule(O.VC, levels, T), levels)
    want = [3 * T // 4] * (levels - 1) + [T]
    assert tot == want


@pytest.mark.parametrize("levels", [2, 3, 4, 5])
def test_w_cycle_visits_each_coarser_level_twice_per_visit_above(levels):
    st = O.schedule(O.WC, levels, 4096)
    # each visit of depth d restricts once and visits depth d+1 twice: depth d
    # is visited 2^d times
    visits = [2 ** d for d in range(levels)]
    for d in range(levels - 1):
        assert sum(1 for k, dd, _ in st if k == "restrict" and dd == d) == visits[d]
        assert sum(1 for k, dd, c in st if k == "run" and dd == d + 1) >= visits[d + 1]
    # transfers balance and the walk starts and ends on the finest level
    depth = 0
    for kind, d, _ in st:
        if kind == "restrict":
            assert depth == d
            depth += 1
        elif kind == "prolong":
            assert depth == d + 1
            depth -= 1
        else:
            assert depth == d
    assert depth == 0


def test_w_cycle_two_levels_written_out():
    T = 16
    assert O.schedule(O.WC, 2, T) == [("run", 0, 4), ("restrict", 0, 0), ("run", 1, 8),
                                      ("run", 1, 8), ("prolong", 0, 0), ("run", 0, 8)]
