"""Pins of the oracle's error measures (``oracle/metrics.py``) on inputs
whose results are worked out by hand, so that a swapped argument, a missing
absolute value or an off-by-one interpolation fails here before it can hide
in a GPU parity assertion.

* relative L1 E = sum |a - ref| / sum |ref| (the paper's E of Sect. V.A,
  summed along x at one row);
* Linf = max |a - ref|;
* crossing: the position where a profile passes a level, linearly
  interpolated between cell centres (the shock position of a density jump).
"""
import numpy as np
import pytest

from oracle import metrics


def test_rel_l1_hand_values():
    # |1-1| + |2-1| + |3-4| = 2 over |1| + |1| + |4| = 6
    assert metrics.rel_l1([1.0, 2.0, 3.0], [1.0, 1.0, 4.0]) == pytest.approx(1.0 / 3.0, rel=1e-15)
    # the denominator is the reference's: a = 2 ref gives 1, not 1/2
    assert metrics.rel_l1([2.0, 2.0], [1.0, 1.0]) == 1.0
    assert metrics.rel_l1([1.0, 1.0], [2.0, 2.0]) == 0.5
    # signs: |(-1) - (-2)| + |2 - 2| = 1 over |-2| + |2| = 4
    assert metrics.rel_l1([-1.0, 2.0], [-2.0, 2.0]) == 0.25
    # a sign error alone is not cancelled: |1 - (-1)| / |-1| = 2
    assert metrics.rel_l1([1.0], [-1.0]) == 2.0


def test_rel_l1_fields_and_zero_reference():
    a = np.array([[1.0, 0.0], [0.0, -1.0]])
    ref = np.array([[1.5, 0.0], [0.0, -0.5]])
    # 0.5 + 0.5 over 1.5 + 0.5
    assert metrics.rel_l1(a, ref) == 0.5
    # an all-zero reference: the absolute L1 sum is returned
    assert metrics.rel_l1([0.25, -0.5], [0.0, 0.0]) == 0.75
    assert metrics.rel_l1(ref, ref) == 0.0


def test_paper_error_is_the_relative_l1_along_a_row():
    num = [1.0, 0.9, 0.5, 0.125]
    exact = [1.0, 1.0, 0.4, 0.125]
    # 0.1 + 0.1 over 2.525
    assert metrics.paper_error(num, exact) == pytest.approx(0.2 / 2.525, rel=1e-15)
    assert metrics.paper_error(num, exact) == metrics.rel_l1(num, exact)


def test_linf_hand_values():
    assert metrics.linf([1.0, -3.0, 2.0], [0.0, 0.0, 0.0]) == 3.0
    assert metrics.linf([[1.0, 2.0], [3.0, 4.0]], [[1.0, 2.5], [2.0, 4.0]]) == 1.0
    assert metrics.linf([-1.0], [1.0]) == 2.0


def test_crossing_on_a_ramp():
    x = np.arange(5) + 0.5  # cell centres 0.5 .. 4.5
    y = 2.0 * x             # 1, 3, 5, 7, 9
    # y = 4 between x = 1.5 (3) and 2.5 (5): halfway
    assert metrics.crossing(x, y, 4.0) == pytest.approx(2.0, abs=1e-15)
    # y = 3.5 a quarter of the way from 1.5 to 2.5
    assert metrics.crossing(x, y, 3.5) == pytest.approx(1.75, abs=1e-15)
    # a level met exactly at a node returns that node
    assert metrics.crossing(x, y, 5.0) == 2.5
    # no crossing
    assert metrics.crossing(x, y, 10.0) is None
    assert metrics.crossing(x, y, 0.5) is None


def test_crossing_of_a_falling_jump_and_window():
    # a shock: high state on the left, low on the right, with a one-cell ramp
    x = np.arange(8) * 0.1
    y = np.array([4.0, 4.0, 4.0, 4.0, 1.0, 1.0, 1.0, 1.0])
    # level 2.5 halfway between x = 0.3 and 0.4
    assert metrics.crossing(x, y, 2.5) == pytest.approx(0.35, abs=1e-15)
    # level 3.25 a quarter of the way down
    assert metrics.crossing(x, y, 3.25) == pytest.approx(0.325, abs=1e-15)
    # a window that excludes the jump finds nothing
    assert metrics.crossing(x, y, 2.5, lo=0.45, hi=0.7) is None


def test_crossing_first_and_last():
    # a tent crosses 1.5 going up (between 0 and 1) and going down (3 and 4)
    x = np.arange(5, dtype=float)
    y = np.array([1.0, 2.0, 3.0, 2.0, 1.0])
    assert metrics.crossing(x, y, 1.5, last=False) == pytest.approx(0.5, abs=1e-15)
    assert metrics.crossing(x, y, 1.5) == pytest.approx(3.5, abs=1e-15)
    # restricted to the rising side
    assert metrics.crossing(x, y, 1.5, hi=2.0) == pytest.approx(0.5, abs=1e-15)
