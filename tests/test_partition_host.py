"""Host logic of the cost-balanced core partition (gdm_rcb_partition, the
bisection behind gdm_balanced_cores; runs on the host, no GPU): against the
oracle's bisection (identical parts: integer output of the same rule),
hand-worked cuts, balance bounds and argument errors."""
import math

import numpy as np
import pytest

from oracle import graph as og
from paper_2606_03140_amd._lib import GDMError, rcb_partition


def test_hand_worked_cuts():
    # four points on x: the widest axis is x, half the weight at the middle
    x = np.array([[3.0, 0, 0], [0.0, 0, 0], [2.0, 0, 0], [1.0, 0, 0]])
    assert list(rcb_partition(x, 2)) == [1, 0, 1, 0]
    # heavy point at x = 0 alone against three light ones
    w = np.array([1.0, 3.0, 1.0, 1.0])
    assert list(rcb_partition(x, 2, w)) == [1, 0, 1, 1]
    # the widest axis wins: spread along z
    y = np.array([[0.1, 0, 5.0], [0.2, 0, 0.0], [0.0, 0, 9.0], [0.3, 0, 1.0]])
    assert list(rcb_partition(y, 2)) == [1, 0, 1, 0]
    # three parts of six points: a third, then halves of the rest
    z = np.array([[float(i), 0, 0] for i in range(6)])
    assert list(rcb_partition(z, 3)) == [0, 0, 1, 1, 2, 2]


@pytest.mark.parametrize("k", [1, 2, 3, 7, 8, 27, 100])
def test_matches_oracle_and_balances(k):
    rng = np.random.default_rng(k)
    pts = rng.uniform(0, 20, size=(1000, 3)) * np.array([1.0, 0.7, 1.3])
    w = rng.integers(1, 12, size=1000).astype(np.float64)
    part = rcb_partition(pts, k, w)
    ref = og.rcb_parts(pts.tolist(), w.tolist(), k)
    assert np.array_equal(part, np.array(ref))
    sums = np.bincount(part, weights=w, minlength=k)
    assert part.min() == 0 and part.max() == k - 1 and np.all(np.bincount(part, minlength=k) > 0)
    depth = math.ceil(math.log2(k)) if k > 1 else 0
    assert np.abs(sums - w.sum() / k).max() <= depth * w.max()
    # unit weights: sizes within the depth of the tree
    cnt = np.bincount(rcb_partition(pts, k), minlength=k)
    assert cnt.max() - cnt.min() <= max(depth, 0) + 1


def test_errors():
    x = np.zeros((5, 3))
    for bad in (0, 6):
        with pytest.raises(GDMError):
            rcb_partition(x, bad)
    with pytest.raises(GDMError):
        rcb_partition(x, 2, np.array([1.0, 1.0, -1.0, 1.0, 1.0]))
    with pytest.raises(GDMError):
        rcb_partition(np.array([[0, 0, np.nan]] * 5), 2)
