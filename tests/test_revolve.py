"""The checkpointing schedule of hlb_adjoint_run (no GPU): its forward-step
count (hlb_revolve_forward_steps, a dry run of the same recursion) against

  * the minimum over all checkpoint placements, by brute-force dynamic
    programming written here: reversing l steps with s free slots costs
    T(l, s) = min over 1 <= m < l of  m + T(l - m, s - 1) + T(m, s)
    (reach a checkpoint m steps ahead, reverse the part after it with one
    slot less, then the part before it with the slot freed again), and
    T(l, 0) = l (l - 1) / 2 (every step recomputed from the start);
  * Griewank & Walther's closed form for binomial checkpointing,
    r n - C(S + r, r - 1), r the least integer with C(S + r, S) >= n, S the
    number of slots with the start state's.
"""
from functools import lru_cache
from math import comb

import pytest

from paper_2202_11770_amd import hlb


@lru_cache(maxsize=None)
def _dp(l, s):
    if l <= 1:
        return 0
    if s == 0:
        return l * (l - 1) // 2
    return min(m + _dp(l - m, s - 1) + _dp(m, s) for m in range(1, l))


def _closed(n, S):
    if n <= 1:
        return 0
    r = 0
    while comb(S + r, S) < n:
        r += 1
    return r * n - comb(S + r, r - 1)


def test_schedule_is_optimal_small():
    for n_snap in range(1, 8):
        for n in range(1, 121):
            got = hlb.hlb_revolve_forward_steps(n, n_snap)
            assert got == _dp(n, n_snap - 1), (n, n_snap)


@pytest.mark.parametrize("n,n_snap", [(40, 10), (300, 10), (1000, 7), (3000, 30), (3000, 4), (100000, 50),
                                      (100000, 2), (20000, 4096), (5, 1), (1, 1), (64, 65)])
def test_schedule_meets_closed_form(n, n_snap):
    assert hlb.hlb_revolve_forward_steps(n, n_snap) == _closed(n, n_snap)


def test_arguments():
    for n, s in ((0, 4), (10, 0), (10, 4097)):
        with pytest.raises(hlb.HLBError):
            hlb.hlb_revolve_forward_steps(n, s)
