"""Hand-worked sequences for the archive updates (Algorithms 4 and 5)."""
import numpy as np


def _x(m, v):
    x = np.zeros(m, np.uint8)
    x[v % m] = 1
    return x


def test_dominance_relations(orc):
    assert orc.dominates((1, 1), (2, 2))
    assert orc.dominates((1, 2), (1, 3))
    assert not orc.dominates((1, 1), (1, 1))      # equivalent is not dominance
    assert not orc.dominates((1, 3), (2, 2))      # mutually non-dominated
    assert not orc.dominates((2, 2), (1, 1))


def test_explore_sequence(orc):
    A = orc.Archive(3, 4)
    assert A.explore(5, 5, _x(4, 0)) == 0          # empty: append
    assert A.explore(6, 4, _x(4, 1)) == 1          # non-dominated: append
    assert A.explore(5, 5, _x(4, 2)) == 2          # equivalent point: append (not full)
    assert A.entries() == [(5, 5), (6, 4), (5, 5)]
    assert A.explore(4, 4, _x(4, 3)) == 0          # dominates slots 0, 1, 2: first one replaced
    assert A.entries() == [(4, 4), (6, 4), (5, 5)]
    assert np.array_equal(A.x[0], _x(4, 3))
    assert A.explore(7, 7, _x(4, 0)) == -1         # full and dominates nothing
    assert A.explore(9, 1, _x(4, 0)) == -1         # non-dominated but full: dropped
    assert A.explore(5, 4, _x(4, 1)) == 1          # dominates (6,4) at 1 and (5,5) at 2 -> slot 1
    assert A.entries() == [(4, 4), (5, 4), (5, 5)]
    assert A.explore(3, 9, _x(4, 2)) == -1
    assert A.size == 3


def test_exploit_sequence(orc):
    A = orc.Archive(3, 4)
    assert A.exploit(5, 5, _x(4, 0), 0) == 0       # append
    assert A.exploit(6, 6, _x(4, 1), 0) == -1      # dominated by (5,5): rejected
    assert A.exploit(4, 6, _x(4, 2), 0) == 1       # non-dominated, B empty: append
    assert A.entries() == [(5, 5), (4, 6)]
    # x = (4,5) dominates both members: B = [0, 1]; w picks floor(w*2/2^32)
    B = orc.Archive(3, 4)
    B.exploit(5, 5, _x(4, 0), 0)
    B.exploit(4, 6, _x(4, 2), 0)
    assert B.exploit(4, 5, _x(4, 3), 0x7FFFFFFF) == 0
    assert B.entries() == [(4, 5), (4, 6)]
    C = orc.Archive(3, 4)
    C.exploit(5, 5, _x(4, 0), 0)
    C.exploit(4, 6, _x(4, 2), 0)
    assert C.exploit(4, 5, _x(4, 3), 0x80000000) == 1
    assert C.entries() == [(5, 5), (4, 5)]
    # (4,5) dominates (5,5) only: B = [0] whatever w is
    assert C.exploit(4, 5, _x(4, 1), 0xFFFFFFFF) == 0
    assert C.entries() == [(4, 5), (4, 5)]
    # equivalent point: nothing dominates it and it dominates nothing -> appended
    assert C.exploit(4, 5, _x(4, 2), 0) == 2
    assert C.size == 3
    # full: a non-dominated point that dominates nothing is dropped
    assert C.exploit(3, 9, _x(4, 1), 0) == -1
    assert C.entries() == [(4, 5), (4, 5), (4, 5)]
