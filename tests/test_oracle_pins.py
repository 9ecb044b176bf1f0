"""Hand-computed pins of the oracle's penalty weight, default schedule and int32
row-bound flag (CPU).  Each expected value below is worked out by hand from the
definitions it cites, not by calling the function under test.

Bits of an n = 2 instance: 0 = (facility 0, location 0), 1 = (0, 1),
2 = (1, 0), 3 = (1, 1).  Upper-triangular cost QUBO of Sec. 2.2:
C_aa = F_ii D_uu and C_ab = F_ij D_uv + F_ji D_vu for a < b.  Constraint QUBO
(Eq. gqap): G_aa = -2, G_ab = 2 for the row pairs (0,1), (2,3) and the column
pairs (0,2), (1,3); constant 2n.
"""
import numpy as np
import pytest

from tests.golden.fixtures import worked_example


def test_alpha_worked_example(orc):
    """Sec. 2.2 worked example: the largest |C| entry printed is 24, so the
    benchmark weight is alpha = 2 * 24 = 48 and the constant of Y = C + alpha G
    (Eq. wqubom) is q = alpha * p_g = 48 * 6 = 288."""
    ex = worked_example()
    H = ex["H"].astype(np.int32)
    D = ex["D"].astype(np.int32)
    assert orc.penalty_2max(orc.cost_qubo(H, D)) == 48
    q = orc.Qubo(H, H, D)
    assert q.alpha == (48, 48)
    assert q.q == (288, 288)
    assert q.maxabs_c == 24
    # Y_00 = C_00 + alpha G_00 = 0 - 96; Y_01 = 0 + 2 alpha (row pair);
    # Y_04 = C_04 = 6 (neither row nor column pair)
    Y = q.Y(1)
    assert (Y[0, 0], Y[0, 1], Y[0, 4], Y[0, 8]) == (-96, 96, 6, 16)


def test_alpha_signed_entries(orc):
    """F = [[0, -7], [2, 0]], D = [[0, 3], [5, 0]]:
    C_03 = F01 D01 + F10 D10 = -21 + 10 = -11,
    C_12 = F01 D10 + F10 D01 = -35 + 6 = -29, every other entry 0.
    The weight uses the absolute value: alpha = 2 * 29 = 58 (a signed maximum
    would give 0), q = 58 * 2n = 232."""
    F = np.array([[0, -7], [2, 0]], np.int32)
    D = np.array([[0, 3], [5, 0]], np.int32)
    C = orc.cost_qubo(F, D)
    assert C[0, 3] == -11 and C[1, 2] == -29
    assert orc.penalty_2max(C) == 58
    q = orc.Qubo(F, F, D)
    assert q.alpha == (58, 58) and q.q == (232, 232)
    Y = q.Y(1)
    assert (Y[0, 0], Y[0, 1], Y[0, 2], Y[1, 2], Y[0, 3]) == (-116, 116, 116, -29, -11)


def test_alpha_diagonal_maximum(orc):
    """F = [[5, 1], [1, 0]], D = [[6, 1], [1, 0]]: C_00 = F00 D00 = 30,
    C_01 = F00 (D01 + D10) = 10, C_02 = (F01 + F10) D00 = 12, C_03 = C_12 = 2.
    The largest entry is on the diagonal: alpha = 60, q = 240."""
    F = np.array([[5, 1], [1, 0]], np.int32)
    D = np.array([[6, 1], [1, 0]], np.int32)
    C = orc.cost_qubo(F, D)
    assert (C[0, 0], C[0, 1], C[0, 2], C[0, 3], C[1, 2]) == (30, 10, 12, 2, 2)
    q = orc.Qubo(F, np.zeros_like(F), D)
    assert q.alpha == (60, 0) and q.q == (240, 0)


def test_default_schedule_values(orc):
    """Table (param): delta0 = 1e9, delta_f = 1e4, xi = 0.001 for coefficients
    scaled to 2^23, here scaled by M / 2^23 with M = max|C|; beta is
    max(1, floor(delta0 / steps))."""
    # M = 2^23: the paper's own numbers; I_max at n = 25 is 0.25 * 625^2 = 97656
    # (rounded down), and 1e9 / 97656 = 10240.03
    assert orc.default_schedule(2 ** 23, 97656) == (1e9, 1e4, 0.001, 10240)
    # M = 24 (the worked example): 24e9 / 2^23 = 5859375 / 2^11 = 2861.02294921875,
    # 24e4 / 2^23 = 1875 / 2^16 = 0.0286102294921875 (both exact in binary)
    d0, df, xi, beta = orc.default_schedule(24, 1000)
    assert (d0, df, xi, beta) == (2861.02294921875, 0.0286102294921875, 0.001, 2)
    # 2861.02 / 10^4 < 1, so beta is held at 1
    assert orc.default_schedule(24, 10 ** 4)[3] == 1


@pytest.mark.parametrize("a, bound", [(14, 2 ** 31 - 2), (15, 2 ** 31 - 1), (16, 2 ** 31)])
def test_row_bound_flag(orc, a, bound):
    """F = [[a, f], [f, 0]], D = [[1, 1], [1, 0]], f = 76695844, a <= f:
    C_00 = a, C_01 = 2a, C_02 = C_03 = C_12 = 2f, the rest 0, so M = 2f and
    alpha = 4f.  Y_00 = a - 2 alpha, Y_01 = 2a + 2 alpha, Y_02 = 2f + 2 alpha,
    Y_03 = 2f, and bit 0 has the largest row bound
    |Y_00| + |Y_01| + |Y_02| + |Y_03| = 6 alpha + a + 4f = 28f + a.
    28 f = 2147483632, so a = 14, 15, 16 put it at 2^31 - 2, 2^31 - 1 and 2^31.
    The flag is raised exactly when some local-field value could leave int32,
    i.e. when the bound exceeds 2^31 - 1."""
    f = 76695844
    F = np.array([[a, f], [f, 0]], np.int32)
    D = np.array([[1, 1], [1, 0]], np.int32)
    q = orc.Qubo(F, F, D)
    assert q.alpha == (4 * f, 4 * f)
    P = q.P(1)
    assert int(np.abs(P).sum(axis=1).max()) == bound == 28 * f + a
    assert q.overflow == (bound > 2 ** 31 - 1)
