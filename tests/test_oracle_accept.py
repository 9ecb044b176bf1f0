"""Special cases of the multi-objective acceptance rules (Section 3.3)."""
import math

import numpy as np
import pytest


def _freq(orc, dE1, dE2, Eoff, T, mode):
    L = orc.lnt()
    return sum(orc.accept(dE1, dE2, Eoff, T, int(L[k]), mode) for k in range(4096)) / 4096.0


def test_strict_with_zero_second_objective_is_single_objective(orc):
    """Strict rule with Z = 0 reduces to Eq. (paccepts) of the single-objective
    DA, offset included: the decision equals the one-objective test on dE1."""
    rng = np.random.default_rng(0)
    L = orc.lnt()
    for _ in range(3000):
        dE1 = int(rng.integers(-5000, 5000))
        Eoff = int(rng.integers(0, 3000))
        T = int(rng.integers(0, 500 * 256))
        k = int(rng.integers(0, 4096))
        one = max(0, dE1 - Eoff) <= (T * int(L[k])) >> 24   # Eq. (paccepts) in fixed point
        assert orc.accept(dE1, 0, Eoff, T, int(L[k]), orc.STRICT) == one


def test_zero_temperature_is_greedy(orc):
    """delta = 0: strict accepts exactly when both D_k <= 0, lenient when either is."""
    L = orc.lnt()
    for dE1 in (-3, 0, 4):
        for dE2 in (-2, 0, 5):
            for Eoff in (0, 3):
                for k in (0, 2000, 4095):
                    s = orc.accept(dE1, dE2, Eoff, 0, int(L[k]), orc.STRICT)
                    l = orc.accept(dE1, dE2, Eoff, 0, int(L[k]), orc.LENIENT)
                    assert s == (dE1 - Eoff <= 0 and dE2 - Eoff <= 0)
                    assert l == (dE1 - Eoff <= 0 or dE2 - Eoff <= 0)


def test_lenient_with_zero_second_objective_accepts_all(orc):
    L = orc.lnt()
    for dE1 in (-10, 0, 10**6):
        for k in (0, 4095):
            assert orc.accept(dE1, 0, 0, 256, int(L[k]), orc.LENIENT)


@pytest.mark.parametrize("d1,d2", [(300, 500), (0, 800), (1200, 100), (-50, 400)])
def test_strict_is_product_lenient_is_max(orc, d1, d2):
    """Eq. (pacceptms): the product of the per-objective probabilities;
    Eq. (pacceptml): their maximum (frequencies over all uniform indices)."""
    delta = 700.0
    T = int(delta * 256)
    p1 = math.exp(-max(0, d1) / delta)
    p2 = math.exp(-max(0, d2) / delta)
    tol = 2.0 / 4096 + 2.0 / delta
    assert abs(_freq(orc, d1, d2, 0, T, orc.STRICT) - p1 * p2) <= tol
    assert abs(_freq(orc, d1, d2, 0, T, orc.LENIENT) - max(p1, p2)) <= tol


def test_offset_shifts_both_objectives(orc):
    """The offset lowers both energy differences by the same amount (Eq. paccepts)."""
    delta = 300.0
    T = int(delta * 256)
    a = _freq(orc, 900, 700, 400, T, orc.STRICT)
    b = _freq(orc, 500, 300, 0, T, orc.STRICT)
    assert a == b
