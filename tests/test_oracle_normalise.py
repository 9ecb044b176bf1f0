"""Pins of the oracle's objective normalisation (Sec. Parameter Settings: the
largest coefficient of each objective QUBO is set to 2^23)."""
import numpy as np
import pytest

import oracle
import synth


def test_hand_computed_n2():
    # n = 2, zero diagonals: the only non-zero coefficients of the cost QUBO are
    # ((0,0),(1,1)) = F01 D01 + F10 D10 = 3*5 + 1*2 = 17 and
    # ((0,1),(1,0)) = F01 D10 + F10 D01 = 3*2 + 1*5 = 11, so max|C| = 17
    F = np.array([[0, 3], [1, 0]], np.int32)
    D = np.array([[0, 5], [2, 0]], np.int32)
    assert int(np.abs(oracle.cost_qubo(F, D)).max()) == 17
    Fs, s = oracle.normalise_flows(F, D, 10)
    assert s == 1024.0 / 17.0
    # 3 * 1024 / 17 = 180.7 -> 181; 1024 / 17 = 60.2 -> 60
    assert np.array_equal(Fs, np.array([[0, 181], [60, 0]], np.int32))


def test_already_at_target_is_unchanged():
    # max|C| = 4*8 + 4*8 = 64 = 2^6
    F = np.array([[0, 4], [4, 0]], np.int32)
    D = np.array([[0, 8], [8, 0]], np.int32)
    Fs, s = oracle.normalise_flows(F, D, 6)
    assert s == 1.0 and np.array_equal(Fs, F)


def test_rounding_to_nearest_halves_up():
    D = np.array([[0, 1], [0, 0]], np.int32)
    # C = {F01 D01 + F10 D10, F01 D10 + F10 D01} = {F01, F10}: max|C| = max(F01, F10)
    Fs, s = oracle.normalise_flows(np.array([[0, 3], [1, 0]], np.int32), D, 0)
    assert s == 1.0 / 3.0                                  # 3 -> 1, 1/3 -> 0
    assert np.array_equal(Fs, np.array([[0, 1], [0, 0]], np.int32))
    Fs, s = oracle.normalise_flows(np.array([[0, 8], [3, 0]], np.int32), D, 2)
    assert s == 0.5                                        # 8 -> 4, 1.5 -> 2 (half up)
    assert np.array_equal(Fs, np.array([[0, 4], [2, 0]], np.int32))
    Fs, s = oracle.normalise_flows(np.array([[0, 8], [5, 0]], np.int32), D, 2)
    assert np.array_equal(Fs, np.array([[0, 4], [3, 0]], np.int32))   # 2.5 -> 3
    Fs, s = oracle.normalise_flows(np.array([[0, 1], [0, 0]], np.int32), D, 1)
    assert s == 2.0 and np.array_equal(Fs, np.array([[0, 2], [0, 0]], np.int32))


def test_scale_invariance():
    # the scaled flows depend only on the direction of F: doubling F halves s
    inst = synth.make_instance(7, 0.3, seed=71)
    a, sa = oracle.normalise_flows(inst.F1, inst.D, 15)
    b, sb = oracle.normalise_flows(2 * inst.F1, inst.D, 15)
    assert np.array_equal(a, b) and sb == sa / 2


@pytest.mark.parametrize("n,rho,L", [(6, 0.0, 12), (9, -0.75, 16), (12, 0.75, 20), (8, 0.0, 23)])
def test_largest_coefficient_within_rounding(n, rho, L):
    # every scaled flow is within 1/2 of s F, so every coefficient of the new QUBO,
    # F'ij Duv + F'ji Dvu, is within (Duv + Dvu) / 2 <= max D of s C
    inst = synth.make_instance(n, rho, seed=100 + n)
    for F in (inst.F1, inst.F2):
        Fs, s = oracle.normalise_flows(F, inst.D, L)
        assert np.all(np.abs(Fs - F.astype(np.float64) * s) <= 0.5)
        mx = int(np.abs(oracle.cost_qubo(Fs, inst.D)).max())
        assert abs(mx - 2 ** L) <= int(inst.D.max())


def test_objectives_balanced():
    # before: the two objectives differ in scale by 100x; after: both at 2^18
    inst = synth.make_instance(8, 0.0, seed=81)
    F2 = inst.F2 * 100
    m1 = int(np.abs(oracle.cost_qubo(inst.F1, inst.D)).max())
    m2 = int(np.abs(oracle.cost_qubo(F2, inst.D)).max())
    assert m2 > 50 * m1
    a, _ = oracle.normalise_flows(inst.F1, inst.D, 18)
    b, _ = oracle.normalise_flows(F2, inst.D, 18)
    for Fs in (a, b):
        assert abs(int(np.abs(oracle.cost_qubo(Fs, inst.D)).max()) - 2 ** 18) <= int(inst.D.max())


def test_permutation_costs_scale_linearly():
    # the QAP cost of a permutation is linear in F, so the scaled cost is s times
    # the original up to n^2 max D / 2 (each of the n^2 flows moves by <= 1/2)
    rng = np.random.default_rng(5)
    inst = synth.make_instance(6, 0.0, seed=61)
    Fs, s = oracle.normalise_flows(inst.F1, inst.D, 22)
    bound = 36 * int(inst.D.max()) / 2
    for _ in range(50):
        p = rng.permutation(6).astype(np.int32)
        c0 = oracle.qap_cost(inst.F1, inst.D, p)
        c1 = oracle.qap_cost(Fs, inst.D, p)
        assert abs(c1 - s * c0) <= bound
