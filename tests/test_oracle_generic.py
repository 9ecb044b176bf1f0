"""Pins of the oracle's K-objective MDA on a generic QUBO (readings G1-G3 of
the oracle header; the Conclusion's extension to more than two objectives).

  * dominance and both archive rules on hand-worked K = 3 sequences;
  * the acceptance rule against the two-objective rule pinned elsewhere (K = 2,
    both modes) and against its one-objective special case (Eq. paccepts);
  * invariants that reduce a K-objective run to a one-objective run: the
    lenient rule with K copies of one QUBO, and the strict rule with the other
    objectives zero, give the same trajectory;
  * a brute-force validator that re-derives every step of short runs from the
    definitions: energies from Eq. (qubo) on the given Q (no local fields), the
    draws from Philox, acceptance, choice, move and archive.
"""
import math

import numpy as np
import pytest


def test_gdominates_hand_cases(orc):
    assert orc.gdominates([1, 2, 3], [1, 2, 4])
    assert orc.gdominates([0, 0, 0], [1, 1, 1])
    assert not orc.gdominates([1, 2, 3], [1, 2, 3])          # equal: no
    assert not orc.gdominates([1, 2, 5], [1, 3, 4])          # worse in one
    assert not orc.gdominates([2, 2, 3], [1, 9, 9])
    assert orc.gdominates([5], [6]) and not orc.gdominates([6], [5])
    # K = 2 agrees with the two-objective dominance
    rng = np.random.default_rng(0)
    for _ in range(200):
        p, q = rng.integers(0, 4, 2), rng.integers(0, 4, 2)
        assert orc.gdominates(p, q) == orc.dominates(p, q)


def test_garchive_explore_sequence(orc):
    """Algorithm 4 with K = 3: replace the first dominated member, else append."""
    A = orc.GArchive(3, 2, 3)
    x = np.zeros(2, np.uint8)
    assert A.explore([5, 5, 5], x) == 0
    assert A.explore([6, 4, 5], x) == 1          # incomparable: appended
    assert A.explore([4, 4, 5], x) == 0          # dominates both; the first (slot 0) is replaced
    assert A.entries() == [(4, 4, 5), (6, 4, 5)]
    assert A.explore([6, 4, 5], x) == 2          # equivalent to slot 1, dominates nothing: appended
    assert A.explore([9, 9, 0], x) == -1         # full and dominates nothing
    assert A.explore([5, 4, 5], x) == 1          # dominates slots 1 and 2: the first is replaced
    assert A.explore([3, 3, 3], x) == 0
    assert A.entries() == [(3, 3, 3), (5, 4, 5), (6, 4, 5)]


def test_garchive_exploit_sequence(orc):
    """Algorithm 5 with K = 3: rejected when dominated; a random member of B replaced."""
    A = orc.GArchive(4, 2, 3)
    x = np.zeros(2, np.uint8)
    for e in ([5, 5, 5], [7, 1, 9], [2, 8, 8]):
        A.exploit(e, x, 0)
    assert A.entries() == [(5, 5, 5), (7, 1, 9), (2, 8, 8)]
    assert A.exploit([6, 6, 6], x, 0) == -1      # dominated by (5, 5, 5)
    # (1, 1, 5) dominates (5, 5, 5) and (7, 1, 9) but not (2, 8, 8): B = {0, 1};
    # w = 2^31 picks floor(2^31 * 2 / 2^32) = 1 -> slot 1
    assert A.exploit([1, 1, 5], x, 1 << 31) == 1
    assert A.entries() == [(5, 5, 5), (1, 1, 5), (2, 8, 8)]
    assert A.exploit([0, 9, 9], x, 0) == 3       # dominates nothing: appended


@pytest.mark.parametrize("mode", [0, 1])
def test_gaccept_matches_two_objective_rule(orc, mode):
    rng = np.random.default_rng(10 + mode)
    L = orc.lnt()
    for _ in range(3000):
        d = rng.integers(-50_000, 50_000, 2)
        eoff = int(rng.integers(0, 30_000))
        T = int(rng.integers(0, 5_000_000))
        k = int(rng.integers(0, 4096))
        assert orc.gaccept(d, eoff, T, int(L[k]), mode) == orc.accept(d[0], d[1], eoff, T, int(L[k]), mode)


def test_gaccept_one_objective_is_paccepts(orc):
    """K = 1: accept iff max(0, dE - E_offset) <= (T * LNT[k]) >> 24 (Eq. paccepts)."""
    L = orc.lnt()
    rng = np.random.default_rng(3)
    for _ in range(2000):
        d = int(rng.integers(-1000, 100_000))
        eoff = int(rng.integers(0, 1000))
        T = int(rng.integers(0, 2_000_000))
        k = int(rng.integers(0, 4096))
        want = max(0, d - eoff) <= (T * int(L[k])) >> 24
        assert orc.gaccept([d], eoff, T, int(L[k]), 0) == want
    # three objectives: the strict statistic is the sum, the lenient one the least
    T, Lk = 1 << 24, 100
    assert orc.gaccept([40, 30, 30], 0, T, Lk, 0) and not orc.gaccept([40, 30, 31], 0, T, Lk, 0)
    assert orc.gaccept([500, 100, 300], 0, T, Lk, 1) and not orc.gaccept([500, 101, 300], 0, T, Lk, 1)


def _rand_q(rng, K, m, lo=-20, hi=21):
    return rng.integers(lo, hi, size=(K, m, m)).astype(np.int32)


def test_lenient_copies_reduce_to_one_objective(orc):
    """Lenient rule, K copies of one QUBO: min_k max(0, D_k) = max(0, D), and
    dominance between equal-coordinate vectors is one-objective dominance."""
    rng = np.random.default_rng(21)
    Q1 = _rand_q(rng, 1, 9)
    g1 = orc.GQubo(Q1)
    g3 = orc.GQubo(np.concatenate([Q1] * 3))
    d0, df, xi, beta = orc.gdefault_schedule(g1.maxabs_c, 800)
    for r in range(3):
        a = orc.run_greplica(g1, r, 800, d0, df, xi, beta, 99, accept=orc.LENIENT, trace=True)
        b = orc.run_greplica(g3, r, 800, d0, df, xi, beta, 99, accept=orc.LENIENT, trace=True)
        assert np.array_equal(a["trace"], b["trace"]) and a["moves"] > 0
        assert b["E"] == a["E"] * 3
        assert np.array_equal(b["arch_e"][:, 0], a["arch_e"][:, 0])


def test_strict_zero_objectives_reduce_to_one(orc):
    """Strict rule with objectives 2..K zero: max(0, 0 - E_offset) = 0, so the
    statistic is objective 1's alone, and the archive compares E_1 only."""
    rng = np.random.default_rng(22)
    Q1 = _rand_q(rng, 1, 10)
    g1 = orc.GQubo(Q1)
    g3 = orc.GQubo(np.concatenate([Q1, np.zeros_like(Q1), np.zeros_like(Q1)]), q=[0, 5, 7])
    d0, df, xi, beta = orc.gdefault_schedule(g1.maxabs_c, 900)
    for r in range(3):
        a = orc.run_greplica(g1, r, 900, d0, df, xi, beta, 7, trace=True)
        b = orc.run_greplica(g3, r, 900, d0, df, xi, beta, 7, trace=True)
        assert np.array_equal(a["trace"], b["trace"]) and a["moves"] > 0
        assert b["E"] == [a["E"][0], 5, 7]
        assert np.array_equal(b["arch_e"][:, 0], a["arch_e"][:, 0])


def _validate(orc, Q, q, steps, seed, r, accept, archive, escape, d0, df, xi, beta, s=0):
    """Every step re-derived from the definitions (energies by Eq. qubo)."""
    K, m = Q.shape[0], Q.shape[1]
    g = orc.GQubo(Q, q)
    res = orc.run_greplica(g, r, steps, d0, df, xi, beta, seed, accept=accept, archive=archive, escape=escape,
                           archive_size=s, trace=True)
    Qs = [Q[k].astype(np.int64) for k in range(K)]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    L = orc.lnt()
    x = np.zeros(m, np.uint8)
    for a in range(m):
        o = orc.philox([a >> 7, 0, r, 2], key)
        x[a] = (int(o[(a >> 5) & 3]) >> (a & 31)) & 1

    def energies(v):
        return [orc.qubo_energy(Qs[k], int(q[k]), v) for k in range(K)]

    E = energies(x)
    Eoff, moves = 0, 0
    A = orc.GArchive(s if s > 0 else m, m, K)
    delta = d0
    for t in range(1, steps + 1):
        if delta > df:
            delta = delta * (1.0 - xi)
        T = int(math.floor(delta * 256.0))
        acc, dEs = [], []
        for a in range(m):
            y = x.copy()
            y[a] ^= 1
            Ey = energies(y)
            d = [Ey[k] - E[k] for k in range(K)]
            dEs.append(d)
            o = orc.philox([a >> 3, t, r, 0], key)
            f = a & 7
            idx = (int(o[f >> 1]) >> (16 * (f & 1) + 4)) & 0xFFF
            if orc.gaccept(d, Eoff, T, int(L[idx]), accept):
                acc.append(a)
        if acc:
            w = int(orc.philox([0, t, r, 1], key)[0])
            j = acc[(w * len(acc)) >> 32]
            assert res["trace"][t - 1] == j, t
            x[j] ^= 1
            E = [E[k] + dEs[j][k] for k in range(K)]
            Eoff = 0
            moves += 1
            if archive == orc.EXPLOIT:
                A.exploit(E, x, int(orc.philox([0, t, r, 3], key)[0]))
            else:
                A.explore(E, x)
        else:
            assert res["trace"][t - 1] == -1, t
            if escape == orc.ESC_OFFSET:
                Eoff += beta
            elif A.size > 0:
                w = int(orc.philox([0, t, r, 3], key)[1])
                x = A.x[(w * A.size) >> 32].copy()
                E = energies(x)
    assert np.array_equal(res["x"], x)
    assert res["E"] == E and (res["Eoff"], res["moves"]) == (Eoff, moves)
    assert res["arch_size"] == A.size
    assert [tuple(int(v) for v in row) for row in res["arch_e"]] == A.entries()
    assert np.array_equal(res["arch_x"], A.x[:A.size])
    # the maintained fields equal offdiag(P_k) x
    for k in range(K):
        P = g.P(k)
        Pz = P.copy()
        np.fill_diagonal(Pz, 0)
        assert np.array_equal(res["h"][k], Pz @ x.astype(np.int64))
    return res


@pytest.mark.parametrize("K,m,accept,archive,escape", [
    (1, 7, 0, 0, 0), (2, 9, 1, 0, 0), (3, 8, 0, 1, 0), (3, 10, 1, 0, 1), (4, 6, 0, 0, 1), (2, 11, 0, 1, 1)])
def test_trajectory_bruteforce(orc, K, m, accept, archive, escape):
    rng = np.random.default_rng(100 * K + m)
    Q = _rand_q(rng, K, m)
    q = rng.integers(-50, 50, K)
    g = orc.GQubo(Q, q)
    d0, df, xi, beta = orc.gdefault_schedule(g.maxabs_c, 250)
    res = _validate(orc, Q, q, 250, (5 << 32) | (17 + m), 1, accept, archive, escape, d0, df, 0.02, 3,
                    s=5 if archive else 0)
    assert res["moves"] > 10
