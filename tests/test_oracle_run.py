"""Pins of the oracle's whole annealing run (Algorithm 3 and the readings it takes).

The step-by-step validator recomputes every energy difference by brute force from
Eq. (qubo) (no local fields), so it checks the oracle's field bookkeeping, energy
tracking, selection order, offset and archive handling against the definitions.
"""
import math

import numpy as np
import pytest

import synth


def _small_instance(n, seed, fmax=99):
    rng = np.random.default_rng(seed)
    F1 = np.triu(rng.integers(0, fmax + 1, size=(n, n)), 1)
    F2 = np.triu(rng.integers(0, fmax + 1, size=(n, n)), 1)
    F1 = (F1 + F1.T).astype(np.int32)
    F2 = (F2 + F2.T).astype(np.int32)
    D = synth.distances(n, rng)
    return F1, F2, D


def _init_x(orc, n, r, key):
    x = np.zeros(n * n, np.uint8)
    for i in range(n):
        for u in range(n):
            o = orc.philox([((i >> 7) << 16) | u, 0, r, 2], key)
            x[i * n + u] = (int(o[(i >> 5) & 3]) >> (i & 31)) & 1
    return x


def _validate(orc, F1, F2, D, steps, seed, r, accept, archive, escape, d0, df, xi, beta, s=0, table=None):
    n = D.shape[0]
    m = n * n
    q = orc.Qubo(F1, F2, D)
    res = orc.run_replica(q, r, steps, d0, df, xi, beta, seed, accept=accept, archive=archive,
                          escape=escape, archive_size=s, trace=True, temp_table=table)
    Y = [q.Y(1), q.Y(2)]
    qc = list(q.q)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    L = orc.lnt()
    x = _init_x(orc, n, r, key)

    def energies(v):
        return [orc.qubo_energy(Y[k], qc[k], v) for k in range(2)]

    E = energies(x)
    Eoff = 0
    A = orc.Archive(s if s > 0 else m, m)
    delta = d0
    moves = 0
    for t in range(1, steps + 1):
        if delta > df:
            delta = delta * (1.0 - xi)
        T = int(math.floor(delta * 256.0)) if table is None else int(table[t - 1])
        acc = []
        dEs = []
        for a in range(m):
            y = x.copy()
            y[a] ^= 1
            Ey = energies(y)
            d = (Ey[0] - E[0], Ey[1] - E[1])
            dEs.append(d)
            i, u = divmod(a, n)
            o = orc.philox([((i >> 3) << 16) | u, t, r, 0], key)
            f = i & 7
            k = (int(o[f >> 1]) >> (16 * (f & 1))) & 0xFFF
            if orc.accept(d[0], d[1], Eoff, T, int(L[k]), accept):
                acc.append(a)
        if acc:
            w = int(orc.philox([0, t, r, 1], key)[0])
            j = acc[(w * len(acc)) >> 32]
            assert res["trace"][t - 1] == j, t
            x[j] ^= 1
            E = [E[0] + dEs[j][0], E[1] + dEs[j][1]]
            Eoff = 0
            moves += 1
            if archive == orc.EXPLOIT:
                A.exploit(E[0], E[1], x, int(orc.philox([0, t, r, 3], key)[0]))
            else:
                A.explore(E[0], E[1], x)
        else:
            assert res["trace"][t - 1] == -1, t
            if escape == orc.ESC_OFFSET:
                Eoff += beta
            elif A.size > 0:
                w = int(orc.philox([0, t, r, 3], key)[1])
                x = A.x[(w * A.size) >> 32].copy()
                E = energies(x)
    assert np.array_equal(res["x"], x)
    assert (res["E1"], res["E2"], res["Eoff"], res["moves"]) == (E[0], E[1], Eoff, moves)
    assert res["arch_size"] == A.size
    assert list(zip(res["arch_e1"], res["arch_e2"])) == A.entries()
    assert np.array_equal(res["arch_x"], A.x[:A.size])
    return res


@pytest.mark.parametrize("accept,archive,escape", [
    (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)])
def test_trajectory_bruteforce_n3(orc, accept, archive, escape):
    F1, F2, D = _small_instance(3, 1)
    q = orc.Qubo(F1, F2, D)
    d0, df, xi, _ = orc.default_schedule(q.maxabs_c, 400)
    _validate(orc, F1, F2, D, 400, 12345 + accept, 2, accept, archive, escape, d0, df, 0.02, 37, s=5)


def test_trajectory_bruteforce_n4(orc):
    F1, F2, D = _small_instance(4, 2)
    q = orc.Qubo(F1, F2, D)
    d0, df, xi, beta = orc.default_schedule(q.maxabs_c, 300)
    res = _validate(orc, F1, F2, D, 300, (7 << 32) | 99, 5, 0, 0, 0, d0, df, 0.01, beta)
    assert res["moves"] > 50


def test_trajectory_bruteforce_given_schedule(orc):
    """The schedule as input data: T_t read from a table (cooling with a
    reheat half-way and a stretch at T = 0) instead of the geometric loop."""
    F1, F2, D = _small_instance(3, 4)
    q = orc.Qubo(F1, F2, D)
    d0, df, xi, beta = orc.default_schedule(q.maxabs_c, 400)
    t = np.arange(400)
    table = np.floor(d0 * 256.0 * 0.98 ** (t % 200)).astype(np.int64)
    table[300:340] = 0
    res = _validate(orc, F1, F2, D, 400, 4242, 1, 0, 0, 0, d0, df, xi, beta, table=table)
    # the table, not the geometric loop, drove the run
    other = orc.run_replica(q, 1, 400, d0, df, xi, beta, 4242, trace=True)
    assert not np.array_equal(res["trace"], other["trace"])


def _fields(P, x):
    Pz = P.copy()
    np.fill_diagonal(Pz, 0)
    return Pz @ x.astype(np.int64)


@pytest.mark.parametrize("accept,archive,escape", [(0, 0, 0), (1, 1, 0), (0, 0, 1)])
def test_state_invariants(orc, accept, archive, escape):
    """h_k = offdiag(P_k) x and E_k = x^T Y_k x + q_k at the end of a run; every
    archive member's energies are those of its stored solution."""
    inst = synth.make_instance(6, 0.5, seed=31)
    q = orc.Qubo(inst.F1, inst.F2, inst.D)
    d0, df, xi, beta = orc.default_schedule(q.maxabs_c, 3000)
    res = orc.run_replica(q, 3, 3000, d0, df, xi, beta, 77, accept=accept, archive=archive,
                          escape=escape)
    for k, h in ((1, res["h1"]), (2, res["h2"])):
        assert np.array_equal(h, _fields(q.P(k), res["x"]))
    assert res["E1"] == orc.qubo_energy(q.Y(1), q.q[0], res["x"])
    assert res["E2"] == orc.qubo_energy(q.Y(2), q.q[1], res["x"])
    for e1, e2, xs in zip(res["arch_e1"], res["arch_e2"], res["arch_x"]):
        assert e1 == orc.qubo_energy(q.Y(1), q.q[0], xs)
        assert e2 == orc.qubo_energy(q.Y(2), q.q[1], xs)


def test_selection_uniform(orc):
    """Reading R6: with every bit accepted, the chosen flip is uniform over all m
    bits (chi-square, 15 degrees of freedom, p = 0.001 bound 37.7)."""
    n, m, steps = 4, 16, 16000
    F1, F2, D = _small_instance(n, 3, fmax=1)
    D = np.minimum(D, 2).astype(np.int32)
    q = orc.Qubo(F1, F2, D)
    res = orc.run_replica(q, 0, steps, 1e9, 1e8, 0.0, 1, 5, trace=True)
    tr = res["trace"]
    assert np.all(tr >= 0)
    cnt = np.bincount(tr, minlength=m)
    exp = steps / m
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    assert chi2 < 37.7, chi2


def test_replicas_independent_and_deterministic(orc):
    inst = synth.make_instance(5, 0.0, seed=4)
    q = orc.Qubo(inst.F1, inst.F2, inst.D)
    d0, df, xi, beta = orc.default_schedule(q.maxabs_c, 500)
    a = orc.run_replica(q, 1, 500, d0, df, xi, beta, 9, trace=True)
    b = orc.run_replica(q, 1, 500, d0, df, xi, beta, 9, trace=True)
    c = orc.run_replica(q, 2, 500, d0, df, xi, beta, 9, trace=True)
    assert np.array_equal(a["trace"], b["trace"]) and a["E1"] == b["E1"]
    assert not np.array_equal(a["trace"], c["trace"])
