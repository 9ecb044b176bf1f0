"""Pins of the oracle's QUBO of the bi-objective QAP (Section 2 of the paper)."""
import itertools

import numpy as np

from tests.golden.fixtures import worked_example


def test_worked_example_matrices(orc):
    """Section 2.2: C, p_c, G, p_g exactly as printed for the n = 3 example."""
    ex = worked_example()
    C = orc.cost_qubo(ex["H"], ex["D"])
    assert np.array_equal(C, ex["C"])
    G, pg = orc.constraint_qubo(3)
    assert np.array_equal(G, ex["G"])
    assert pg == ex["pg"]
    assert ex["pc"] == 0


def test_worked_example_solutions(orc):
    """Section 2.2: f(sigma), x^T C x, x^T G x and g(x) of both printed solutions."""
    ex = worked_example()
    C = orc.cost_qubo(ex["H"], ex["D"])
    G, pg = orc.constraint_qubo(3)
    for sol in ex["solutions"]:
        perm = [s - 1 for s in sol["sigma"]]
        assert orc.qap_cost(ex["H"], ex["D"], perm) == sol["f"]
        assert orc.qubo_energy(C, 0, sol["x"]) == sol["xCx"]
        assert orc.qubo_energy(G, 0, sol["x"]) == sol["xGx"]
        assert orc.qubo_energy(G, pg, sol["x"]) == sol["g"]
        assert orc.constraint_direct(3, sol["x"]) == sol["g"]
        assert orc.cost_direct(ex["H"], ex["D"], sol["x"]) == sol["xCx"]


def _rand_flows(n, rng, symmetric=True, diag=False, neg=False):
    lo = -20 if neg else 0
    F = rng.integers(lo, 50, size=(n, n)).astype(np.int32)
    if symmetric:
        F = np.triu(F, 1)
        F = F + F.T
    if not diag:
        np.fill_diagonal(F, 0)
    return F.astype(np.int32)


def test_bruteforce_n4_all_states(orc):
    """Eqs. (nqap), (cqap), (gqap), (qubo): for all 2^16 states of an n = 4
    instance, x^T C x = c(x) and x^T G x + 2n = g(x); every permutation matrix has
    g = 0 and c = f(sigma); every other state has g > 0."""
    rng = np.random.default_rng(7)
    n, m = 4, 16
    H = _rand_flows(n, rng, symmetric=False, diag=True)
    D = _rand_flows(n, rng, symmetric=False, diag=True)
    C = orc.cost_qubo(H, D)
    G, pg = orc.constraint_qubo(n)
    perms = {}
    for p in itertools.permutations(range(n)):
        x = np.zeros(m, np.uint8)
        for i, u in enumerate(p):
            x[i * n + u] = 1
        perms[x.tobytes()] = p
    Cs = C.astype(np.int64)
    Gs = G.astype(np.int64)
    for bits in range(1 << m):
        x = np.array([(bits >> a) & 1 for a in range(m)], np.uint8)
        xi = x.astype(np.int64)
        c = int(xi @ Cs @ xi)
        g = int(xi @ Gs @ xi) + pg
        if bits % 4099 == 0:
            assert c == orc.cost_direct(H, D, x)
            assert g == orc.constraint_direct(n, x)
        key = x.tobytes()
        if key in perms:
            assert g == 0
            assert c == orc.qap_cost(H, D, list(perms[key]))
        else:
            assert g > 0
    # the quadruple-sum definitions on every permutation
    for key, p in perms.items():
        x = np.frombuffer(key, np.uint8)
        assert orc.cost_direct(H, D, x) == orc.qap_cost(H, D, list(p))
        assert orc.constraint_direct(n, x) == 0


def test_delta_energy_identity_exhaustive(orc):
    """Eq. (cale): E(x with bit a flipped) = E(x) + dE_a for every x and a
    (n = 3, all 512 states), for Y = C + alpha G and for a general non-symmetric Q."""
    rng = np.random.default_rng(3)
    n, m = 3, 9
    H = _rand_flows(n, rng, symmetric=False, diag=True)
    D = _rand_flows(n, rng, symmetric=False, diag=True)
    C = orc.cost_qubo(H, D)
    G, pg = orc.constraint_qubo(n)
    alpha = orc.penalty_2max(C)
    Y = C + alpha * G
    Qg = rng.integers(-30, 30, size=(m, m)).astype(np.int64)
    for Q, q in ((Y, alpha * pg), (Qg, 5)):
        for bits in range(1 << m):
            x = np.array([(bits >> a) & 1 for a in range(m)], np.uint8)
            dE = orc.delta_energy(Q, x)
            e0 = orc.qubo_energy(Q, q, x)
            for a in range(m):
                y = x.copy()
                y[a] ^= 1
                assert orc.qubo_energy(Q, q, y) - e0 == dE[a]


def test_delta_energy_identity_random(orc):
    rng = np.random.default_rng(11)
    for n in (5, 7):
        m = n * n
        H = _rand_flows(n, rng, symmetric=False, diag=True, neg=True)
        D = _rand_flows(n, rng, symmetric=False, diag=True)
        C = orc.cost_qubo(H, D)
        G, pg = orc.constraint_qubo(n)
        Y = C + 3 * G
        for _ in range(20):
            x = rng.integers(0, 2, size=m).astype(np.uint8)
            dE = orc.delta_energy(Y, x)
            e0 = orc.qubo_energy(Y, 3 * pg, x)
            for a in rng.choice(m, size=5, replace=False):
                y = x.copy()
                y[a] ^= 1
                assert orc.qubo_energy(Y, 3 * pg, y) - e0 == dE[a]


def test_penalty_vl_bruteforce(orc):
    """Eq. (vermap): w bounds the change of c(x) caused by one flip, and is attained."""
    rng = np.random.default_rng(5)
    n, m = 3, 9
    H = _rand_flows(n, rng, symmetric=False, diag=True, neg=True)
    D = _rand_flows(n, rng, symmetric=True, diag=False)
    C = orc.cost_qubo(H, D)
    w = orc.penalty_vl_w(C)
    best = -10**18
    for bits in range(1 << m):
        x = np.array([(bits >> a) & 1 for a in range(m)], np.uint8)
        dE = orc.delta_energy(C, x)
        best = max(best, int(np.max(np.abs(dE))))
    assert best == w


def test_build_matches_definition(orc):
    """The oracle's Y_k (upper triangle of P_k) equals C_k + alpha_k G with the
    per-objective 2max weight, and q_k = alpha_k * 2n (Eq. wqubom)."""
    rng = np.random.default_rng(2)
    n = 4
    F1 = _rand_flows(n, rng)
    F2 = _rand_flows(n, rng)
    D = _rand_flows(n, rng)
    q = orc.Qubo(F1, F2, D)
    G, pg = orc.constraint_qubo(n)
    for k, F in ((1, F1), (2, F2)):
        C = orc.cost_qubo(F, D)
        a = orc.penalty_2max(C)
        assert q.alpha[k - 1] == a
        assert np.array_equal(q.Y(k), C + a * G)
        assert q.q[k - 1] == a * pg
        P = q.P(k)
        assert np.array_equal(P, P.T)
    qv = orc.Qubo(F1, F2, D, penalty=orc.PEN_VL)
    C1 = orc.cost_qubo(F1, D)
    assert qv.alpha[0] == (orc.penalty_vl_w(C1) + 1) // 2
