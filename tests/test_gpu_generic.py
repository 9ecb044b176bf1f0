"""K objectives on a generic QUBO (the Conclusion's extension beyond two
objectives) on the GPU, bit for bit against the oracle's K-objective MDA.

  * every replica's trajectory, final state (x, K local fields, K energies,
    offset, moves) and raw archive, for K = 1..4, both acceptance rules, both
    archive methods and both escapes, at sizes from m = 2 to the largest each K
    takes, every slot count, ragged last lanes;
  * the merged non-dominated front over all replicas and each replica's own
    front against the front of the oracle's archives, and at scale (256
    replicas) against its definition over every raw archive entry;
  * a temperature table given as data;
  * properties at the largest sizes: energies of the final states and of every
    archived solution from Eq. (qubo) directly; the lenient rule with K copies
    of one QUBO runs the one-objective trajectory;
  * argument errors.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import decode_bits
from tests.oracle_jobs import run_greplicas

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _energies(Q, q, x):
    """E_k = x^T Q_k x + q_k (Eq. qubo), exact in int64."""
    xv = x.astype(np.int64)
    return [int(xv @ Q[k].astype(np.int64) @ xv) + int(q[k]) for k in range(Q.shape[0])]


def _run_both(mda, Q, q, R, steps, seed, accept=0, archive=0, escape=0, asize=0, xi=0.02, trace=True,
              picks=None, temp_table=None):
    K, m = Q.shape[0], Q.shape[1]
    print("generic case K=%d m=%d R=%d steps=%d seed=%d accept=%d archive=%d escape=%d s=%d"
          % (K, m, R, steps, seed, accept, archive, escape, asize), flush=True)
    g = mda.GQubo(Q, q)
    og = oracle.GQubo(Q, q)
    assert g.info() == dict(m=m, K=K, maxabs_c=og.maxabs_c)
    d0, df, _, _ = oracle.gdefault_schedule(og.maxabs_c, steps)
    beta = max(1, int(d0 // steps))
    run = mda.gda_run(g, mda.make_params(R, steps, seed, delta0=d0, deltaf=df, xi=xi, beta=beta, accept=accept,
                                         archive=archive, escape=escape, archive_size=asize,
                                         trace_replicas=R if trace else 0, temp_table=temp_table))
    run.sync()
    reps = list(range(R)) if picks is None else picks
    res = run_greplicas(Q, q, reps, steps=steps, delta0=d0, deltaf=df, xi=xi, beta=beta, seed=seed, accept=accept,
                        archive=archive, escape=escape, archive_size=asize, trace=trace, temp_table=temp_table)
    for r in reps:
        _compare(run, res[r], r, trace)
    return g, run, res


def _compare(run, o, r, trace):
    gs = run.state(r, trace=trace)
    tag = "K=%d m=%d replica %d" % (run.qubo.K, run.qubo.m, r)
    if trace:
        gt, ot = gs["trace"], o["trace"]
        if not np.array_equal(gt, ot):
            k = int(np.argmax(gt != ot))
            raise AssertionError("%s: trajectory differs first at step %d (gpu %d, oracle %d)" % (tag, k + 1, gt[k], ot[k]))
    assert np.array_equal(gs["x"], o["x"]), tag + ": x"
    assert np.array_equal(gs["h"], o["h"]), tag + ": h"
    assert (gs["E"], gs["Eoff"], gs["moves"]) == (o["E"], o["Eoff"], o["moves"]), tag
    a = run.archive(r, raw=True)
    assert len(a) == o["arch_size"], tag + ": archive size"
    assert np.array_equal(a.e, o["arch_e"]), tag + ": archive energies"
    assert np.array_equal(decode_bits(a.xbits, run.qubo.m), o["arch_x"]), tag + ": archive solutions"
    assert np.array_equal(a.slot, np.arange(len(a))) and np.all(a.replica == r)


CASES = [
    # K, m, accept, archive, escape, archive size, replicas, steps, density, rho
    (1, 2, 0, 0, 0, 0, 8, 300, 1.0, 0.0),
    (1, 7, 1, 1, 0, 3, 8, 1500, 1.0, 0.0),
    (2, 100, 1, 0, 0, 0, 16, 3000, 0.5, -0.5),
    (3, 300, 0, 1, 0, 9, 12, 3000, 0.3, 0.0),
    (4, 513, 1, 0, 1, 0, 8, 3000, 0.2, 0.5),
    (1, 600, 0, 1, 1, 20, 8, 4000, 0.1, 0.0),
    (2, 1030, 0, 0, 0, 0, 6, 4000, 0.05, 0.0),
    (3, 1024, 1, 1, 0, 0, 6, 3000, 0.05, 0.7),
    (4, 1024, 0, 0, 1, 0, 6, 3000, 0.05, 0.0),
    (1, 2100, 0, 0, 0, 0, 4, 3000, 0.02, 0.0),
    (2, 2048, 1, 1, 1, 40, 3, 2000, 0.02, -0.3),
    (1, 4096, 0, 0, 0, 0, 2, 1500, 0.01, 0.0),
]


@pytest.mark.parametrize("K,m,accept,archive,escape,asize,R,steps,density,rho", CASES)
def test_generic_parity(mda, K, m, accept, archive, escape, asize, R, steps, density, rho):
    Q, q = synth.make_gqubo(K, m, seed=1000 * K + m, density=density, rho=rho)
    _, run, res = _run_both(mda, Q, q, R, steps, 31 + m, accept, archive, escape, asize)
    assert sum(o["moves"] for o in res.values()) > 0


def _front(entries, K):
    """Non-dominated entries (E, replica, slot), equal vectors reduced to the lowest (replica, slot)."""
    best = {}
    for e, r, s in entries:
        key = tuple(int(v) for v in e)
        if key not in best or (r, s) < best[key]:
            best[key] = (r, s)
    keys = list(best)
    E = np.array(keys, np.int64).reshape(-1, K)
    keep = oracle.gnondominated(E)
    return sorted((keys[i], best[keys[i]]) for i in keep)


@pytest.mark.parametrize("K,accept,archive", [(2, 0, 0), (3, 1, 1), (4, 0, 1)])
def test_generic_fronts(mda, K, accept, archive):
    m, R, steps = 150, 24, 2500
    Q, q = synth.make_gqubo(K, m, seed=77 + K, density=0.4, rho=-0.3)
    _, run, res = _run_both(mda, Q, q, R, steps, 900 + K, accept, archive, 0, 12, trace=False)
    allent = []
    for r in range(R):
        ent = [(res[r]["arch_e"][i], r, i) for i in range(res[r]["arch_size"])]
        allent += ent
        mine = run.archive(r)
        want = _front(ent, K)
        got = sorted((tuple(int(v) for v in mine.e[i]), (int(mine.replica[i]), int(mine.slot[i])))
                     for i in range(len(mine)))
        assert got == want, r
    f = run.archive(-1)
    want = _front(allent, K)
    got = [(tuple(int(v) for v in f.e[i]), (int(f.replica[i]), int(f.slot[i]))) for i in range(len(f))]
    assert got == want                        # also in lexicographic order
    X = decode_bits(f.xbits, m)
    for i in range(len(f)):
        assert _energies(Q, q, X[i]) == list(got[i][0])


@pytest.mark.parametrize("K", [2, 3, 4])
def test_generic_merged_front_at_scale(mda, K):
    """The merged front of many replicas against its definition over every raw
    archive entry: no entry dominates a front entry, every entry is dominated
    by or equal to a front entry, equal energy vectors appear once with their
    lowest (replica, slot), sorted lexicographically."""
    m, R, steps = 512, 256, 20000
    Q, q = synth.make_gqubo(K, m, seed=600 + K, density=0.1, rho=-0.4)
    g = mda.GQubo(Q, q)
    print("generic front K=%d m=%d R=%d steps=%d" % (K, m, R, steps), flush=True)
    run = mda.gda_run(g, mda.make_params(R, steps, 17, xi=0.002, delta0=0.0))
    run.sync()
    E, key = [], []
    for r in range(R):
        a = run.archive(r, raw=True, bits=False)
        E.append(a.e)
        key.append(np.stack([np.full(len(a), r), np.arange(len(a))], axis=1))
    E = np.concatenate(E)
    key = np.concatenate(key)
    f = run.archive(-1)
    F = f.e
    assert len(F) > 10
    for i in range(len(F)):
        dom = np.all(E <= F[i], axis=1) & np.any(E < F[i], axis=1)
        assert not dom.any(), i
        same = np.all(E == F[i], axis=1)
        lowest = min(tuple(k) for k in key[same])
        assert (int(f.replica[i]), int(f.slot[i])) == lowest, i
    covered = np.zeros(len(E), bool)
    for i in range(len(F)):
        covered |= np.all(F[i] <= E, axis=1)
    assert covered.all()
    rows = [tuple(v) + (int(f.replica[i]), int(f.slot[i])) for i, v in enumerate(F.tolist())]
    assert rows == sorted(rows) and len({tuple(v) for v in F.tolist()}) == len(F)
    X = decode_bits(f.xbits, m)
    for i in range(0, len(F), max(1, len(F) // 16)):
        assert _energies(Q, q, X[i]) == [int(v) for v in F[i]]


def test_generic_temp_table(mda):
    K, m, R, steps = 2, 257, 8, 3000
    Q, q = synth.make_gqubo(K, m, seed=5, density=0.3)
    rng = np.random.default_rng(4)
    tt = np.sort(rng.integers(0, 40_000, steps))[::-1].astype(np.int64)
    tt[::97] = 0
    _run_both(mda, Q, q, R, steps, 11, accept=1, temp_table=tt)


@pytest.mark.parametrize("K,m,density", [(1, 4096, 0.01), (2, 2048, 0.02), (3, 1024, 0.05), (4, 1024, 0.05)])
def test_generic_energy_property_at_max_size(mda, K, m, density):
    """Energies of every final state and every archived solution from Eq.
    (qubo) directly, at the largest m each K takes and the full step count
    0.25 m^2 / 16 (a sixteenth of Table param's I_max)."""
    Q, q = synth.make_gqubo(K, m, seed=4242 + K, density=density)
    g = mda.GQubo(Q, q)
    R, steps = 64, m * m // 64
    print("generic property K=%d m=%d R=%d steps=%d" % (K, m, R, steps), flush=True)
    run = mda.gda_run(g, mda.make_params(R, steps, 3, xi=0.002, delta0=0.0))
    run.sync()
    for r in range(0, R, 9):
        s = run.state(r)
        assert s["E"] == _energies(Q, q, s["x"]), r
        a = run.archive(r, raw=True)
        X = decode_bits(a.xbits, m)
        for i in range(0, len(a), max(1, len(a) // 8)):
            assert list(a.e[i]) == _energies(Q, q, X[i]), (r, i)


def test_generic_lenient_copies_equal_one_objective(mda):
    """Lenient rule, K copies of one QUBO: the same trajectory as K = 1 (no oracle, full size)."""
    m, R, steps = 1024, 32, 20000
    Q1, q1 = synth.make_gqubo(1, m, seed=12, density=0.05)
    runs = []
    for K in (1, 3):
        g = mda.GQubo(np.concatenate([Q1] * K), np.repeat(q1, K))
        run = mda.gda_run(g, mda.make_params(R, steps, 8, accept=mda.LENIENT, trace_replicas=R, xi=0.003,
                                             delta0=0.0))
        run.sync()
        runs.append(run)
    for r in range(R):
        a, b = runs[0].state(r, trace=True), runs[1].state(r, trace=True)
        assert np.array_equal(a["trace"], b["trace"]), r
        assert b["E"] == [a["E"][0]] * 3 and a["moves"] == b["moves"], r


def test_generic_errors(mda):
    Q, q = synth.make_gqubo(1, 8, seed=1)
    for K, m in ((1, 4097), (2, 2049), (3, 1025), (4, 1025)):
        with pytest.raises(mda.MdaError) as e:
            mda.GQubo(np.zeros((K, m, m), np.int32))
        assert e.value.code == mda.MDA_EINVAL, (K, m)
    with pytest.raises(mda.MdaError) as e:
        mda.GQubo(np.zeros((5, 8, 8), np.int32))
    assert e.value.code == mda.MDA_EINVAL
    with pytest.raises(mda.MdaError) as e:
        mda.GQubo(np.zeros((1, 1, 1), np.int32))
    assert e.value.code == mda.MDA_EINVAL
    big = np.zeros((2, 8, 8), np.int32)
    big[1, 0, 1:] = 1 << 29                  # row 0 of P_2: 7 * 2^29 > 2^31 - 2
    with pytest.raises(mda.MdaError) as e:
        mda.GQubo(big)
    assert e.value.code == mda.MDA_EOVERFLOW
    g = mda.GQubo(Q, q)
    for kw in (dict(variant=mda.VARIANT_PLAIN), dict(waves_per_replica=2), dict(accept=7), dict(steps=0, replicas=0)):
        args = dict(replicas=2, steps=10)
        args.update({k: v for k, v in kw.items() if k in ("steps", "replicas")})
        extra = {k: v for k, v in kw.items() if k not in ("steps", "replicas")}
        with pytest.raises(mda.MdaError) as e:
            mda.gda_run(g, mda.make_params(args["replicas"], args["steps"], 1, **extra))
        assert e.value.code == mda.MDA_EINVAL, kw
    g3 = mda.GQubo(np.zeros((3, 64, 64), np.int32))
    with pytest.raises(mda.MdaError) as e:            # 5462 x 3 energies exceed a wave's LDS share
        mda.gda_run(g3, mda.make_params(2, 10, 1, archive_size=5462))
    assert e.value.code == mda.MDA_EINVAL
    run = mda.gda_run(g3, mda.make_params(2, 10, 1, archive_size=5461))   # the largest: one wave per block
    run.sync()
    run = mda.gda_run(g, mda.make_params(2, 10, 1))
    with pytest.raises(mda.MdaError):
        run.state(2)
    with pytest.raises(mda.MdaError):
        run.state(0, trace=True)             # not traced
    p = run.params
    assert p.steps == 10 and p.archive_size == 8 and p.delta0 == pytest.approx(1e9 * g.info()["maxabs_c"] / 2 ** 23)
