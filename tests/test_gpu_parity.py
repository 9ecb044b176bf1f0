"""GPU (HIP through the C ABI) against the CPU oracle, bit for bit.

Every case is seeded and synthetic (see synth/).  Small cases compare every
replica's whole trajectory; the benchmark-sized cases run at full size in the
benchmark's launch configuration and compare a deterministic replica sample.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs, sample_replicas
from tests.oracle_jobs import run_replicas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _run(mda, inst, R, steps, seed, path=0, trace=None, **kw):
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path, penalty=kw.pop("penalty", 0))
    p = mda.make_params(R, steps, seed, trace_replicas=R if trace is None else trace, **kw)
    run = mda.da_run(q, p)
    run.sync()
    return q, run


def _check_all(mda, inst, R, steps, seed, path=0, penalty=0, **kw):
    q, run = _run(mda, inst, R, steps, seed, path=path, penalty=penalty, **kw)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D, penalty)
    okw = oracle_kwargs(oq, steps, seed, accept=kw.get("accept", 0), archive=kw.get("archive", 0),
                        escape=kw.get("escape", 0), archive_size=kw.get("archive_size", 0))
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), penalty=penalty, **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="n=%d path=%d" % (inst.n, path))
    return q, run, res


@pytest.mark.parametrize("path", [1, 2])
def test_plain_config_n8_all_replicas(mda, path):
    """n = 8 (64 bits), uniform flows, 16 replicas x 10^4 steps, seed 0; dense and Kronecker."""
    inst = synth.make_instance(8, 0.0, seed=0, structured=False)
    q, run, res = _check_all(mda, inst, 16, 10000, 0, path=path)
    assert q.info().path == path


@pytest.mark.parametrize("n,path,accept,archive,escape,asize", [
    (5, 1, 1, 0, 0, 0), (5, 2, 0, 1, 0, 6), (6, 2, 0, 0, 1, 8), (11, 1, 1, 1, 1, 12),
    (11, 2, 0, 0, 0, 5), (13, 2, 1, 1, 0, 0), (17, 1, 0, 0, 1, 0), (3, 2, 0, 1, 1, 3)])
def test_modes(mda, n, path, accept, archive, escape, asize):
    inst = synth.make_instance(n, 0.3, seed=100 + n)
    _check_all(mda, inst, 6, 2500, 7 + n, path=path, accept=accept, archive=archive, escape=escape,
               archive_size=asize)


@pytest.mark.parametrize("n,path,accept,archive,escape", [
    (5, 1, 0, 0, 0), (9, 2, 1, 0, 0), (17, 2, 0, 1, 1), (24, 1, 1, 1, 0), (33, 2, 0, 0, 1), (50, 2, 1, 0, 0),
    (64, 1, 0, 0, 0)])
def test_final_temperature_thresholds(mda, n, path, accept, archive, escape):
    """A fast schedule (xi = 0.02) that reaches its final temperature after a
    few hundred steps: most steps take their thresholds from the table of the
    final temperature in LDS; every replica against the oracle."""
    inst = synth.make_instance(n, -0.3, seed=300 + n)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D, 0)
    steps, seed = 3000, 40 + n
    d0, df, _, _ = oracle.default_schedule(oq.maxabs_c, steps)
    beta = max(1, int(d0 // steps))
    R = 6 if n < 40 else 3
    q, run = _run(mda, inst, R, steps, seed, path=path, delta0=d0, deltaf=df, xi=0.02, beta=beta, accept=accept,
                  archive=archive, escape=escape)
    assert run.params.steps == steps
    okw = oracle_kwargs(oq, steps, seed, accept=accept, archive=archive, escape=escape,
                        schedule=(d0, df, 0.02, beta))
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="n=%d path=%d xi=0.02" % (n, path))


@pytest.mark.parametrize("n,path,accept,general", [
    (49, 1, 0, False), (52, 2, 1, False), (51, 2, 0, True), (52, 1, 1, True), (53, 2, 0, False),
    (25, 2, 0, False), (28, 1, 1, False), (27, 2, 1, True), (29, 2, 0, False)])
def test_half_group_slot_tiles(mda, n, path, accept, general):
    """25 to 28 and 49 to 52 facilities run on 28 and 52 register slots,
    whose last group of 8 holds 4 (29 and 53 go to 32 and 56): dense and
    Kronecker columns, both rules, the two-product column on non-symmetric
    operands; every replica against the oracle, full trajectories."""
    if general:
        rng = np.random.default_rng(n)
        F1, F2 = (rng.integers(0, 40, size=(n, n)).astype(np.int32) for _ in range(2))
        D = rng.integers(0, 60, size=(n, n)).astype(np.int32)
        inst = synth.Instance(n, F1, F2, D, 0.0, 0)
    else:
        inst = synth.make_instance(n, 0.4, seed=520 + n)
    q, run, _ = _check_all(mda, inst, 3, 2000, 52 + n, path=path, accept=accept)
    want = {25: 28, 27: 28, 28: 28, 29: 32, 53: 56}.get(n, 52)
    assert mda.run_layout(q, mda.make_params(3, 2000, 52 + n)).gns == want
    assert q.info().symmetric == (0 if general else 1)


@pytest.mark.parametrize("n", [4, 7, 9])
def test_general_kronecker_nonsymmetric(mda, n):
    """Non-symmetric flows and distances with non-zero diagonals (two-product column)."""
    rng = np.random.default_rng(n)
    F1 = rng.integers(0, 60, size=(n, n)).astype(np.int32)
    F2 = rng.integers(0, 60, size=(n, n)).astype(np.int32)
    D = rng.integers(0, 90, size=(n, n)).astype(np.int32)
    inst = synth.Instance(n, F1, F2, D, 0.0, 0)
    for path in (1, 2):
        q, run, _ = _check_all(mda, inst, 4, 2000, 3, path=path)
        assert q.info().symmetric == 0


def test_vl_penalty(mda):
    inst = synth.make_instance(6, -0.5, seed=9)
    _check_all(mda, inst, 4, 2000, 11, path=2, penalty=1)


@pytest.mark.parametrize("penalty", [0, 1])
def test_negative_entries(mda, penalty):
    """Flows and distances of both signs: the builder's general scans (penalty
    weight and field bound) against the oracle's, on both update paths."""
    rng = np.random.default_rng(60 + penalty)
    n = 7
    F1 = rng.integers(-40, 60, size=(n, n)).astype(np.int32)
    F2 = rng.integers(-50, 50, size=(n, n)).astype(np.int32)
    D = rng.integers(-20, 90, size=(n, n)).astype(np.int32)
    inst = synth.Instance(n, F1, F2, D, 0.0, 0)
    for path in (1, 2):
        q, run, _ = _check_all(mda, inst, 4, 2000, 5 + penalty, path=path, penalty=penalty)
        oq = oracle.Qubo(F1, F2, D, penalty)
        assert (q.info().alpha1, q.info().alpha2) == (oq.alpha[0], oq.alpha[1])


@pytest.mark.parametrize("path", [1, 2])
def test_plain_form_against_oracle(mda, path):
    """The plain form (one launch per annealing step, state in HBM) on the
    n = 8 configuration (16 replicas x 10^4 steps, seed 0), every replica
    bit-exact against the oracle: trajectory, final state, raw archive."""
    inst = synth.make_instance(8, 0.0, seed=0, structured=False)
    _check_all(mda, inst, 16, 10000, 0, path=path, variant=mda.VARIANT_PLAIN)


def test_plain_form_equals_persistent(mda):
    inst = synth.make_instance(9, 0.0, seed=5)
    steps, R = 1200, 5
    _, a = _run(mda, inst, R, steps, 21, path=2)
    _, b = _run(mda, inst, R, steps, 21, path=2, variant=mda.VARIANT_PLAIN)
    for r in range(R):
        sa, sb = a.state(r, trace=True), b.state(r, trace=True)
        assert np.array_equal(sa["trace"], sb["trace"])
        assert (sa["E1"], sa["E2"], sa["Eoff"]) == (sb["E1"], sb["E2"], sb["Eoff"])
        ea, eb = a.archive(r, raw=True), b.archive(r, raw=True)
        assert np.array_equal(ea.e1, eb.e1) and np.array_equal(ea.xbits, eb.xbits)


@pytest.mark.parametrize("path,accept,general", [(1, 0, False), (1, 1, False), (2, 0, False), (2, 1, False),
                                                   (2, 0, True), (2, 1, True)])
def test_plain_form_every_step_variant(mda, path, accept, general):
    """The plain form's step kernel is built per step variant (update path x
    acceptance rule; the general Kronecker column for non-symmetric factors):
    each build against the oracle, every replica, trajectory included."""
    n = 9
    if general:
        rng = np.random.default_rng(90 + accept)
        F1 = rng.integers(0, 60, size=(n, n)).astype(np.int32)
        F2 = rng.integers(0, 60, size=(n, n)).astype(np.int32)
        D = rng.integers(0, 90, size=(n, n)).astype(np.int32)
        inst = synth.Instance(n, F1, F2, D, 0.0, 0)
    else:
        inst = synth.make_instance(n, 0.4, seed=90 + accept)
    q, run, _ = _check_all(mda, inst, 4, 1500, 13 + accept, path=path, accept=accept,
                           variant=mda.VARIANT_PLAIN)
    assert q.info().symmetric == (0 if general else 1)


def test_launch_shape_invariance(mda):
    inst = synth.make_instance(10, 0.5, seed=6)
    outs = []
    for wpb in (1, 2, 3, 4, 8):
        _, run = _run(mda, inst, 9, 1500, 4, path=2, waves_per_block=wpb)
        outs.append([run.state(r, trace=True)["trace"] for r in range(9)])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_batch_equals_single(mda):
    """Instances of different sizes in one launch give the results of separate runs."""
    insts = [synth.make_instance(n, 0.2, seed=40 + n) for n in (7, 12, 20, 3)]
    steps = 1500
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=1 + (k % 2)) for k, i in enumerate(insts)]
    ps = [mda.make_params(3 + k, steps, 1000 + k, trace_replicas=3 + k) for k in range(len(insts))]
    runs = mda.da_run_batch(qs, ps)
    for k, (inst, run) in enumerate(zip(insts, runs)):
        run.sync()
        oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
        okw = oracle_kwargs(oq, steps, 1000 + k)
        res = run_replicas(inst.F1, inst.F2, inst.D, range(3 + k), **okw)
        for r in range(3 + k):
            compare_replica(run, res[r], r, label="batch %d" % k)


@pytest.mark.parametrize("pair", [(50, 54), (26, 31)])
def test_half_tile_joins_full_tile_in_a_batch(mda, pair):
    """Beside a run of 54 (31) facilities with the same variant, a run of 50
    (26) goes on 56 (32) slots instead of 52 (28): one launch, not two; alone
    it keeps the smaller tile.  All replicas of both, and of the lone run,
    against the oracle."""
    insts = [synth.make_instance(n, 0.1, seed=60 + n) for n in pair]
    steps = 1500
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=2) for i in insts]
    ps = [mda.make_params(3, steps, 2000 + k, trace_replicas=3) for k in range(2)]
    runs = mda.da_run_batch(qs, ps)
    alone = mda.da_run(qs[0], ps[0])
    alone.sync()
    for k, (inst, run) in enumerate(zip(insts, runs)):
        run.sync()
        okw = oracle_kwargs(oracle.Qubo(inst.F1, inst.F2, inst.D), steps, 2000 + k)
        res = run_replicas(inst.F1, inst.F2, inst.D, range(3), **okw)
        for r in range(3):
            compare_replica(run, res[r], r, label="batch n=%d" % inst.n)
            if k == 0:
                compare_replica(alone, res[r], r, label="alone n=%d" % inst.n)


def test_merged_archive(mda):
    """archive_get(-1): non-dominated union over replicas, duplicates dropped, sorted."""
    inst = synth.make_instance(8, 0.0, seed=0, structured=False)
    steps, R = 3000, 16
    q, run = _run(mda, inst, R, steps, 0, path=1, trace=0)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), **oracle_kwargs(oq, steps, 0, trace=False))
    pts = {}
    for r in range(R):
        for s, (e1, e2) in enumerate(zip(res[r]["arch_e1"], res[r]["arch_e2"])):
            pts.setdefault((int(e1), int(e2)), (r, s))
    keys = list(pts)
    nd = sorted(k for k in keys if not any(oracle.dominates(o, k) for o in keys))
    got = run.archive(-1)
    assert [(int(a), int(b)) for a, b in zip(got.e1, got.e2)] == nd
    assert [(int(r), int(s)) for r, s in zip(got.replica, got.slot)] == [pts[k] for k in nd]
    for k in range(len(got)):
        x = np.array([(got.xbits[k, a >> 5] >> (a & 31)) & 1 for a in range(64)], np.uint8)
        assert got.feasible[k] == (oracle.constraint_direct(8, x) == 0)


def test_free_after_allocator_reinstalled(mda):
    """A run allocated before the allocator is installed again is released
    through the callbacks it was allocated with."""
    import gc
    inst = synth.make_instance(5, 0.0, seed=1)
    q, run = _run(mda, inst, 2, 50, 1, trace=0)
    mda.use_hip_allocator()
    mda.use_torch_allocator()
    del run, q
    gc.collect()
