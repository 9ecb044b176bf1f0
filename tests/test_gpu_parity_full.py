"""Benchmark-sized runs against the oracle, in the launch configuration the
benchmark times.

  n = 25, rho = 0.75, 1024 replicas x 10^5 steps, dense and Kronecker updates:
      every replica bit-exact against the oracle (final state, raw archive),
      16 of them also step by step (whole trajectory); the two update paths
      identical on every replica.
  n = 50, rho in {-0.75, 0, 0.75}, 4096 replicas x 10^5 steps, the three
      instances in one persistent launch: 16 replicas per instance (0, 1,
      R - 1 and 13 seeded picks) bit-exact against the oracle (final state and
      raw archive); the merged front checked for the properties that hold at
      any size.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs, sample_replicas
from tests.oracle_jobs import run_replicas

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

STEPS = 100_000


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


# ---------------------------------------------------------------- n = 25

@pytest.fixture(scope="module")
def n25(mda):
    inst = synth.make_instance(25, 0.75, seed=synth.instance_seed(1, 0))
    R = 1024
    runs = {}
    for path in (1, 2):
        print("n=25 path=%d: %d replicas x %d steps" % (path, R, STEPS), flush=True)
        q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
        assert q.info().path == path
        run = mda.da_run(q, mda.make_params(R, STEPS, inst.seed, trace_replicas=R))
        run.sync()
        runs[path] = run
    picks = sample_replicas(R, extra=13, seed=25)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    print("n=25: oracle on all %d replicas" % R, flush=True)
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), **oracle_kwargs(oq, STEPS, inst.seed, trace=False))
    print("n=25: oracle trajectories of %d replicas" % len(picks), flush=True)
    traced = run_replicas(inst.F1, inst.F2, inst.D, picks, **oracle_kwargs(oq, STEPS, inst.seed))
    return inst, R, runs, res, traced


@pytest.mark.parametrize("path", [1, 2])
def test_n25_all_replicas(n25, path):
    inst, R, runs, res, traced = n25
    assert len(res) == R
    for r in range(R):
        compare_replica(runs[path], res[r], r, trace=False, label="n=25 path=%d" % path)


@pytest.mark.parametrize("path", [1, 2])
def test_n25_sampled_trajectories(n25, path):
    inst, R, runs, res, traced = n25
    assert len(traced) == 16
    for r, o in traced.items():
        compare_replica(runs[path], o, r, label="n=25 path=%d" % path)


def test_n25_dense_equals_kronecker(n25):
    inst, R, runs, res, traced = n25
    for r in range(R):
        a, b = runs[1].state(r, trace=True), runs[2].state(r, trace=True)
        assert np.array_equal(a["trace"], b["trace"]), r
        assert (a["E1"], a["E2"], a["Eoff"], a["moves"]) == (b["E1"], b["E2"], b["Eoff"], b["moves"]), r
        assert np.array_equal(a["h1"], b["h1"]) and np.array_equal(a["h2"], b["h2"]), r
    fa, fb = runs[1].archive(-1), runs[2].archive(-1)
    assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2)
    assert np.array_equal(fa.replica, fb.replica) and np.array_equal(fa.slot, fb.slot)
    assert np.array_equal(fa.xbits, fb.xbits)


def test_n25_front_equals_union_of_archives(n25):
    """The merged front (filtered on the device, merged on the host) equals the
    non-dominated set of the union of every replica's raw archive."""
    inst, R, runs, res, traced = n25
    e1, e2, rep, slot = [], [], [], []
    for r in range(R):
        a = runs[2].archive(r, raw=True, bits=False)
        e1.append(a.e1)
        e2.append(a.e2)
        rep.append(np.full(len(a), r, np.int64))
        slot.append(np.arange(len(a), dtype=np.int64))
    e1, e2, rep, slot = map(np.concatenate, (e1, e2, rep, slot))
    order = np.lexsort((slot, rep, e2, e1))
    best = np.iinfo(np.int64).max
    keep = []
    for k in order:
        if e2[k] < best:
            keep.append(k)
            best = e2[k]
    f = runs[2].archive(-1, bits=False)
    assert np.array_equal(f.e1, e1[keep]) and np.array_equal(f.e2, e2[keep])
    assert np.array_equal(f.replica, rep[keep]) and np.array_equal(f.slot, slot[keep])


# ---------------------------------------------------------------- n = 50

@pytest.fixture(scope="module")
def n50(mda):
    insts = [synth.make_instance(50, rho, seed=synth.instance_seed(2, k))
             for k, rho in enumerate((-0.75, 0.0, 0.75))]
    R = 4096
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=2) for i in insts]
    ps = [mda.make_params(R, STEPS, i.seed) for i in insts]
    print("n=50: 3 instances x %d replicas x %d steps in one launch" % (R, STEPS), flush=True)
    runs = mda.da_run_batch(qs, ps)
    for r in runs:
        r.sync()
    print("n=50: device %.1f ms" % runs[0].elapsed_ms(), flush=True)
    return insts, R, qs, runs


@pytest.mark.parametrize("k", [0, 1, 2])
def test_n50_sampled_replicas(n50, k):
    insts, R, qs, runs = n50
    inst = insts[k]
    picks = sample_replicas(R, extra=13, seed=50 + k)
    assert len(picks) == 16
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    res = run_replicas(inst.F1, inst.F2, inst.D, picks, **oracle_kwargs(oq, STEPS, inst.seed, trace=False))
    for r, o in res.items():
        compare_replica(runs[k], o, r, trace=False, label="n=50 instance %d" % k)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_n50_merged_front(n50, k):
    """The merged front is sorted, mutually non-dominated, made of raw archive
    entries, and weakly dominates every archive entry of sampled replicas."""
    insts, R, qs, runs = n50
    run = runs[k]
    f = run.archive(-1)
    assert len(f) > 0
    assert np.all(np.diff(f.e1) > 0) and np.all(np.diff(f.e2) < 0)
    for r in sample_replicas(R, extra=5, seed=500 + k):
        a = run.archive(r, raw=True, bits=False)
        for e1, e2 in zip(a.e1, a.e2):
            assert np.any((f.e1 <= e1) & (f.e2 <= e2)), (r, e1, e2)
    for idx in range(0, len(f), max(1, len(f) // 8)):
        r, s = int(f.replica[idx]), int(f.slot[idx])
        a = run.archive(r, raw=True)
        assert (a.e1[s], a.e2[s]) == (f.e1[idx], f.e2[idx])
        assert np.array_equal(a.xbits[s], f.xbits[idx])
