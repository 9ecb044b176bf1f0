"""Many instances of uneven size in one graph launch, against the oracle.

256 bQAP instances, n uniform on {10..60}, rho uniform on [-0.75, 0.75]
(synth.mixed_batch), 64 replicas x 10^5 steps each, Kronecker updates, all in
one da_run_batch captured as a HIP graph (one persistent launch per register
tile).  Checked: sampled replicas of sampled instances bit-exact against the
oracle; the same instances run alone (same seeds, direct launch) give the same
replicas and fronts; the whole batch launched directly gives the same results
as the graph.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs, sample_replicas
from tests.oracle_jobs import run_replicas

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

STEPS = 100_000
R = 64


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _launch(mda, insts, qs, graph, stream):
    ps = [mda.make_params(R, STEPS, i.seed, graph=graph, stream=stream) for i in insts]
    runs = mda.da_run_batch(qs, ps)
    for r in runs:
        r.sync()
    return runs


@pytest.fixture(scope="module")
def batch(mda):
    import torch
    insts = synth.mixed_batch()
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=mda.PATH_KRON) for i in insts]
    stream = torch.cuda.Stream()
    print("mixed batch: %d instances, n in [%d, %d], %d replicas x %d steps, graph launch"
          % (len(insts), min(i.n for i in insts), max(i.n for i in insts), R, STEPS), flush=True)
    runs = _launch(mda, insts, qs, True, stream.cuda_stream)
    print("mixed batch: graph %.1f ms" % runs[0].kernel_ms(), flush=True)
    return insts, qs, runs, stream


def _picks(insts, count=10, seed=3):
    ns = [i.n for i in insts]
    rng = np.random.default_rng(seed)
    picks = {int(np.argmin(ns)), int(np.argmax(ns))}
    while len(picks) < count:
        picks.add(int(rng.integers(0, len(insts))))
    return sorted(picks)


def test_sampled_instances_against_oracle(batch):
    """12 instances (the smallest, the largest and 10 seeded picks), 16
    replicas each (0, 1, R - 1 and 13 seeded picks)."""
    insts, qs, runs, _ = batch
    for k in _picks(insts, count=12):
        inst = insts[k]
        oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
        reps = sample_replicas(R, extra=13, seed=300 + k)
        assert len(reps) == 16
        res = run_replicas(inst.F1, inst.F2, inst.D, reps, **oracle_kwargs(oq, STEPS, inst.seed, trace=False))
        for r in reps:
            compare_replica(runs[k], res[r], r, trace=False, label="batch instance %d (n=%d)" % (k, inst.n))


def test_alone_equals_batched(mda, batch):
    insts, qs, runs, stream = batch
    for k in _picks(insts, count=6, seed=4):
        alone = mda.da_run(qs[k], mda.make_params(R, STEPS, insts[k].seed, stream=stream.cuda_stream))
        alone.sync()
        for r in range(R):
            a, b = alone.state(r), runs[k].state(r)
            assert (a["E1"], a["E2"], a["Eoff"], a["moves"]) == (b["E1"], b["E2"], b["Eoff"], b["moves"]), (k, r)
            assert np.array_equal(a["x"], b["x"]), (k, r)
        fa, fb = alone.archive(-1), runs[k].archive(-1)
        assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2) and np.array_equal(fa.xbits, fb.xbits)


def test_direct_launch_equals_graph(mda, batch):
    insts, qs, runs, stream = batch
    direct = _launch(mda, insts, qs, False, stream.cuda_stream)
    for k in range(len(insts)):
        assert direct[k].stats() == runs[k].stats(), k
        fa, fb = direct[k].archive(-1, bits=False), runs[k].archive(-1, bits=False)
        assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2), k
        assert np.array_equal(fa.replica, fb.replica) and np.array_equal(fa.slot, fb.slot), k


def test_graph_needs_created_stream(mda, batch):
    insts, qs, _, _ = batch
    with pytest.raises(mda.MdaError) as e:
        mda.da_run(qs[0], mda.make_params(2, 10, 1, graph=True, stream=0))
    assert e.value.code == mda.MDA_EINVAL
