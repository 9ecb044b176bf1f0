"""The workgroup form (one replica over several waves) against the oracle.

Instances beyond one wave's 64 locations (n = 65 .. 100: 2 x 2 waves) and
smaller ones forced onto 2 to 4 waves, on both update paths and in every mode;
every replica's trajectory, final state and raw archive bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs
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


CASES = [
    # n, path, waves per replica (0 = automatic), accept, archive, escape, archive size
    (9, 2, 2, 0, 0, 0, 0),
    (33, 2, 3, 1, 1, 0, 0),
    (50, 2, 2, 0, 0, 0, 0),
    (50, 1, 4, 0, 0, 1, 30),
    (65, 2, 0, 0, 0, 0, 0),
    (80, 1, 0, 1, 0, 0, 0),
    (100, 2, 0, 0, 0, 0, 0),
    (100, 2, 4, 0, 1, 1, 50),
]


@pytest.mark.parametrize("n,path,wpr,accept,archive,escape,asize", CASES)
def test_group_against_oracle(mda, n, path, wpr, accept, archive, escape, asize):
    R, steps, seed = 3, 2000, 500 + n
    inst = synth.make_instance(n, 0.25, seed=seed)
    print("group case n=%d path=%d waves=%d modes=%d%d%d s=%d" % (n, path, wpr, accept, archive, escape, asize),
          flush=True)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
    run = mda.da_run(q, mda.make_params(R, steps, seed, trace_replicas=R, waves_per_replica=wpr, accept=accept,
                                        archive=archive, escape=escape, archive_size=asize))
    run.sync()
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    okw = oracle_kwargs(oq, steps, seed, accept=accept, archive=archive, escape=escape, archive_size=asize)
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), workers=min(R, 3), **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="group n=%d waves=%d" % (n, wpr))


def test_group_equals_one_wave(mda):
    """n = 40 on one wave and on 2 and 4 waves: identical replicas and fronts."""
    inst = synth.make_instance(40, -0.5, seed=40)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=2)
    runs = [mda.da_run(q, mda.make_params(16, 3000, 41, trace_replicas=16, waves_per_replica=w)) for w in (1, 2, 4)]
    for r in range(16):
        ref = runs[0].state(r, trace=True)
        for run in runs[1:]:
            g = run.state(r, trace=True)
            assert np.array_equal(g["trace"], ref["trace"]) and np.array_equal(g["x"], ref["x"]), r
            assert np.array_equal(g["h1"], ref["h1"]) and np.array_equal(g["h2"], ref["h2"]), r
    f0 = runs[0].archive(-1)
    for run in runs[1:]:
        f = run.archive(-1)
        assert np.array_equal(f.e1, f0.e1) and np.array_equal(f.xbits, f0.xbits)


def test_mixed_layouts_in_one_batch(mda):
    """One-wave and workgroup runs in one batch give their separate results."""
    insts = [synth.make_instance(n, 0.0, seed=700 + n) for n in (12, 70, 30)]
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=2) for i in insts]
    ps = [mda.make_params(4, 1500, 800 + k, trace_replicas=4, waves_per_replica=(2 if k == 2 else 0))
          for k in range(3)]
    runs = mda.da_run_batch(qs, ps)
    for k, (q, p) in enumerate(zip(qs, ps)):
        alone = mda.da_run(q, mda.make_params(4, 1500, 800 + k, trace_replicas=4,
                                              waves_per_replica=(2 if k == 2 else 0)))
        for r in range(4):
            assert np.array_equal(alone.state(r, trace=True)["trace"], runs[k].state(r, trace=True)["trace"])
