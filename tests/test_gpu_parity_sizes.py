"""GPU against the oracle across problem sizes: the smallest instance, the
benchmark sizes (n = 25, 50) on short runs, a ragged register tile (n = 33)
and the largest instance one wave holds (n = 64).  Every replica's whole
trajectory, final state and raw archive are compared bit for bit."""
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


def _check(mda, inst, R, steps, seed, path, **kw):
    print("case n=%d rho=%g seed=%d path=%d R=%d steps=%d %s" % (inst.n, inst.rho, seed, path, R, steps, kw),
          flush=True)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
    run = mda.da_run(q, mda.make_params(R, steps, seed, trace_replicas=R, **kw))
    run.sync()
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    okw = oracle_kwargs(oq, steps, seed, accept=kw.get("accept", 0), archive=kw.get("archive", 0),
                        escape=kw.get("escape", 0), archive_size=kw.get("archive_size", 0))
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="n=%d path=%d" % (inst.n, path))
    return run, res


def test_n2_smallest(mda):
    inst = synth.make_instance(2, 0.0, seed=2)
    for path in (1, 2):
        _check(mda, inst, 5, 500, 3, path)


@pytest.mark.parametrize("path", [1, 2])
def test_n25_short(mda, path):
    inst = synth.make_instance(25, 0.75, seed=synth.instance_seed(1, 0))
    _check(mda, inst, 6, 4000, inst.seed, path)


def test_n33_ragged(mda):
    inst = synth.make_instance(33, -0.3, seed=33)
    _check(mda, inst, 4, 3000, 33, 2, accept=1, archive=1)


@pytest.mark.parametrize("rho_idx", [0, 1, 2])
def test_n50_short(mda, rho_idx):
    rho = (-0.75, 0.0, 0.75)[rho_idx]
    inst = synth.make_instance(50, rho, seed=synth.instance_seed(2, rho_idx))
    run, res = _check(mda, inst, 4, 3000, inst.seed, 2)
    assert sum(r["moves"] for r in res.values()) > 0


def test_n50_escape_archive(mda):
    inst = synth.make_instance(50, 0.0, seed=synth.instance_seed(2, 1))
    _check(mda, inst, 3, 3000, 77, 2, escape=1, archive_size=40)


def test_n64_largest(mda):
    inst = synth.make_instance(64, 0.5, seed=64)
    _check(mda, inst, 3, 2000, 64, 2)


def test_n101_rejected(mda):
    inst = synth.make_instance(101, 0.0, seed=101)
    with pytest.raises(mda.MdaError) as e:
        mda.Qubo(inst.F1, inst.F2, inst.D)
    assert e.value.code == mda.MDA_EINVAL


def test_one_wave_beyond_64_rejected(mda):
    inst = synth.make_instance(65, 0.0, seed=65)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=2)
    with pytest.raises(mda.MdaError) as e:
        mda.da_run(q, mda.make_params(2, 10, 1, waves_per_replica=1))
    assert e.value.code == mda.MDA_EINVAL
