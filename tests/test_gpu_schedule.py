"""The schedule as input data (Table param): mda_params.temp_table replaces the
geometric cooling of delta0, deltaf and xi.

  - the oracle's own geometric table fed to both sides gives the oracle's run
    and the library's default run, bit for bit;
  - a schedule that is not geometric (cooling with periodic reheating, and a
    stretch at temperature 0) fed to both sides gives identical trajectories,
    final states and raw archives, on both update paths.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs
from tests.oracle_jobs import run_replicas

pytestmark = pytest.mark.gpu

R, STEPS = 8, 4000


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _both(mda, inst, table, path, seed):
    print("case n=%d path=%d seed=%d table[0]=%d" % (inst.n, path, seed, int(table[0])), flush=True)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    okw = oracle_kwargs(oq, STEPS, seed)
    run = mda.da_run(q, mda.make_params(R, STEPS, seed, trace_replicas=R, beta=okw["beta"], temp_table=table))
    run.sync()
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), temp_table=table, **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="n=%d path=%d" % (inst.n, path))
    return q, run


@pytest.mark.parametrize("path", [1, 2])
def test_oracle_table_equals_default(mda, path):
    inst = synth.make_instance(12, 0.4, seed=1212)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    d0, df, xi, beta = oracle.default_schedule(oq.maxabs_c, STEPS)
    table = oracle.temperature(d0, df, xi, STEPS)
    q, run = _both(mda, inst, table, path, 77)
    plain = mda.da_run(q, mda.make_params(R, STEPS, 77, trace_replicas=R))
    for r in range(R):
        a, b = run.state(r, trace=True), plain.state(r, trace=True)
        assert np.array_equal(a["trace"], b["trace"]) and (a["E1"], a["E2"]) == (b["E1"], b["E2"])
    assert run.params.temp_table is None


@pytest.mark.parametrize("path", [1, 2])
def test_reheating_schedule(mda, path):
    inst = synth.make_instance(11, -0.2, seed=1111)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    d0, df, xi, _ = oracle.default_schedule(oq.maxabs_c, STEPS)
    t = np.arange(STEPS)
    # geometric cooling restarted every 1000 steps, then 300 steps at T = 0
    table = np.floor(d0 * 256.0 * 0.995 ** (t % 1000)).astype(np.int64)
    table[2000:2300] = 0
    _both(mda, inst, table, path, 91)
