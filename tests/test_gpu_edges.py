"""Edge cases of the GPU path against the oracle.

  - the smallest run: one replica, one step;
  - a one-entry archive, in both archive methods and both escapes;
  - the default step count (0 selects m^2 / 4, Table param), with a trace sized
    from the parameters the library resolved;
  - degenerate instances: every flow zero (both objectives vanish, only the
    penalty is left), and equal objectives (F1 = F2, so e1 = e2 on every state
    and the merged front is a single point);
  - the argument errors of da_run, da_state_get and archive_get (including a
    step count of 2^32 - 1 and temperature tables out of range).
Every replica's trajectory, final state and raw archive are compared bit for bit.
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


def _check(mda, F1, F2, D, R, steps, seed, path=2, oracle_steps=None, schedule=None, **kw):
    n = D.shape[0]
    print("case n=%d R=%d steps=%d seed=%d path=%d schedule=%s %s" % (n, R, steps, seed, path, schedule, kw),
          flush=True)
    q = mda.Qubo(F1, F2, D, path=path)
    if schedule:
        kw.update(zip(("delta0", "deltaf", "xi", "beta"), schedule))
    run = mda.da_run(q, mda.make_params(R, steps, seed, trace_replicas=R, **kw))
    run.sync()
    oq = oracle.Qubo(F1, F2, D)
    okw = oracle_kwargs(oq, oracle_steps or steps, seed, accept=kw.get("accept", 0), archive=kw.get("archive", 0),
                        escape=kw.get("escape", 0), archive_size=kw.get("archive_size", 0), schedule=schedule)
    res = run_replicas(F1, F2, D, range(R), **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="n=%d" % n)
    return run, res


@pytest.mark.parametrize("path", [1, 2])
def test_one_replica_one_step(mda, path):
    inst = synth.make_instance(6, 0.2, seed=601)
    run, res = _check(mda, inst.F1, inst.F2, inst.D, 1, 1, 602, path=path)
    assert run.state(0, trace=True)["trace"].shape == (1,)


@pytest.mark.parametrize("archive,escape", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_archive_of_one_entry(mda, archive, escape):
    inst = synth.make_instance(7, -0.5, seed=701)
    mx = oracle.Qubo(inst.F1, inst.F2, inst.D).maxabs_c
    # cool enough that a fifth of the steps move (the default schedule, made
    # for 10^5 steps and more, accepts every flip this early)
    run, res = _check(mda, inst.F1, inst.F2, inst.D, 4, 3000, 702 + 2 * archive + escape,
                      schedule=(4.0 * mx, mx / 8.0, 0.002, 1), archive=archive, escape=escape, archive_size=1)
    for r in range(4):
        assert len(run.archive(r, raw=True, bits=False)) == 1
        assert 0 < res[r]["moves"] < 3000


def test_default_step_count(mda):
    inst = synth.make_instance(4, 0.0, seed=401)
    m = inst.m
    run, res = _check(mda, inst.F1, inst.F2, inst.D, 3, 0, 402, oracle_steps=m * m // 4)
    p = run.params
    assert p.steps == m * m // 4 and p.archive_size == m and p.waves_per_replica == 1
    d0, df, xi, beta = oracle.default_schedule(oracle.Qubo(inst.F1, inst.F2, inst.D).maxabs_c, m * m // 4)
    assert (p.delta0, p.deltaf, p.xi, p.beta) == (d0, df, xi, beta)
    assert run.state(2, trace=True)["trace"].shape == (m * m // 4,)


@pytest.mark.parametrize("path", [1, 2])
def test_zero_flows(mda, path):
    inst = synth.make_instance(5, 0.0, seed=501)
    Z = np.zeros_like(inst.F1)
    run, res = _check(mda, Z, Z, inst.D, 4, 2000, 502, path=path)
    for r in range(4):
        a = run.archive(r, raw=True, bits=False)
        assert np.array_equal(a.e1, a.e2)


def test_equal_objectives(mda):
    inst = synth.make_instance(9, 0.0, seed=901)
    run, res = _check(mda, inst.F1, inst.F1, inst.D, 8, 4000, 902)
    lows = []
    for r in range(8):
        a = run.archive(r, raw=True, bits=False)
        assert np.array_equal(a.e1, a.e2)
        lows.append(int(a.e1.min()))
    f = run.archive(-1, bits=False)
    assert len(f) == 1 and f.e1[0] == f.e2[0] == min(lows)


def test_argument_errors(mda):
    inst = synth.make_instance(6, 0.0, seed=611)
    q = mda.Qubo(inst.F1, inst.F2, inst.D)

    def code(**kw):
        base = dict(replicas=2, steps=100, seed=1)
        base.update(kw)
        with pytest.raises(mda.MdaError) as e:
            mda.da_run(q, mda.make_params(base.pop("replicas"), base.pop("steps"), base.pop("seed"), **base))
        return e.value.code

    assert code(replicas=0) == mda.MDA_EINVAL
    assert code(steps=-1) == mda.MDA_EINVAL
    assert code(steps=1 << 32) == mda.MDA_EINVAL
    assert code(steps=(1 << 32) - 1) == mda.MDA_EINVAL             # t would wrap before reaching it
    assert code(steps=10, temp_table=np.full(10, 1 << 44)) == mda.MDA_EOVERFLOW
    assert code(steps=10, temp_table=np.full(10, -1)) == mda.MDA_EOVERFLOW
    assert code(accept=2) == mda.MDA_EINVAL
    assert code(archive=2) == mda.MDA_EINVAL
    assert code(escape=2) == mda.MDA_EINVAL
    assert code(archive_size=-1) == mda.MDA_EINVAL
    assert code(trace_replicas=3) == mda.MDA_EINVAL
    assert code(xi=1.0) == mda.MDA_EINVAL
    assert code(waves_per_replica=9) == mda.MDA_EINVAL
    assert code(delta0=1e20, deltaf=1.0) == mda.MDA_EOVERFLOW    # above 2^35
    assert code(delta0=float("nan"), deltaf=1.0) == mda.MDA_EOVERFLOW

    run = mda.da_run(q, mda.make_params(2, 100, 1, trace_replicas=1))
    run.sync()
    for bad in (-1, 2):
        with pytest.raises(mda.MdaError) as e:
            run.state(bad)
        assert e.value.code == mda.MDA_EINVAL
    with pytest.raises(mda.MdaError) as e:
        run.state(1, trace=True)                      # replica 1 was not traced
    assert e.value.code == mda.MDA_EINVAL
    with pytest.raises(mda.MdaError) as e:
        run.archive(2)
    assert e.value.code == mda.MDA_EINVAL
    with pytest.raises(mda.MdaError) as e:
        run.archive(-1, raw=True)                     # the raw archive is per replica
    assert e.value.code == mda.MDA_EINVAL
    assert len(run.state(0, trace=True)["trace"]) == 100


def test_batch_members_resolve_their_own_defaults(mda):
    """In one batched launch, a member with the default step count (m^2 / 4)
    and one with an explicit count each report their own resolved parameters
    and equal their single runs."""
    a = synth.make_instance(4, 0.3, seed=441)
    b = synth.make_instance(6, -0.3, seed=661)
    qa, qb = mda.Qubo(a.F1, a.F2, a.D, path=2), mda.Qubo(b.F1, b.F2, b.D, path=2)
    pa = mda.make_params(3, 0, 11, trace_replicas=3)
    pb = mda.make_params(5, 700, 12, trace_replicas=5, archive_size=9)
    ra, rb = mda.da_run_batch([qa, qb], [pa, pb])
    assert ra.params.steps == 16 * 16 // 4 and ra.params.archive_size == 16
    assert rb.params.steps == 700 and rb.params.archive_size == 9
    for q, p, run, R in ((qa, pa, ra, 3), (qb, pb, rb, 5)):
        alone = mda.da_run(q, p)
        for r in range(R):
            x, y = alone.state(r, trace=True), run.state(r, trace=True)
            assert len(x["trace"]) == run.params.steps
            assert np.array_equal(x["trace"], y["trace"]) and (x["E1"], x["E2"]) == (y["E1"], y["E2"])
