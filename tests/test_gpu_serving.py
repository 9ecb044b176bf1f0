"""The serving engine: requests of different n submitted at once, staggered,
or under a memory budget that admits one at a time.  Each served result must
equal a da_run of the same instance, parameters and seed (trajectories, final
states, fronts), and one is checked against the oracle directly."""
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs
from tests.oracle_jobs import run_replicas

pytestmark = pytest.mark.gpu

R, STEPS = 8, 3000


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _requests():
    out = []
    for k, n in enumerate((12, 40, 70, 25, 90, 8)):
        inst = synth.make_instance(n, 0.5 - 0.2 * k, seed=4_000_000 + k)
        out.append((inst, 0 if k % 2 == 0 else 2))   # automatic (dense up to the budget) or Kronecker path
    return out


def _same_as_alone(mda, inst, path, run, steps=STEPS):
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
    alone = mda.da_run(q, mda.make_params(R, steps, inst.seed, trace_replicas=R))
    for r in range(R):
        a, b = alone.state(r, trace=True), run.state(r, trace=True)
        assert np.array_equal(a["trace"], b["trace"]), (inst.n, r)
        assert (a["E1"], a["E2"], a["moves"]) == (b["E1"], b["E2"], b["moves"]), (inst.n, r)
    fa, fb = alone.archive(-1), run.archive(-1)
    assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2) and np.array_equal(fa.xbits, fb.xbits)


def _serve(mda, srv, reqs, gap=0.0, steps=STEPS):
    tickets = []
    for inst, path in reqs:
        tickets.append(srv.submit(inst.F1, inst.F2, inst.D, mda.make_params(R, steps, inst.seed, trace_replicas=R),
                                  path=path))
        if gap:
            time.sleep(gap)
    return [srv.wait(t, timeout=120.0) for t in tickets]


def test_mix_at_once(mda):
    srv = mda.Server()
    reqs = _requests()
    got = _serve(mda, srv, reqs)
    for (inst, path), (run, info) in zip(reqs, got):
        assert info["status"] == 2 and info["t_done"] >= info["t_launch"] >= info["t_admit"] >= info["t_submit"]
        _same_as_alone(mda, inst, path, run)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["pending"] == 0
    srv.close()


def test_staggered_arrivals_overlap(mda):
    """Requests arriving while earlier ones are on the device are launched on
    another stream before those finish, and each result is the one it has alone."""
    srv = mda.Server(max_inflight=4)
    reqs = _requests()
    got = _serve(mda, srv, reqs, gap=0.002, steps=20000)
    for (inst, path), (run, info) in zip(reqs, got):
        _same_as_alone(mda, inst, path, run, steps=20000)
    assert srv.stats()["launches"] >= 2
    infos = [info for _, info in got]
    overlapped = [(i, j) for i in range(len(infos)) for j in range(i + 1, len(infos))
                  if infos[j]["t_launch"] < infos[i]["t_done"] and infos[j]["slot"] != infos[i]["slot"]
                  and infos[j]["t_launch"] > infos[i]["t_launch"]]
    assert overlapped, [(k["t_launch"], k["t_done"], k["slot"]) for k in infos]
    srv.close()


def test_budget_limits_admission(mda):
    """With room for the largest request only, it cannot share a launch with
    the requests admitted before it.  A collected run keeps its memory, so its
    footprint stays on the budget until the run is freed."""
    import gc
    reqs = _requests()
    sizes = [mda.footprint(i.n, mda.make_params(R, STEPS, 1, trace_replicas=R), path=p) for i, p in reqs]
    big = int(np.argmax(sizes))
    srv = mda.Server(hbm_budget=max(sizes) + 1, max_inflight=4)
    got = []
    for k, (inst, path) in enumerate(reqs):
        t = srv.submit(inst.F1, inst.F2, inst.D, mda.make_params(R, STEPS, inst.seed, trace_replicas=R), path=path)
        run, info = srv.wait(t, timeout=120.0)
        assert info["footprint"] == sizes[k]
        _same_as_alone(mda, inst, path, run)
        # the collected run still holds its memory
        assert srv.stats()["hbm_used"] == sizes[k]
        run.close()
        del run
        gc.collect()
        assert srv.stats()["hbm_used"] == 0
        got.append(info)
    # all at once: the largest cannot share a launch; each run is closed as it
    # is collected, which returns its memory to the budget for the next ones
    tickets = [srv.submit(i.F1, i.F2, i.D, mda.make_params(R, STEPS, i.seed, trace_replicas=R), path=p)
               for i, p in reqs]
    infos = []
    for t in tickets:
        run, info = srv.wait(t, timeout=120.0)
        run.close()
        infos.append(info)
    assert infos[big]["batch"] == 1
    assert srv.stats()["launches"] >= 2 and srv.stats()["hbm_used"] == 0
    srv.close()


def test_held_runs_keep_their_footprint(mda):
    """Runs the client holds count against the budget until they are freed."""
    reqs = _requests()
    sizes = [mda.footprint(i.n, mda.make_params(R, STEPS, 1, trace_replicas=R), path=p) for i, p in reqs]
    srv = mda.Server(max_inflight=4)
    got = _serve(mda, srv, reqs)
    assert srv.stats()["hbm_used"] == sum(sizes)
    for k, (run, _) in enumerate(got):
        run.close()
        assert srv.stats()["hbm_used"] == sum(sizes[k + 1:])
    srv.close()


def test_oversized_request_fails(mda):
    inst = synth.make_instance(30, 0.0, seed=30)
    srv = mda.Server(hbm_budget=1 << 20)
    t = srv.submit(inst.F1, inst.F2, inst.D, mda.make_params(R, STEPS, 1))
    with pytest.raises(mda.MdaError) as e:
        srv.wait(t, timeout=30.0)
    assert e.value.code == mda.MDA_ENOMEM
    srv.close()


def test_served_request_against_oracle(mda):
    inst = synth.make_instance(70, -0.3, seed=70)
    srv = mda.Server()
    t = srv.submit(inst.F1, inst.F2, inst.D, mda.make_params(3, 2000, inst.seed, trace_replicas=3), path=2)
    run, info = srv.wait(t, timeout=120.0)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    res = run_replicas(inst.F1, inst.F2, inst.D, range(3), workers=3, **oracle_kwargs(oq, 2000, inst.seed))
    for r in range(3):
        compare_replica(run, res[r], r, label="served n=70")
    srv.close()


def test_served_normalised_request(mda):
    """A request with objective normalisation equals a direct run on the
    QUBO built with the same option."""
    inst = synth.make_instance(30, 0.2, seed=3030)
    srv = mda.Server()
    t = srv.submit(inst.F1, inst.F2, inst.D, mda.make_params(R, STEPS, inst.seed, trace_replicas=R), path=2,
                   normalise=mda.NORM_AUTO)
    run, info = srv.wait(t, timeout=120.0)
    assert info["status"] == 2
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=2, normalise=mda.NORM_AUTO)
    assert q.info().normalise_log2 >= 1
    alone = mda.da_run(q, mda.make_params(R, STEPS, inst.seed, trace_replicas=R))
    for r in range(R):
        a, b = alone.state(r, trace=True), run.state(r, trace=True)
        assert np.array_equal(a["trace"], b["trace"]), r
        assert (a["E1"], a["E2"], a["moves"]) == (b["E1"], b["E2"], b["moves"]), r
    fa, fb = alone.archive(-1), run.archive(-1)
    assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2)
    srv.close()
