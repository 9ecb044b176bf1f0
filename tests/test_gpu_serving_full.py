"""The serving workload at its own size, against the oracle.

Twelve bQAP solve requests from the seeded serving mix (n uniform on
{10..100}, rho uniform on [-0.75, 0.75]), 256 replicas x 5 * 10^4 steps each,
arriving as a Poisson stream (mean gap 40 ms) at a server whose dense-row
budget is 64 MB, so that the requests above n of about 45 take the Kronecker
update path and the smaller ones dense rows, in the same mix.  Checked:
  * three requests (the largest n, the smallest n and the largest n on dense
    rows): replicas 0, 1, R - 1 and 13 seeded picks bit-exact against the
    oracle (final state and raw archive);
  * the same three requests run alone (da_run, same seed): every replica and
    the merged front identical to the served result;
  * later arrivals were launched on other streams while earlier ones ran.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs, sample_replicas
from tests.oracle_jobs import run_replicas

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

R, STEPS = 256, 50_000
DENSE_BUDGET = 64 << 20
COUNT = 12


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


@pytest.fixture(scope="module")
def served(mda):
    import time
    insts = synth.mixed_batch(count=COUNT, n_lo=10, n_hi=100, config=4)
    gaps = np.random.default_rng(4).exponential(0.040, size=COUNT)
    srv = mda.Server(max_inflight=4)
    print("serving: %d requests, n = %s, %d replicas x %d steps" % (COUNT, [i.n for i in insts], R, STEPS), flush=True)
    tickets = []
    for inst, gap in zip(insts, gaps):
        tickets.append(srv.submit(inst.F1, inst.F2, inst.D, mda.make_params(R, STEPS, inst.seed),
                                  dense_budget=DENSE_BUDGET))
        time.sleep(float(gap))
    got = [srv.wait(t, timeout=600.0) for t in tickets]
    print("serving: done, %d launches" % srv.stats()["launches"], flush=True)
    paths = [mda.Qubo(i.F1, i.F2, i.D, dense_budget=DENSE_BUDGET).info().path for i in insts]
    yield insts, got, paths
    for run, _ in got:
        run.close()
    srv.close()


def _checked(insts, paths):
    ns = [i.n for i in insts]
    dense = [k for k in range(len(insts)) if paths[k] == 1]
    picks = [int(np.argmax(ns)), int(np.argmin(ns)), max(dense, key=lambda k: ns[k])]
    return sorted(set(picks))


def test_paths_in_the_mix(mda, served):
    insts, got, paths = served
    assert set(paths) == {mda.PATH_DENSE, mda.PATH_KRON}


def test_arrivals_overlap(served):
    insts, got, paths = served
    infos = [info for _, info in got]
    assert all(i["status"] == 2 for i in infos)
    overlapped = [(i, j) for i in range(len(infos)) for j in range(i + 1, len(infos))
                  if infos[i]["t_launch"] < infos[j]["t_launch"] < infos[i]["t_done"]
                  and infos[i]["slot"] != infos[j]["slot"]]
    assert overlapped


@pytest.mark.parametrize("which", [0, 1, 2])
def test_served_against_oracle(served, which):
    insts, got, paths = served
    picks = _checked(insts, paths)
    if which >= len(picks):
        pytest.skip("fewer distinct requests")
    k = picks[which]
    inst = insts[k]
    run = got[k][0]
    reps = sample_replicas(R, extra=13, seed=4000 + k)
    assert len(reps) == 16
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D)
    print("oracle: request %d (n=%d), %d replicas" % (k, inst.n, len(reps)), flush=True)
    workers = 8 if inst.n >= 70 else None   # the oracle's dense P is 1.6 GB per process at n = 100
    res = run_replicas(inst.F1, inst.F2, inst.D, reps, workers=workers,
                       **oracle_kwargs(oq, STEPS, inst.seed, trace=False))
    for r in reps:
        compare_replica(run, res[r], r, trace=False, label="served request %d (n=%d)" % (k, inst.n))


@pytest.mark.parametrize("which", [0, 1, 2])
def test_served_equals_alone(mda, served, which):
    insts, got, paths = served
    picks = _checked(insts, paths)
    if which >= len(picks):
        pytest.skip("fewer distinct requests")
    k = picks[which]
    inst = insts[k]
    run = got[k][0]
    q = mda.Qubo(inst.F1, inst.F2, inst.D, dense_budget=DENSE_BUDGET)
    alone = mda.da_run(q, mda.make_params(R, STEPS, inst.seed))
    alone.sync()
    for r in range(R):
        a, b = alone.state(r), run.state(r)
        assert (a["E1"], a["E2"], a["Eoff"], a["moves"]) == (b["E1"], b["E2"], b["Eoff"], b["moves"]), (k, r)
        assert np.array_equal(a["x"], b["x"]), (k, r)
    fa, fb = alone.archive(-1), run.archive(-1)
    assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2) and np.array_equal(fa.xbits, fb.xbits)
