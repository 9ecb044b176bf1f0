"""Quiet steps against the oracle, bit for bit.

With the offset escape a step whose cheap test fails only raises the offset
by beta; the kernels take such steps without the wave, one by one while the
temperature changes and a whole stretch at once (computed from the replica's
least combined difference) at the final temperature.  These cases push that
arithmetic to its edges, each against the oracle's step-by-step run with full
trajectories:
- beta = 1 with a fast schedule: stretches of thousands of steps, many of
  which run into the last step of the run;
- beta above 2^32: the 64-bit division, and an offset beyond every int32
  difference after one quiet step;
on the one-wave kernel, the workgroup kernel (n > 64 and a small instance
forced onto two waves) and the K-objective kernel.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, decode_bits, oracle_kwargs
from tests.oracle_jobs import run_greplicas, run_replicas

pytestmark = pytest.mark.gpu

HUGE_BETA = (1 << 33) + 7


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _beta(mode):
    return 1 if mode == "one" else HUGE_BETA


@pytest.mark.parametrize("n,path,accept,mode,wpr", [
    (9, 2, 0, "one", 0), (24, 1, 1, "one", 0), (50, 2, 0, "one", 0), (17, 2, 1, "huge", 0), (50, 1, 0, "huge", 0),
    (70, 2, 0, "one", 0), (20, 2, 0, "huge", 2), (20, 1, 1, "one", 2)])
def test_quiet_steps_against_oracle(mda, n, path, accept, mode, wpr):
    inst = synth.make_instance(n, 0.2, seed=700 + n)
    oq = oracle.Qubo(inst.F1, inst.F2, inst.D, 0)
    steps, seed = 3000, 70 + n
    d0, df, _, _ = oracle.default_schedule(oq.maxabs_c, steps)
    beta = _beta(mode)
    R = 6 if n < 40 else 2
    print("quiet case n=%d path=%d accept=%d beta=%d waves=%d" % (n, path, accept, beta, wpr), flush=True)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
    run = mda.da_run(q, mda.make_params(R, steps, seed, delta0=d0, deltaf=df, xi=0.02, beta=beta, accept=accept,
                                        trace_replicas=R, waves_per_replica=wpr))
    run.sync()
    okw = oracle_kwargs(oq, steps, seed, accept=accept, schedule=(d0, df, 0.02, beta))
    res = run_replicas(inst.F1, inst.F2, inst.D, range(R), **okw)
    for r in range(R):
        compare_replica(run, res[r], r, label="quiet n=%d beta=%d" % (n, beta))
    if mode == "one":
        # some run ends inside a stretch: the stretch was cut at the last step
        assert any(res[r]["trace"][-1] == -1 for r in range(R))
    else:
        # an offset beyond every difference makes the next step accept: no
        # two quiet steps in a row
        for r in range(R):
            t = res[r]["trace"]
            assert not np.any((t[1:] == -1) & (t[:-1] == -1))


@pytest.mark.parametrize("K,m,accept,mode", [(2, 300, 0, "one"), (3, 200, 0, "one"), (2, 300, 0, "huge")])
def test_quiet_steps_k_objectives(mda, K, m, accept, mode):
    Q, qk = synth.make_gqubo(K, m, seed=80 + m, density=0.3)
    g = mda.GQubo(Q, qk)
    og = oracle.GQubo(Q, qk)
    steps, seed, R = 3000, 90 + K, 6
    d0, df, _, _ = oracle.gdefault_schedule(og.maxabs_c, steps)
    beta = _beta(mode)
    print("quiet K-objective case K=%d m=%d accept=%d beta=%d" % (K, m, accept, beta), flush=True)
    run = mda.gda_run(g, mda.make_params(R, steps, seed, delta0=d0, deltaf=df, xi=0.02, beta=beta, accept=accept,
                                         trace_replicas=R))
    run.sync()
    res = run_greplicas(Q, qk, list(range(R)), steps=steps, delta0=d0, deltaf=df, xi=0.02, beta=beta, seed=seed,
                        accept=accept, archive=0, escape=0, archive_size=0, trace=True)
    for r in range(R):
        gs = run.state(r, trace=True)
        o = res[r]
        tag = "K=%d m=%d beta=%d replica %d" % (K, m, beta, r)
        if not np.array_equal(gs["trace"], o["trace"]):
            k = int(np.argmax(gs["trace"] != o["trace"]))
            raise AssertionError("%s: trajectory differs first at step %d" % (tag, k + 1))
        assert np.array_equal(gs["x"], o["x"]) and np.array_equal(gs["h"], o["h"]), tag
        assert (gs["E"], gs["Eoff"], gs["moves"]) == (o["E"], o["Eoff"], o["moves"]), tag
        a = run.archive(r, raw=True)
        assert np.array_equal(a.e, o["arch_e"]), tag + ": archive energies"
        assert np.array_equal(decode_bits(a.xbits, m), o["arch_x"]), tag + ": archive solutions"
    if mode == "one":
        assert any(res[r]["trace"][-1] == -1 for r in range(R))
