"""SB-DA (the scalarisation-based DA) on the same kernels, against the oracle:
every weight's run bit-exact on the scalarised instance (second objective
zero, Verma-Lewis penalty), each replica's best solution the oracle archive's
least-energy entry, and the reported objective values the oracle's QAP costs."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs
from tests.oracle_jobs import run_replicas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda, sbda
    mda.use_torch_allocator()
    return mda, sbda


def test_sbda_against_oracle(mods):
    mda, sbda = mods
    inst = synth.make_instance(8, -0.5, seed=88)
    R, steps, seed = 4, 3000, 123
    res = sbda.sbda(inst.F1, inst.F2, inst.D, R, steps, seed)
    zero = np.zeros_like(inst.F1)
    for w, g in enumerate(res.weights):
        Fg = (g * inst.F1.astype(np.int64) + (10 - g) * inst.F2.astype(np.int64)).astype(np.int32)
        oq = oracle.Qubo(Fg, zero, inst.D, 1)
        assert oq.alpha[1] == 0
        out = run_replicas(Fg, zero, inst.D, range(R), penalty=1, workers=4,
                           **oracle_kwargs(oq, steps, seed + g, trace=False))
        for r in range(R):
            compare_replica(res.runs[w], out[r], r, trace=False, label="SB-DA weight %d" % g)
            assert np.all(out[r]["arch_e2"] == 0)
            # da_best: the least energy and its first slot in the oracle's archive
            assert res.best[w, r, 0] == out[r]["arch_e1"].min()
            assert res.best[w, r, 1] == int(np.argmin(out[r]["arch_e1"]))
    for r in range(R):
        assert len(res.points[r]) >= 1
        for (f1, f2), perm in zip(res.points[r], res.perms[r]):
            assert f1 == oracle.qap_cost(inst.F1, inst.D, perm)
            assert f2 == oracle.qap_cost(inst.F2, inst.D, perm)
        # mutually non-dominated
        p = res.points[r]
        for a in range(len(p)):
            for b in range(len(p)):
                if a != b:
                    assert not (p[b][0] <= p[a][0] and p[b][1] <= p[a][1])


def test_sbda_normalised_against_oracle(mods):
    """R and S normalised to one 2^L before aggregation (Sec. Parameter
    Settings): every weight bit-exact against the oracle on the aggregated
    oracle-normalised flows; points still in the true objectives."""
    mda, sbda = mods
    inst = synth.make_instance(8, 0.5, seed=89)
    R, steps, seed = 3, 3000, 321
    res = sbda.sbda(inst.F1, inst.F2, inst.D, R, steps, seed, normalise=mda.NORM_AUTO)
    L = res.normalise_log2
    print("SB-DA normalised to 2^%d" % L, flush=True)
    assert 1 <= L <= 23
    if L < 23:
        with pytest.raises((mda.MdaError, ValueError)):
            sbda.normalised_qubos(inst.F1, inst.F2, inst.D, L + 1)
    A, _ = oracle.normalise_flows(inst.F1, inst.D, L)
    B, _ = oracle.normalise_flows(inst.F2, inst.D, L)
    zero = np.zeros_like(inst.F1)
    for w, g in enumerate(res.weights):
        Fg = (g * A.astype(np.int64) + (10 - g) * B.astype(np.int64)).astype(np.int32)
        oq = oracle.Qubo(Fg, zero, inst.D, 1)
        out = run_replicas(Fg, zero, inst.D, range(R), penalty=1, workers=4,
                           **oracle_kwargs(oq, steps, seed + g, trace=False))
        for r in range(R):
            compare_replica(res.runs[w], out[r], r, trace=False, label="normalised SB-DA weight %d" % g)
    for r in range(R):
        for (f1, f2), perm in zip(res.points[r], res.perms[r]):
            assert f1 == oracle.qap_cost(inst.F1, inst.D, perm)
            assert f2 == oracle.qap_cost(inst.F2, inst.D, perm)


def test_scalarised_build_errors_and_best_of_empty(mods):
    mda, _ = mods
    inst = synth.make_instance(6, 0.0, seed=6)
    for g in (-1, 11):
        with pytest.raises(mda.MdaError) as e:
            mda.Qubo(inst.F1, inst.F2, inst.D, scalarise=g)
        assert e.value.code == mda.MDA_EINVAL
    big = np.full((6, 6), 2 ** 28, np.int32)
    with pytest.raises(mda.MdaError) as e:        # 10 * 2^28 > 2^31 - 1
        mda.Qubo(big, big, inst.D, scalarise=5)
    assert e.value.code == mda.MDA_EOVERFLOW
    # weight 10 is objective 1 alone: the same QUBO as the plain build with a zero second objective
    zero = np.zeros_like(inst.F1)
    a = mda.Qubo(inst.F1 * 10, zero, inst.D, penalty=mda.PEN_VL)
    b = mda.Qubo(inst.F1, inst.F2, inst.D, penalty=mda.PEN_VL, scalarise=10)
    ia, ib = a.info(), b.info()
    assert (ia.alpha1, ia.alpha2, ia.maxabs_c) == (ib.alpha1, ib.alpha2, ib.maxabs_c)
    # one step from a random start may leave an archive empty: slot -1
    run = mda.da_run(b, mda.make_params(8, 1, 3))
    e1, slot = run.best()
    for r in range(8):
        a_r = run.archive(r, raw=True, bits=False)
        if len(a_r) == 0:
            assert slot[r] == -1 and e1[r] == np.iinfo(np.int64).max
        else:
            assert e1[r] == a_r.e1.min() and slot[r] == int(np.argmin(a_r.e1))
