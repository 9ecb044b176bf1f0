"""Objective normalisation (Sec. Parameter Settings) on the GPU path: the
library's scales, penalty weights and largest coefficient equal the oracle's
for the oracle-normalised flows, and runs on the normalised QUBOs are
bit-exact against the oracle on those flows.  The paper's 2^23 is taken as
given for small n; the automatic choice (the largest 2^L <= 2^23 whose fields
fit int32) at the benchmark sizes."""
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


def _check(mda, inst, R, steps, seed, norm, path=2):
    print("case n=%d rho=%g normalise=%d path=%d R=%d steps=%d" % (inst.n, inst.rho, norm, path, R, steps),
          flush=True)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path, normalise=norm)
    info = q.info()
    L = info.normalise_log2
    F1s, s1 = oracle.normalise_flows(inst.F1, inst.D, L)
    F2s, s2 = oracle.normalise_flows(inst.F2, inst.D, L)
    assert (info.scale1, info.scale2) == (s1, s2)
    oq = oracle.Qubo(F1s, F2s, inst.D)
    assert info.maxabs_c == oq.maxabs_c and (info.alpha1, info.alpha2) == oq.alpha
    run = mda.da_run(q, mda.make_params(R, steps, seed, trace_replicas=R))
    run.sync()
    res = run_replicas(F1s, F2s, inst.D, range(R), **oracle_kwargs(oq, steps, seed))
    for r in range(R):
        compare_replica(run, res[r], r, label="n=%d normalised 2^%d" % (inst.n, L))
    return L


@pytest.mark.parametrize("path", [1, 2])
def test_paper_target_small_n(mda, path):
    inst = synth.make_instance(8, -0.75, seed=808)
    assert _check(mda, inst, 6, 3000, 11, 23, path=path) == 23


@pytest.mark.parametrize("n,rho,k", [(25, 0.75, 0), (50, -0.75, 1)])
def test_automatic_target(mda, n, rho, k):
    inst = synth.make_instance(n, rho, seed=synth.instance_seed(1 if n == 25 else 2, k))
    L = _check(mda, inst, 4, 2000, 12 + n, mda.NORM_AUTO)
    assert 1 <= L <= 23
    if L < 23:
        # one power more does not fit int32 fields (it runs on int64 ones)
        with pytest.raises(mda.MdaError) as e:
            mda.Qubo(inst.F1, inst.F2, inst.D, path=2, normalise=L + 1, fields=32)
        assert e.value.code == mda.MDA_EOVERFLOW
        assert mda.Qubo(inst.F1, inst.F2, inst.D, path=2, normalise=L + 1).info().fields == 64


def test_unbalanced_objectives_are_equalised(mda):
    inst = synth.make_instance(10, 0.0, seed=1010)
    F2 = (inst.F2 * 50).astype(np.int32)
    q0 = mda.Qubo(inst.F1, F2, inst.D, path=2)
    q = mda.Qubo(inst.F1, F2, inst.D, path=2, normalise=mda.NORM_AUTO)
    i0, i = q0.info(), q.info()
    assert i0.normalise_log2 == 0 and (i0.scale1, i0.scale2) == (1.0, 1.0)
    assert i.scale1 > 40 * i.scale2                    # the weak objective is scaled up
    for F, s in ((inst.F1, i.scale1), (F2, i.scale2)):
        Fs, so = oracle.normalise_flows(F, inst.D, i.normalise_log2)
        assert so == s
        assert abs(int(np.abs(oracle.cost_qubo(Fs, inst.D)).max()) - 2 ** i.normalise_log2) <= int(inst.D.max())
