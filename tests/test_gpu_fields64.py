"""int64 energy differences on the GPU path, bit for bit against the oracle
(whose arithmetic is int64 throughout).

The library keeps the local fields in int32 while every bit's
|P_aa| + sum_b |P_ab| fits (the build-time bound) and switches to int64 beyond
it.  Checked here:
  * int64 forced on small instances, every update path, acceptance rule,
    archive method and escape: every replica's trajectory, final state and
    raw archive against the oracle;
  * the same instance with int32 and with int64 differences: identical runs;
  * the paper's normalisation to 2^23 (Sec. Parameter Settings) at the
    benchmark sizes n = 25 (dense and Kronecker) and n = 50, which needs int64
    fields: the library's scales and weights equal the oracle's, and sampled
    replicas are bit-exact against the oracle on the normalised flows;
  * SB-DA (Alg. SB-DA) at the paper's size n = 50, whose scalarised QUBOs need
    int64 fields: every weight against the oracle;
  * the argument errors of the field width.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import compare_replica, oracle_kwargs, sample_replicas
from tests.oracle_jobs import run_replicas

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _check(mda, F1, F2, D, R, steps, seed, path, fields, picks=None, penalty=0, trace=True, **kw):
    n = D.shape[0]
    print("case n=%d R=%d steps=%d seed=%d path=%d fields=%d penalty=%d %s"
          % (n, R, steps, seed, path, fields, penalty, kw), flush=True)
    q = mda.Qubo(F1, F2, D, path=path, fields=fields, penalty=penalty)
    assert q.info().fields == (64 if fields == 64 else 32)
    run = mda.da_run(q, mda.make_params(R, steps, seed, trace_replicas=R if trace else 0, **kw))
    run.sync()
    oq = oracle.Qubo(F1, F2, D, penalty)
    schedule = None
    if "delta0" in kw:   # an explicit schedule; beta resolved as the library does
        schedule = (kw["delta0"], kw["deltaf"], kw["xi"], max(1, int(kw["delta0"] // steps)))
    okw = oracle_kwargs(oq, steps, seed, accept=kw.get("accept", 0), archive=kw.get("archive", 0),
                        escape=kw.get("escape", 0), archive_size=kw.get("archive_size", 0), trace=trace,
                        schedule=schedule)
    reps = list(range(R)) if picks is None else picks
    res = run_replicas(F1, F2, D, reps, penalty=penalty, **okw)
    for r in reps:
        compare_replica(run, res[r], r, trace=trace, label="n=%d fields=%d" % (n, fields))
    return q, run


@pytest.mark.parametrize("n,path,accept,archive,escape,asize", [
    (5, 1, 0, 0, 0, 0), (6, 2, 1, 0, 0, 0), (9, 2, 0, 1, 0, 7), (11, 1, 1, 1, 1, 12),
    (13, 2, 0, 0, 1, 0), (17, 1, 0, 1, 0, 0), (23, 2, 1, 0, 0, 0), (33, 2, 0, 0, 0, 0),
    (57, 2, 0, 0, 0, 0), (64, 1, 0, 0, 0, 0)])
def test_forced_int64_modes(mda, n, path, accept, archive, escape, asize):
    inst = synth.make_instance(n, 0.2, seed=6400 + n)
    R = 6 if n < 40 else 3
    _check(mda, inst.F1, inst.F2, inst.D, R, 2500, 64 + n, path, 64, accept=accept, archive=archive,
           escape=escape, archive_size=asize)


@pytest.mark.parametrize("n", [4, 7])
def test_forced_int64_general_kronecker(mda, n):
    """Non-symmetric flows and distances with non-zero diagonals (two products per column entry)."""
    rng = np.random.default_rng(640 + n)
    F1 = rng.integers(0, 60, size=(n, n)).astype(np.int32)
    F2 = rng.integers(0, 60, size=(n, n)).astype(np.int32)
    D = rng.integers(0, 90, size=(n, n)).astype(np.int32)
    for path in (1, 2):
        _check(mda, F1, F2, D, 4, 2000, 3, path, 64)


@pytest.mark.parametrize("path", [1, 2])
def test_int32_equals_int64(mda, path):
    inst = synth.make_instance(20, -0.4, seed=2020)
    runs = []
    for fields in (32, 64):
        q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path, fields=fields)
        assert q.info().fields == fields
        run = mda.da_run(q, mda.make_params(16, 4000, 77, trace_replicas=16))
        run.sync()
        runs.append(run)
    for r in range(16):
        a, b = runs[0].state(r, trace=True), runs[1].state(r, trace=True)
        assert np.array_equal(a["trace"], b["trace"]), r
        assert (a["E1"], a["E2"], a["Eoff"], a["moves"]) == (b["E1"], b["E2"], b["Eoff"], b["moves"]), r
        assert np.array_equal(a["h1"], b["h1"]) and np.array_equal(a["h2"], b["h2"]), r
    fa, fb = runs[0].archive(-1), runs[1].archive(-1)
    assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.e2, fb.e2) and np.array_equal(fa.xbits, fb.xbits)


@pytest.mark.parametrize("n,rho,k,path", [(25, 0.75, 0, 1), (25, 0.75, 0, 2), (50, 0.0, 1, 2)])
def test_paper_normalisation_at_benchmark_sizes(mda, n, rho, k, path):
    """Both objectives scaled to a largest coefficient of 2^23 (Sec. Parameter
    Settings) with the paper's delta0 = 1e9 and delta_f = 1e4 on that scale
    (Table param): the fields need int64 at these sizes."""
    inst = synth.make_instance(n, rho, seed=synth.instance_seed(1 if n == 25 else 2, k))
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path, normalise=23)
    info = q.info()
    assert info.normalise_log2 == 23 and info.fields == 64
    F1s, s1 = oracle.normalise_flows(inst.F1, inst.D, 23)
    F2s, s2 = oracle.normalise_flows(inst.F2, inst.D, 23)
    assert (info.scale1, info.scale2) == (s1, s2)
    oq = oracle.Qubo(F1s, F2s, inst.D)
    assert oq.overflow                                  # beyond the int32 bound: the reason for int64
    assert info.maxabs_c == oq.maxabs_c and (info.alpha1, info.alpha2) == oq.alpha
    R, steps = (64, 20000) if n == 25 else (32, 10000)
    picks = sample_replicas(R, extra=13, seed=2300 + n + path)
    _check(mda, F1s, F2s, inst.D, R, steps, 23 + n, path, 64, picks=picks, trace=False,
           delta0=1e9, deltaf=1e4, xi=0.001)


def test_sbda_at_paper_size(mda):
    """SB-DA at n = 50 (the paper's larger size): the scalarised flows
    g F1 + (10 - g) F2 with the Verma-Lewis penalty need int64 fields (at
    n = 25 they still fit int32)."""
    from paper_2205_13399_amd import sbda
    inst = synth.make_instance(50, 0.0, seed=2525)
    R, steps, seed = 2, 2000, 555
    res = sbda.sbda(inst.F1, inst.F2, inst.D, R, steps, seed)
    assert any(r.qubo.info().fields == 64 for r in res.runs)
    zero = np.zeros_like(inst.F1)
    for w, g in enumerate(res.weights):
        Fg = (g * inst.F1.astype(np.int64) + (10 - g) * inst.F2.astype(np.int64)).astype(np.int32)
        oq = oracle.Qubo(Fg, zero, inst.D, 1)
        out = run_replicas(Fg, zero, inst.D, range(R), penalty=1, workers=3,
                           **oracle_kwargs(oq, steps, seed + g, trace=False))
        for r in range(R):
            compare_replica(res.runs[w], out[r], r, trace=False, label="SB-DA n=50 weight %d" % g)
            assert res.best[w, r, 0] == out[r]["arch_e1"].min()


def test_field_width_errors(mda):
    inst = synth.make_instance(25, 0.75, seed=25)
    with pytest.raises(mda.MdaError) as e:
        mda.Qubo(inst.F1, inst.F2, inst.D, normalise=23, fields=32)
    assert e.value.code == mda.MDA_EOVERFLOW
    with pytest.raises(mda.MdaError) as e:
        mda.Qubo(inst.F1, inst.F2, inst.D, fields=7)
    assert e.value.code == mda.MDA_EINVAL
    big = synth.make_instance(70, 0.0, seed=70)
    with pytest.raises(mda.MdaError) as e:
        mda.Qubo(big.F1, big.F2, big.D, fields=64)
    assert e.value.code == mda.MDA_EOVERFLOW
    q = mda.Qubo(inst.F1, inst.F2, inst.D, fields=64)
    for kw in (dict(waves_per_replica=2), dict(variant=mda.VARIANT_PLAIN)):
        with pytest.raises(mda.MdaError) as e:
            mda.da_run(q, mda.make_params(2, 10, 1, **kw))
        assert e.value.code == mda.MDA_EINVAL
