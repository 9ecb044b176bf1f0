"""da_run_noalloc: the run of da_run written into caller-owned device buffers,
with the launch's own data in the library's fixed scratch area (no
allocation).  Each call is compared with da_run of the same QUBO and
parameters: final solutions, local fields, energies, offsets, counters,
trajectories, raw archives (energies and solutions) and the non-dominated
flags.  Two calls in a row share the scratch area, the second with a smaller
instance, fewer replicas and fewer steps; a third uses the workgroup layout.
The buffers start filled with garbage, so nothing relies on cleared memory.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_13399_amd import mda as m
    m.use_torch_allocator()
    return m


def _noalloc(mda, q, p):
    import torch
    lay = mda.run_layout(q, p)
    assert 0 < lay.scratch_bytes <= mda.NOALLOC_SCRATCH_BYTES
    dev = torch.device("cuda")
    spec = dict(x=(lay.n_x, torch.int64), h=(lay.n_h, torch.int64), st=(lay.n_st, torch.int64),
                arch_e=(lay.n_arch_e, torch.int64), arch_x=(lay.n_arch_x, torch.int64),
                nd=(lay.n_nd, torch.uint8), trace=(max(1, lay.n_trace), torch.int32))
    bufs = {k: torch.full((cnt,), 0x5A, dtype=dt, device=dev) for k, (cnt, dt) in spec.items()}
    torch.cuda.synchronize()
    mda.da_run_noalloc(q, p, **{k: v.data_ptr() for k, v in bufs.items()})
    torch.cuda.synchronize()
    return lay, {k: v.cpu().numpy() for k, v in bufs.items()}


def _bits(words, lay, n):
    """One stored solution (its uint64 words) as m bytes, bit a = i*n + u."""
    w = words.view(np.uint64)
    x = np.zeros(n * n, np.uint8)
    for i in range(n):
        for u in range(n):
            if lay.wr * lay.wc == 1:
                word, bit = u, i
            else:
                pr, c = i // lay.gns, u // 64
                word, bit = (pr * lay.wc + c) * 64 + (u % 64), i - pr * lay.gns
            x[i * n + u] = (int(w[word]) >> bit) & 1
    return x


def _compare(mda, inst, R, steps, seed, path, **kw):
    import torch
    print("case n=%d R=%d steps=%d seed=%d path=%d %s" % (inst.n, R, steps, seed, path, kw), flush=True)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=path)
    stream = torch.cuda.current_stream().cuda_stream
    p = mda.make_params(R, steps, seed, trace_replicas=R, stream=stream, **kw)
    lay, b = _noalloc(mda, q, p)
    ref = mda.da_run(q, p)
    ref.sync()
    n, m, s = inst.n, inst.m, lay.archive_size
    assert (lay.n, lay.replicas, lay.steps) == (n, R, steps)
    st = b["st"].reshape(R, 16)
    for r in range(R):
        g = ref.state(r, trace=True)
        tag = "n=%d replica %d" % (n, r)
        assert np.array_equal(_bits(b["x"][r * lay.x_words:(r + 1) * lay.x_words], lay, n), g["x"]), tag
        h = b["h"].reshape(R, 2, m)[r]
        assert np.array_equal(h[0], g["h1"]) and np.array_equal(h[1], g["h2"]), tag
        assert tuple(int(v) for v in st[r, :6]) == (g["E1"], g["E2"], g["Eoff"], g["moves"], g["scanned"],
                                                     g["rng_blocks"]), tag
        assert np.array_equal(b["trace"][r * steps:(r + 1) * steps], g["trace"]), tag
        a = ref.archive(r, raw=True)
        k = int(st[r, 6])
        assert k == len(a), tag
        ae = b["arch_e"].reshape(R, s, 2)[r, :k]
        assert np.array_equal(ae[:, 0], a.e1) and np.array_equal(ae[:, 1], a.e2), tag
        ax = b["arch_x"].reshape(R, s, lay.arch_x_words)[r]
        for slot in range(k):
            want = np.array([(int(a.xbits[slot, j >> 5]) >> (j & 31)) & 1 for j in range(m)], np.uint8)
            assert np.array_equal(_bits(ax[slot], lay, n), want), (tag, slot)
        nd = b["nd"].reshape(R, s)[r, :k]
        assert int(st[r, 8]) == int(nd.sum()), tag
        front = ref.archive(r, raw=False, bits=False)
        flagged = {(int(x), int(y)) for x, y, f in zip(ae[:, 0], ae[:, 1], nd) if f}
        assert flagged == {(int(x), int(y)) for x, y in zip(front.e1, front.e2)}, tag


def test_two_calls_in_a_row(mda):
    """A larger run, then a smaller one through the same scratch area."""
    _compare(mda, synth.make_instance(40, 0.3, seed=4040), 24, 4000, 17, path=2)
    _compare(mda, synth.make_instance(9, -0.4, seed=909), 5, 1500, 18, path=1, archive=1, escape=1)


def test_workgroup_layout(mda):
    _compare(mda, synth.make_instance(70, 0.1, seed=7070), 4, 1200, 19, path=2)


def test_errors(mda):
    inst = synth.make_instance(6, 0.0, seed=66)
    q = mda.Qubo(inst.F1, inst.F2, inst.D)
    with pytest.raises(mda.MdaError) as e:
        mda.run_layout(q, mda.make_params(600_000, 10, 1))     # work list beyond the scratch area
    assert e.value.code == mda.MDA_ERANGE
    p = mda.make_params(2, 10, 1, trace_replicas=1)
    with pytest.raises(mda.MdaError) as e:
        mda.da_run_noalloc(q, p, 1, 1, 1, 1, 1, 1, 0)          # traced replicas need a trace buffer
    assert e.value.code == mda.MDA_EINVAL
    with pytest.raises(mda.MdaError) as e:
        mda.da_run_noalloc(q, mda.make_params(2, 10, 1, variant=mda.VARIANT_PLAIN), 1, 1, 1, 1, 1, 1)
    assert e.value.code == mda.MDA_EINVAL
