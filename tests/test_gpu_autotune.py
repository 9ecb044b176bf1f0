"""Launch-shape autotuner: it times every valid shape, returns the fastest,
remembers it, and the tuned shape gives the same results as the default."""
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


def test_autotune_picks_fastest_and_keeps_results(mda):
    inst = synth.make_instance(30, 0.2, seed=31)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=2)
    p = mda.make_params(256, 3000, 7)
    t = mda.autotune(q, p, probe_steps=500)
    shapes = {(w, b, o) for w, b, o, _ in t["candidates"]}
    # n = 30: 32 slots, the one- and two-waves-per-SIMD builds
    assert {(1, 1, 1), (1, 1, 2), (1, 2, 1), (1, 2, 2), (1, 4, 1), (1, 4, 2), (2, 0, 0), (4, 0, 0)} <= shapes
    assert t["best_ms"] == min(ms for _, _, _, ms in t["candidates"])
    assert (t["waves_per_replica"], t["waves_per_block"], t["occupancy"]) in shapes
    again = mda.autotune(q, p, probe_steps=500)
    assert again["cached"] and again["waves_per_replica"] == t["waves_per_replica"]
    a = mda.da_run(q, p)
    b = mda.da_run(q, mda.tuned(p, t))
    for r in (0, 17, 255):
        sa, sb = a.state(r), b.state(r)
        assert (sa["E1"], sa["E2"], sa["moves"]) == (sb["E1"], sb["E2"], sb["moves"])
        assert np.array_equal(sa["x"], sb["x"])
    fa, fb = a.archive(-1), b.archive(-1)
    assert np.array_equal(fa.e1, fb.e1) and np.array_equal(fa.xbits, fb.xbits)


def test_autotune_beyond_one_wave(mda):
    inst = synth.make_instance(80, 0.0, seed=81)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=2)
    t = mda.autotune(q, mda.make_params(64, 400, 3), probe_steps=300)
    assert t["waves_per_replica"] == 4 and [c[0] for c in t["candidates"]] == [4]


def test_autotune_times_both_occupancy_builds(mda):
    """n = 40 (40 slots): the one- and two-waves-per-SIMD builds are both
    candidates; every forced build gives the same results."""
    inst = synth.make_instance(40, 0.0, seed=41)
    q = mda.Qubo(inst.F1, inst.F2, inst.D, path=2)
    p = mda.make_params(2048, 600, 5)
    t = mda.autotune(q, p, probe_steps=300)
    occs = {o for w, _, o, _ in t["candidates"] if w == 1}
    assert occs == {1, 2}
    runs = [mda.da_run(q, mda.make_params(2048, 600, 5, occupancy=o)) for o in (0, 1, 2)]
    for r in (0, 1000, 2047):
        s0 = runs[0].state(r)
        for other in runs[1:]:
            s1 = other.state(r)
            assert (s0["E1"], s0["E2"], s0["moves"]) == (s1["E1"], s1["E2"], s1["moves"])
    with pytest.raises(mda.MdaError) as e:
        mda.da_run(q, mda.make_params(4, 10, 1, occupancy=3))
    assert e.value.code == mda.MDA_EINVAL
