"""Shared helpers of the GPU parity tests (GPU side through the C ABI, oracle beside it)."""
import numpy as np

import oracle


def decode_bits(xbits, m):
    out = np.zeros((xbits.shape[0], m), np.uint8)
    for a in range(m):
        out[:, a] = (xbits[:, a >> 5] >> (a & 31)) & 1
    return out


def compare_replica(run, o, r, trace=True, label=""):
    """Bit-exact comparison of one replica: trajectory, final state, raw archive."""
    g = run.state(r, trace=trace)
    tag = "%s replica %d" % (label, r)
    if trace:
        gt, ot = g["trace"], o["trace"]
        if not np.array_equal(gt, ot):
            k = int(np.argmax(gt != ot))
            raise AssertionError("%s: trajectory differs first at step %d (gpu %d, oracle %d)"
                                 % (tag, k + 1, gt[k], ot[k]))
    assert np.array_equal(g["x"], o["x"]), tag + ": x"
    assert np.array_equal(g["h1"].astype(np.int64), o["h1"]), tag + ": h1"
    assert np.array_equal(g["h2"].astype(np.int64), o["h2"]), tag + ": h2"
    assert (g["E1"], g["E2"], g["Eoff"], g["moves"]) == (o["E1"], o["E2"], o["Eoff"], o["moves"]), tag
    a = run.archive(r, raw=True)
    assert len(a) == o["arch_size"], tag + ": archive size"
    assert np.array_equal(a.e1, o["arch_e1"]) and np.array_equal(a.e2, o["arch_e2"]), tag + ": archive energies"
    assert np.array_equal(decode_bits(a.xbits, run.qubo.m), o["arch_x"]), tag + ": archive solutions"
    return g


def oracle_kwargs(oq, steps, seed, accept=0, archive=0, escape=0, archive_size=0, trace=True,
                  schedule=None):
    d0, df, xi, beta = schedule if schedule else oracle.default_schedule(oq.maxabs_c, steps)
    return dict(steps=steps, delta0=d0, deltaf=df, xi=xi, beta=beta, seed=seed, accept=accept,
                archive=archive, escape=escape, archive_size=archive_size, trace=trace)


def sample_replicas(R, extra=5, seed=1):
    rng = np.random.default_rng(seed)
    picks = {0, 1, R - 1}
    while len(picks) < min(R, 3 + extra):
        picks.add(int(rng.integers(0, R)))
    return sorted(picks)
