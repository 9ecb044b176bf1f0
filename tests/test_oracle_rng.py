"""Pins of the oracle's random numbers and host tables."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_philox_published_vectors(orc):
    """Known-answer vectors of Philox4x32-10 distributed with the generator's
    publication (Random123, Salmon et al. SC'11): all-zero and all-ones inputs."""
    assert [int(v) for v in orc.philox([0, 0, 0, 0], [0, 0])] == \
        [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert [int(v) for v in orc.philox([0xffffffff] * 4, [0xffffffff] * 2)] == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("rr") / "rocrand_philox")
    src = os.path.join(ROOT, "tests", "refsrc", "rocrand_philox.cpp")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I/opt/rocm/include",
                           "-o", out, src], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out


def test_philox_matches_rocrand(orc, rocrand_ref):
    """The oracle's Philox equals rocRAND's independent implementation on 2000
    random counters and keys (host-side call of its engine, no device)."""
    rng = np.random.default_rng(1)
    rows = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64).astype(np.uint32)
    rows[:10, :4] = 0
    text = "\n".join(" ".join("%x" % v for v in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(rows)
    for r, ln in zip(rows, lines):
        ref = [int(v, 16) for v in ln.split()]
        assert [int(v) for v in orc.philox(r[:4], r[4:])] == ref


def test_threshold_table_is_quantised_minus_log(orc):
    """LNT encodes -ln(u) at the 4096 midpoints in 2^-16 units: each entry is
    within 0.5 of the exact value (round to nearest), and it decreases strictly."""
    L = orc.lnt()
    assert L.shape == (4096,)
    assert np.all(np.diff(L) < 0)
    for k in (0, 1, 2, 100, 2047, 4000, 4095):
        exact = -math.log((k + 0.5) / 4096.0) * 65536.0
        assert abs(L[k] - exact) <= 0.5


@pytest.mark.parametrize("delta", [50.0, 1000.0, 3.3e4])
def test_acceptance_frequency(orc, delta):
    """Eq. (paccepts): over the 4096 equiprobable uniform indices the accepted
    fraction approaches exp(-S/delta) (within the 1/4096 quantisation and the
    one-unit floor of the threshold), for every S."""
    L = orc.lnt()
    T = int(math.floor(delta * 256.0))
    for S in [0, 1, 7, int(delta / 3), int(delta), int(2.5 * delta), int(6 * delta), int(12 * delta)]:
        freq = sum(orc.accept(S, 0, 0, T, int(L[k])) for k in range(0, 4096, 1)) / 4096.0
        lo = math.exp(-(S + 1) / delta) - 1.0 / 4096
        hi = math.exp(-S / delta) + 1.0 / 4096
        assert lo - 1e-12 <= freq <= hi + 1e-12, (S, freq, math.exp(-S / delta))


def test_temperature_closed_form(orc):
    """Algorithm 3 (cooling): delta_t = delta0 (1-xi)^t until it first drops to
    delta_f or below, constant afterwards; T_t = floor(256 delta_t)."""
    d0, df, xi, steps = 2.0e6, 20.0, 0.001, 15000
    T = orc.temperature(d0, df, xi, steps)
    tc = math.ceil(math.log(df / d0) / math.log(1.0 - xi))
    for t in (1, 2, 10, 1000, 5000, tc - 5):
        exact = d0 * (1.0 - xi) ** t * 256.0
        assert abs(T[t - 1] - exact) <= 1.0 + 1e-9 * exact
    assert np.all(np.diff(T) <= 0)
    assert T[-1] == T[tc + 2]
    assert abs(int(np.argmax(T == T[-1])) + 1 - tc) <= 1
    assert T[-1] <= df * 256 and T[-1] > df * 256 * (1 - xi) - 1
