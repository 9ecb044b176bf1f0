"""CPU checks of the C ABI library: it loads, exports every declared entry point,
and its host tables equal the oracle's (no device call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mda():
    from paper_2205_13399_amd import mda as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libmda.so is not built (run __graft_entry__.build())")
    m.lib()
    return m


def _declared():
    text = open(os.path.join(ROOT, "include", "mda.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(ln for ln in text.split("\n") if not ln.lstrip().startswith("typedef"))
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(mda):
    lib = ctypes.CDLL(mda.LIB_PATH)
    declared = _declared()
    assert "qubo_build_bqap" in declared and "da_run" in declared and "archive_get" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(mda.EXPORTED)


def test_threshold_table_matches_oracle(mda, orc):
    assert np.array_equal(mda.threshold_table(), orc.lnt())


@pytest.mark.parametrize("d0,df,xi,steps", [(2.9e6, 29.5, 0.001, 20000), (1e5, 1e5, 0.001, 50),
                                            (5e4, 10.0, 0.01, 3000), (123.0, 1.0, 0.0, 100)])
def test_temperature_table_matches_oracle(mda, orc, d0, df, xi, steps):
    assert np.array_equal(mda.temperature_table(d0, df, xi, steps), orc.temperature(d0, df, xi, steps))


def test_params_default(mda):
    p = mda.make_params(3, 100, 5)
    assert p.replicas == 3 and p.steps == 100 and p.accept == mda.STRICT and p.archive == mda.EXPLORE
    assert p.escape == mda.ESC_OFFSET and p.beta == -1


def test_errors_without_device(mda):
    h = ctypes.c_void_p()
    F = np.zeros((3, 3), np.int32)
    rc = mda.lib().qubo_build_bqap(1, F.ctypes.data_as(ctypes.c_void_p), F.ctypes.data_as(ctypes.c_void_p),
                                   F.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(h))
    assert rc == mda.MDA_EINVAL
    assert b"n = 1" in mda.lib().mda_last_error()
    rc = mda.lib().qubo_build_bqap(3, None, None, None, None, None, ctypes.byref(h))
    assert rc == mda.MDA_EINVAL
    for bad in (-2, 31):   # normalise_log2 outside [-1, 30], rejected before any device call
        bo = mda.BuildOpts(mda.PEN_2MAX, mda.PATH_AUTO, 0, bad, 0)
        rc = mda.lib().qubo_build_bqap(3, F.ctypes.data_as(ctypes.c_void_p), F.ctypes.data_as(ctypes.c_void_p),
                                       F.ctypes.data_as(ctypes.c_void_p), ctypes.byref(bo), None, ctypes.byref(h))
        assert rc == mda.MDA_EINVAL and b"normalise_log2" in mda.lib().mda_last_error()
    assert mda.lib().da_run(None, None, None) == mda.MDA_EINVAL
    assert mda.lib().archive_get(None, 0, 0, None, None) == mda.MDA_EINVAL
    mda.lib().da_run_free(None)
    mda.lib().qubo_free(None)


def test_torch_allocator_installed_once(mda):
    """Every device buffer keeps the release callback it was allocated with, so
    installing the allocator again must not drop the callbacks already handed out."""
    pytest.importorskip("torch")
    mda.use_torch_allocator()
    first = mda._torch_installed
    kept = len(mda._alloc_keep)
    mda.use_hip_allocator()
    mda.use_torch_allocator()
    assert mda._torch_installed is first
    assert len(mda._alloc_keep) == kept and all(f in mda._alloc_keep for f in first)


def test_footprint_counts_archives_and_operands(mda):
    """mda_footprint: replicas x archive slots x (energies + stored solution)
    dominate; the dense rows (2 m^2 int32) are counted only when the build
    would pick them."""
    p = mda.make_params(4096, 100000, 1)
    kron = mda.footprint(50, p, path=mda.PATH_KRON)
    m = 2500
    assert kron >= 4096 * m * (16 + 50 * 8)          # archives of every replica
    assert kron < 4096 * m * (16 + 50 * 8) * 1.2
    dense = mda.footprint(50, p, path=mda.PATH_DENSE)
    assert dense - kron >= 8 * m * m                  # two objectives' rows of m entries (no padding)
    assert dense - kron < 8 * m * m * 1.1
    # the automatic path takes dense rows only within an explicit budget
    assert mda.footprint(50, p) == kron
    assert mda.footprint(50, p, dense_budget=8 * m * m) == dense
    # beyond 64 facilities a solution is stored as 2 x 2 wave blocks of 64 words
    p100 = mda.make_params(256, 50000, 1)
    assert mda.footprint(100, p100, path=mda.PATH_KRON) >= 256 * 10000 * (16 + 256 * 8)
    with pytest.raises(mda.MdaError):
        mda.footprint(101, p100)


def test_server_needs_device(mda):
    import torch
    if torch.cuda.is_available():
        pytest.skip("device present")
    with pytest.raises(mda.MdaError) as e:
        mda.Server()
    assert e.value.code == mda.MDA_EDEVICE
