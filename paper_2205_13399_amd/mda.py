"""Python binding of the MI355X multi-objective Digital Annealer C ABI (``include/mda.h``).

Argument marshalling only: every step of the annealing path runs in the HIP
kernels of ``libmda.so``.  PyTorch supplies device memory (through the caching
allocator hook) and streams.  The library must be built (``build.py``); importing
this module without it raises, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmda.so")

MDA_OK, MDA_EINVAL, MDA_EOVERFLOW, MDA_ENOMEM, MDA_EDEVICE, MDA_ERANGE, MDA_EBUSY = 0, -1, -2, -3, -4, -5, -6
PEN_2MAX, PEN_VL = 0, 1
NORM_NONE, NORM_AUTO = 0, -1   # normalise: or L in [1, 30] for max|C_k| = 2^L
FIELDS_AUTO, FIELDS_32, FIELDS_64 = 0, 32, 64   # width of the energy differences
PATH_AUTO, PATH_DENSE, PATH_KRON = 0, 1, 2
STRICT, LENIENT = 0, 1
EXPLORE, EXPLOIT = 0, 1
ESC_OFFSET, ESC_ARCHIVE = 0, 1
VARIANT_AUTO, VARIANT_PERSISTENT, VARIANT_PLAIN = 0, 1, 2

_ERRNAMES = {MDA_EINVAL: "EINVAL", MDA_EOVERFLOW: "EOVERFLOW", MDA_ENOMEM: "ENOMEM",
             MDA_EDEVICE: "EDEVICE", MDA_ERANGE: "ERANGE", MDA_EBUSY: "EBUSY"}


class MdaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class BuildOpts(C.Structure):
    _fields_ = [("penalty", C.c_int32), ("path", C.c_int32), ("dense_budget", C.c_int64),
                ("normalise_log2", C.c_int32), ("fields", C.c_int32)]


class QuboInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("path", C.c_int32), ("symmetric", C.c_int32),
                ("alpha1", C.c_int64), ("alpha2", C.c_int64), ("q1", C.c_int64), ("q2", C.c_int64),
                ("maxabs_c", C.c_int64), ("device_bytes", C.c_int64), ("normalise_log2", C.c_int32),
                ("fields", C.c_int32), ("scale1", C.c_double), ("scale2", C.c_double)]


class Params(C.Structure):
    _fields_ = [("replicas", C.c_int32), ("archive_size", C.c_int32), ("steps", C.c_int64),
                ("delta0", C.c_double), ("deltaf", C.c_double), ("xi", C.c_double),
                ("beta", C.c_int64), ("accept", C.c_int32), ("archive", C.c_int32),
                ("escape", C.c_int32), ("variant", C.c_int32), ("seed", C.c_uint64),
                ("trace_replicas", C.c_int32), ("waves_per_block", C.c_int32),
                ("stream", C.c_void_p), ("graph", C.c_int32), ("waves_per_replica", C.c_int32),
                ("temp_table", C.c_void_p), ("occupancy", C.c_int32)]


class ArchiveOut(C.Structure):
    _fields_ = [("cap", C.c_int64), ("e1", C.c_void_p), ("e2", C.c_void_p), ("replica", C.c_void_p),
                ("slot", C.c_void_p), ("feasible", C.c_void_p), ("xbits", C.c_void_p),
                ("perm", C.c_void_p)]


class State(C.Structure):
    _fields_ = [("x", C.c_void_p), ("h1", C.c_void_p), ("h2", C.c_void_p), ("e1", C.c_int64),
                ("e2", C.c_int64), ("e_offset", C.c_int64), ("moves", C.c_int64),
                ("scanned", C.c_int64), ("rng_blocks", C.c_int64), ("trace", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("waves_per_replica", C.c_int32), ("candidates", C.c_int32),
                ("cached", C.c_int32), ("best_ms", C.c_double), ("probe_steps", C.c_int64),
                ("probe_replicas", C.c_int32), ("occupancy", C.c_int32), ("cand_wpb", C.c_int32 * 16),
                ("cand_wpr", C.c_int32 * 16), ("probe_ms", C.c_double * 16), ("cand_occ", C.c_int32 * 16)]


class RunLayout(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("replicas", C.c_int32), ("archive_size", C.c_int32),
                ("steps", C.c_int64), ("trace_replicas", C.c_int32), ("wr", C.c_int32), ("wc", C.c_int32),
                ("gns", C.c_int32), ("x_words", C.c_int64), ("arch_x_words", C.c_int64),
                ("n_x", C.c_int64), ("n_h", C.c_int64), ("n_st", C.c_int64), ("n_arch_e", C.c_int64),
                ("n_arch_x", C.c_int64), ("n_nd", C.c_int64), ("n_trace", C.c_int64),
                ("scratch_bytes", C.c_int64)]


class RunBuffers(C.Structure):
    _fields_ = [("x", C.c_void_p), ("h", C.c_void_p), ("st", C.c_void_p), ("arch_e", C.c_void_p),
                ("arch_x", C.c_void_p), ("nd", C.c_void_p), ("trace", C.c_void_p)]


NOALLOC_SCRATCH_BYTES = 4 << 20


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_inflight", C.c_int32), ("max_batch", C.c_int32),
                ("device", C.c_int32), ("reserved", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("n", C.c_int32), ("status", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_launch", C.c_double),
                ("t_done", C.c_double), ("bit_trials", C.c_int64), ("footprint", C.c_int64),
                ("batch", C.c_int32), ("slot", C.c_int32)]


class ServerCounters(C.Structure):
    _fields_ = [("launches", C.c_int64), ("completed", C.c_int64), ("bit_trials", C.c_int64),
                ("pending", C.c_int64), ("in_flight", C.c_int64), ("hbm_used", C.c_int64),
                ("hbm_budget", C.c_int64), ("now", C.c_double), ("first_launch", C.c_double),
                ("last_done", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Loads ``libmda.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmda.so not found at %s: run paper_2205_13399_amd/build.py" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.qubo_build_bqap.argtypes = [i32, vp, vp, vp, C.POINTER(BuildOpts), vp, C.POINTER(vp)]
    L.qubo_build_bqap.restype = C.c_int
    L.qubo_build_scalarised.argtypes = [i32, vp, vp, vp, i32, C.POINTER(BuildOpts), vp, C.POINTER(vp)]
    L.qubo_build_scalarised.restype = C.c_int
    L.da_best.argtypes = [vp, vp, vp]
    L.da_best.restype = C.c_int
    L.qubo_flows.argtypes = [vp, vp, vp]
    L.qubo_flows.restype = C.c_int
    L.qubo_info.argtypes = [vp, C.POINTER(QuboInfo)]
    L.qubo_info.restype = C.c_int
    L.qubo_free.argtypes = [vp]
    L.qubo_free.restype = None
    L.mda_params_default.argtypes = [C.POINTER(Params)]
    L.mda_params_default.restype = None
    L.da_run.argtypes = [vp, C.POINTER(Params), C.POINTER(vp)]
    L.da_run.restype = C.c_int
    L.da_run_batch.argtypes = [C.POINTER(vp), C.POINTER(Params), i32, C.POINTER(vp)]
    L.da_run_batch.restype = C.c_int
    L.da_sync.argtypes = [vp]
    L.da_sync.restype = C.c_int
    L.da_elapsed_ms.argtypes = [vp, C.POINTER(C.c_double)]
    L.da_elapsed_ms.restype = C.c_int
    L.da_kernel_ms.argtypes = [vp, C.POINTER(C.c_double)]
    L.da_kernel_ms.restype = C.c_int
    L.archive_get.argtypes = [vp, i32, i32, C.POINTER(ArchiveOut), C.POINTER(i64)]
    L.archive_get.restype = C.c_int
    L.da_state_get.argtypes = [vp, i32, C.POINTER(State)]
    L.da_state_get.restype = C.c_int
    L.da_params_get.argtypes = [vp, C.POINTER(Params)]
    L.da_params_get.restype = C.c_int
    L.da_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.da_stats.restype = C.c_int
    L.da_run_free.argtypes = [vp]
    L.da_run_free.restype = None
    L.mda_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    L.mda_set_allocator.restype = C.c_int
    L.mda_last_error.argtypes = []
    L.mda_last_error.restype = C.c_char_p
    L.mda_threshold_table.argtypes = [vp]
    L.mda_threshold_table.restype = C.c_int
    L.mda_temperature_table.argtypes = [C.c_double, C.c_double, C.c_double, i64, vp]
    L.mda_temperature_table.restype = C.c_int
    L.mda_autotune.argtypes = [vp, C.POINTER(Params), i64, i32, C.POINTER(Tuning)]
    L.mda_autotune.restype = C.c_int
    L.mda_footprint.argtypes = [i32, C.POINTER(Params), C.POINTER(BuildOpts)]
    L.mda_footprint.restype = C.c_int64
    L.da_run_layout.argtypes = [vp, C.POINTER(Params), C.POINTER(RunLayout)]
    L.da_run_layout.restype = C.c_int
    L.da_run_noalloc.argtypes = [vp, C.POINTER(Params), C.POINTER(RunBuffers)]
    L.da_run_noalloc.restype = C.c_int
    L.mda_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(vp)]
    L.mda_server_create.restype = C.c_int
    L.mda_server_submit.argtypes = [vp, i32, vp, vp, vp, C.POINTER(BuildOpts), C.POINTER(Params), C.POINTER(i64)]
    L.mda_server_submit.restype = C.c_int
    L.mda_server_wait.argtypes = [vp, i64, C.c_double, C.POINTER(vp), C.POINTER(RequestInfo)]
    L.mda_server_wait.restype = C.c_int
    L.mda_server_stats.argtypes = [vp, C.POINTER(ServerCounters)]
    L.mda_server_stats.restype = C.c_int
    L.mda_server_destroy.argtypes = [vp]
    L.mda_server_destroy.restype = None
    L.gqubo_build.argtypes = [i32, i32, vp, vp, vp, C.POINTER(vp)]
    L.gqubo_build.restype = C.c_int
    L.gqubo_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)]
    L.gqubo_info.restype = C.c_int
    L.gqubo_free.argtypes = [vp]
    L.gqubo_free.restype = None
    L.gda_run.argtypes = [vp, C.POINTER(Params), C.POINTER(vp)]
    L.gda_run.restype = C.c_int
    L.gda_params_get.argtypes = [vp, C.POINTER(Params)]
    L.gda_params_get.restype = C.c_int
    L.gda_kernel_ms.argtypes = [vp, C.POINTER(C.c_double)]
    L.gda_kernel_ms.restype = C.c_int
    L.gda_state_get.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.gda_state_get.restype = C.c_int
    L.garchive_get.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, C.POINTER(i64)]
    L.garchive_get.restype = C.c_int
    L.gda_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.gda_stats.restype = C.c_int
    L.gda_run_free.argtypes = [vp]
    L.gda_run_free.restype = None
    _lib = L
    return L


EXPORTED = ["qubo_build_bqap", "qubo_build_scalarised", "da_best", "qubo_flows", "qubo_info", "qubo_free", "mda_params_default", "da_run", "da_run_batch",
            "da_sync", "da_elapsed_ms", "da_kernel_ms", "archive_get", "da_state_get", "da_params_get", "da_stats", "da_run_free",
            "mda_set_allocator", "mda_last_error", "mda_threshold_table", "mda_temperature_table",
            "mda_autotune", "mda_footprint", "da_run_layout", "da_run_noalloc", "mda_server_create", "mda_server_submit", "mda_server_wait", "mda_server_stats",
            "mda_server_destroy", "gqubo_build", "gqubo_info", "gqubo_free", "gda_run", "gda_params_get", "gda_kernel_ms",
            "gda_state_get", "garchive_get", "gda_stats", "gda_run_free"]


def _check(rc: int):
    if rc != MDA_OK:
        raise MdaError(rc, lib().mda_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- allocator

# Callbacks handed to the library stay alive for the life of the process: every
# device buffer keeps the release function it was allocated with, so a buffer
# allocated under one allocator is released through it even after another one
# has been installed.
_alloc_keep = []
_torch_installed = None


def use_torch_allocator():
    """Routes the library's device allocations through PyTorch's caching
    allocator, on the stream the library names (idempotent)."""
    global _torch_installed
    import torch

    if _torch_installed is not None:
        _check(lib().mda_set_allocator(_torch_installed[0], _torch_installed[1], None))
        return

    def _alloc(nbytes, stream, ctx):
        try:
            s = torch.cuda.ExternalStream(stream) if stream else torch.cuda.current_stream()
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=s))
        except Exception:
            return None

    def _free(ptr, nbytes, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    _alloc_keep.extend([fa, ff])
    _torch_installed = (fa, ff)
    _check(lib().mda_set_allocator(fa, ff, None))


def use_hip_allocator():
    _check(lib().mda_set_allocator(ALLOC_FN(), FREE_FN(), None))


def current_stream_handle() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


# ---------------------------------------------------------------- host tables

def threshold_table() -> np.ndarray:
    out = np.zeros(4096, np.int32)
    _check(lib().mda_threshold_table(_ptr(out)))
    return out


def temperature_table(delta0: float, deltaf: float, xi: float, steps: int) -> np.ndarray:
    out = np.zeros(int(steps), np.int64)
    _check(lib().mda_temperature_table(float(delta0), float(deltaf), float(xi), int(steps), _ptr(out)))
    return out


# ---------------------------------------------------------------- handles

class Qubo:
    """qubo_build_bqap: the penalised QUBOs Y, Z of one bi-objective QAP instance;
    with scalarise = g10 (0..10), qubo_build_scalarised: the single-objective
    QUBO of SB-DA's weight gamma = g10 / 10."""

    def __init__(self, F1, F2, D, penalty: int = PEN_2MAX, path: int = PATH_AUTO,
                 dense_budget: int = 0, stream: Optional[int] = None, normalise: int = NORM_NONE,
                 fields: int = FIELDS_AUTO, scalarise: Optional[int] = None):
        F1 = np.ascontiguousarray(F1, np.int32)
        F2 = np.ascontiguousarray(F2, np.int32)
        D = np.ascontiguousarray(D, np.int32)
        n = int(D.shape[0])
        if F1.shape != (n, n) or F2.shape != (n, n) or D.shape != (n, n):
            raise ValueError("F1, F2, D must be n x n")
        self._h = C.c_void_p()
        opts = BuildOpts(int(penalty), int(path), int(dense_budget), int(normalise), int(fields))
        s = current_stream_handle() if stream is None else stream
        if scalarise is None:
            _check(lib().qubo_build_bqap(n, _ptr(F1), _ptr(F2), _ptr(D), C.byref(opts),
                                         C.c_void_p(s) if s else None, C.byref(self._h)))
        else:
            _check(lib().qubo_build_scalarised(n, _ptr(F1), _ptr(F2), _ptr(D), int(scalarise), C.byref(opts),
                                               C.c_void_p(s) if s else None, C.byref(self._h)))
        self.n = n
        self.m = n * n

    @property
    def handle(self):
        return self._h

    def flows(self):
        """qubo_flows: (F1, F2) as built, after normalisation."""
        F1 = np.zeros((self.n, self.n), np.int32)
        F2 = np.zeros((self.n, self.n), np.int32)
        _check(lib().qubo_flows(self._h, _ptr(F1), _ptr(F2)))
        return F1, F2

    def info(self) -> QuboInfo:
        inf = QuboInfo()
        _check(lib().qubo_info(self._h, C.byref(inf)))
        return inf

    def close(self):
        if self._h:
            lib().qubo_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(replicas: int, steps: int, seed: int, *, archive_size: int = 0,
                delta0: float = 0.0, deltaf: float = 0.0, xi: float = 0.001, beta: int = -1,
                accept: int = STRICT, archive: int = EXPLORE, escape: int = ESC_OFFSET,
                variant: int = VARIANT_AUTO, trace_replicas: int = 0, waves_per_block: int = 0,
                stream: Optional[int] = None, graph: bool = False, waves_per_replica: int = 0,
                temp_table: Optional[np.ndarray] = None, occupancy: int = 0) -> Params:
    """A parameter block (mda_params).  temp_table: steps int64 entries of T_t
    (fixed point, 8 fractional bits) in place of the geometric schedule; the
    array is kept alive with the returned block and copied by the library when
    a run starts."""
    p = Params()
    lib().mda_params_default(C.byref(p))
    p.replicas = int(replicas)
    p.archive_size = int(archive_size)
    p.steps = int(steps)
    p.delta0 = float(delta0)
    p.deltaf = float(deltaf)
    p.xi = float(xi)
    p.beta = int(beta)
    p.accept = int(accept)
    p.archive = int(archive)
    p.escape = int(escape)
    p.variant = int(variant)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    p.trace_replicas = int(trace_replicas)
    p.waves_per_block = int(waves_per_block)
    p.graph = 1 if graph else 0
    p.waves_per_replica = int(waves_per_replica)
    p.occupancy = int(occupancy)
    s = current_stream_handle() if stream is None else stream
    p.stream = C.c_void_p(s) if s else None
    if temp_table is not None:
        tt = np.ascontiguousarray(temp_table, np.int64)
        if tt.shape != (int(steps),):
            raise ValueError("temp_table needs one entry per step")
        p._temp_keep = tt
        p.temp_table = tt.ctypes.data
    return p


@dataclass
class ArchiveResult:
    e1: np.ndarray
    e2: np.ndarray
    replica: np.ndarray
    slot: np.ndarray
    feasible: np.ndarray
    xbits: Optional[np.ndarray]
    perm: Optional[np.ndarray]

    def __len__(self):
        return len(self.e1)


class Run:
    """One da_run (or one member of a da_run_batch)."""

    def __init__(self, handle: C.c_void_p, qubo: Qubo):
        self._h = handle
        self.qubo = qubo           # keeps the QUBO alive on the Python side too
        self.params = Params()     # as resolved by the library (steps, schedule, archive size)
        _check(lib().da_params_get(self._h, C.byref(self.params)))

    def sync(self):
        _check(lib().da_sync(self._h))

    def elapsed_ms(self) -> float:
        ms = C.c_double()
        _check(lib().da_elapsed_ms(self._h, C.byref(ms)))
        return float(ms.value)

    def kernel_ms(self) -> float:
        ms = C.c_double()
        _check(lib().da_kernel_ms(self._h, C.byref(ms)))
        return float(ms.value)

    def archive(self, replica: int = -1, raw: bool = False, bits: bool = True) -> ArchiveResult:
        cnt = C.c_int64()
        _check(lib().archive_get(self._h, int(replica), int(raw), None, C.byref(cnt)))
        k = int(cnt.value)
        n, m = self.qubo.n, self.qubo.m
        words = (m + 31) // 32
        e1 = np.zeros(k, np.int64)
        e2 = np.zeros(k, np.int64)
        rep = np.zeros(k, np.int32)
        slot = np.zeros(k, np.int32)
        feas = np.zeros(k, np.uint8)
        xb = np.zeros((k, words), np.uint32) if bits else None
        perm = np.zeros((k, n), np.int32) if bits else None
        out = ArchiveOut(k, _ptr(e1).value, _ptr(e2).value, _ptr(rep).value, _ptr(slot).value,
                         _ptr(feas).value, _ptr(xb).value if bits else None,
                         _ptr(perm).value if bits else None)
        _check(lib().archive_get(self._h, int(replica), int(raw), C.byref(out), C.byref(cnt)))
        return ArchiveResult(e1, e2, rep, slot, feas, xb, perm)

    def state(self, replica: int, trace: bool = False) -> dict:
        m = self.qubo.m
        x = np.zeros(m, np.uint8)
        h1 = np.zeros(m, np.int64)
        h2 = np.zeros(m, np.int64)
        tr = np.zeros(int(self.params.steps), np.int32) if trace else None
        st = State(_ptr(x).value, _ptr(h1).value, _ptr(h2).value, 0, 0, 0, 0, 0, 0,
                   _ptr(tr).value if trace else None)
        _check(lib().da_state_get(self._h, int(replica), C.byref(st)))
        res = dict(x=x, h1=h1, h2=h2, E1=int(st.e1), E2=int(st.e2), Eoff=int(st.e_offset),
                   moves=int(st.moves), scanned=int(st.scanned), rng_blocks=int(st.rng_blocks))
        if trace:
            res["trace"] = tr
        return res

    def best(self):
        """da_best: per replica the archive entry of least E1 (first slot on
        ties) as (e1, slot) arrays; slot -1 for an empty archive."""
        R = int(self.params.replicas)
        e1 = np.zeros(R, np.int64)
        slot = np.zeros(R, np.int32)
        _check(lib().da_best(self._h, _ptr(e1), _ptr(slot)))
        return e1, slot

    def stats(self) -> dict:
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().da_stats(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return dict(moves=int(a.value), scanned=int(b.value), rng_blocks=int(c.value),
                    archived=int(d.value))

    def close(self):
        if self._h:
            lib().da_run_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def da_run(q: Qubo, params: Params) -> Run:
    h = C.c_void_p()
    _check(lib().da_run(q.handle, C.byref(params), C.byref(h)))
    return Run(h, q)


def da_run_batch(qs: Sequence[Qubo], params: Sequence[Params]) -> list:
    k = len(qs)
    if k != len(params) or k == 0:
        raise ValueError("one parameter block per QUBO")
    harr = (C.c_void_p * k)(*[q.handle for q in qs])
    parr = (Params * k)(*params)
    outs = (C.c_void_p * k)()
    _check(lib().da_run_batch(harr, parr, k, outs))
    return [Run(C.c_void_p(outs[i]), qs[i]) for i in range(k)]


class GQubo:
    """gqubo_build: K objectives x^T Q_k x + q_k on m bits (a generic QUBO)."""

    def __init__(self, Q, q=None, stream: Optional[int] = None):
        Q = np.ascontiguousarray(Q, np.int32)
        if Q.ndim == 2:
            Q = Q[None]
        if Q.ndim != 3 or Q.shape[1] != Q.shape[2]:
            raise ValueError("Q must be K x m x m")
        K, m = int(Q.shape[0]), int(Q.shape[1])
        qq = np.zeros(K, np.int64) if q is None else np.ascontiguousarray(q, np.int64)
        if qq.shape != (K,):
            raise ValueError("q needs K entries")
        self._h = C.c_void_p()
        s = current_stream_handle() if stream is None else stream
        _check(lib().gqubo_build(m, K, _ptr(Q), _ptr(qq), C.c_void_p(s) if s else None, C.byref(self._h)))
        self.m, self.K = m, K

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        m, K, mx = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().gqubo_info(self._h, C.byref(m), C.byref(K), C.byref(mx)))
        return dict(m=int(m.value), K=int(K.value), maxabs_c=int(mx.value))

    def close(self):
        if self._h:
            lib().gqubo_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class GArchiveResult:
    e: np.ndarray               # count x K energies
    replica: np.ndarray
    slot: np.ndarray
    xbits: Optional[np.ndarray]

    def __len__(self):
        return len(self.e)


class GRun:
    """One gda_run: K-objective replicas on a generic QUBO."""

    def __init__(self, handle: C.c_void_p, g: GQubo):
        self._h = handle
        self.qubo = g
        self.params = Params()
        _check(lib().gda_params_get(self._h, C.byref(self.params)))

    def kernel_ms(self) -> float:
        ms = C.c_double()
        _check(lib().gda_kernel_ms(self._h, C.byref(ms)))
        return float(ms.value)

    def sync(self):
        self.kernel_ms()

    def state(self, replica: int, trace: bool = False) -> dict:
        m, K = self.qubo.m, self.qubo.K
        x = np.zeros(m, np.uint8)
        h = np.zeros((K, m), np.int64)
        E = np.zeros(K, np.int64)
        eo, mv = C.c_int64(), C.c_int64()
        tr = np.zeros(int(self.params.steps), np.int32) if trace else None
        _check(lib().gda_state_get(self._h, int(replica), _ptr(x), _ptr(h), _ptr(E), C.byref(eo), C.byref(mv),
                                   _ptr(tr) if trace else None))
        res = dict(x=x, h=h, E=[int(v) for v in E], Eoff=int(eo.value), moves=int(mv.value))
        if trace:
            res["trace"] = tr
        return res

    def stats(self) -> dict:
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().gda_stats(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return dict(moves=int(a.value), scanned=int(b.value), rng_blocks=int(c.value), archived=int(d.value))

    def archive(self, replica: int = -1, raw: bool = False, bits: bool = True) -> GArchiveResult:
        cnt = C.c_int64()
        _check(lib().garchive_get(self._h, int(replica), int(raw), 0, None, None, None, None, C.byref(cnt)))
        k, K, m = int(cnt.value), self.qubo.K, self.qubo.m
        e = np.zeros((k, K), np.int64)
        rep = np.zeros(k, np.int32)
        slot = np.zeros(k, np.int32)
        xb = np.zeros((k, (m + 31) // 32), np.uint32) if bits else None
        _check(lib().garchive_get(self._h, int(replica), int(raw), k, _ptr(e), _ptr(rep), _ptr(slot),
                                  _ptr(xb) if bits else None, C.byref(cnt)))
        return GArchiveResult(e, rep, slot, xb)

    def close(self):
        if self._h:
            lib().gda_run_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gda_run(g: GQubo, params: Params) -> GRun:
    h = C.c_void_p()
    _check(lib().gda_run(g.handle, C.byref(params), C.byref(h)))
    return GRun(h, g)


def run_layout(q: Qubo, params: Params) -> RunLayout:
    """da_run_layout: sizes of the buffers da_run_noalloc writes."""
    lay = RunLayout()
    _check(lib().da_run_layout(q.handle, C.byref(params), C.byref(lay)))
    return lay


def da_run_noalloc(q: Qubo, params: Params, x: int, h: int, st: int, arch_e: int, arch_x: int, nd: int,
                   trace: int = 0) -> None:
    """da_run_noalloc: the run of da_run written into caller-owned device
    buffers (raw device addresses, sized by run_layout); asynchronous on the
    parameters' stream."""
    b = RunBuffers(x, h, st, arch_e, arch_x, nd, trace or None)
    _check(lib().da_run_noalloc(q.handle, C.byref(params), C.byref(b)))


# ---------------------------------------------------------------- footprint and serving

def footprint(n: int, params: Params, path: int = PATH_AUTO, penalty: int = PEN_2MAX, dense_budget: int = 0) -> int:
    """mda_footprint: device bytes a run of an n-facility instance holds."""
    v = int(lib().mda_footprint(int(n), C.byref(params), C.byref(BuildOpts(int(penalty), int(path), int(dense_budget)))))
    if v < 0:
        _check(v)
    return v


class _Shape:
    def __init__(self, n):
        self.n = n
        self.m = n * n


class Server:
    """The serving engine: submit solves at any time, collect their runs."""

    def __init__(self, hbm_budget: int = 0, max_inflight: int = 0, max_batch: int = 0, device: int = -1):
        self._h = C.c_void_p()
        opts = ServerOpts(int(hbm_budget), int(max_inflight), int(max_batch), int(device), 0)
        _check(lib().mda_server_create(C.byref(opts), C.byref(self._h)))
        self._n = {}            # ticket -> n of the submitted instance

    def submit(self, F1, F2, D, params: Params, path: int = PATH_AUTO, penalty: int = PEN_2MAX,
               dense_budget: int = 0, normalise: int = NORM_NONE, fields: int = FIELDS_AUTO) -> int:
        F1 = np.ascontiguousarray(F1, np.int32)
        F2 = np.ascontiguousarray(F2, np.int32)
        D = np.ascontiguousarray(D, np.int32)
        n = int(D.shape[0])
        t = C.c_int64()
        bo = BuildOpts(int(penalty), int(path), int(dense_budget), int(normalise), int(fields))
        _check(lib().mda_server_submit(self._h, n, _ptr(F1), _ptr(F2), _ptr(D), C.byref(bo), C.byref(params),
                                       C.byref(t)))
        self._n[int(t.value)] = n
        return int(t.value)

    def wait(self, ticket: int, timeout: float = -1.0, keep: bool = True):
        """Returns (Run or None, info dict); raises MdaError on failure or timeout."""
        h = C.c_void_p()
        info = RequestInfo()
        rc = lib().mda_server_wait(self._h, int(ticket), float(timeout), C.byref(h) if keep else None,
                                   C.byref(info))
        _check(rc)
        n = self._n.pop(int(ticket))
        d = {k: getattr(info, k) for k, _ in RequestInfo._fields_ if k != "reserved"}
        run = Run(h, _Shape(n)) if keep else None
        return run, d

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib().mda_server_stats(self._h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in ServerCounters._fields_}

    def close(self):
        if self._h:
            lib().mda_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(q: Qubo, params: Params, probe_steps: int = 2000, probe_replicas: int = 0) -> dict:
    """mda_autotune: the fastest launch shape for q and params (see mda.h)."""
    t = Tuning()
    _check(lib().mda_autotune(q.handle, C.byref(params), int(probe_steps), int(probe_replicas), C.byref(t)))
    k = int(t.candidates)
    return {"waves_per_block": int(t.waves_per_block), "waves_per_replica": int(t.waves_per_replica),
            "occupancy": int(t.occupancy), "cached": bool(t.cached), "best_ms": float(t.best_ms),
            "candidates": [(int(t.cand_wpr[i]), int(t.cand_wpb[i]), int(t.cand_occ[i]), float(t.probe_ms[i]))
                           for i in range(k)]}


def tuned(params: Params, tuning: dict) -> Params:
    """A copy of params with the tuned launch shape."""
    p = Params.from_buffer_copy(params)
    p.waves_per_block = tuning["waves_per_block"]
    p.waves_per_replica = tuning["waves_per_replica"]
    p.occupancy = tuning["occupancy"]
    return p
