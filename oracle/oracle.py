"""ctypes wrapper of the C oracle (TEST INFRASTRUCTURE ONLY).

Every function forwards to ``mda_oracle.c`` except ``normalise_flows``, plain
numpy over the oracle's own cost QUBO; see the C file's header for the readings
of the paper (arXiv:2205.13399) it implements.  Arrays are numpy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

__all__ = [
    "build", "lib", "qap_cost", "cost_direct", "constraint_direct", "cost_qubo",
    "constraint_qubo", "normalise_flows", "qubo_energy", "delta_energy", "penalty_2max", "penalty_vl_w",
    "philox", "lnt", "temperature", "accept", "dominates", "Archive", "Qubo", "run_replica",
    "default_schedule", "STRICT", "LENIENT", "EXPLORE", "EXPLOIT", "ESC_OFFSET",
    "ESC_ARCHIVE", "PEN_2MAX", "PEN_VL", "nondominated",
    "GQubo", "run_greplica", "gaccept", "gdominates", "GArchive", "gdefault_schedule", "gnondominated",
]

STRICT, LENIENT = 0, 1
EXPLORE, EXPLOIT = 0, 1
ESC_OFFSET, ESC_ARCHIVE = 0, 1
PEN_2MAX, PEN_VL = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mda_oracle.c")
_SO = os.path.join(_HERE, "libmda_oracle.so")

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    stale = os.path.exists(_SO) and any(
        os.path.getmtime(src) > os.path.getmtime(_SO) for src in (_SRC, os.path.join(_HERE, "mda_oracle.h")))
    if force or stale or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Qubo(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("m", C.c_int32),
        ("alpha1", C.c_int64), ("alpha2", C.c_int64), ("q1", C.c_int64), ("q2", C.c_int64),
        ("maxabs_c", C.c_int64),
        ("P1", C.c_void_p), ("P2", C.c_void_p),
        ("overflow", C.c_int32),
    ]


class _Params(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("delta0", C.c_double), ("deltaf", C.c_double), ("xi", C.c_double),
        ("beta", C.c_int64), ("accept", C.c_int32), ("archive", C.c_int32),
        ("escape", C.c_int32), ("archive_size", C.c_int32), ("seed", C.c_uint64),
        ("temp_table", C.c_void_p),
    ]


class _ReplicaOut(C.Structure):
    _fields_ = [
        ("x", C.c_void_p), ("h1", C.c_void_p), ("h2", C.c_void_p), ("state", C.c_void_p),
        ("arch_size", C.c_void_p), ("arch_e", C.c_void_p), ("arch_x", C.c_void_p),
        ("trace", C.c_void_p),
    ]


class _GQubo(C.Structure):
    _fields_ = [("m", C.c_int32), ("K", C.c_int32), ("P", C.c_void_p), ("q", C.c_void_p),
                ("maxabs_c", C.c_int64), ("overflow", C.c_int32)]


class _GArchive(C.Structure):
    _fields_ = [("size", C.c_int32), ("cap", C.c_int32), ("m", C.c_int32), ("K", C.c_int32),
                ("e", C.c_void_p), ("x", C.c_void_p)]


class _GReplicaOut(C.Structure):
    _fields_ = [("x", C.c_void_p), ("h", C.c_void_p), ("state", C.c_void_p), ("arch_size", C.c_void_p),
                ("arch_e", C.c_void_p), ("arch_x", C.c_void_p), ("trace", C.c_void_p)]


class _Archive(C.Structure):
    _fields_ = [("size", C.c_int32), ("cap", C.c_int32), ("m", C.c_int32),
                ("e1", C.c_void_p), ("e2", C.c_void_p), ("x", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = C.CDLL(_SO)
        L.orc_qap_cost.restype = C.c_int64
        L.orc_qap_cost.argtypes = [C.c_int32, _i32p, _i32p, _i32p]
        L.orc_cost_direct.restype = C.c_int64
        L.orc_cost_direct.argtypes = [C.c_int32, _i32p, _i32p, _u8p]
        L.orc_constraint_direct.restype = C.c_int64
        L.orc_constraint_direct.argtypes = [C.c_int32, _u8p]
        L.orc_cost_qubo.restype = None
        L.orc_cost_qubo.argtypes = [C.c_int32, _i32p, _i32p, _i64p]
        L.orc_constraint_qubo.restype = None
        L.orc_constraint_qubo.argtypes = [C.c_int32, _i64p, C.POINTER(C.c_int64)]
        L.orc_qubo_energy.restype = C.c_int64
        L.orc_qubo_energy.argtypes = [C.c_int32, _i64p, C.c_int64, _u8p]
        L.orc_delta_energy.restype = None
        L.orc_delta_energy.argtypes = [C.c_int32, _i64p, _u8p, _i64p]
        L.orc_penalty_2max.restype = C.c_int64
        L.orc_penalty_2max.argtypes = [C.c_int32, _i64p]
        L.orc_penalty_vl_w.restype = C.c_int64
        L.orc_penalty_vl_w.argtypes = [C.c_int32, _i64p]
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_lnt.restype = None
        L.orc_lnt.argtypes = [_i32p]
        L.orc_temperature.restype = None
        L.orc_temperature.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int64, _i64p]
        L.orc_accept.restype = C.c_int
        L.orc_accept.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32]
        L.orc_dominates.restype = C.c_int
        L.orc_dominates.argtypes = [C.c_int64] * 4
        L.orc_archive_explore.restype = C.c_int32
        L.orc_archive_explore.argtypes = [C.POINTER(_Archive), C.c_int64, C.c_int64, _u8p]
        L.orc_archive_exploit.restype = C.c_int32
        L.orc_archive_exploit.argtypes = [C.POINTER(_Archive), C.c_int64, C.c_int64, _u8p, C.c_uint32]
        L.orc_build.restype = C.c_int
        L.orc_build.argtypes = [C.c_int32, _i32p, _i32p, _i32p, C.c_int32, C.POINTER(_Qubo)]
        L.orc_free.restype = None
        L.orc_free.argtypes = [C.POINTER(_Qubo)]
        L.orc_mda_replica.restype = C.c_int
        L.orc_mda_replica.argtypes = [C.POINTER(_Qubo), C.POINTER(_Params), C.c_int32,
                                      C.POINTER(_ReplicaOut)]
        L.orc_gbuild.restype = C.c_int
        L.orc_gbuild.argtypes = [C.c_int32, C.c_int32, _i32p, C.c_void_p, C.POINTER(_GQubo)]
        L.orc_gfree.restype = None
        L.orc_gfree.argtypes = [C.POINTER(_GQubo)]
        L.orc_gdominates.restype = C.c_int
        L.orc_gdominates.argtypes = [C.c_int32, _i64p, _i64p]
        L.orc_gaccept.restype = C.c_int
        L.orc_gaccept.argtypes = [C.c_int32, _i64p, C.c_int64, C.c_int64, C.c_int32, C.c_int32]
        L.orc_garchive_explore.restype = C.c_int32
        L.orc_garchive_explore.argtypes = [C.POINTER(_GArchive), _i64p, _u8p]
        L.orc_garchive_exploit.restype = C.c_int32
        L.orc_garchive_exploit.argtypes = [C.POINTER(_GArchive), _i64p, _u8p, C.c_uint32]
        L.orc_gmda_replica.restype = C.c_int
        L.orc_gmda_replica.argtypes = [C.POINTER(_GQubo), C.POINTER(_Params), C.c_int32,
                                       C.POINTER(_GReplicaOut)]
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def qap_cost(H, D, perm) -> int:
    H, D = _i32(H), _i32(D)
    return int(lib().orc_qap_cost(H.shape[0], H, D, _i32(perm)))


def cost_direct(H, D, x) -> int:
    H, D = _i32(H), _i32(D)
    return int(lib().orc_cost_direct(H.shape[0], H, D, _u8(x)))


def constraint_direct(n, x) -> int:
    return int(lib().orc_constraint_direct(n, _u8(x)))


def cost_qubo(H, D) -> np.ndarray:
    H, D = _i32(H), _i32(D)
    n = H.shape[0]
    out = np.zeros((n * n, n * n), np.int64)
    lib().orc_cost_qubo(n, H, D, out)
    return out


def constraint_qubo(n):
    out = np.zeros((n * n, n * n), np.int64)
    pg = C.c_int64(0)
    lib().orc_constraint_qubo(n, out, C.byref(pg))
    return out, int(pg.value)


def normalise_flows(F, D, log2: int):
    """Objective normalisation (Sec. Parameter Settings): the objective QUBO is
    scaled so that its largest coefficient is 2^log2 (the paper uses 2^23).
    The cost QUBO of Sec. 2.2 is linear in the flows, so the flows are scaled by
    s = 2^log2 / max|C| (C the upper-triangular cost QUBO) and rounded to the
    nearest integer, halves up.  Returns (scaled flows, s); a flow matrix whose
    QUBO vanishes is returned unchanged with s = 1."""
    F = _i32(F)
    mx = int(np.abs(cost_qubo(F, D)).max())
    if mx == 0:
        return F.copy(), 1.0
    s = float(2 ** int(log2)) / float(mx)
    r = np.floor(F.astype(np.float64) * s + 0.5)
    if np.abs(r).max() > np.iinfo(np.int32).max:
        raise OverflowError("scaled flow beyond int32")
    return r.astype(np.int32), s


def qubo_energy(Q, q, x) -> int:
    Q = np.ascontiguousarray(Q, np.int64)
    return int(lib().orc_qubo_energy(Q.shape[0], Q, int(q), _u8(x)))


def delta_energy(Q, x) -> np.ndarray:
    Q = np.ascontiguousarray(Q, np.int64)
    out = np.zeros(Q.shape[0], np.int64)
    lib().orc_delta_energy(Q.shape[0], Q, _u8(x), out)
    return out


def penalty_2max(Cm) -> int:
    Cm = np.ascontiguousarray(Cm, np.int64)
    return int(lib().orc_penalty_2max(Cm.shape[0], Cm))


def penalty_vl_w(Cm) -> int:
    Cm = np.ascontiguousarray(Cm, np.int64)
    return int(lib().orc_penalty_vl_w(Cm.shape[0], Cm))


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                            np.ascontiguousarray(key, np.uint32), out)
    return out


def lnt() -> np.ndarray:
    out = np.zeros(4096, np.int32)
    lib().orc_lnt(out)
    return out


def temperature(delta0, deltaf, xi, steps) -> np.ndarray:
    out = np.zeros(int(steps), np.int64)
    lib().orc_temperature(float(delta0), float(deltaf), float(xi), int(steps), out)
    return out


def accept(dE1, dE2, Eoff, T, lnt_k, mode=STRICT) -> bool:
    return bool(lib().orc_accept(int(dE1), int(dE2), int(Eoff), int(T), int(lnt_k), int(mode)))


def dominates(p, q) -> bool:
    return bool(lib().orc_dominates(int(p[0]), int(p[1]), int(q[0]), int(q[1])))


class Archive:
    """A fixed-capacity archive driven through the oracle's update rules."""

    def __init__(self, cap: int, m: int):
        self.e1 = np.zeros(cap, np.int64)
        self.e2 = np.zeros(cap, np.int64)
        self.x = np.zeros((cap, m), np.uint8)
        self._s = _Archive(0, cap, m, self.e1.ctypes.data, self.e2.ctypes.data, self.x.ctypes.data)

    @property
    def size(self) -> int:
        return int(self._s.size)

    def explore(self, e1, e2, x) -> int:
        return int(lib().orc_archive_explore(C.byref(self._s), int(e1), int(e2), _u8(x)))

    def exploit(self, e1, e2, x, w) -> int:
        return int(lib().orc_archive_exploit(C.byref(self._s), int(e1), int(e2), _u8(x), int(w) & 0xFFFFFFFF))

    def entries(self):
        k = self.size
        return [(int(self.e1[i]), int(self.e2[i])) for i in range(k)]


class Qubo:
    """Y and Z of Eq. (wqubom) for one bi-objective QAP instance, built by the oracle."""

    def __init__(self, F1, F2, D, penalty: int = PEN_2MAX):
        self.F1, self.F2, self.D = _i32(F1), _i32(F2), _i32(D)
        self.n = self.D.shape[0]
        self._q = _Qubo()
        rc = lib().orc_build(self.n, self.F1, self.F2, self.D, penalty, C.byref(self._q))
        if rc != 0:
            raise MemoryError("oracle QUBO build failed")

    def __del__(self):
        try:
            lib().orc_free(C.byref(self._q))
        except Exception:
            pass

    @property
    def m(self):
        return self._q.m

    @property
    def alpha(self):
        return int(self._q.alpha1), int(self._q.alpha2)

    @property
    def q(self):
        return int(self._q.q1), int(self._q.q2)

    @property
    def maxabs_c(self):
        return int(self._q.maxabs_c)

    @property
    def overflow(self):
        return bool(self._q.overflow)

    def P(self, k: int) -> np.ndarray:
        """Copy of the symmetric matrix P_k (diagonal = Y_aa)."""
        m = self.m
        ptr = self._q.P1 if k == 1 else self._q.P2
        buf = (C.c_int64 * (m * m)).from_address(ptr)
        return np.frombuffer(buf, dtype=np.int64).reshape(m, m).copy()

    def Y(self, k: int) -> np.ndarray:
        return np.triu(self.P(k))


def default_schedule(maxabs_c: int, steps: int):
    """The schedule of Table (param) scaled to unnormalised coefficients: the paper
    uses delta0 = 1e9 and deltaf = 1e4 on QUBOs whose largest coefficient is 2^23;
    here both are scaled by max|C| / 2^23.  beta = max(1, floor(delta0 / steps))."""
    d0 = 1e9 * float(maxabs_c) / 8388608.0
    df = 1e4 * float(maxabs_c) / 8388608.0
    beta = max(1, int(np.floor(d0 / max(1, steps))))
    return d0, df, 0.001, beta


def run_replica(q: Qubo, r: int, steps: int, delta0: float, deltaf: float, xi: float,
                beta: int, seed: int, accept: int = STRICT, archive: int = EXPLORE,
                escape: int = ESC_OFFSET, archive_size: int = 0, trace: bool = False,
                temp_table=None) -> dict:
    """Runs replica r of Algorithm 3 and returns its final state and raw archive.
    temp_table (steps int64 entries, T_t in fixed point) replaces the geometric
    schedule of delta0, deltaf and xi when given."""
    m = q.m
    s = archive_size if archive_size > 0 else m
    x = np.zeros(m, np.uint8)
    h1 = np.zeros(m, np.int64)
    h2 = np.zeros(m, np.int64)
    state = np.zeros(4, np.int64)
    asz = np.zeros(1, np.int32)
    ae = np.zeros(2 * s, np.int64)
    ax = np.zeros((s, m), np.uint8)
    tr = np.zeros(int(steps), np.int32) if trace else None
    out = _ReplicaOut(x.ctypes.data, h1.ctypes.data, h2.ctypes.data, state.ctypes.data,
                      asz.ctypes.data, ae.ctypes.data, ax.ctypes.data,
                      tr.ctypes.data if trace else None)
    tt = None
    if temp_table is not None:
        tt = np.ascontiguousarray(temp_table, np.int64)
        if tt.shape != (int(steps),):
            raise ValueError("temp_table needs one entry per step")
    p = _Params(int(steps), float(delta0), float(deltaf), float(xi), int(beta), accept, archive,
                escape, int(archive_size), int(seed) & 0xFFFFFFFFFFFFFFFF,
                tt.ctypes.data if tt is not None else None)
    rc = lib().orc_mda_replica(C.byref(q._q), C.byref(p), int(r), C.byref(out))
    if rc != 0:
        raise ValueError("oracle run failed: %d" % rc)
    k = int(asz[0])
    res = dict(x=x, h1=h1, h2=h2, E1=int(state[0]), E2=int(state[1]), Eoff=int(state[2]),
               moves=int(state[3]), arch_size=k, arch_e1=ae[0:2 * k:2].copy(),
               arch_e2=ae[1:2 * k:2].copy(), arch_x=ax[:k].copy())
    if trace:
        res["trace"] = tr
    return res


def nondominated(e1, e2):
    """Indices of entries that no other entry dominates (Section 3.3), ascending."""
    e1 = np.asarray(e1, np.int64)
    e2 = np.asarray(e2, np.int64)
    keep = []
    for i in range(len(e1)):
        dominated = False
        for j in range(len(e1)):
            if j != i and dominates((e1[j], e2[j]), (e1[i], e2[i])):
                dominated = True
                break
        if not dominated:
            keep.append(i)
    return keep


# ---------------------------------------------------------------- K objectives on a generic QUBO

class GQubo:
    """K objectives x^T Q_k x + q_k over m bits (readings G1-G3 of the C header)."""

    def __init__(self, Q, q=None):
        Q = np.ascontiguousarray(Q, np.int32)
        if Q.ndim != 3 or Q.shape[1] != Q.shape[2]:
            raise ValueError("Q must be K x m x m")
        self.K, self.m = int(Q.shape[0]), int(Q.shape[1])
        self.Q = Q
        self.q0 = np.zeros(self.K, np.int64) if q is None else np.ascontiguousarray(q, np.int64)
        self._g = _GQubo()
        rc = lib().orc_gbuild(self.m, self.K, Q, self.q0.ctypes.data, C.byref(self._g))
        if rc != 0:
            raise MemoryError("oracle generic QUBO build failed")

    def __del__(self):
        try:
            lib().orc_gfree(C.byref(self._g))
        except Exception:
            pass

    @property
    def maxabs_c(self):
        return int(self._g.maxabs_c)

    @property
    def overflow(self):
        return bool(self._g.overflow)

    def P(self, k: int) -> np.ndarray:
        """Copy of the symmetric form P_k (k = 0..K-1)."""
        m = self.m
        buf = (C.c_int64 * (self.K * m * m)).from_address(self._g.P)
        return np.frombuffer(buf, dtype=np.int64).reshape(self.K, m, m)[k].copy()


def gdefault_schedule(maxabs_c: int, steps: int):
    """Table (param) scaled by max|C| / 2^23, as for the bQAP."""
    return default_schedule(maxabs_c, steps)


def gdominates(p, q) -> bool:
    p = np.ascontiguousarray(p, np.int64)
    q = np.ascontiguousarray(q, np.int64)
    return bool(lib().orc_gdominates(len(p), p, q))


def gaccept(dE, Eoff, T, lnt_k, mode=STRICT) -> bool:
    dE = np.ascontiguousarray(dE, np.int64)
    return bool(lib().orc_gaccept(len(dE), dE, int(Eoff), int(T), int(lnt_k), int(mode)))


class GArchive:
    """A fixed-capacity K-objective archive driven through the oracle's rules."""

    def __init__(self, cap: int, m: int, K: int):
        self.e = np.zeros((cap, K), np.int64)
        self.x = np.zeros((cap, m), np.uint8)
        self.K = K
        self._s = _GArchive(0, cap, m, K, self.e.ctypes.data, self.x.ctypes.data)

    @property
    def size(self) -> int:
        return int(self._s.size)

    def explore(self, e, x) -> int:
        return int(lib().orc_garchive_explore(C.byref(self._s), np.ascontiguousarray(e, np.int64), _u8(x)))

    def exploit(self, e, x, w) -> int:
        return int(lib().orc_garchive_exploit(C.byref(self._s), np.ascontiguousarray(e, np.int64), _u8(x),
                                              int(w) & 0xFFFFFFFF))

    def entries(self):
        return [tuple(int(v) for v in self.e[i]) for i in range(self.size)]


def run_greplica(g: GQubo, r: int, steps: int, delta0: float, deltaf: float, xi: float, beta: int, seed: int,
                 accept: int = STRICT, archive: int = EXPLORE, escape: int = ESC_OFFSET, archive_size: int = 0,
                 trace: bool = False, temp_table=None) -> dict:
    """Replica r of the K-objective MDA; returns its final state and raw archive."""
    m, K = g.m, g.K
    s = archive_size if archive_size > 0 else m
    x = np.zeros(m, np.uint8)
    h = np.zeros((K, m), np.int64)
    state = np.zeros(K + 2, np.int64)
    asz = np.zeros(1, np.int32)
    ae = np.zeros((s, K), np.int64)
    ax = np.zeros((s, m), np.uint8)
    tr = np.zeros(int(steps), np.int32) if trace else None
    tt = None
    if temp_table is not None:
        tt = np.ascontiguousarray(temp_table, np.int64)
    out = _GReplicaOut(x.ctypes.data, h.ctypes.data, state.ctypes.data, asz.ctypes.data, ae.ctypes.data,
                       ax.ctypes.data, tr.ctypes.data if trace else None)
    p = _Params(int(steps), float(delta0), float(deltaf), float(xi), int(beta), accept, archive,
                escape, int(archive_size), int(seed) & 0xFFFFFFFFFFFFFFFF, tt.ctypes.data if tt is not None else None)
    rc = lib().orc_gmda_replica(C.byref(g._g), C.byref(p), int(r), C.byref(out))
    if rc != 0:
        raise ValueError("oracle run failed: %d" % rc)
    k = int(asz[0])
    res = dict(x=x, h=h, E=[int(v) for v in state[:K]], Eoff=int(state[K]), moves=int(state[K + 1]),
               arch_size=k, arch_e=ae[:k].copy(), arch_x=ax[:k].copy())
    if trace:
        res["trace"] = tr
    return res


def gnondominated(E):
    """Indices of rows of E (N x K) that no other row dominates, ascending."""
    E = np.asarray(E, np.int64)
    keep = []
    for i in range(len(E)):
        if not any(j != i and gdominates(E[j], E[i]) for j in range(len(E))):
            keep.append(i)
    return keep
