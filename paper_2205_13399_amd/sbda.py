"""Scalarisation-based DA (Algorithm SB-DA of Section 3.2) on the same kernels.

For each weight gamma = g / 10, g = 0..10, the aggregated cost QUBO
C = gamma R + (1 - gamma) S (scaled by 10 to stay integer: the cost QUBO of
the flows 10 gamma F1 + (10 - 10 gamma) F2, since C is linear in the flows;
built by the library's qubo_build_scalarised) gets its own penalty (Eq.
vermap / wvermaa) and is solved by the DA (Algorithm 1).  The DA is the multi-objective annealer with a second
objective identically zero: the strict rule then reduces to Eq. paccepts and
the archive holds the lowest-energy states, so each replica's best solution
is its archive entry of least E1 (found on the device by da_best).  Every weight runs in one batched launch;
replica r of every weight together form SB-DA run r, whose result is the
non-dominated subset of its 11 solutions in the true objectives (f1, f2).

With normalisation (Sec. Parameter Settings), R and S are first put on the
same scale -- both flow matrices scaled so that max|R| = max|S| = 2^L -- and
the aggregation uses the scaled flows; the points are still reported in the
true objectives.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import mda, quality

WEIGHTS = tuple(range(11))   # 10 gamma


def qap_cost(F: np.ndarray, D: np.ndarray, perm: np.ndarray) -> int:
    """Eq. nqap: sum_ij F[i][j] D[perm i][perm j]."""
    p = np.asarray(perm, np.int64)
    return int((np.asarray(F, np.int64) * np.asarray(D, np.int64)[np.ix_(p, p)]).sum())


@dataclass
class SbdaResult:
    runs: list                # one mda.Run per weight
    weights: tuple
    best: np.ndarray          # [weights, replicas, 2] archive energy (E1, slot) of each replica's best
    points: List[np.ndarray]  # per SB-DA run (replica): non-dominated (f1, f2) of its feasible solutions
    perms: List[np.ndarray]   # per SB-DA run: the permutations of those points
    normalise_log2: int = 0   # L of the normalisation applied (0: none)


def _aggregated_qubos(F1, F2, D, weights, penalty, path, stream):
    """qubo_build_scalarised for every weight."""
    return [mda.Qubo(F1, F2, D, penalty=penalty, path=path, stream=stream, scalarise=g) for g in weights]


def normalised_qubos(F1, F2, D, normalise: int, weights: Sequence[int] = WEIGHTS, penalty: int = mda.PEN_VL,
                     path: int = mda.PATH_KRON, stream: Optional[int] = None):
    """The aggregated QUBOs of normalised R and S: L = normalise, or with
    NORM_AUTO the largest L <= 23 for which the normalisation and every
    aggregated QUBO pass the library's bounds (int64 fields where the int32
    ones fail).  Returns (qubos, L)."""
    for L in ([normalise] if normalise > 0 else range(23, 0, -1)):
        try:
            q = mda.Qubo(F1, F2, D, penalty=penalty, path=path, stream=stream, normalise=L)
            A, B = q.flows()
            q.close()
            return _aggregated_qubos(A, B, D, weights, penalty, path, stream), L
        except mda.MdaError as e:
            if normalise > 0 or e.code != mda.MDA_EOVERFLOW:
                raise
    raise mda.MdaError(mda.MDA_EOVERFLOW, "no normalisation 2^L, 1 <= L <= 23, fits every aggregated QUBO")


def sbda(F1, F2, D, replicas: int, steps: int, seed: int, weights: Sequence[int] = WEIGHTS,
         penalty: int = mda.PEN_VL, path: int = mda.PATH_KRON, stream: Optional[int] = None,
         graph: bool = False, normalise: int = mda.NORM_NONE) -> SbdaResult:
    """Runs SB-DA: weight g uses Philox key seed + g."""
    F1 = np.asarray(F1, np.int32)
    F2 = np.asarray(F2, np.int32)
    D = np.asarray(D, np.int32)
    n = D.shape[0]
    if normalise == mda.NORM_NONE:
        qs, L = _aggregated_qubos(F1, F2, D, weights, penalty, path, stream), 0
    else:
        qs, L = normalised_qubos(F1, F2, D, normalise, weights, penalty, path, stream)
    ps = [mda.make_params(replicas, steps, seed + g, stream=stream, graph=graph) for g in weights]
    runs = mda.da_run_batch(qs, ps)
    best = np.zeros((len(weights), replicas, 2), np.int64)
    cand = [[] for _ in range(replicas)]
    for w, run in enumerate(runs):
        e1, slot = run.best()                     # da_best: least E1, first slot on ties
        best[w, :, 0] = e1
        best[w, :, 1] = slot
        for r in range(replicas):
            if slot[r] < 0:
                continue
            a = run.archive(r, raw=True)
            k = int(slot[r])
            if a.feasible[k]:
                perm = a.perm[k]
                cand[r].append((qap_cost(F1, D, perm), qap_cost(F2, D, perm), perm.copy()))
    points, perms = [], []
    for r in range(replicas):
        if not cand[r]:
            points.append(np.zeros((0, 2), np.int64))
            perms.append(np.zeros((0, n), np.int32))
            continue
        pts = np.array([(c[0], c[1]) for c in cand[r]], np.int64)
        nd = quality.nondominated(pts)
        points.append(pts[nd])
        perms.append(np.array([cand[r][k][2] for k in nd], np.int32))
    return SbdaResult(runs=runs, weights=tuple(weights), best=best, points=points, perms=perms, normalise_log2=L)
