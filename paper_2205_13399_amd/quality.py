"""Quality of bi-objective solution sets (minimisation): non-dominated
filtering and the 2-D hypervolume with the normalisation used by the paper's
evaluation (Section 4: every energy mapped to [1, 2] over all compared sets,
reference point (2.1, 2.1), largest possible value 1.21).  Host-side
reporting on results already copied from the device."""
from __future__ import annotations

from typing import Iterable, List, Sequence, Tuple

import numpy as np


def nondominated(points: np.ndarray) -> np.ndarray:
    """Indices of the points no other point dominates (Section 3.3: <= in both
    objectives and < in one), duplicates reduced to their first occurrence,
    in ascending (f1, f2) order."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    if len(p) == 0:
        return np.zeros(0, np.int64)
    order = np.lexsort((np.arange(len(p)), p[:, 1], p[:, 0]))
    keep = []
    best2 = np.inf
    for k in order:
        if p[k, 1] < best2:
            keep.append(k)
            best2 = p[k, 1]
    return np.asarray(keep, np.int64)


def hypervolume_2d(points: np.ndarray, ref: Tuple[float, float] = (2.1, 2.1)) -> float:
    """Area dominated by the points and bounded by ref (minimisation)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    p = p[(p[:, 0] < ref[0]) & (p[:, 1] < ref[1])]
    if len(p) == 0:
        return 0.0
    nd = p[nondominated(p)]           # ascending f1, strictly descending f2
    hv, prev2 = 0.0, ref[1]
    for f1, f2 in nd:
        hv += (ref[0] - f1) * (prev2 - f2)
        prev2 = f2
    return float(hv)


def normaliser(point_sets: Iterable[np.ndarray]):
    """Affine map of each objective onto [1, 2] over the union of the sets."""
    allp = np.concatenate([np.asarray(s, np.float64).reshape(-1, 2) for s in point_sets])
    lo, hi = allp.min(axis=0), allp.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    return lambda s: 1.0 + (np.asarray(s, np.float64).reshape(-1, 2) - lo) / span


def compare(sets: Sequence[np.ndarray]) -> List[dict]:
    """Non-dominated count and normalised hypervolume of each set, the
    normalisation taken over all of them together."""
    norm = normaliser(sets)
    out = []
    for s in sets:
        s = np.asarray(s, np.float64).reshape(-1, 2)
        nd = s[nondominated(s)] if len(s) else s
        out.append({"nondominated": int(len(nd)), "hypervolume": hypervolume_2d(norm(nd)) if len(nd) else 0.0})
    return out
