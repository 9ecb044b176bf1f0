"""Seeded synthetic bi-objective QAP instances.

This module only draws inputs (flow matrices F1, F2 and a distance matrix D); it
holds none of the annealer's arithmetic and is shared by the oracle tests, the
GPU tests and the benchmark.  The paper evaluates on the structured qapStr
benchmark instances of Section 4.1 (n in {25, 50}, objective correlation
rho in {-0.75, 0, 0.75}); those instances are not available here, so these
seeded stand-ins with the same sizes and correlation levels take their place.

Recipe (all integers, deterministic for a given seed):
  * D: n points drawn uniformly on the integer grid {0..99}^2; D[u][v] is the
    Euclidean distance rounded to the nearest integer, computed exactly in
    integer arithmetic; symmetric with a zero diagonal.
  * F1, F2 ("structured"): for every pair i < j a standard bivariate normal
    (z1, z2) with correlation rho is mapped through the normal CDF to (p1, p2);
    F_k = 0 when p_k < 0.5 (half of all pairs), else min(99, floor(200 (p_k - 0.5))),
    so non-zero flows are uniform on {0..99}.  Mirrored to j > i, zero diagonal.
  * F1, F2 ("uniform", the small plain case): independent uniform {0..99} entries
    for i < j, mirrored, zero diagonal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["Instance", "make_instance", "distances", "instance_seed"]


@dataclass
class Instance:
    n: int
    F1: np.ndarray   # int32 n x n
    F2: np.ndarray   # int32 n x n
    D: np.ndarray    # int32 n x n
    rho: float
    seed: int

    @property
    def m(self) -> int:
        return self.n * self.n


def _round_sqrt(k: int) -> int:
    """Nearest integer to sqrt(k) for a non-negative integer k (never a tie)."""
    r = math.isqrt(k)
    return r + 1 if k - r * r > r else r


def distances(n: int, rng: np.random.Generator) -> np.ndarray:
    pts = rng.integers(0, 100, size=(n, 2))
    D = np.zeros((n, n), np.int32)
    for u in range(n):
        for v in range(n):
            dx = int(pts[u, 0] - pts[v, 0])
            dy = int(pts[u, 1] - pts[v, 1])
            D[u, v] = _round_sqrt(dx * dx + dy * dy)
    return D


def _norm_cdf(z: np.ndarray) -> np.ndarray:
    from scipy.special import ndtr
    return ndtr(z)


def make_instance(n: int, rho: float = 0.0, seed: int = 0, structured: bool = True) -> Instance:
    """One seeded instance; see the module docstring for the recipe."""
    if n < 2:
        raise ValueError("n must be >= 2")
    rng = np.random.Generator(np.random.PCG64(seed))
    D = distances(n, rng)
    iu, ju = np.triu_indices(n, k=1)
    npairs = iu.size
    if structured:
        g1 = rng.standard_normal(npairs)
        g2 = rng.standard_normal(npairs)
        z1 = g1
        z2 = rho * g1 + math.sqrt(max(0.0, 1.0 - rho * rho)) * g2
        vals = []
        for z in (z1, z2):
            p = _norm_cdf(z)
            f = np.where(p < 0.5, 0, np.minimum(99, np.floor(200.0 * (p - 0.5)))).astype(np.int32)
            vals.append(f)
    else:
        vals = [rng.integers(0, 100, size=npairs).astype(np.int32) for _ in range(2)]
    Fs = []
    for v in vals:
        F = np.zeros((n, n), np.int32)
        F[iu, ju] = v
        F[ju, iu] = v
        Fs.append(F)
    return Instance(n=n, F1=Fs[0], F2=Fs[1], D=D, rho=float(rho), seed=int(seed))


def instance_seed(config: int, index: int) -> int:
    """Seed convention: config * 1e6 + instance index (config 0 uses seed 0)."""
    return int(config) * 1_000_000 + int(index)
