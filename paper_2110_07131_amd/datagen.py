"""Seeded synthetic inputs for reverse k-MIPS workloads.

This module only draws random vectors; it contains none of the method's
arithmetic and is shared by the HIP path's callers and by the CPU oracle's
tests.  It imports nothing from the native library.

Vector recipe (the paper evaluates on 50-dimensional matrix-factorisation
vectors of MovieLens/Netflix/Amazon/Yahoo!, Section 5.1 / Table 2; those
factors are not available, so seeded synthetic vectors of the same shape stand
in for them):

    x ~ N(0, I_d),  r ~ LogNormal(0, sigma),  v = r * x / ||x||

so every vector's norm is r (before rounding) and its direction is uniform on
the sphere.  Vectors are stored as float32 (round to nearest even).  Users,
items and query indices come from three independent PCG64 streams spawned from
one SeedSequence.  Queries are items drawn uniformly from P without
replacement, as in the paper's protocol (Section 5.1).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["vectors", "Workload", "workload", "CONFIGS", "small_int_vectors"]


def vectors(n: int, d: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """n float32 vectors of dimension d with log-normal norms (see module doc)."""
    if n == 0:
        return np.zeros((0, d), np.float32)
    x = rng.standard_normal((n, d))
    r = rng.lognormal(0.0, sigma, n)
    nx = np.linalg.norm(x, axis=1)
    nx[nx == 0.0] = 1.0
    v = x * (r / nx)[:, None]
    return np.ascontiguousarray(v.astype(np.float32))


@dataclasses.dataclass
class Workload:
    Q: np.ndarray          # users, float32 [n, d]
    P: np.ndarray          # items, float32 [m, d]
    qidx: np.ndarray       # int64 [nq]: query items are P[qidx]
    ks: np.ndarray         # int32 [nq]: k of each query (may be all equal)

    @property
    def queries(self) -> np.ndarray:
        return np.ascontiguousarray(self.P[self.qidx])


def workload(n: int, m: int, d: int, sigma: float, n_queries: int, seed: int = 0,
             k_choices=None, k_max: int | None = None) -> Workload:
    """Draw users, items and query indices from three spawned PCG64 streams.

    k_choices: None (every query at k = k_max), an int (fixed k), a list of k
    values (every query item is evaluated at every listed k: the query list is
    the cross product, item-major), or the string "uniform" (k ~ U{1..k_max},
    drawn from the query stream).
    """
    ss = np.random.SeedSequence(seed).spawn(3)
    gq = np.random.Generator(np.random.PCG64(ss[0]))
    gp = np.random.Generator(np.random.PCG64(ss[1]))
    gi = np.random.Generator(np.random.PCG64(ss[2]))
    Q = vectors(n, d, sigma, gq)
    P = vectors(m, d, sigma, gp)
    nq = min(n_queries, m)
    qidx = gi.choice(m, nq, replace=False) if nq > 0 else np.zeros(0, np.int64)
    if k_choices is None:
        ks = np.full(nq, k_max if k_max else 1, np.int32)
    elif isinstance(k_choices, (int, np.integer)):
        ks = np.full(nq, int(k_choices), np.int32)
    elif isinstance(k_choices, str) and k_choices == "uniform":
        ks = gi.integers(1, int(k_max) + 1, nq).astype(np.int32)
    else:
        kl = np.asarray(k_choices, np.int32)
        qidx = np.repeat(np.asarray(qidx, np.int64), len(kl))
        ks = np.tile(kl, nq)
    return Workload(Q, P, np.asarray(qidx, np.int64), ks)


def small_int_vectors(n: int, d: int, lo: int, hi: int, rng: np.random.Generator) -> np.ndarray:
    """Integer-valued float32 vectors in [lo, hi]; all dot products are exact
    in float32, bfloat16 products and float64, and ties are frequent."""
    return rng.integers(lo, hi + 1, (n, d)).astype(np.float32)


# Workload shapes.  "parity" is the small case the oracle finishes in
# seconds; the others are the evaluation workloads (user/item counts,
# dimension, log-normal sigma, k_max, query count, k values).
CONFIGS = {
    "parity": dict(n=2000, m=1000, d=50, sigma=0.5, k_max=10, n_queries=20, ks=[1]),
    "plain": dict(n=100_000, m=20_000, d=50, sigma=0.5, k_max=25, n_queries=1000, ks=[1, 5, 10, 25]),
    "precision": dict(n=1_000_000, m=100_000, d=100, sigma=0.5, k_max=25, n_queries=1000, ks=[1, 10, 25]),
    "batched": dict(n=500_000, m=50_000, d=200, sigma=0.8, k_max=50, n_queries=4096, ks="uniform"),
    "serve_small": dict(n=50_000, m=10_000, d=50, sigma=0.5, k_max=25, n_queries=10_000, ks="uniform"),
    "serve_mid": dict(n=500_000, m=50_000, d=100, sigma=0.5, k_max=25, n_queries=10_000, ks="uniform"),
    "serve_large": dict(n=2_000_000, m=100_000, d=200, sigma=0.5, k_max=25, n_queries=10_000, ks="uniform"),
}


def config_workload(name: str, seed: int = 0, n_queries: int | None = None) -> Workload:
    c = CONFIGS[name]
    ks = c["ks"]
    nq = c["n_queries"] if n_queries is None else n_queries
    return workload(c["n"], c["m"], c["d"], c["sigma"], nq, seed,
                    k_choices=ks, k_max=c["k_max"])
