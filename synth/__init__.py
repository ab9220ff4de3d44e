"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers only. It holds none of the search method's
arithmetic: no distances, no graphs, no selection. Both the HIP path and the
CPU oracle take its arrays as plain inputs.

The data stand in for the paper's evaluation sets (Sift, Gist, Deep, Wiki;
Table 2), which are not available here. They are Gaussian mixtures with the
shapes, dimensions and value scale of those workloads:

    centers ~ N(0, 1)^{C x d}
    x       = centers[comp] + sigma * N(0, 1)^d,   comp ~ U{0..C-1}

Generation is chunked in blocks of 2^20 rows, each block drawing from its own
PCG64 stream keyed by (seed, block index), so any row range can be produced
without generating the rows before it, and the result does not depend on how
many rows are requested at once.
"""
from __future__ import annotations

import numpy as np

CHUNK = 1 << 20

# Seed roles (one stream per role).
SEED_CENTERS = 0
SEED_BASE = 1
SEED_QUERIES = 2
SEED_HELDOUT = 3
SEED_ARRIVALS = 7


def centers(C: int, d: int, seed: int = SEED_CENTERS) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((C, d)).astype(np.float32)


def mixture(n: int, d: int, C: int, sigma: float, seed: int,
            centers_seed: int = SEED_CENTERS, start: int = 0) -> np.ndarray:
    """Rows [start, start+n) of the mixture stream `seed` (float32, row-major)."""
    cen = centers(C, d, centers_seed)
    out = np.empty((n, d), dtype=np.float32)
    row = start
    end = start + n
    while row < end:
        blk = row // CHUNK
        b0 = blk * CHUNK
        rng = np.random.Generator(np.random.PCG64([seed, blk]))
        comp = rng.integers(0, C, CHUNK)
        lo = row - b0
        hi = min(end - b0, CHUNK)
        # draw the whole block's noise so that a row's value is independent of the range asked for
        noise = rng.standard_normal((CHUNK, d), dtype=np.float32)
        out[row - start: row - start + (hi - lo)] = cen[comp[lo:hi]] + np.float32(sigma) * noise[lo:hi]
        row = b0 + hi
    return out


def mixture_small(n: int, d: int, C: int, sigma: float, seed: int,
                  centers_seed: int = SEED_CENTERS) -> np.ndarray:
    """Small-n variant: one stream, no block padding (cheap for tests)."""
    cen = centers(C, d, centers_seed)
    rng = np.random.Generator(np.random.PCG64([seed, 0x5EED]))
    comp = rng.integers(0, C, n)
    noise = rng.standard_normal((n, d), dtype=np.float32)
    return (cen[comp] + np.float32(sigma) * noise).astype(np.float32)


def to_u8(x: np.ndarray) -> np.ndarray:
    """Quantise-and-clip map used for the uint8 workload: clip(rint(128 + 32 x), 0, 255)."""
    return np.clip(np.rint(128.0 + 32.0 * x.astype(np.float64)), 0, 255).astype(np.uint8)


def uniform_ints(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi, n)


def random_graph(n: int, deg: int, seed: int) -> np.ndarray:
    """A random fixed-degree digraph with distinct, non-self neighbours per row (test input)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.empty((n, deg), dtype=np.uint32)
    for u in range(n):
        cand = rng.choice(n - 1, size=deg, replace=False)
        cand[cand >= u] += 1
        g[u] = cand
    return g


# Workload recipes (sizes of the paper-shaped configurations).
WORKLOADS = {
    "tiny": dict(N=10_000, d=128, C=32, sigma=0.3, dtype="f32", deg=32, nq=1_000, k=10, itopk=64),
    "sharded1m": dict(N=1_000_000, d=96, C=1_000, sigma=0.25, dtype="f32", deg=32, nq=10_000, k=10,
                      shards=4, ghost_ratio=0.01),
    "lowprec5m": dict(N=5_000_000, d=256, C=2_000, sigma=0.2, dtype="f32", deg=64, nq=100_000, k=10),
    "learned10m": dict(N=10_000_000, d=96, C=4_000, sigma=0.25, dtype="f32", deg=32, nq=100_000, k=10,
                       ghosts=4096),
    "serving20m": dict(N=20_000_000, d=128, C=4_000, sigma=0.25, dtype="u8", deg=64),
}
