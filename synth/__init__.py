"""Seeded synthetic instances shaped like the paper's workloads.

This module only produces inputs (graphs as symmetric CSR, dense coupling
matrices, request streams).  It holds none of the annealing method's
arithmetic and uses numpy's PCG64 generator, so both the CPU oracle and the
GPU library can be fed the same instance.

Shapes (the paper's G-set graphs are not available, so these stand in):
  * random sparse Max-Cut graph with n vertices and m distinct edges drawn
    uniformly from all vertex pairs, weight +1 (the G1-like shape, n = 800,
    m = 19,176);
  * a 2-D toroidal grid with +-1 weights (the degree-4 G-set tori, e.g.
    100 x 200 = 20,000 vertices);
  * a dense +-1 coupling matrix with zero diagonal (stand-in for the
    fully-connected 100,000-spin instance);
  * a Poisson stream of mixed Max-Cut requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    w: np.ndarray        # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def edges(self) -> int:
        return self.nnz // 2


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray) -> Graph:
    """Symmetric CSR (both directions) with columns sorted in each row."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    w = np.asarray(w, np.int32)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32), ww.astype(np.int32))


def _unrank_pairs(idx: np.ndarray, n: int):
    """Map k in [0, n(n-1)/2) to the k-th pair (i < j) in row-major order."""
    idx = np.asarray(idx, np.int64)
    # row i holds pairs (i, i+1..n-1): start(i) = i*n - i*(i+1)/2
    i = (n - 2 - np.floor(np.sqrt(-8.0 * idx + 4.0 * n * (n - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
    start = i * n - i * (i + 1) // 2
    # guard against floating error at row boundaries
    fix_lo = idx < start
    while np.any(fix_lo):
        i[fix_lo] -= 1
        start = i * n - i * (i + 1) // 2
        fix_lo = idx < start
    nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
    fix_hi = idx >= nxt
    while np.any(fix_hi):
        i[fix_hi] += 1
        start = i * n - i * (i + 1) // 2
        nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
        fix_hi = idx >= nxt
    j = idx - start + i + 1
    return i, j


def random_graph(n: int, m: int, seed: int, weights: str = "one") -> Graph:
    """G(n, m): m distinct unordered pairs uniform over all n(n-1)/2 pairs."""
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("too many edges")
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.choice(total, size=m, replace=False)
    i, j = _unrank_pairs(idx, n)
    if weights == "one":
        w = np.ones(m, np.int32)
    else:
        w = np.where(rng.integers(0, 2, size=m) == 1, 1, -1).astype(np.int32)
    return csr_from_edges(n, i, j, w)


def torus(width: int, height: int, seed: int, weights: str = "pm1") -> Graph:
    """width x height periodic grid; vertex id = y*width + x; edges to
    (x+1 mod width, y) and (x, y+1 mod height)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ys, xs = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    vid = (ys * width + xs).ravel()
    right = (ys * width + (xs + 1) % width).ravel()
    down = (((ys + 1) % height) * width + xs).ravel()
    u = np.concatenate([vid, vid])
    v = np.concatenate([right, down])
    if weights == "pm1":
        w = np.where(rng.integers(0, 2, size=u.size) == 1, 1, -1).astype(np.int32)
    else:
        w = np.ones(u.size, np.int32)
    return csr_from_edges(width * height, u, v, w)


def dense_pm1(n: int, seed: int) -> np.ndarray:
    """Symmetric int8 matrix with +-1 off-diagonal entries, zero diagonal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    up = np.where(rng.integers(0, 2, size=(n, n)) == 1, 1, -1).astype(np.int8)
    up = np.triu(up, 1)
    return (up + up.T).astype(np.int8)


def csr_from_dense(J: np.ndarray) -> Graph:
    i, j = np.nonzero(np.triu(J, 1))
    return csr_from_edges(J.shape[0], i, j, J[i, j].astype(np.int32))


# ---------------------------------------------------------------- configs
def config_c1_graph(seed: int = 1) -> Graph:
    """Plain-PAMC sparse Max-Cut instance: n = 800, 19,176 edges, w = +1."""
    return random_graph(800, 19176, seed)


def config_c2_graph(seed: int = 1) -> Graph:
    """100 x 200 torus with +-1 weights (n = 20,000, degree 4)."""
    return torus(100, 200, seed)


def config_c4_graph(seed: int = 1) -> Graph:
    """Max-3-Cut source graph: n = 7,000, average degree 6 (21,000 edges)."""
    return random_graph(7000, 21000, seed)


@dataclass
class Request:
    index: int
    arrival_s: float
    graph: Graph
    seed: int


def request_stream(count: int, rate_per_s: float, seed: int, n_min: int = 800, n_max: int = 20000):
    """Mixed Max-Cut requests: n log-uniform in [n_min, n_max]; even index a
    random graph with average degree U[4, 50] and w = +1, odd index a torus
    with +-1 weights (even sides, so the torus is bipartite)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_per_s) if rate_per_s > 0 else 0.0
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        gseed = int(rng.integers(0, 2**31))
        if i % 2 == 0:
            d = rng.uniform(4.0, 50.0)
            m = min(int(round(n * d / 2)), n * (n - 1) // 2)
            g = random_graph(n, m, gseed)
        else:
            h = max(4, 2 * int(round(math.sqrt(n / 2) / 2)))
            wdt = max(4, 2 * int(round(n / (2 * h))))
            g = torus(wdt, h, gseed)
        out.append(Request(i, t, g, seed * 100003 + i))
    return out
