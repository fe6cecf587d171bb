"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds none of the diffusion arithmetic: it only draws graphs, seed
nodes, tolerances, arrival times and edge-insert batches.

Graph recipe (undirected Chung-Lu, power-law expected degrees):

* target weights ``w_i = (i+1)^(-1/(gamma-1))`` scaled to mean ``2E/n``, capped at
  ``sqrt(n * 2E/n)`` (structural cut-off); three rescale-and-cap passes;
* exactly ``E`` distinct undirected edges drawn i.i.d. proportional to ``w``
  (self-loops and repeats skipped, first occurrences in sampling order win);
* a seeded random relabelling of the nodes, so ids carry no degree order;
* symmetric int32 CSR with ascending neighbour lists (``nnz = 2E``).

Random streams: ``numpy.random.SeedSequence(seed)`` spawns the children
[graph, seeds, eps, arrivals, inserts]; the graph stream drives the native
SplitMix64 sampler in ``chung_lu.c``.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chung_lu.c")
_LIB = os.path.join(_HERE, "libchunglu.so")
_lock = threading.Lock()
_lib = None

STREAMS = ("graph", "seeds", "eps", "arrivals", "inserts")


def build(force: bool = False) -> str:
    """Compile the native sampler (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB)
            p = C.c_void_p
            lib.cl_sample_edges.argtypes = [C.c_int64, p, C.c_int64, C.c_uint64, p]
            lib.cl_sample_edges.restype = C.c_int64
            lib.cl_permutation.argtypes = [C.c_int64, C.c_uint64, p]
            lib.cl_permutation.restype = None
            lib.cl_build_csr.argtypes = [C.c_int64, C.c_int64, p, p, p, p]
            lib.cl_build_csr.restype = C.c_int
            lib.cl_components.argtypes = [C.c_int64, p, p, p]
            lib.cl_components.restype = None
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def streams(seed: int) -> dict:
    """One independent ``numpy.random.Generator`` per input stream."""
    children = np.random.SeedSequence(seed).spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(c)) for name, c in zip(STREAMS, children)}


def power_law_weights(n: int, E: int, gamma: float) -> np.ndarray:
    """Expected-degree sequence w_i ∝ (i+1)^(-1/(gamma-1)), mean 2E/n, capped."""
    dbar = 2.0 * E / n
    w = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
    cap = np.sqrt(n * dbar)
    for _ in range(3):
        w *= dbar / w.mean()
        w = np.minimum(w, cap)
    return w


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [2E]
    gamma: float
    seed: int

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(self.row_ptr.tobytes())
        h.update(self.col_idx.tobytes())
        return h.hexdigest()

    def summary(self) -> dict:
        d = self.degrees
        return dict(n=self.n, edges=self.nnz // 2, nnz=self.nnz, d_max=int(d.max()), d_mean=float(d.mean()),
                    isolated=int((d == 0).sum()), gamma=self.gamma, seed=self.seed)


def chung_lu(n: int, E: int, gamma: float, seed: int = 42) -> Graph:
    """Undirected Chung-Lu power-law graph with exactly E edges (see module doc)."""
    if n < 2 or E < 1 or E > n * (n - 1) // 4:
        raise ValueError("need n >= 2 and 1 <= E <= n(n-1)/4")
    lib = _load()
    g = streams(seed)["graph"]
    s_edges, s_perm = (int(v) for v in g.integers(0, 2**63 - 1, size=2))
    w = np.ascontiguousarray(power_law_weights(n, E, gamma))
    keys = np.empty(E, dtype=np.uint64)
    got = lib.cl_sample_edges(n, _ptr(w), E, s_edges, _ptr(keys))
    if got != E:
        raise RuntimeError("edge sampling failed")
    perm = np.empty(n, dtype=np.int32)
    lib.cl_permutation(n, s_perm, _ptr(perm))
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col_idx = np.empty(2 * E, dtype=np.int32)
    if lib.cl_build_csr(n, E, _ptr(keys), _ptr(perm), _ptr(row_ptr), _ptr(col_idx)) != 0:
        raise RuntimeError("CSR build failed")
    return Graph(n, row_ptr, col_idx, gamma, seed)


def from_edges(n: int, edges) -> Graph:
    """Symmetric CSR of a small hand-written undirected edge list (tests)."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    for u in range(n):
        row_ptr[u + 1] = row_ptr[u] + len(adj[u])
    col_idx = np.array([v for u in range(n) for v in sorted(adj[u])], dtype=np.int32)
    return Graph(n, row_ptr, col_idx, 0.0, 0)


def from_edge_arrays(n: int, u, v) -> Graph:
    """Symmetric CSR (ascending neighbour lists) of the undirected edges
    (u[i], v[i]); the edges must be distinct and free of self-loops."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.lexsort((dst, src))
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(np.bincount(src, minlength=n))
    return Graph(n, row_ptr, dst[order].astype(np.int32), 0.0, 0)


def edge_arrays(graph: Graph):
    """The undirected edges (u < v) of a symmetric CSR, in CSR order."""
    src = np.repeat(np.arange(graph.n, dtype=np.int64), np.diff(graph.row_ptr))
    keep = src < graph.col_idx
    return src[keep].astype(np.int32), graph.col_idx[keep].astype(np.int32)


def snapshots(graph: Graph, k: int = 16, initial: float = 0.179, delete_frac: float = 0.0, seed: int = 42,
              protect=()):
    """Dynamic-graph workload in the manner of the paper's snapshot experiment
    (Sec. 5, 16 snapshots, 17.9% of the edges at the start): the edges in a
    seeded random order, the first `initial` share as graph 0, the rest in k
    equal insertion batches; with delete_frac > 0 every batch also deletes that
    share of its size from the edges present before it, never an edge at a node
    of `protect` (so that query seeds keep their edges).  Graph 0 does not
    depend on delete_frac or protect.  Returns (graph 0,
    [(insert_u, insert_v, delete_u, delete_v)] * k)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    u, v = edge_arrays(graph)
    perm = rng.permutation(len(u))
    u, v = u[perm], v[perm]
    m0 = int(round(initial * len(u)))
    present = np.zeros(len(u), dtype=bool)
    present[:m0] = True
    guard = np.zeros(graph.n, dtype=bool)
    guard[np.asarray(list(protect), dtype=np.int64)] = True
    deletable = ~(guard[u] | guard[v])
    g0 = from_edge_arrays(graph.n, u[:m0], v[:m0])
    bounds = np.linspace(m0, len(u), k + 1).round().astype(np.int64)
    out = []
    for b in range(k):
        lo, hi = bounds[b], bounds[b + 1]
        nd = int(round(delete_frac * (hi - lo)))
        dels = rng.choice(np.flatnonzero(present & deletable), nd, replace=False) if nd else np.zeros(0, np.int64)
        present[dels] = False
        present[lo:hi] = True
        out.append((u[lo:hi], v[lo:hi], u[dels], v[dels]))
    return g0, out


def grid_2d(rows: int, cols: int) -> Graph:
    """The rows x cols 4-neighbour grid graph (node (i, j) has id i * cols + j):
    1000 x 1000 gives 10^6 nodes and 1,998,000 edges, the grid of the paper's
    App. C experiment on graph types.  Neighbour lists are ascending."""
    n = rows * cols
    ids = np.arange(n, dtype=np.int64)
    i, j = ids // cols, ids % cols
    cand = np.stack([np.where(i > 0, ids - cols, -1), np.where(j > 0, ids - 1, -1),
                     np.where(j < cols - 1, ids + 1, -1), np.where(i < rows - 1, ids + cols, -1)], axis=1)
    valid = cand >= 0
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(valid.sum(axis=1))
    col_idx = cand[valid].astype(np.int32)
    return Graph(n, row_ptr, col_idx, 0.0, 0)


def components(graph: Graph) -> np.ndarray:
    lib = _load()
    label = np.empty(graph.n, dtype=np.int32)
    lib.cl_components(graph.n, _ptr(graph.row_ptr), _ptr(graph.col_idx), _ptr(label))
    return label


def largest_component_nodes(graph: Graph) -> np.ndarray:
    label = components(graph)
    d = graph.degrees
    lab = label[d > 0]
    big = np.bincount(lab).argmax()
    return np.flatnonzero((label == big) & (d > 0)).astype(np.int32)


def uniform_seeds(graph: Graph, k: int, seed: int = 42) -> np.ndarray:
    """k distinct seed nodes, uniform over the largest connected component."""
    pool = largest_component_nodes(graph)
    rng = streams(seed)["seeds"]
    return np.sort(rng.choice(pool, size=min(k, len(pool)), replace=False)).astype(np.int32)


def stratified_seeds(graph: Graph, k: int, bins: int = 16, seed: int = 42) -> np.ndarray:
    """Degree-stratified seeds: log2-spaced degree bins, equal numbers per bin
    (nodes drawn uniformly inside a bin; short bins are topped up from the others)."""
    pool = largest_component_nodes(graph)
    rng = streams(seed)["seeds"]
    d = graph.degrees[pool].astype(np.float64)
    edges = np.logspace(0, np.log2(d.max() + 1), bins + 1, base=2.0)
    which = np.clip(np.searchsorted(edges, d, side="right") - 1, 0, bins - 1)
    per = k // bins
    out = []
    for b in range(bins):
        cand = pool[which == b]
        take = min(per, len(cand))
        if take:
            out.extend(rng.choice(cand, size=take, replace=False).tolist())
    rest = np.setdiff1d(pool, np.array(out, dtype=np.int32))
    if len(out) < k:
        out.extend(rng.choice(rest, size=k - len(out), replace=False).tolist())
    return np.array(out, dtype=np.int32)


def log_uniform_eps(k: int, lo: float = 1e-7, hi: float = 1e-4, seed: int = 42) -> np.ndarray:
    rng = streams(seed)["eps"]
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=k)


def seed_set(graph: Graph, anchor: int, size: int = 8, rng=None) -> tuple[np.ndarray, np.ndarray]:
    """A seed set: the anchor plus up to size-1 of its neighbours, topped up from
    its 2-hop neighbourhood, then uniformly; equal weights 1/size."""
    rng = rng or np.random.default_rng(anchor)
    rp, ci = graph.row_ptr, graph.col_idx
    chosen = [int(anchor)]
    nb = ci[rp[anchor]:rp[anchor + 1]]
    for v in rng.permutation(nb)[: size - 1]:
        chosen.append(int(v))
    if len(chosen) < size:
        two = set()
        for v in nb:
            two.update(int(w) for w in ci[rp[v]:rp[v + 1]])
        two -= set(chosen)
        two = [w for w in sorted(two) if rp[w + 1] > rp[w]]
        for w in rng.permutation(np.array(two, dtype=np.int64))[: size - len(chosen)]:
            chosen.append(int(w))
    d = graph.degrees
    while len(chosen) < size:
        w = int(rng.integers(0, graph.n))
        if d[w] > 0 and w not in chosen:
            chosen.append(w)
    idx = np.array(sorted(chosen), dtype=np.int32)
    return idx, np.full(len(idx), 1.0 / len(idx))


def poisson_arrivals(qps: float, duration_s: float, seed: int = 42) -> np.ndarray:
    rng = streams(seed)["arrivals"]
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / qps)
        if t >= duration_s:
            break
        out.append(t)
    return np.array(out)


def insert_batch(graph: Graph, k: int, rng, existing=None) -> tuple[np.ndarray, np.ndarray]:
    """k new undirected edges, endpoints drawn proportional to degree+1, no
    self-loops and no edge already in ``graph`` or in ``existing`` (a set of
    canonical (u, v) pairs that is updated in place).  Candidates are drawn in
    vectorised rounds and kept in draw order."""
    d = graph.degrees.astype(np.float64) + 1.0
    cdf = np.cumsum(d)
    cdf /= cdf[-1]
    rp, ci = graph.row_ptr, graph.col_idx
    existing = existing if existing is not None else set()
    us, vs = [], []
    while len(us) < k:
        m = 2 * (k - len(us)) + 16
        cand = np.minimum(np.searchsorted(cdf, rng.random(2 * m), side="right"), graph.n - 1).reshape(m, 2)
        for u, v in cand:
            if len(us) == k:
                break
            a, b = (int(u), int(v)) if u < v else (int(v), int(u))
            if a == b or (a, b) in existing:
                continue
            row = ci[rp[a]:rp[a + 1]]
            j = np.searchsorted(row, b)
            if j < len(row) and row[j] == b:
                continue
            existing.add((a, b))
            us.append(a)
            vs.append(b)
    return np.array(us, dtype=np.int32), np.array(vs, dtype=np.int32)
