"""Seeded synthetic workloads: directed graphs (out-adjacency CSR), weights, seed vectors.

Inputs only.  Nothing here computes PageRank or D-Iteration quantities; the
HIP library and the CPU oracle both take their inputs from this module and
share nothing else.

Workload recipes (sizes follow the paper's setting of d = 0.85 with a uniform
or topic-sensitive default distribution Z, Section 2.1 and Section 4.1):

* ``tiny_zipf``  - n = 10,000, 10% dangling nodes, out-degree power law 2.1 on
  [1, 1000], targets uniform, unweighted.
* ``webgen``     - web-like stand-in for the paper's crawl (Section 4): hosts of
  log-uniform size 10..999 numbered contiguously, 15% dangling nodes, out-degree
  power law 2.4 on [5, 1000] (mean ~14, m ~ 12 n), 80% of links inside the host,
  targets drawn proportionally to a power-law (2.1) attractiveness capped at
  n^0.75, rows sorted by target; optional LogNormal(0, 1) float32 weights.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwebgen.so")
_lib = None


def build_library(force: bool = False) -> str:
    """Compile webgen.c into libwebgen.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "webgen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # DI_WEBGEN_LIB names another build of the same source (the sanitizer test uses it)
    path = os.environ.get("DI_WEBGEN_LIB")
    if not path:
        if not os.path.exists(_LIB_PATH):
            build_library()
        path = _LIB_PATH
    lib = ctypes.CDLL(path)
    i64, u64, dbl, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    lib.wl_hash.restype = u64
    lib.wl_hash.argtypes = [u64, u64, u64, u64]
    lib.wl_degrees.restype = i64
    lib.wl_degrees.argtypes = [i64, u64, dbl, dbl, i64, i64, vp]
    lib.wl_targets_uniform.argtypes = [i64, u64, vp, vp]
    lib.wl_targets_web.argtypes = [i64, u64, dbl, dbl, dbl, vp, vp]
    lib.wl_host_count.restype = i64
    lib.wl_host_count.argtypes = [i64, u64]
    lib.wl_hosts.argtypes = [i64, u64, vp]
    lib.wl_lognormal_weights.argtypes = [u64, i64, vp]
    lib.wl_normal_vector.argtypes = [u64, i64, vp]
    lib.wl_seed_nodes.argtypes = [u64, i64, i64, i64, vp]
    lib.wl_batch_sizes.argtypes = [u64, i64, dbl, dbl, vp, vp]
    lib.wl_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """Directed graph as out-adjacency CSR (rows = sources, sorted targets)."""

    n: int
    out_ptr: np.ndarray  # int64[n+1]
    out_idx: np.ndarray  # int32[m]
    w: Optional[np.ndarray] = None  # float32[m] or None (unweighted)
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.out_ptr[-1])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.out_ptr)


def hash64(seed: int, stream: int, a: int, b: int) -> int:
    return int(_load().wl_hash(seed, stream, a, b))


def _degrees(n, seed, p_dang, alpha, dmin, dmax):
    lib = _load()
    out_ptr = np.empty(n + 1, dtype=np.int64)
    m = lib.wl_degrees(n, seed, p_dang, alpha, dmin, dmax, _p(out_ptr))
    if m < 0:
        raise MemoryError("wl_degrees failed")
    return out_ptr, int(m)


def tiny_zipf(n: int = 10_000, seed: int = 1) -> Graph:
    """Unweighted graph with power-law out-degrees and uniform targets."""
    out_ptr, m = _degrees(n, seed, 0.10, 2.1, 1, 1000)
    out_idx = np.empty(m, dtype=np.int32)
    _load().wl_targets_uniform(n, seed, _p(out_ptr), _p(out_idx))
    return Graph(n, out_ptr, out_idx, None, "tiny_zipf(n=%d,seed=%d)" % (n, seed))


def webgen(n: int, seed: int, weighted: bool = False) -> Graph:
    """Web-like graph: host locality, power-law in-degree, dangling nodes."""
    out_ptr, m = _degrees(n, seed, 0.15, 2.4, 5, 1000)
    out_idx = np.empty(m, dtype=np.int32)
    if _load().wl_targets_web(n, seed, 2.1, 0.75, 0.8, _p(out_ptr), _p(out_idx)) != 0:
        raise MemoryError("wl_targets_web failed")
    w = None
    if weighted:
        w = np.empty(m, dtype=np.float32)
        _load().wl_lognormal_weights(seed, m, _p(w))
    return Graph(n, out_ptr, out_idx, w, "webgen(n=%d,seed=%d%s)" % (n, seed, ",w" if weighted else ""))


def host_ptr(n: int, seed: int) -> np.ndarray:
    lib = _load()
    nh = int(lib.wl_host_count(n, seed))
    hp = np.empty(nh + 1, dtype=np.int64)
    lib.wl_hosts(n, seed, _p(hp))
    return hp


def lognormal_weights(m: int, seed: int) -> np.ndarray:
    w = np.empty(m, dtype=np.float32)
    _load().wl_lognormal_weights(seed, m, _p(w))
    return w


def normal_vector(n: int, seed: int) -> np.ndarray:
    c = np.empty(n, dtype=np.float64)
    _load().wl_normal_vector(seed, n, _p(c))
    return c


def ppr_seeds(n: int, k: int = 64, per_column: int = 16, seed: int = 4) -> np.ndarray:
    out = np.empty((k, per_column), dtype=np.int64)
    if _load().wl_seed_nodes(seed, n, k, per_column, _p(out)) != 0:
        raise ValueError("more seeds than nodes")
    return out


def ppr_Z(n: int, k: int = 64, per_column: int = 16, seed: int = 4) -> np.ndarray:
    """n x k column-major right-hand sides, each uniform over `per_column` seed nodes."""
    s = ppr_seeds(n, k, per_column, seed)
    Z = np.zeros((n, k), dtype=np.float64, order="F")
    for c in range(k):
        Z[s[c], c] = 1.0 / per_column
    return Z


def batch_sizes(count: int, seed: int, lo: float = 1e3, hi: float = 2e5):
    sizes = np.empty(count, dtype=np.int64)
    seeds = np.empty(count, dtype=np.uint64)
    _load().wl_batch_sizes(seed, count, lo, hi, _p(sizes), _p(seeds))
    return sizes, seeds


def union(graphs) -> tuple[Graph, np.ndarray]:
    """Block-diagonal union; returns the graph and graph_ptr (node offsets)."""
    ns = [g.n for g in graphs]
    gptr = np.zeros(len(graphs) + 1, dtype=np.int64)
    gptr[1:] = np.cumsum(ns)
    ms = [g.m for g in graphs]
    eoff = np.zeros(len(graphs) + 1, dtype=np.int64)
    eoff[1:] = np.cumsum(ms)
    out_ptr = np.empty(int(gptr[-1]) + 1, dtype=np.int64)
    out_idx = np.empty(int(eoff[-1]), dtype=np.int32)
    weighted = all(g.w is not None for g in graphs)
    w = np.empty(int(eoff[-1]), dtype=np.float32) if weighted else None
    for k, g in enumerate(graphs):
        out_ptr[gptr[k]:gptr[k + 1]] = g.out_ptr[:-1] + eoff[k]
        out_idx[eoff[k]:eoff[k + 1]] = g.out_idx + np.int32(gptr[k])
        if weighted:
            w[eoff[k]:eoff[k + 1]] = g.w
    out_ptr[-1] = eoff[-1]
    return Graph(int(gptr[-1]), out_ptr, out_idx, w, "union(%d)" % len(graphs)), gptr


def multigraph_batch(count: int = 256, seed: int = 4) -> tuple[Graph, np.ndarray]:
    """`count` independent web-like graphs of log-uniform size 1k..200k, as one union."""
    sizes, seeds = batch_sizes(count, seed)
    graphs = [webgen(int(sizes[g]), int(seeds[g])) for g in range(count)]
    return union(graphs)


def induced_bfs_subgraph(g: Graph, size: int = 200, seed: int = 5) -> tuple[Graph, np.ndarray]:
    """First `size` nodes reached by BFS on the undirected view from a seeded start node.

    Returns the induced subgraph (nodes relabelled by ascending original id, rows
    sorted by target, weights kept) and the original ids of its nodes.
    """
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.out_ptr))
    dst = g.out_idx.astype(np.int64)
    und_src = np.concatenate([src, dst])
    und_dst = np.concatenate([dst, src])
    order = np.argsort(und_src, kind="stable")
    und_src, und_dst = und_src[order], und_dst[order]
    ptr = np.zeros(g.n + 1, dtype=np.int64)
    np.add.at(ptr, und_src + 1, 1)
    ptr = np.cumsum(ptr)
    start = hash64(seed, 9, 0, 0) % g.n
    seen = {start}
    order_nodes = [start]
    head = 0
    while head < len(order_nodes) and len(order_nodes) < size:
        u = order_nodes[head]
        head += 1
        for v in und_dst[ptr[u]:ptr[u + 1]]:
            v = int(v)
            if v not in seen:
                seen.add(v)
                order_nodes.append(v)
                if len(order_nodes) >= size:
                    break
    nodes = np.array(sorted(order_nodes), dtype=np.int64)
    remap = -np.ones(g.n, dtype=np.int64)
    remap[nodes] = np.arange(len(nodes))
    keep = (remap[src] >= 0) & (remap[dst] >= 0)
    s2, d2 = remap[src[keep]], remap[dst[keep]]
    w2 = g.w[keep] if g.w is not None else None
    o = np.lexsort((d2, s2))
    s2, d2 = s2[o], d2[o]
    if w2 is not None:
        w2 = w2[o]
    n2 = len(nodes)
    out_ptr = np.zeros(n2 + 1, dtype=np.int64)
    np.add.at(out_ptr, s2 + 1, 1)
    out_ptr = np.cumsum(out_ptr)
    return Graph(n2, out_ptr, d2.astype(np.int32), w2, "bfs%d(%s)" % (n2, g.name)), nodes


def from_edges(n: int, src, dst, w=None, name: str = "") -> Graph:
    """Graph from an edge list (rows sorted by target, stable for duplicates)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    o = np.lexsort((dst, src))
    src, dst = src[o], dst[o]
    out_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(out_ptr, src + 1, 1)
    out_ptr = np.cumsum(out_ptr)
    wv = None if w is None else np.asarray(w, dtype=np.float32)[o]
    return Graph(n, out_ptr, dst.astype(np.int32), wv, name)


def edit_graph(g: Graph, seed: int, frac: float = 0.01) -> Graph:
    """An edited copy of g on the same nodes (input for graph updates): a share `frac` of
    the edges get a new target drawn between their row neighbours' targets (rows stay
    sorted), frac/2 of the edges are dropped (some sources become dangling), and a tenth
    of the dangling nodes get one edge to a uniform target.  Edges keep their weights; added
    edges draw LogNormal(0, 1) weights.  Seeded numpy generator; O(m)."""
    rng = np.random.default_rng([seed, 0xD1])
    n, m = g.n, g.m
    ptr = g.out_ptr
    idx = g.out_idx.astype(np.int64)
    w = None if g.w is None else g.w.copy()
    # moved targets, between the row neighbours' targets
    mv = np.unique(rng.integers(0, m, size=int(frac * m))) if m else np.zeros(0, np.int64)
    if len(mv) > 1:  # no two moved edges side by side, so the new targets keep the row order
        gap = np.diff(mv) > 1
        mv = mv[np.concatenate([[True], gap]) & np.concatenate([gap, [True]])]
    row = np.searchsorted(ptr, mv, side="right") - 1
    lo = np.where(mv > ptr[row], idx[np.maximum(mv - 1, 0)], 0)
    hi = np.where(mv + 1 < ptr[row + 1], idx[np.minimum(mv + 1, m - 1)], n - 1)
    idx[mv] = lo + (rng.random(len(mv)) * (hi - lo + 1)).astype(np.int64).clip(0, hi - lo)
    # dropped edges
    keep = np.ones(m, dtype=bool)
    if m:
        keep[rng.integers(0, m, size=int(frac / 2 * m))] = False
    drops = np.bincount(np.searchsorted(ptr, np.flatnonzero(~keep), side="right") - 1, minlength=n)
    # one edge for a tenth of the dangling nodes (their rows are empty, so stay sorted)
    dang = np.flatnonzero(np.diff(ptr) == 0)
    add = np.sort(rng.choice(dang, size=len(dang) // 10, replace=False)) if len(dang) >= 10 else dang[:0]
    add_t = rng.integers(0, n, size=len(add))
    kept_idx = idx[keep]
    kept_ptr = np.concatenate([[0], np.cumsum(np.diff(ptr) - drops)])
    new_idx = np.insert(kept_idx, kept_ptr[add], add_t)
    deg = np.diff(kept_ptr)
    deg[add] += 1
    new_ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    new_w = None
    if w is not None:
        new_w = np.insert(w[keep], kept_ptr[add], rng.lognormal(0.0, 1.0, size=len(add)).astype(np.float32))
    return Graph(n, new_ptr, new_idx.astype(np.int32), new_w, "edit(%s,%g)" % (g.name, frac))


# Named configurations of the paper's setting (d = 0.85; uniform Z unless noted).
def config_graph(name: str) -> Graph:
    if name == "tiny":
        return tiny_zipf(10_000, 1)
    if name == "web1m":
        return webgen(1_000_000, 2)
    if name == "web50m":
        return webgen(50_000_000, 3)
    if name == "web4m":
        return webgen(4_000_000, 4)
    if name == "web2m_w":
        return webgen(2_000_000, 5, weighted=True)
    raise KeyError(name)
