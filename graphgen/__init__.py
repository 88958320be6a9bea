"""Seeded synthetic inputs: graphs in CSR form and node types.

The heavy lifting is in ``graphgen.cpp`` (built into ``libgraphgen.so`` next
to this file by ``graphgen.build()``).  This module holds only input
generation; it contains no graphlet-counting arithmetic, so the oracle tests
and the GPU path can both draw their inputs from it.

Named workloads (``workload(name)``) fix every recipe constant: model, sizes,
exponents, degree caps, type distributions and seeds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp, i64, f64, u64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_int
    lib.gg_chung_lu.restype = vp
    lib.gg_chung_lu.argtypes = [i64, f64, f64, f64, u64]
    lib.gg_kpartite_cl.restype = vp
    lib.gg_kpartite_cl.argtypes = [i32, vp, vp, vp, vp, i64, u64]
    lib.gg_gnp.restype = vp
    lib.gg_gnp.argtypes = [i64, f64, u64]
    for nm in ("gg_num_nodes", "gg_num_slots"):
        getattr(lib, nm).restype = i64
        getattr(lib, nm).argtypes = [vp]
    for nm in ("gg_row_ptr", "gg_col_idx", "gg_parts"):
        getattr(lib, nm).restype = vp
        getattr(lib, nm).argtypes = [vp]
    lib.gg_has_parts.restype = i32
    lib.gg_has_parts.argtypes = [vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_types_uniform.restype = None
    lib.gg_types_uniform.argtypes = [i64, i32, u64, vp]
    lib.gg_types_zipf.restype = None
    lib.gg_types_zipf.argtypes = [i64, i32, f64, u64, vp]
    lib.gg_types_homophily.restype = None
    lib.gg_types_homophily.argtypes = [i64, vp, vp, i32, f64, f64, u64, vp]
    lib.gg_batch_gnp.restype = vp
    lib.gg_batch_gnp.argtypes = [i64, f64, f64, f64, f64, i32, i32, u64]
    lib.gg_batch_num_graphs.restype = i64
    lib.gg_batch_num_graphs.argtypes = [vp]
    for nm in ("gg_batch_node_off", "gg_batch_slot_off", "gg_batch_row_ptr", "gg_batch_col_idx",
               "gg_batch_types", "gg_batch_L"):
        getattr(lib, nm).restype = vp
        getattr(lib, nm).argtypes = [vp]
    lib.gg_batch_free.restype = None
    lib.gg_batch_free.argtypes = [vp]
    _lib = lib
    return lib


def _view(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    ct = np.ctypeslib.as_ctypes_type(np.dtype(dtype))
    arr = (ct * n).from_address(ptr)
    return np.frombuffer(arr, dtype=dtype, count=n).copy()


def _take_graph(h):
    lib = _load()
    if not h:
        raise ValueError("graph generator rejected its arguments")
    try:
        n = lib.gg_num_nodes(h)
        nnz = lib.gg_num_slots(h)
        row_ptr = _view(lib.gg_row_ptr(h), n + 1, np.int32)
        col_idx = _view(lib.gg_col_idx(h), nnz, np.int32)
        parts = _view(lib.gg_parts(h), n, np.uint8) if lib.gg_has_parts(h) else None
    finally:
        lib.gg_free(h)
    return row_ptr, col_idx, parts


def chung_lu(n, gamma, wmax, mean_deg, seed):
    """Chung-Lu graph (Miller-Hagberg sampling), ids shuffled. Returns (row_ptr, col_idx)."""
    rp, ci, _ = _take_graph(_load().gg_chung_lu(int(n), float(gamma), float(wmax), float(mean_deg), int(seed)))
    return rp, ci


def kpartite_cl(sizes, gammas, wmaxs, means, m, seed):
    """k-partite Chung-Lu. Returns (row_ptr, col_idx, part_of_node)."""
    k = len(sizes)
    a = np.asarray(sizes, dtype=np.int64)
    g = np.asarray(gammas, dtype=np.float64)
    w = np.asarray(wmaxs, dtype=np.float64)
    mu = np.asarray(means, dtype=np.float64)
    h = _load().gg_kpartite_cl(k, a.ctypes.data, g.ctypes.data, w.ctypes.data, mu.ctypes.data, int(m), int(seed))
    return _take_graph(h)


def gnp(n, p, seed):
    """Erdos-Renyi G(n, p). Returns (row_ptr, col_idx)."""
    rp, ci, _ = _take_graph(_load().gg_gnp(int(n), float(p), int(seed)))
    return rp, ci


def types_uniform(n, L, seed):
    out = np.empty(int(n), dtype=np.uint8)
    _load().gg_types_uniform(int(n), int(L), int(seed), out.ctypes.data)
    return out


def types_zipf(n, L, s, seed):
    out = np.empty(int(n), dtype=np.uint8)
    _load().gg_types_zipf(int(n), int(L), float(s), int(seed), out.ctypes.data)
    return out


def types_homophily(row_ptr, col_idx, L, s, p_follow, seed):
    n = len(row_ptr) - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    out = np.empty(n, dtype=np.uint8)
    _load().gg_types_homophily(n, rp.ctypes.data, ci.ctypes.data, int(L), float(s), float(p_follow), int(seed),
                               out.ctypes.data)
    return out


@dataclass
class Batch:
    """Concatenated small graphs with local node ids.

    Graph g owns nodes [node_off[g], node_off[g+1]) and CSR slots
    [slot_off[g], slot_off[g+1]); its local row pointer (n_g + 1 entries,
    starting at 0) sits at row_ptr[node_off[g] + g : node_off[g+1] + g + 1].
    """
    node_off: np.ndarray
    slot_off: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    types: np.ndarray
    L: np.ndarray

    @property
    def G(self):
        return len(self.L)

    def graph(self, g):
        n0, n1 = int(self.node_off[g]), int(self.node_off[g + 1])
        s0, s1 = int(self.slot_off[g]), int(self.slot_off[g + 1])
        rp = self.row_ptr[n0 + g:n1 + g + 1].copy()
        return rp, self.col_idx[s0:s1].copy(), self.types[n0:n1].copy(), int(self.L[g])


def batch_gnp(G, nmin, nmax, rmin, rmax, lmin, lmax, seed) -> Batch:
    lib = _load()
    h = lib.gg_batch_gnp(int(G), float(nmin), float(nmax), float(rmin), float(rmax), int(lmin), int(lmax), int(seed))
    if not h:
        raise ValueError("batch generator rejected its arguments")
    try:
        node_off = _view(lib.gg_batch_node_off(h), G + 1, np.int64)
        slot_off = _view(lib.gg_batch_slot_off(h), G + 1, np.int64)
        N = int(node_off[-1])
        S = int(slot_off[-1])
        b = Batch(node_off=node_off, slot_off=slot_off,
                  row_ptr=_view(lib.gg_batch_row_ptr(h), N + G, np.int32),
                  col_idx=_view(lib.gg_batch_col_idx(h), S, np.int32),
                  types=_view(lib.gg_batch_types(h), N, np.uint8),
                  L=_view(lib.gg_batch_L(h), G, np.uint8))
    finally:
        lib.gg_batch_free(h)
    return b


@dataclass
class Graph:
    name: str
    row_ptr: np.ndarray
    col_idx: np.ndarray
    types: np.ndarray
    L: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return len(self.row_ptr) - 1

    @property
    def m(self):
        return len(self.col_idx) // 2


# ---------------------------------------------------------------------------
# Workload recipes.  Every constant of every input lives here.

def orient(row_ptr, col_idx, seed, p_both=0.2):
    """Seeded orientation of an undirected CSR graph into a directed one:
    each edge {u, v} becomes reciprocal with probability p_both, else one arc
    in a uniformly random direction.  Returns the per-slot direction bits
    (uint8 [nnz]; bit 0: row -> column, bit 1: column -> row), consistent on
    the two slots of every edge."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    n = len(rp) - 1
    if len(ci) == 0:
        return np.zeros(0, np.uint8)
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    lo, hi = np.minimum(u, ci), np.maximum(u, ci)
    order = np.argsort(lo * n + hi, kind="stable")   # the two slots of an edge end up side by side
    rng = np.random.default_rng(seed)
    m = len(ci) // 2
    both = rng.random(m) < p_both
    fwd = rng.integers(1, 3, size=m)                  # 1: low id -> high id, 2: high -> low
    code = np.where(both, 3, fwd).astype(np.uint8)    # relative to (low, high)
    per_slot = np.repeat(code, 2)
    out = np.empty(len(ci), np.uint8)
    out[order] = per_slot
    swap = u > ci                                     # slot read from the high end: swap the two bits
    out[swap] = ((out[swap] & 1) << 1) | ((out[swap] >> 1) & 1)
    return out


def tiny_digraph(idx: int):
    """(Graph, slot direction bits) of the idx-th tiny directed test graph."""
    g = tiny_graph(idx)
    return g, orient(g.row_ptr, g.col_idx, 5000 + idx, p_both=0.25)


def tiny_graph(idx: int) -> Graph:
    """One of the 200 brute-force-checkable graphs: G(n, p), n ~ U{6..12},
    p ~ U(0.2, 0.8), L ~ U{1..4}, uniform types; seed 1000 + idx."""
    seed = 1000 + idx
    rng = np.random.Generator(np.random.Philox(seed))
    n = int(rng.integers(6, 13))
    p = float(rng.uniform(0.2, 0.8))
    L = int(rng.integers(1, 5))
    rp, ci = gnp(n, p, seed)
    ty = types_uniform(n, L, seed)
    return Graph(f"tiny{idx}", rp, ci, ty, L, dict(model="gnp", n=n, p=p, seed=seed))


def chung_lu_small() -> Graph:
    """Chung-Lu, n=2000, ~10k edges, exponent 2.5, max expected degree 200,
    mean 10, L=3 uniform types, seed 1."""
    rp, ci = chung_lu(2000, 2.5, 200.0, 10.0, 1)
    ty = types_uniform(2000, 3, 1)
    return Graph("cl-2k", rp, ci, ty, 3, dict(model="chung-lu", gamma=2.5, wmax=200, mean=10.0, seed=1))


# Mean expected degree for the 1M-node graph, calibrated so that the realised
# edge count after probability capping is close to 10M.
CL1M_MEAN = 20.0


def chung_lu_1m(mean=None) -> Graph:
    """Chung-Lu, n=1M, exponent 2.2, max expected degree 50k, L=5 types,
    Zipf(1.2) with homophily 0.7, seed 2."""
    mu = CL1M_MEAN if mean is None else mean
    rp, ci = chung_lu(1_000_000, 2.2, 50_000.0, mu, 2)
    ty = types_homophily(rp, ci, 5, 1.2, 0.7, 2)
    return Graph("cl-1m", rp, ci, ty, 5, dict(model="chung-lu", gamma=2.2, wmax=50000, mean=mu, seed=2,
                                             types="zipf1.2+homophily0.7"))


# Expected edge count before probability capping for the bipartite graph,
# calibrated so that the realised count is close to 50M (50,003,127 edges,
# maximum degree 81,476).
BIP50M_PRECAP_M = 53_600_000


def bipartite_50m() -> Graph:
    """Bipartite Chung-Lu user-item graph: 2M type-0 nodes (exponent 2.1,
    mean 25, max expected degree 2e4) and 500k type-1 nodes (exponent 1.8,
    mean 100, max expected degree 1e5), about 50M edges, only between the two
    sides; L=2 with the side as the type; seed 31."""
    rp, ci, parts = kpartite_cl([2_000_000, 500_000], [2.1, 1.8], [2e4, 1e5], [25.0, 100.0], BIP50M_PRECAP_M, 31)
    return Graph("bip-50m", rp, ci, parts, 2, dict(model="bipartite-chung-lu", sizes=[2_000_000, 500_000],
                                                  gamma=[2.1, 1.8], wmax=[2e4, 1e5], mean=[25, 100],
                                                  precap_m=BIP50M_PRECAP_M, seed=31))


def tripartite_30m() -> Graph:
    """3-partite Chung-Lu graph: parts of 1M, 1M and 200k nodes (types 0, 1,
    2), power-law weights with exponent 2.1 and max expected degree 2e4 in
    every part, 30M expected edges, only between different parts; seed 32."""
    rp, ci, parts = kpartite_cl([1_000_000, 1_000_000, 200_000], [2.1, 2.1, 2.1], [2e4, 2e4, 2e4],
                                [27.3, 27.3, 27.3], 30_000_000, 32)
    return Graph("tri-30m", rp, ci, parts, 3, dict(model="3-partite-chung-lu", sizes=[1_000_000, 1_000_000, 200_000],
                                                  gamma=2.1, wmax=2e4, seed=32))


# Mean expected degree of the 20M-node graph, calibrated so that the
# realised edge count after probability capping is close to 300M
# (300,032,326 edges, maximum degree 296,629).
CL20M_MEAN = 32.85


def chung_lu_20m() -> Graph:
    """Chung-Lu, n=20M, exponent 2.0, max expected degree 5e5, mean 32.85
    (about 3.0e8 edges after probability capping), L=8 types iid Zipf(1.0),
    seed 5."""
    rp, ci = chung_lu(20_000_000, 2.0, 5e5, CL20M_MEAN, 5)
    ty = types_zipf(20_000_000, 8, 1.0, 5)
    return Graph("cl-20m", rp, ci, ty, 8, dict(model="chung-lu", gamma=2.0, wmax=5e5, mean=CL20M_MEAN, seed=5,
                                              types="zipf1.0"))


WORKLOADS = {
    "cl-2k": chung_lu_small,
    "cl-1m": chung_lu_1m,
    "bip-50m": bipartite_50m,
    "tri-30m": tripartite_30m,
    "cl-20m": chung_lu_20m,
}


def workload(name: str) -> Graph:
    return WORKLOADS[name]()
