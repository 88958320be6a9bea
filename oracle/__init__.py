"""Oracle for per-edge typed graphlet counts (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never links, loads or calls it, and
it shares no code with the GPU path.

``oracle.c`` holds two independent CPU counters (brute force over all 3/4-node
subsets, and the paper's Algorithms 1-3 with Eqs. 7-17); this module builds
that file with gcc and wraps it with ctypes.  ``directed.py`` holds the
directed typed 3-node counters (plain Python).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SHAPES = ("wedge", "triangle", "path4", "star4", "cycle4", "tailed_triangle", "chordal_cycle", "clique4")
SHAPE_EDGES = (2, 3, 3, 3, 4, 4, 5, 6)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    for nm in ("or_num_keys", "or_row_width", "or_orbit_row_width"):
        getattr(lib, nm).restype = i64
        getattr(lib, nm).argtypes = [i32]
    lib.or_typed_per_shape.restype = i64
    lib.or_typed_per_shape.argtypes = [i32, i32]
    lib.or_rank.restype = i64
    lib.or_rank.argtypes = [i32, vp]
    lib.or_key.restype = i64
    lib.or_key.argtypes = [i32, i32, vp]
    lib.or_shape_offset.restype = i64
    lib.or_shape_offset.argtypes = [i32, i32]
    lib.or_row_key.restype = i64
    lib.or_row_key.argtypes = [i32, i32, i32, i64]
    lib.or_brute.restype = i32
    lib.or_brute.argtypes = [i64, vp, vp, vp, i32, vp, vp, vp]
    lib.or_count_edges.restype = i32
    lib.or_count_edges.argtypes = [i64, vp, vp, vp, i32, i64, vp, vp, vp, vp, i32]
    lib.or_count_all.restype = i32
    lib.or_count_all.argtypes = [i64, vp, vp, vp, i32, vp, vp, i32]
    lib.or_count_batch.restype = i32
    lib.or_count_batch.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, i32]
    _lib = lib
    return lib


def num_keys(L):
    return int(_load().or_num_keys(L))


def row_width(L):
    return int(_load().or_row_width(L))


def orbit_row_width(L):
    return int(_load().or_orbit_row_width(L))


def typed_per_shape(L, K):
    return int(_load().or_typed_per_shape(L, K))


def rank(types):
    t = np.ascontiguousarray(types, dtype=np.int32)
    return int(_load().or_rank(len(t), t.ctypes.data))


def key(L, shape, types):
    t = np.ascontiguousarray(types, dtype=np.int32)
    return int(_load().or_key(L, shape, t.ctypes.data))


def shape_offset(L, shape):
    return int(_load().or_shape_offset(L, shape))


def row_key(L, phi_i, phi_j, col):
    return int(_load().or_row_key(L, phi_i, phi_j, col))


def _arrs(row_ptr, col_idx, types):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    ty = np.ascontiguousarray(types, dtype=np.uint8)
    return rp, ci, ty


def canonical_edges(row_ptr, col_idx):
    """(i, j) with i < j in row-major CSR order."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    src = np.repeat(np.arange(len(rp) - 1, dtype=np.int64), np.diff(rp))
    keep = ci > src
    return src[keep].astype(np.int32), ci[keep].astype(np.int32)


def brute(row_ptr, col_idx, types, L, orbits=False):
    """Brute-force enumeration (n <= 64). Returns (rows, orbit_rows or None, global)."""
    rp, ci, ty = _arrs(row_ptr, col_idx, types)
    n = len(rp) - 1
    m = len(ci) // 2
    rows = np.zeros((m, row_width(L)), dtype=np.uint64)
    orows = np.zeros((m, orbit_row_width(L)), dtype=np.uint64) if orbits else None
    glob = np.zeros(num_keys(L), dtype=np.uint64)
    st = _load().or_brute(n, rp.ctypes.data, ci.ctypes.data, ty.ctypes.data, L, rows.ctypes.data,
                          orows.ctypes.data if orbits else None, glob.ctypes.data)
    if st != 0:
        raise ValueError(f"or_brute failed with status {st}")
    return rows, orows, glob


def count_edges(row_ptr, col_idx, types, L, ei, ej, orbits=False, nthreads=1):
    """Paper-method rows for an explicit list of edges. Returns (rows, orbit_rows or None)."""
    rp, ci, ty = _arrs(row_ptr, col_idx, types)
    ei = np.ascontiguousarray(ei, dtype=np.int32)
    ej = np.ascontiguousarray(ej, dtype=np.int32)
    ne = len(ei)
    rows = np.zeros((ne, row_width(L)), dtype=np.uint64)
    orows = np.zeros((ne, orbit_row_width(L)), dtype=np.uint64) if orbits else None
    st = _load().or_count_edges(len(rp) - 1, rp.ctypes.data, ci.ctypes.data, ty.ctypes.data, L, ne,
                                ei.ctypes.data, ej.ctypes.data, rows.ctypes.data,
                                orows.ctypes.data if orbits else None, int(nthreads))
    if st != 0:
        raise ValueError(f"or_count_edges failed with status {st}")
    return rows, orows


def count_all(row_ptr, col_idx, types, L, per_edge=True, nthreads=1):
    """Paper-method counts for every canonical edge plus global counts (Eq. 17).
    Returns (rows or None, global)."""
    rp, ci, ty = _arrs(row_ptr, col_idx, types)
    m = len(ci) // 2
    rows = np.zeros((m, row_width(L)), dtype=np.uint64) if per_edge else None
    glob = np.zeros(num_keys(L), dtype=np.uint64)
    st = _load().or_count_all(len(rp) - 1, rp.ctypes.data, ci.ctypes.data, ty.ctypes.data, L,
                              rows.ctypes.data if per_edge else None, glob.ctypes.data, int(nthreads))
    if st != 0:
        raise ValueError(f"or_count_all failed with status {st}")
    return rows, glob


def count_batch(node_off, slot_off, row_ptr, col_idx, types, Ls, nthreads=1):
    """Global counts (Eq. 17) of every graph of a batch (layout as in
    graphgen.Batch), graph-parallel over nthreads.  Returns (counts, key_off)
    with graph g's K(L_g) counts at counts[key_off[g]:key_off[g+1]]."""
    Ls = np.ascontiguousarray(Ls, dtype=np.uint8)
    G = len(Ls)
    key_off = np.zeros(G + 1, dtype=np.int64)
    if G:
        key_off[1:] = np.cumsum([num_keys(int(x)) for x in Ls])
    node_off = np.ascontiguousarray(node_off, dtype=np.int64)
    slot_off = np.ascontiguousarray(slot_off, dtype=np.int64)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    ty = np.ascontiguousarray(types, dtype=np.uint8)
    out = np.zeros(int(key_off[-1]), dtype=np.uint64)
    st = _load().or_count_batch(G, node_off.ctypes.data, slot_off.ctypes.data, rp.ctypes.data, ci.ctypes.data,
                                ty.ctypes.data, Ls.ctypes.data, key_off.ctypes.data, out.ctypes.data, int(nthreads))
    if st != 0:
        raise ValueError(f"or_count_batch failed with status {st}")
    return out, key_off
