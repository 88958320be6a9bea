"""Oracle for directed typed 4-node graphlets (test infrastructure only).

Only the test-suite and the benchmark may import this module; the product
library never calls it and shares no code with it.

The Directed Typed Graphlets subsection splits every typed neighbour set
into typed out- and in-neighbour sets and asks for a unique id per directed
typed motif.  This module writes the 4-node case out from the definitions:

* nodes 0..3 of a 4-node digraph in a fixed order; its arc code holds one
  bit per ordered pair (x, y), x != y, in the order of ORDERED_PAIRS; its
  full code adds the four node types, 4 bits each, above bit 12;
* canonical code: the smallest full code over the 24 orderings of the nodes;
* keys of L types: the canonical codes of weakly connected 4-node digraphs
  with types below L, numbered in increasing order (199 classes for L = 1,
  the connected directed 4-node graphs);
* per-edge row of support edge (i, j), i < j (an edge of the undirected
  support graph, with both directions of a reciprocal pair on one support
  edge): for every pair of other nodes {k, l} whose induced subgraph on
  {i, j, k, l} is weakly connected, the column of its canonical key gains
  one;
* global count of a key: the number of 4-node sets inducing it; each is seen
  from each of its support edges (Eq. 17's argument), so global = row sums /
  support edges.

Two independent counters: `brute_global` over all 4-node sets and
`edge_rows` per support edge, plus `rows_to_global`.
"""
from __future__ import annotations

import itertools

import numpy as np

ORDERED_PAIRS = [(x, y) for x in range(4) for y in range(4) if x != y]
_BIT = {xy: b for b, xy in enumerate(ORDERED_PAIRS)}
UNORDERED = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def code4(arcs, types):
    """Full code of the digraph on ordered nodes 0..3: arcs is a set of
    ordered pairs (x, y), types four ints below 16."""
    c = 0
    for xy in arcs:
        c |= 1 << _BIT[xy]
    for p in range(4):
        c |= int(types[p]) << (12 + 4 * p)
    return c


def decode4(code):
    arcs = {xy for xy, b in _BIT.items() if code >> b & 1}
    return arcs, tuple((code >> (12 + 4 * p)) & 15 for p in range(4))


def _perm_tables():
    """For each of the 24 node orderings: the new bit of every old arc bit
    and the old node placed at each new position."""
    out = []
    for perm in itertools.permutations(range(4)):
        inv = {perm[p]: p for p in range(4)}  # old node -> new position
        bitmap = [_BIT[(inv[x], inv[y])] for (x, y) in ORDERED_PAIRS]
        out.append((bitmap, perm))
    return out


_PERMS = _perm_tables()


def canonical4(code):
    arcs_bits = code & 0xFFF
    types = [(code >> (12 + 4 * p)) & 15 for p in range(4)]
    best = None
    for bitmap, perm in _PERMS:
        a = 0
        for b in range(12):
            if arcs_bits >> b & 1:
                a |= 1 << bitmap[b]
        c = a
        for p in range(4):
            c |= types[perm[p]] << (12 + 4 * p)
        best = c if best is None else min(best, c)
    return best


def canonical_all(L):
    """Canonical codes of every full code with types below L, vectorised
    over the 4096 arc sets and L^4 typings: an array indexed by
    arc_bits + 4096 * (t0 + L t1 + L^2 t2 + L^3 t3)."""
    arcs = np.arange(4096, dtype=np.int64)
    typings = np.array(list(itertools.product(range(L), repeat=4)), dtype=np.int64)  # (t0, t1, t2, t3)
    # typing index t0 + L t1 + L^2 t2 + L^3 t3 for the order of `typings`
    tidx = typings[:, 0] + L * typings[:, 1] + L * L * typings[:, 2] + L ** 3 * typings[:, 3]
    best = np.full((len(typings), 4096), np.iinfo(np.int64).max, dtype=np.int64)
    for bitmap, perm in _PERMS:
        a = np.zeros(4096, dtype=np.int64)
        for b in range(12):
            a |= ((arcs >> b) & 1) << bitmap[b]
        tv = np.zeros(len(typings), dtype=np.int64)
        for p in range(4):
            tv |= typings[:, perm[p]] << (12 + 4 * p)
        best = np.minimum(best, a[None, :] | tv[:, None])
    out = np.empty(4096 * len(typings), dtype=np.int64)
    for q in range(len(typings)):
        out[4096 * tidx[q]:4096 * (tidx[q] + 1)] = best[q]
    return out


def weakly_connected(arc_bits):
    adj = [set() for _ in range(4)]
    for b, (x, y) in enumerate(ORDERED_PAIRS):
        if arc_bits >> b & 1:
            adj[x].add(y)
            adj[y].add(x)
    seen, stack = {0}, [0]
    while stack:
        v = stack.pop()
        for w in adj[v]:
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return len(seen) == 4


def support_edges4(code):
    return sum(1 for (x, y) in UNORDERED if code >> _BIT[(x, y)] & 1 or code >> _BIT[(y, x)] & 1)


_CONNECTED = np.array([weakly_connected(a) for a in range(4096)])


def keys(L):
    """Sorted canonical codes of the weakly connected typed 4-node digraphs
    with types below L."""
    can = canonical_all(L)
    conn = np.tile(_CONNECTED, len(can) // 4096)
    return np.unique(can[conn])


class KeyTable:
    """Key index of every full code with types below L (or -1 when the
    digraph is not weakly connected)."""

    def __init__(self, L):
        self.L = L
        self.keys = keys(L)
        can = canonical_all(L)
        idx = np.searchsorted(self.keys, can)
        idx[~np.tile(_CONNECTED, len(can) // 4096)] = -1
        self.index = idx
        self.support = np.array([support_edges4(int(c)) for c in self.keys], dtype=np.int64)

    def key(self, arc_bits, types):
        L = self.L
        t = types[0] + L * types[1] + L * L * types[2] + L ** 3 * types[3]
        return int(self.index[arc_bits + 4096 * t])


def arcs_from_csr(row_ptr, col_idx, slot_dir):
    """Set of arcs (u, v) from the support CSR and its per-slot direction
    bits (bit 0: row -> column, bit 1: column -> row)."""
    arcs = set()
    for u in range(len(row_ptr) - 1):
        for s in range(row_ptr[u], row_ptr[u + 1]):
            v = int(col_idx[s])
            if slot_dir[s] & 1:
                arcs.add((u, v))
            if slot_dir[s] & 2:
                arcs.add((v, u))
    return arcs


def _local_bits(arcs, nodes):
    b = 0
    for q, (x, y) in enumerate(ORDERED_PAIRS):
        if (nodes[x], nodes[y]) in arcs:
            b |= 1 << q
    return b


def brute_global(n, arcs, types, L, table=None):
    """Global counts by enumerating every 4-node set (small n)."""
    T = table or KeyTable(L)
    g = np.zeros(len(T.keys), dtype=np.uint64)
    for nodes in itertools.combinations(range(n), 4):
        bits = _local_bits(arcs, nodes)
        k = T.key(bits, [int(types[v]) for v in nodes])
        if k >= 0:
            g[k] += 1
    return g


def edge_rows(row_ptr, col_idx, slot_dir, types, L, pairs=None, table=None):
    """Per support edge (i, j), i < j in row-major CSR order (or the listed
    pairs): the row over keys by the definition above.  The candidates for
    {k, l} are the neighbours U of i and j and, for k in U, the neighbours of
    k: a weakly connected 4-node set through (i, j) has a node of U, and the
    other node is in U or adjacent to it."""
    T = table or KeyTable(L)
    arcs = arcs_from_csr(row_ptr, col_idx, slot_dir)
    n = len(row_ptr) - 1
    nbr = [set(int(x) for x in col_idx[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]
    if pairs is None:
        pairs = [(i, int(j)) for i in range(n) for j in col_idx[row_ptr[i]:row_ptr[i + 1]] if j > i]
    rows = np.zeros((len(pairs), len(T.keys)), dtype=np.uint64)
    for e, (i, j) in enumerate(pairs):
        U = (nbr[i] | nbr[j]) - {i, j}
        seen = set()
        for k in U:
            for l in (U | nbr[k]) - {i, j, k}:
                pr = (min(k, l), max(k, l))
                if pr in seen:
                    continue
                seen.add(pr)
                nodes = (i, j, pr[0], pr[1])
                key = T.key(_local_bits(arcs, nodes), [int(types[v]) for v in nodes])
                if key >= 0:
                    rows[e, key] += 1
    return rows, pairs


def rows_to_global(rows, table):
    sums = rows.astype(object).sum(axis=0)
    out = np.zeros(len(table.keys), dtype=np.uint64)
    for q in range(len(table.keys)):
        d = int(table.support[q])
        assert sums[q] % d == 0, "a key's row sum is not a multiple of its support edge count"
        out[q] = sums[q] // d
    return out
