"""Small hand-built graphs for closed-form checks (test helpers only)."""
import itertools

import numpy as np


def csr_from_edges(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a == b:
            raise ValueError("self loop")
        adj[a].add(b)
        adj[b].add(a)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for v in range(n):
        nb = sorted(adj[v])
        cols.extend(nb)
        row_ptr[v + 1] = row_ptr[v] + len(nb)
    return row_ptr, np.array(cols, dtype=np.int32)


def csr_from_arcs(n, arcs):
    """Support CSR of a set of arcs (u, v) and its per-slot direction bits
    (bit 0: row -> column, bit 1: column -> row)."""
    row_ptr, col_idx = csr_from_edges(n, {(min(u, v), max(u, v)) for (u, v) in arcs})
    sd = np.zeros(len(col_idx), np.uint8)
    for u in range(n):
        for s in range(row_ptr[u], row_ptr[u + 1]):
            v = int(col_idx[s])
            sd[s] = (1 if (u, v) in arcs else 0) | (2 if (v, u) in arcs else 0)
    return row_ptr, col_idx, sd


def complete(n):
    return csr_from_edges(n, itertools.combinations(range(n), 2))


def star(s):
    return csr_from_edges(s + 1, [(0, v) for v in range(1, s + 1)])


def path(n):
    return csr_from_edges(n, [(v, v + 1) for v in range(n - 1)])


def cycle(n):
    return csr_from_edges(n, [(v, (v + 1) % n) for v in range(n)])


def complete_bipartite(a, b):
    return csr_from_edges(a + b, [(x, a + y) for x in range(a) for y in range(b)])


def tailed_triangle():
    # triangle 0,1,2 ; tail 2-3
    return csr_from_edges(4, [(0, 1), (0, 2), (1, 2), (2, 3)])


def diamond():
    # K4 minus edge 2-3 ; chord 0-1
    return csr_from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)])


def all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield csr_from_edges(n, [p for q, p in enumerate(pairs) if (mask >> q) & 1])


def relabel(row_ptr, col_idx, perm):
    """Node v becomes perm[v]."""
    n = len(row_ptr) - 1
    edges = []
    for v in range(n):
        for s in range(row_ptr[v], row_ptr[v + 1]):
            if col_idx[s] > v:
                edges.append((int(perm[v]), int(perm[col_idx[s]])))
    return csr_from_edges(n, edges)
