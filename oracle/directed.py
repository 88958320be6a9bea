"""Oracle for directed typed 3-node graphlets (test infrastructure only).

Only the test-suite and the benchmark may import this module; the product
library never calls it and shares no code with it.

The paper's directed variant replaces each typed neighbour set by its typed
out- and in-neighbour sets (the Directed Typed Graphlets subsection).  For 3
nodes that gives, for a support edge (i, j) and a third node k, the direction
codes of the pairs (i, k) and (j, k); this module writes the definitions out
plainly:

* direction code of an ordered pair (u, v): [u -> v] + 2 [v -> u], 0..3;
* a directed typed triad on ordered nodes (a, b, c): six arc bits (a->b,
  b->a, a->c, c->a, b->c, c->b) in bits 0..5 and the three types in bits
  6-9, 10-13 and 14-17; its canonical code is the smallest code over the six
  orderings of the nodes; the keys of L types are the canonical codes of
  weakly connected triads with types below L, numbered in increasing order
  (the "unique id" that the subsection asks for);
* per-edge row of support edge (i, j), i < j: for every k with c(i,k) or
  c(j,k) nonzero, column ((4 c(i,k) + c(j,k)) - 1) L + phi_k gains one;
* global count of a key: the number of node triples whose induced triad has
  that canonical code.

Two independent counters: `brute_global` over all node triples, and
`edge_rows` per support edge with `rows_to_global` (each triad is seen from
each of its 2 or 3 support edges).
"""
from __future__ import annotations

import itertools

import numpy as np

# arc bits of the ordered node pairs (x, y) -> bit for x -> y
_BIT = {(0, 1): 0, (1, 0): 1, (0, 2): 2, (2, 0): 3, (1, 2): 4, (2, 1): 5}


def triad_code(arcs, types):
    """Code of the triad on ordered nodes 0, 1, 2: arcs is a set of (x, y)."""
    adj = 0
    for (x, y) in arcs:
        adj |= 1 << _BIT[(x, y)]
    return adj | (types[0] << 6) | (types[1] << 10) | (types[2] << 14)


def decode(code):
    arcs = {xy for xy, b in _BIT.items() if code >> b & 1}
    return arcs, ((code >> 6) & 15, (code >> 10) & 15, (code >> 14) & 15)


def canonical(code):
    arcs, types = decode(code)
    best = None
    for perm in itertools.permutations(range(3)):
        # node perm[p] of the old order becomes node p of the new one
        inv = {perm[p]: p for p in range(3)}
        c = triad_code({(inv[x], inv[y]) for (x, y) in arcs}, [types[perm[p]] for p in range(3)])
        best = c if best is None else min(best, c)
    return best


def support_edges(code):
    arcs, _ = decode(code)
    return len({frozenset(a) for a in arcs})


def keys(L):
    """Sorted canonical codes of the weakly connected typed triads with L
    types (the directed 3-node key list)."""
    out = set()
    for adj in range(64):
        if support_edges(adj) < 2:
            continue
        for t in itertools.product(range(L), repeat=3):
            out.add(canonical(adj | (t[0] << 6) | (t[1] << 10) | (t[2] << 14)))
    return np.array(sorted(out), dtype=np.int64)


def key_index(L):
    ks = keys(L)
    return {int(c): q for q, c in enumerate(ks)}


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


def brute_global(n, arcs, types, L):
    """Global counts by enumerating every node triple (small n)."""
    idx = key_index(L)
    g = np.zeros(len(idx), dtype=np.uint64)
    nbr = [set() for _ in range(n)]
    for (u, v) in arcs:
        nbr[u].add(v)
        nbr[v].add(u)
    for a, b, c in itertools.combinations(range(n), 3):
        nodes = (a, b, c)
        local = {(x, y) for x in range(3) for y in range(3) if x != y and (nodes[x], nodes[y]) in arcs}
        code = triad_code(local, [int(types[v]) for v in nodes])
        if support_edges(code) >= 2:
            g[idx[canonical(code)]] += 1
    return g


def dir_code(arcs, u, v):
    return (1 if (u, v) in arcs else 0) + (2 if (v, u) in arcs else 0)


def edge_rows(row_ptr, col_idx, slot_dir, types, L):
    """Per support edge (i, j), i < j in row-major CSR order: the 15 L row by
    the definition above, and the edge's own direction code c(i, j)."""
    arcs = arcs_from_csr(row_ptr, col_idx, slot_dir)
    n = len(row_ptr) - 1
    nbr = [set(int(x) for x in col_idx[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]
    rows, codes, ends = [], [], []
    for i in range(n):
        for s in range(row_ptr[i], row_ptr[i + 1]):
            j = int(col_idx[s])
            if j <= i:
                continue
            row = np.zeros(15 * L, dtype=np.uint64)
            for k in (nbr[i] | nbr[j]) - {i, j}:
                a, b = dir_code(arcs, i, k), dir_code(arcs, j, k)
                row[(4 * a + b - 1) * L + int(types[k])] += 1
            rows.append(row)
            codes.append(dir_code(arcs, i, j))
            ends.append((i, j))
    return np.array(rows, dtype=np.uint64).reshape(-1, 15 * L), np.array(codes, np.int64), ends


def rows_for_edges(row_ptr, col_idx, slot_dir, types, L, pairs):
    """Rows of the given support edges (i, j) only, by the same definition,
    reading just the rows of their endpoints (for large graphs)."""
    def row_of(v):
        lo, hi = int(row_ptr[v]), int(row_ptr[v + 1])
        return {int(col_idx[s]): int(slot_dir[s]) for s in range(lo, hi)}
    out = np.zeros((len(pairs), 15 * L), dtype=np.uint64)
    for e, (i, j) in enumerate(pairs):
        ri, rj = row_of(int(i)), row_of(int(j))
        for k in (set(ri) | set(rj)) - {int(i), int(j)}:
            out[e, (4 * ri.get(k, 0) + rj.get(k, 0) - 1) * L + int(types[k])] += 1
    return out


def rows_to_global(rows, codes, ends, types, L):
    """Global counts from per-edge rows: each triad is seen from each of its
    support edges, so the sums are divided by that number."""
    idx = key_index(L)
    sums = np.zeros(len(idx), dtype=object)
    ks = keys(L)
    for e, (i, j) in enumerate(ends):
        cij = int(codes[e])
        for col in np.nonzero(rows[e])[0]:
            cat, t = divmod(int(col), L)
            a, b = divmod(cat + 1, 4)
            # nodes (i, j, k): arcs from the three direction codes
            arcs = set()
            for (x, y, c) in ((0, 1, cij), (0, 2, a), (1, 2, b)):
                if c & 1:
                    arcs.add((x, y))
                if c & 2:
                    arcs.add((y, x))
            code = triad_code(arcs, [int(types[i]), int(types[j]), t])
            sums[idx[canonical(code)]] += int(rows[e, col])
    out = np.zeros(len(idx), dtype=np.uint64)
    for q in range(len(idx)):
        d = support_edges(int(ks[q]))
        assert sums[q] % d == 0, "a triad sum is not a multiple of its support edge count"
        out[q] = sums[q] // d
    return out
