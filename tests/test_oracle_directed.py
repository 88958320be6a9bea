"""Pins of the directed typed 3-node oracle: the triad catalogue, closed
forms, two independent counters agreeing, and the undirected rows recovered
by summing over directions."""
import itertools
import math

import numpy as np

import graphgen
import oracle
from oracle import directed as od


def test_thirteen_connected_triads_without_types():
    # the classic triad census: 16 isomorphism classes on 3 nodes, 3 of them
    # weakly disconnected (empty, one arc, one mutual pair)
    assert len(od.keys(1)) == 13
    divisors = sorted(od.support_edges(int(c)) for c in od.keys(1))
    assert divisors.count(2) == 6 and divisors.count(3) == 7


def test_key_count_with_types():
    # brute force over labelled triads: orbits of the 6 node orderings
    for L in (2, 3):
        seen = set()
        for adj in range(64):
            if od.support_edges(adj) < 2:
                continue
            for t in itertools.product(range(L), repeat=3):
                seen.add(od.canonical(adj | (t[0] << 6) | (t[1] << 10) | (t[2] << 14)))
        assert len(od.keys(L)) == len(seen)
    # Burnside count for L = 2 (orbits of typed connected triads under S3)
    fixed = 0
    for perm in itertools.permutations(range(3)):
        for adj in range(64):
            if od.support_edges(adj) < 2:
                continue
            for t in itertools.product(range(2), repeat=3):
                code = adj | (t[0] << 6) | (t[1] << 10) | (t[2] << 14)
                arcs, types = od.decode(code)
                inv = {perm[p]: p for p in range(3)}
                moved = od.triad_code({(inv[x], inv[y]) for (x, y) in arcs}, [types[perm[p]] for p in range(3)])
                fixed += moved == code
    assert fixed % 6 == 0 and len(od.keys(2)) == fixed // 6


def one_key(L, arcs, types):
    return od.key_index(L)[od.canonical(od.triad_code(arcs, types))]


def test_closed_forms():
    # directed 3-cycle
    g = od.brute_global(3, {(0, 1), (1, 2), (2, 0)}, [0, 0, 0], 1)
    assert g.sum() == 1 and g[one_key(1, {(0, 1), (1, 2), (2, 0)}, [0, 0, 0])] == 1
    # transitive tournament: every triple is transitive
    n = 7
    arcs = {(u, v) for u in range(n) for v in range(u + 1, n)}
    g = od.brute_global(n, arcs, [0] * n, 1)
    assert g[one_key(1, {(0, 1), (0, 2), (1, 2)}, [0, 0, 0])] == math.comb(n, 3) == g.sum()
    # all-mutual complete graph
    arcs = {(u, v) for u in range(n) for v in range(n) if u != v}
    g = od.brute_global(n, arcs, [0] * n, 1)
    assert g[one_key(1, arcs & {(0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1)}, [0, 0, 0])] == math.comb(n, 3)
    # out-star with typed leaves
    s = 6
    arcs = {(0, v) for v in range(1, s + 1)}
    types = [1] + [v % 2 for v in range(1, s + 1)]
    g = od.brute_global(s + 1, arcs, types, 2)
    n1, n0 = sum(t == 1 for t in types[1:]), sum(t == 0 for t in types[1:])
    assert g[one_key(2, {(0, 1), (0, 2)}, [1, 0, 0])] == math.comb(n0, 2)
    assert g[one_key(2, {(0, 1), (0, 2)}, [1, 1, 1])] == math.comb(n1, 2)
    assert g[one_key(2, {(0, 1), (0, 2)}, [1, 0, 1])] == n0 * n1
    assert g.sum() == math.comb(s, 2)


def test_per_edge_counter_agrees_with_brute_force():
    for idx in range(0, 60, 3):
        gr, sd = graphgen.tiny_digraph(idx)
        if gr.m == 0:
            continue
        L = gr.L
        rows, codes, ends = od.edge_rows(gr.row_ptr, gr.col_idx, sd, gr.types, L)
        want = od.brute_global(gr.n, od.arcs_from_csr(gr.row_ptr, gr.col_idx, sd), gr.types, L)
        assert np.array_equal(od.rows_to_global(rows, codes, ends, gr.types, L), want), idx


def test_summing_directions_gives_the_undirected_rows():
    g = graphgen.chung_lu_small()
    sd = graphgen.orient(g.row_ptr, g.col_idx, 77)
    rows, _, ends = od.edge_rows(g.row_ptr, g.col_idx, sd, g.types, g.L)
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    assert [tuple(e) for e in ends] == list(zip(ei.tolist(), ej.tolist()))
    und, _ = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei, ej, nthreads=8)
    L = g.L
    # [e][c(i,k)][c(j,k)][t], with an empty (0, 0) cell put in front
    r = np.concatenate([np.zeros((len(ends), 1, L), np.uint64), rows.reshape(len(ends), 15, L)], axis=1)
    r = r.reshape(len(ends), 4, 4, L)
    wedge = r[:, 1:, 0, :].sum(axis=1) + r[:, 0, 1:, :].sum(axis=1)
    tri = r[:, 1:, 1:, :].sum(axis=(1, 2))
    assert np.array_equal(wedge, und[:, :L]) and np.array_equal(tri, und[:, L:2 * L])


def test_orientation_is_consistent():
    g = graphgen.chung_lu_small()
    sd = graphgen.orient(g.row_ptr, g.col_idx, 3)
    assert (sd > 0).all() and (sd < 4).all()
    arcs = od.arcs_from_csr(g.row_ptr, g.col_idx, sd)
    for u in range(g.n):
        for s in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col_idx[s])
            assert sd[s] == od.dir_code(arcs, u, v)
    assert np.array_equal(sd, graphgen.orient(g.row_ptr, g.col_idx, 3))
    frac_both = (sd == 3).mean()
    assert 0.1 < frac_both < 0.3
