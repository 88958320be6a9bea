"""Pins of the directed typed 4-node oracle (CPU): class counts against
textbook values and Burnside's lemma, the per-edge counter against the
enumeration of every 4-node set, direction-summed rows against the
undirected oracle, and closed forms."""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import directed4 as d4


def burnside_all(L):
    """Typed 4-node digraphs up to isomorphism (connected or not): the
    average over the 24 node permutations of 2^(cycles on ordered pairs) *
    L^(cycles on nodes)."""
    total = 0
    for perm in itertools.permutations(range(4)):
        def cycles(items, f):
            seen, c = set(), 0
            for x in items:
                if x in seen:
                    continue
                c += 1
                while x not in seen:
                    seen.add(x)
                    x = f(x)
            return c
        c_nodes = cycles(range(4), lambda v: perm[v])
        c_pairs = cycles(d4.ORDERED_PAIRS, lambda xy: (perm[xy[0]], perm[xy[1]]))
        total += 2 ** c_pairs * L ** c_nodes
    assert total % 24 == 0
    return total // 24


def test_class_counts():
    # 218 digraphs on 4 nodes up to isomorphism, 199 of them weakly connected
    assert len(np.unique(d4.canonical_all(1))) == 218 == burnside_all(1)
    assert len(d4.keys(1)) == 199
    for L in (2, 3):
        assert len(np.unique(d4.canonical_all(L))) == burnside_all(L)


def test_canonical_is_invariant_and_scalar_matches_vectorised():
    rng = np.random.default_rng(5)
    can = d4.canonical_all(3)
    for _ in range(300):
        arcs = int(rng.integers(0, 4096))
        ty = [int(x) for x in rng.integers(0, 3, size=4)]
        code = arcs | sum(t << (12 + 4 * p) for p, t in enumerate(ty))
        c0 = d4.canonical4(code)
        assert c0 == can[arcs + 4096 * (ty[0] + 3 * ty[1] + 9 * ty[2] + 27 * ty[3])]
        perm = rng.permutation(4)
        a, t = d4.decode4(code)
        moved = d4.code4({(int(perm[x]), int(perm[y])) for x, y in a}, [t[int(np.argwhere(perm == p)[0][0])]
                                                                       for p in range(4)])
        assert d4.canonical4(moved) == c0


def tiny_digraph(idx, L):
    g = graphgen.tiny_graph(idx)
    sd = graphgen.orient(g.row_ptr, g.col_idx, 700 + idx, 0.3)
    ty = (g.types % L).astype(np.uint8)
    return g, sd, ty


@pytest.mark.parametrize("L", [1, 2])
def test_per_edge_rows_equal_enumeration_of_all_sets(L):
    T = d4.KeyTable(L)
    for idx in range(25):
        g, sd, ty = tiny_digraph(idx, L)
        arcs = d4.arcs_from_csr(g.row_ptr, g.col_idx, sd)
        want = d4.brute_global(g.n, arcs, ty, L, table=T)
        rows, _ = d4.edge_rows(g.row_ptr, g.col_idx, sd, ty, L, table=T)
        assert np.array_equal(d4.rows_to_global(rows, T), want), idx


def _undirected_key(L, code):
    arcs, types = d4.decode4(code)
    deg = [0] * 4
    ne = 0
    for x, y in d4.UNORDERED:
        if (x, y) in arcs or (y, x) in arcs:
            ne += 1
            deg[x] += 1
            deg[y] += 1
    maxd = max(deg)
    h = (3 if maxd == 3 else 2) if ne == 3 else ((5 if maxd == 3 else 4) if ne == 4 else (6 if ne == 5 else 7))
    return oracle.key(L, h, list(types))


def test_direction_summed_rows_equal_undirected_rows():
    L = 2
    T = d4.KeyTable(L)
    ukey = np.array([_undirected_key(L, int(c)) for c in T.keys])
    for idx in range(20):
        g, sd, ty = tiny_digraph(idx, L)
        rows, pairs = d4.edge_rows(g.row_ptr, g.col_idx, sd, ty, L, table=T)
        urows, _, _ = oracle.brute(g.row_ptr, g.col_idx, ty, L)
        for e, (i, j) in enumerate(pairs):
            want = {}
            for col in range(2 * L, oracle.row_width(L)):
                v = int(urows[e, col])
                if v:
                    k = oracle.row_key(L, int(ty[i]), int(ty[j]), col)
                    want[k] = want.get(k, 0) + v
            got = {}
            for q in np.nonzero(rows[e])[0]:
                got[int(ukey[q])] = got.get(int(ukey[q]), 0) + int(rows[e, q])
            assert got == want, (idx, e)


def _csr(n, arcs):
    sup = {}
    for u, v in arcs:
        a, b = min(u, v), max(u, v)
        sup[(a, b)] = sup.get((a, b), 0) | (1 if (u, v) == (a, b) else 2)
    rows = [[] for _ in range(n)]
    for (a, b), c in sup.items():
        rows[a].append((b, c))
        rows[b].append((a, ((c & 1) << 1) | (c >> 1)))
    rp, ci, sd = [0], [], []
    for v in range(n):
        for w, c in sorted(rows[v]):
            ci.append(w)
            sd.append(c)
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(sd, np.uint8)


def test_closed_forms():
    T = d4.KeyTable(1)
    # complete mutual digraph on n nodes: C(n, 4) sets, all of one class
    n = 7
    arcs = {(u, v) for u in range(n) for v in range(n) if u != v}
    rp, ci, sd = _csr(n, arcs)
    rows, _ = d4.edge_rows(rp, ci, sd, np.zeros(n, np.uint8), 1, table=T)
    g = d4.rows_to_global(rows, T)
    full = T.key((1 << 12) - 1, [0, 0, 0, 0])
    assert g[full] == math.comb(n, 4) and g.sum() == math.comb(n, 4)
    # transitive tournament: every 4-set is a transitive tournament on 4 nodes
    arcs = {(u, v) for u in range(n) for v in range(n) if u < v}
    rp, ci, sd = _csr(n, arcs)
    rows, _ = d4.edge_rows(rp, ci, sd, np.zeros(n, np.uint8), 1, table=T)
    g = d4.rows_to_global(rows, T)
    tt = T.key(d4.code4({(x, y) for x in range(4) for y in range(4) if x < y}, [0] * 4) & 0xFFF, [0, 0, 0, 0])
    assert g[tt] == math.comb(n, 4) and g.sum() == math.comb(n, 4)
    # directed 4-cycle: one set, the cycle class; each of its 4 support edges sees it once
    arcs = {(0, 1), (1, 2), (2, 3), (3, 0)}
    rp, ci, sd = _csr(4, arcs)
    rows, _ = d4.edge_rows(rp, ci, sd, np.zeros(4, np.uint8), 1, table=T)
    cyc = T.key(d4.code4(arcs, [0] * 4) & 0xFFF, [0, 0, 0, 0])
    assert rows[:, cyc].tolist() == [1, 1, 1, 1] and rows.sum() == 4
