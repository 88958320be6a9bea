"""Pins for the oracle: closed forms, the paper's printed counts, brute force
and invariants.  These run on the CPU only and never touch the GPU library."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import graphgen
import oracle
from _graphs import (all_graphs, complete, complete_bipartite, csr_from_edges, cycle, diamond, path, relabel, star,
                     tailed_triangle)

HERE = os.path.dirname(os.path.abspath(__file__))
W, TRI, PATH, STAR, CYC, TAIL, CHORD, CLIQ = range(8)


def both(rp, ci, ty, L):
    """Brute force and the paper's method on the same graph; asserts they agree."""
    rb, ob, gb = oracle.brute(rp, ci, ty, L, orbits=True)
    ei, ej = oracle.canonical_edges(rp, ci)
    rm, om = oracle.count_edges(rp, ci, ty, L, ei, ej, orbits=True)
    _, gm = oracle.count_all(rp, ci, ty, L)
    assert np.array_equal(rb, rm)
    assert np.array_equal(ob, om)
    assert np.array_equal(gb, gm)
    return rb, ob, gb


def untyped(rp, ci):
    n = len(rp) - 1
    return both(rp, ci, np.zeros(n, np.uint8), 1)


# ---------------------------------------------------------------- keys ----

def test_per_shape_key_counts_match_table2():
    gold = json.load(open(os.path.join(HERE, "golden", "typed_graphlets_per_shape.json")))
    for K, vals in gold["per_shape"].items():
        for L, v in zip(gold["L_values"], vals):
            assert oracle.typed_per_shape(L, int(K)) == v
    g = gold["all_3_and_4_node_keys"]
    assert oracle.num_keys(g["L"]) == g["count"]


@pytest.mark.parametrize("L", range(1, 10))
def test_rank_is_a_bijection_onto_dense_range(L):
    for k in (3, 4):
        ranks = [oracle.rank(c) for c in itertools.combinations_with_replacement(range(L), k)]
        assert sorted(ranks) == list(range(oracle.typed_per_shape(L, k)))
        # order of the input types does not matter
        for c in itertools.combinations_with_replacement(range(L), k):
            for p in set(itertools.permutations(c)):
                assert oracle.rank(p) == oracle.rank(c)


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_row_columns_map_to_distinct_keys_of_the_right_shape(L):
    R = oracle.row_width(L)
    assert R == 2 * L + 3 * L * (L + 1)
    for a in range(L):
        for b in range(L):
            keys = [oracle.row_key(L, a, b, c) for c in range(R)]
            assert len(set(keys)) == R
            for c, k in enumerate(keys):
                shape = c // L if c < 2 * L else 2 + (c - 2 * L) // (L * (L + 1) // 2)
                lo = oracle.shape_offset(L, shape)
                hi = oracle.shape_offset(L, shape + 1) if shape < 7 else oracle.num_keys(L)
                assert lo <= k < hi


# ----------------------------------------------------------- closed forms --

@pytest.mark.parametrize("n", [4, 5, 6, 8])
def test_complete_graph(n):
    rp, ci = complete(n)
    rows, _, glob = untyped(rp, ci)
    for r in rows:
        assert r[TRI] == n - 2 and r[CLIQ] == math.comb(n - 2, 2)
        assert r[[W, PATH, STAR, CYC, TAIL, CHORD]].sum() == 0
    assert glob[TRI] == math.comb(n, 3) and glob[CLIQ] == math.comb(n, 4)
    assert glob.sum() == math.comb(n, 3) + math.comb(n, 4)


def test_complete_graph_typed_closed_form():
    # K_9 with 2/3/4 nodes of types 0/1/2: global (shape, multiset) count of a
    # clique-shaped graphlet is the product of C(c_t, mult_t).
    n, L = 9, 3
    ty = np.array([0, 0, 1, 1, 1, 2, 2, 2, 2], np.uint8)
    rp, ci = complete(n)
    rows, _, glob = both(rp, ci, ty, L)
    c = np.bincount(ty, minlength=L)
    for k, shape in ((3, TRI), (4, CLIQ)):
        for ms in itertools.combinations_with_replacement(range(L), k):
            want = 1
            for t in range(L):
                want *= math.comb(int(c[t]), ms.count(t))
            assert glob[oracle.key(L, shape, ms)] == want
    # per edge: triangle[t] = c_t - [phi_i = t] - [phi_j = t]
    ei, ej = oracle.canonical_edges(rp, ci)
    for e in range(len(ei)):
        for t in range(L):
            assert rows[e, L + t] == c[t] - (ty[ei[e]] == t) - (ty[ej[e]] == t)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 7])
def test_star(s):
    rp, ci = star(s)
    rows, _, glob = untyped(rp, ci)
    for r in rows:
        assert r[W] == s - 1 and r[STAR] == math.comb(s - 1, 2)
        assert r.sum() == r[W] + r[STAR]
    assert glob[W] == math.comb(s, 2) and glob[STAR] == math.comb(s, 3)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 9])
def test_path(n):
    rp, ci = path(n)
    rows, _, glob = untyped(rp, ci)
    assert glob[W] == max(n - 2, 0) and glob[PATH] == max(n - 3, 0)
    assert glob.sum() == glob[W] + glob[PATH]
    for v in range(n - 1):
        assert rows[v, W] == (v > 0) + (v + 2 < n)


@pytest.mark.parametrize("n", [5, 6, 10])
def test_cycle(n):
    rp, ci = cycle(n)
    rows, orows, glob = untyped(rp, ci)
    for r in rows:
        assert r[W] == 2 and r[PATH] == 3 and r.sum() == 5
    # orbit split of the 4-paths: two as end edge (g3), one as centre (g4)
    assert (orows[:, 2] == 2).all() and (orows[:, 3] == 1).all()
    assert glob[W] == n and glob[PATH] == n


def test_four_cycle():
    rp, ci = cycle(4)
    rows, _, glob = untyped(rp, ci)
    for r in rows:
        assert r[W] == 2 and r[CYC] == 1 and r.sum() == 3
    assert glob[W] == 4 and glob[CYC] == 1 and glob.sum() == 5


@pytest.mark.parametrize("a,b", [(2, 2), (2, 3), (3, 4), (1, 5)])
def test_complete_bipartite_typed(a, b):
    rp, ci = complete_bipartite(a, b)
    ty = np.array([0] * a + [1] * b, np.uint8)
    rows, _, glob = both(rp, ci, ty, 2)
    R = oracle.row_width(2)
    P = 3
    for r in rows:
        # relative to (phi_i, phi_j) = (0, 1): wedges towards a type-1 node come
        # from the type-0 end and vice versa
        assert r[0] + r[1] == (a - 1) + (b - 1)
        assert r[2:4].sum() == 0                               # no triangles
        cyc = r[4 + 2 * P:4 + 3 * P].sum()
        assert cyc == (a - 1) * (b - 1)
        assert r[4 + P:4 + 2 * P].sum() == math.comb(a - 1, 2) + math.comb(b - 1, 2)
        assert r[4:4 + P].sum() == 0                           # no 4-paths
        assert r[4 + 3 * P:].sum() == 0                        # nothing with a triangle
        assert r.sum() == (a - 1) + (b - 1) + (a - 1) * (b - 1) + math.comb(a - 1, 2) + math.comb(b - 1, 2)
    assert glob[oracle.key(2, CYC, [0, 0, 1, 1])] == math.comb(a, 2) * math.comb(b, 2)
    assert glob[oracle.key(2, STAR, [0, 1, 1, 1])] == a * math.comb(b, 3)
    assert glob[oracle.key(2, STAR, [0, 0, 0, 1])] == b * math.comb(a, 3)
    assert glob[oracle.key(2, W, [0, 1, 1])] == a * math.comb(b, 2)
    assert glob[oracle.key(2, W, [0, 0, 1])] == b * math.comb(a, 2)
    assert glob.sum() == (math.comb(a, 2) * math.comb(b, 2) + a * math.comb(b, 3) + b * math.comb(a, 3)
                          + a * math.comb(b, 2) + b * math.comb(a, 2))
    assert R == rows.shape[1]


def test_tailed_triangle_by_hand():
    rp, ci = tailed_triangle()          # triangle 0,1,2 ; tail 2-3
    rows, orows, glob = untyped(rp, ci)
    ei, ej = oracle.canonical_edges(rp, ci)
    e = {(int(a), int(b)): q for q, (a, b) in enumerate(zip(ei, ej))}
    g = lambda edge, k: orows[e[edge], k]   # orbit columns: g1,g2,g3..g12 -> 0,1,2..11
    assert rows[e[(0, 1)], TRI] == 1 and g((0, 1), 7) == 1          # g8 tri-centre
    for edge in ((0, 2), (1, 2)):
        assert rows[e[edge], TRI] == 1 and rows[e[edge], W] == 1 and g(edge, 8) == 1   # g9 tri-edge
    assert rows[e[(2, 3)], W] == 2 and g((2, 3), 6) == 1 and rows[e[(2, 3)], STAR] == 0  # g7 tail
    assert glob[TAIL] == 1 and glob[W] == 2 and glob[TRI] == 1 and glob.sum() == 4
    # typed: a=0, b=0, c=1, d=2 -> every edge carries (tailed, {0,0,1,2}) once
    ty = np.array([0, 0, 1, 2], np.uint8)
    rows3, _, glob3 = both(rp, ci, ty, 3)
    k = oracle.key(3, TAIL, [0, 0, 1, 2])
    for q in range(len(ei)):
        keys = {oracle.row_key(3, ty[ei[q]], ty[ej[q]], c): v for c, v in enumerate(rows3[q]) if v}
        assert keys.get(k) == 1
    assert glob3[k] == 1


def test_diamond_by_hand():
    rp, ci = diamond()                  # chord 0-1
    rows, orows, glob = untyped(rp, ci)
    ei, ej = oracle.canonical_edges(rp, ci)
    for q, (a, b) in enumerate(zip(ei, ej)):
        if (a, b) == (0, 1):
            assert rows[q, TRI] == 2 and orows[q, 10] == 1       # g11 chord
        else:
            assert rows[q, TRI] == 1 and rows[q, W] == 1 and orows[q, 9] == 1  # g10 rim
    assert glob[CHORD] == 1 and glob[TRI] == 2 and glob[W] == 2 and glob.sum() == 5


# ------------------------------------------------------------ brute force --

def test_method_equals_brute_force_on_200_tiny_graphs():
    for idx in range(200):
        g = graphgen.tiny_graph(idx)
        both(g.row_ptr, g.col_idx, g.types, g.L)


def test_method_equals_brute_force_on_every_graph_with_5_nodes():
    typings = [np.zeros(5, np.uint8), np.array([0, 1, 0, 1, 2], np.uint8), np.array([2, 1, 0, 1, 1], np.uint8)]
    for rp, ci in all_graphs(5):
        for ty in typings:
            both(rp, ci, ty, 3)


# ---------------------------------------------------------------- invariants

SHAPE_EDGES = (2, 3, 3, 3, 4, 4, 5, 6)
# per-instance multiplicity of each orbit g1..g12: how many edges of one
# instance of its shape sit in that orbit
ORBIT_SHAPE = (0, 1, 2, 2, 3, 4, 5, 5, 5, 6, 6, 7)
ORBIT_MULT = (2, 3, 2, 1, 3, 4, 1, 1, 2, 4, 1, 6)


def test_orbit_multiplicities_and_eq17_divisors():
    for idx in range(0, 200, 7):
        g = graphgen.tiny_graph(idx)
        rows, orows, glob = oracle.brute(g.row_ptr, g.col_idx, np.zeros(g.n, np.uint8), 1, orbits=True)
        assert sum(ORBIT_MULT[q] for q in range(12) if ORBIT_SHAPE[q] == 7) == SHAPE_EDGES[7]
        for q in range(12):
            assert orows[:, q].sum() == ORBIT_MULT[q] * glob[ORBIT_SHAPE[q]]
        for h in range(8):
            assert rows[:, h].sum() == SHAPE_EDGES[h] * glob[h]


def test_typed_counts_sum_to_untyped_counts():
    # Proposition 1: per edge and per shape, the typed counts partition the untyped count
    g = graphgen.chung_lu_small()
    rows, glob = oracle.count_all(g.row_ptr, g.col_idx, g.types, g.L, nthreads=4)
    rows1, glob1 = oracle.count_all(g.row_ptr, g.col_idx, np.zeros(g.n, np.uint8), 1, nthreads=4)
    L, P = g.L, g.L * (g.L + 1) // 2
    assert np.array_equal(rows[:, :L].sum(1), rows1[:, 0])
    assert np.array_equal(rows[:, L:2 * L].sum(1), rows1[:, 1])
    for h in range(6):
        assert np.array_equal(rows[:, 2 * L + h * P:2 * L + (h + 1) * P].sum(1), rows1[:, 2 + h])
    for h in range(8):
        lo = oracle.shape_offset(L, h)
        hi = oracle.shape_offset(L, h + 1) if h < 7 else oracle.num_keys(L)
        assert glob[lo:hi].sum() == glob1[h]


def test_partition_of_neighbourhoods():
    # Property 2 and the degree identity d_i + d_j = 2|T| + |S_i| + |S_j| + 2
    # (the +2 accounts for i in Gamma_j and j in Gamma_i, which belong to none
    # of T, S_i, S_j)
    g = graphgen.chung_lu_small()
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    rows, _ = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei, ej, nthreads=4)
    deg = np.diff(g.row_ptr)
    S = rows[:, :g.L].sum(1).astype(np.int64)
    T = rows[:, g.L:2 * g.L].sum(1).astype(np.int64)
    assert np.array_equal(deg[ei] + deg[ej], 2 * T + S + 2)
    # |I| = |V| - |S_i| - |S_j| - |T| - 2 is never negative
    assert (g.n - S - T - 2 >= 0).all()


def test_node_relabelling_only_permutes_edges():
    g = graphgen.tiny_graph(17)
    perm = np.random.default_rng(5).permutation(g.n)
    rp2, ci2 = relabel(g.row_ptr, g.col_idx, perm)
    ty2 = np.empty_like(g.types)
    ty2[perm] = g.types
    r1, _, g1 = oracle.brute(g.row_ptr, g.col_idx, g.types, g.L)
    r2, _, g2 = both(rp2, ci2, ty2, g.L)
    assert np.array_equal(g1, g2)
    e1 = oracle.canonical_edges(g.row_ptr, g.col_idx)
    e2 = oracle.canonical_edges(rp2, ci2)
    idx2 = {(int(a), int(b)): q for q, (a, b) in enumerate(zip(*e2))}
    for q, (a, b) in enumerate(zip(*e1)):
        pa, pb = int(perm[a]), int(perm[b])
        q2 = idx2[(min(pa, pb), max(pa, pb))]
        # the row is relative to (phi_i, phi_j), which swap when the order flips;
        # compare through global keys instead
        k1 = {oracle.row_key(g.L, g.types[a], g.types[b], c): v for c, v in enumerate(r1[q]) if v}
        k2 = {oracle.row_key(g.L, ty2[min(pa, pb)], ty2[max(pa, pb)], c): v for c, v in enumerate(r2[q2]) if v}
        assert k1 == k2


def test_merging_two_types_sums_their_keys():
    g = graphgen.tiny_graph(3)
    L = 3
    ty = (np.arange(g.n) % L).astype(np.uint8)
    _, _, g3 = both(g.row_ptr, g.col_idx, ty, L)
    merged = np.where(ty == 2, 1, ty).astype(np.uint8)
    _, _, g2 = both(g.row_ptr, g.col_idx, merged, 2)
    acc = np.zeros_like(g2)
    for shape in range(8):
        k = 3 if shape < 2 else 4
        for ms in itertools.combinations_with_replacement(range(L), k):
            mm = [min(t, 1) if t < 2 else 1 for t in ms]
            acc[oracle.key(2, shape, mm)] += g3[oracle.key(L, shape, ms)]
    assert np.array_equal(acc, g2)


def test_dense_random_graph_hits_every_key():
    # G(200, 0.5) with 25 nodes of each of 8 types: every one of the 2220
    # typed 3/4-node graphlets occurs (brute force is too slow here, so only
    # the method runs; it is pinned above)
    n, L = 200, 8
    rp, ci = graphgen.gnp(n, 0.5, 77)
    ty = (np.arange(n) % L).astype(np.uint8)
    _, glob = oracle.count_all(rp, ci, ty, L, per_edge=False, nthreads=8)
    assert len(glob) == 2220 and (glob > 0).all()


# ------------------------------------------------------ cost-model network --

def test_mlp_reference_gradient_matches_finite_differences():
    from oracle import mlp_ref
    rng = np.random.default_rng(11)
    p = rng.normal(0, 0.3, mlp_ref.NPARAM)
    stats = np.concatenate([rng.normal(0, 1, 16), rng.uniform(0.5, 2.0, 16)])
    X = rng.normal(0, 2, (40, 16))
    Y = rng.normal(0, 1, 40)
    g = mlp_ref.gradient(p, stats, X, Y)
    idx = rng.choice(mlp_ref.NPARAM, 300, replace=False)
    h = 1e-6
    for q in idx:
        a = p.copy(); a[q] += h
        b = p.copy(); b[q] -= h
        fd = (mlp_ref.loss(a, stats, X, Y) - mlp_ref.loss(b, stats, X, Y)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 + 1e-5 * abs(g[q]), (q, fd, g[q])


def test_bf16_rounding_reference():
    from oracle import mlp_ref
    x = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.1415926, 1e-40, np.inf], np.float32)
    r = mlp_ref.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0              # tie between 1.0 and 1.0078125 rounds to even
    assert r[2] == np.float32(1.0078125)
    assert r[3] == np.float32(1.0078125)
    assert r[4] == np.float32(-3.140625)
    assert r[6] == np.inf
    assert (r.view(np.uint32) & 0xFFFF == 0).all()


def test_part_structure_forces_zero_keys():
    # On k-partite graphs typed by part, a (shape, multiset) key that no
    # placement can properly colour never occurs (brute force).
    from test_gpu_partite import colourable
    for sizes, seed in (([7, 6], 3), ([5, 4, 4], 4)):
        k = len(sizes)
        rp, ci, parts = graphgen.kpartite_cl(sizes, [2.5] * k, [6.0] * k, [4.0] * k, 3 * sum(sizes), seed)
        rows, _, glob = oracle.brute(rp, ci, parts, k)
        seen = 0
        for key in range(oracle.num_keys(k)):
            shape = next(h for h in range(8) if key < (oracle.shape_offset(k, h + 1) if h < 7
                                                        else oracle.num_keys(k)))
            types = None
            for ms in itertools.combinations_with_replacement(range(k), 3 if shape < 2 else 4):
                if oracle.key(k, shape, ms) == key:
                    types = ms
            if not colourable(shape, types):
                assert glob[key] == 0
            seen += int(glob[key] > 0)
        assert seen > 0


def _typed_sets(rp, ci, ty, L, i, j):
    """|S_i^t|, |S_j^t|, |T_ij^t| of edge (i, j) by the set definitions of
    Section 4.1 (S_i = Gamma_i minus Gamma_j minus {j})."""
    gi = set(ci[rp[i]:rp[i + 1]].tolist()) - {j}
    gj = set(ci[rp[j]:rp[j + 1]].tolist()) - {i}
    cnt = lambda s: np.bincount(ty[sorted(s)].astype(np.int64), minlength=L) if s else np.zeros(L, np.int64)
    return cnt(gi - gj), cnt(gj - gi), cnt(gi & gj)


def _check_eqs_7_to_10(rp, ci, ty, L, orows, ei, ej):
    P = L * (L + 1) // 2
    C = lambda x: x * (x - 1) // 2
    for q, (i, j) in enumerate(zip(ei, ej)):
        Si, Sj, T = _typed_sets(rp, ci, ty, L, int(i), int(j))
        o = orows[q].astype(np.int64)
        g = lambda k, p: int(o[2 * L + (k - 3) * P + p])
        for u in range(L):
            for t in range(u + 1):
                p = u * (u + 1) // 2 + t
                if t == u:
                    want = (Si[t] * Sj[t] - g(6, p), C(Si[t]) + C(Sj[t]) - g(7, p),
                            T[t] * (Si[t] + Sj[t]) - g(10, p), C(T[t]) - g(12, p))
                else:
                    want = (Si[t] * Sj[u] + Si[u] * Sj[t] - g(6, p), Si[t] * Si[u] + Sj[t] * Sj[u] - g(7, p),
                            T[t] * (Si[u] + Sj[u]) + T[u] * (Si[t] + Sj[t]) - g(10, p), T[t] * T[u] - g(12, p))
                assert (g(4, p), g(5, p), g(9, p), g(11, p)) == tuple(int(x) for x in want), (q, t, u)


def test_eqs_7_to_10_hold_for_the_counted_orbits():
    """Eqs. 7-10 derive g4, g5, g9 and g11 of every edge and type pair from
    the typed set sizes and g6, g7, g10, g12.  The oracle counts all twelve
    orbits from the definition (brute force, and the per-edge counter), so
    the identities are checked here, not assumed: on 60 tiny graphs and on
    the 2000-node Chung-Lu graph."""
    for idx in range(60):
        g = graphgen.tiny_graph(idx)
        _, ob, _ = oracle.brute(g.row_ptr, g.col_idx, g.types, g.L, orbits=True)
        ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
        _check_eqs_7_to_10(g.row_ptr, g.col_idx, g.types, g.L, ob, ei, ej)
    g = graphgen.chung_lu_small()
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    sel = np.arange(0, g.m, 13)
    _, om = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei[sel], ej[sel], orbits=True, nthreads=4)
    _check_eqs_7_to_10(g.row_ptr, g.col_idx, g.types, g.L, om, ei[sel], ej[sel])
