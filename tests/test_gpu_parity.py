"""Parity of the gfx950 path (through the C-ABI) with the oracle: bit-exact
per-edge rows and global counts."""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from _gpu import gpu_count, note
from _graphs import all_graphs, complete, complete_bipartite, csr_from_edges, cycle, star

pytestmark = pytest.mark.gpu


def assert_same(got_rows, got_glob, want_rows, want_glob, what):
    if want_glob is not None:
        assert np.array_equal(got_glob, want_glob), f"{what}: global counts differ"
    if want_rows is not None:
        bad = np.nonzero((got_rows != want_rows).any(axis=1))[0]
        assert len(bad) == 0, f"{what}: {len(bad)} edge rows differ, first edge {bad[:5]}"


def test_tiny_graphs_match_brute_force():
    import paper_1901_10026_amd as tg
    probes = tg.Tuning.from_dict({"clique_pass": 0})
    for idx in range(200):
        g = graphgen.tiny_graph(idx)
        note(f"tiny{idx} n={g.n} m={g.m} L={g.L}")
        rb, _, gb = oracle.brute(g.row_ptr, g.col_idx, g.types, g.L)
        for sched in ("none", "degree"):
            gg, rr, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, schedule=sched, validate=True)
            assert_same(rr, gg, rb, gb, f"tiny{idx}/{sched}")
        gg, rr, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, tuning=probes)
        assert_same(rr, gg, rb, gb, f"tiny{idx}/out-list probes")


def test_every_graph_on_five_nodes():
    ty = np.array([0, 1, 0, 1, 2], np.uint8)
    for q, (rp, ci) in enumerate(all_graphs(5)):
        if len(ci) == 0:
            continue
        rb, _, gb = oracle.brute(rp, ci, ty, 3)
        gg, rr, _ = gpu_count(rp, ci, ty, 3)
        assert_same(rr, gg, rb, gb, f"5-node graph {q}")


def test_chung_lu_2k_all_edges():
    g = graphgen.chung_lu_small()
    note(f"cl-2k n={g.n} m={g.m}")
    want_rows, want_glob = oracle.count_all(g.row_ptr, g.col_idx, g.types, g.L, nthreads=8)
    for sched in ("none", "degree"):
        gg, rr, ends = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, schedule=sched, endpoints=True)
        assert_same(rr, gg, want_rows, want_glob, f"cl-2k/{sched}")
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    assert np.array_equal(ends[:, 0], ei) and np.array_equal(ends[:, 1], ej)


def test_edge_ranges_and_global_only():
    g = graphgen.chung_lu_small()
    gg, rr, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L)
    for e0, e1 in ((0, 1), (17, 900), (g.m - 5, g.m), (300, 300)):
        g2, r2, ends = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, edge_range=(e0, e1), endpoints=True)
        assert np.array_equal(g2, gg)
        assert np.array_equal(r2, rr[e0:e1])
        assert ends.shape == (e1 - e0, 2)
    g3, r3, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, per_edge=False)
    assert r3 is None and np.array_equal(g3, gg)


def test_edge_id_sample():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    gg, rr, ee = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, endpoints=True)
    rng = np.random.default_rng(5)
    ids = np.unique(np.concatenate([[0, g.m - 1], rng.choice(g.m, 300, replace=False)]))
    dev_ids = torch.from_numpy(ids.astype(np.int64)).to("cuda:0")
    g2, r2, e2 = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, edge_ids=dev_ids, endpoints=True)
    assert np.array_equal(g2, gg)
    assert np.array_equal(r2, rr[ids])
    assert np.array_equal(e2, ee[ids])
    for bad in ([5, 5], [7, 3], [-1], [g.m]):
        with pytest.raises(tg.TGError, match="INVALID_ARG"):
            gpu_count(g.row_ptr, g.col_idx, g.types, g.L, edge_ids=torch.tensor(bad, dtype=torch.int64,
                                                                               device="cuda:0"))


def test_per_edge_cycle_counters():
    """4-cycle counters kept per edge (the layout for graphs whose per-slot
    counters exceed the memory budget) give the same counts."""
    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    gg, rr, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L)
    t = tg.Tuning.from_dict({"c4_slot_budget_mb": 0, "c4_slices": 8})
    g2, r2, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, tuning=t)
    assert np.array_equal(g2, gg) and np.array_equal(r2, rr)


def test_common_neighbour_lists_or_row_intersection():
    """T_ij read from the lists the typed-triangle pass keeps (the default)
    or found again by intersecting the two rows (no list budget): the same
    counts, with and without rows."""
    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    gg, rr, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L)
    t = tg.Tuning.from_dict({"tlist_budget_mib": 0})
    assert t.tlist_budget_mib == 0 and tg.Tuning.default().tlist_budget_mib > 0
    g2, r2, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, tuning=t)
    assert np.array_equal(g2, gg) and np.array_equal(r2, rr)
    g3, _, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, tuning=t, per_edge=False)
    assert np.array_equal(g3, gg)
    # 1 MiB: above 12 B per edge, below the lists (1.4 MB), so none are kept
    g4, r4, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, tuning=tg.Tuning.from_dict({"tlist_budget_mib": 1}))
    assert np.array_equal(g4, gg) and np.array_equal(r4, rr)


def test_rows_only_counting():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    gg, rr, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L)
    ids = np.arange(3, g.m, 37, dtype=np.int64)
    dev_ids = torch.from_numpy(ids).to("cuda:0")
    g2, r2, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, edge_ids=dev_ids, global_counts=False)
    assert g2 is None and np.array_equal(r2, rr[ids])
    g3, r3, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L, edge_range=(100, 1500), global_counts=False)
    assert g3 is None and np.array_equal(r3, rr[100:1500])


@pytest.mark.parametrize("n,L", [(12, 3), (60, 4), (200, 2), (301, 5), (302, 5), (420, 8)])
def test_complete_graphs_hit_heavy_paths(n, L):
    # |T_ij| = n - 2 exceeds one wavefront's capacity for n >= 131, and the
    # highest-ranked nodes carry enough wedges for the grouped dense path.
    # K_302: the lowest node's 301 higher neighbours take the clique pass's
    # workgroup tier with LDS rows at an odd row count.
    rp, ci = complete(n)
    ty = (np.arange(n) % L).astype(np.uint8)
    note(f"K_{n} L={L}")
    gg, rr, _ = gpu_count(rp, ci, ty, L)
    c = np.bincount(ty, minlength=L)
    for k, shape in ((3, 1), (4, 7)):
        for ms in itertools.combinations_with_replacement(range(L), k):
            want = 1
            for t in range(L):
                want *= math.comb(int(c[t]), ms.count(t))
            assert gg[oracle.key(L, shape, ms)] == want
    assert gg.sum() == math.comb(n, 3) + math.comb(n, 4)
    ei, ej = oracle.canonical_edges(rp, ci)
    sample = np.linspace(0, len(ei) - 1, 40).astype(np.int64)
    want_rows, _ = oracle.count_edges(rp, ci, ty, L, ei[sample], ej[sample])
    assert np.array_equal(rr[sample], want_rows)


@pytest.mark.parametrize("s", [3, 100, 5000])
def test_big_star(s):
    rp, ci = star(s)
    ty = (np.arange(s + 1) % 2).astype(np.uint8)
    note(f"star {s}")
    gg, rr, _ = gpu_count(rp, ci, ty, 2)
    rb_rows, glob = oracle.count_all(rp, ci, ty, 2)
    assert_same(rr, gg, rb_rows, glob, f"star{s}")


@pytest.mark.parametrize("a,b", [(2, 3), (3, 3000), (40, 60)])
def test_complete_bipartite(a, b):
    rp, ci = complete_bipartite(a, b)
    ty = np.array([0] * a + [1] * b, np.uint8)
    note(f"K_{a},{b}")
    gg, rr, _ = gpu_count(rp, ci, ty, 2)
    want_rows, want_glob = oracle.count_all(rp, ci, ty, 2, nthreads=8)
    assert_same(rr, gg, want_rows, want_glob, f"K{a},{b}")
    assert gg[oracle.key(2, 4, [0, 0, 1, 1])] == math.comb(a, 2) * math.comb(b, 2)


def test_cycles_and_l1():
    for n in (4, 5, 9):
        rp, ci = cycle(n)
        ty = np.zeros(n, np.uint8)
        rb, _, gb = oracle.brute(rp, ci, ty, 1)
        gg, rr, _ = gpu_count(rp, ci, ty, 1)
        assert_same(rr, gg, rb, gb, f"C{n}")


@pytest.mark.parametrize("L", [8, 16])
def test_many_types(L):
    # dense random graph with all types present; L = 16 also exercises global
    # accumulation outside LDS
    rp, ci = graphgen.gnp(60, 0.4, 9)
    ty = (np.arange(60) % L).astype(np.uint8)
    want_rows, want_glob = oracle.count_all(rp, ci, ty, L, nthreads=8)
    gg, rr, _ = gpu_count(rp, ci, ty, L)
    assert_same(rr, gg, want_rows, want_glob, f"gnp60/L{L}")


def test_empty_and_edgeless_graphs():
    rp = np.zeros(1, np.int32)
    gg, rr, _ = gpu_count(rp, np.zeros(0, np.int32), np.zeros(0, np.uint8), 3)
    assert (gg == 0).all() and rr.shape == (0, 42)
    rp = np.zeros(6, np.int32)
    gg, rr, _ = gpu_count(rp, np.zeros(0, np.int32), np.zeros(5, np.uint8), 2, validate=True)
    assert (gg == 0).all() and rr.shape == (0, 22)


@pytest.mark.parametrize("case,status", [
    ("unsorted", "TG_ERR_INVALID_GRAPH"), ("asymmetric", "TG_ERR_INVALID_GRAPH"),
    ("selfloop", "TG_ERR_INVALID_GRAPH"), ("duplicate", "TG_ERR_INVALID_GRAPH"),
    ("range", "TG_ERR_INVALID_GRAPH"), ("rowptr", "TG_ERR_INVALID_GRAPH"), ("type", "TG_ERR_TYPE_RANGE"),
])
def test_validation_reports_bad_graphs(case, status):
    import paper_1901_10026_amd as tg
    rp, ci = csr_from_edges(5, [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4)])
    rp, ci = rp.copy(), ci.copy()
    ty = np.zeros(5, np.uint8)
    if case == "unsorted":
        ci[rp[2]], ci[rp[2] + 1] = ci[rp[2] + 1], ci[rp[2]]
    elif case == "asymmetric":
        ci[rp[3]:rp[4]] = [1, 2]   # row 3 was [2, 4]: adds 3->1 without 1->3, drops 3->4
    elif case == "selfloop":
        ci[rp[4]] = 4
    elif case == "duplicate":
        ci[rp[2] + 1] = ci[rp[2]]
    elif case == "range":
        ci[rp[4]] = 9
    elif case == "rowptr":
        rp[2] = rp[3] + 1
    elif case == "type":
        ty[3] = 7
    with pytest.raises(tg.TGError) as e:
        gpu_count(rp, ci, ty, 2, validate=True)
    assert e.value.name == status, str(e.value)


def test_clique_pass_tiers_on_a_dense_graph():
    """G(450, 0.75), L = 8: the lowest nodes have up to ~330 higher
    neighbours; every clique-pass tier (wavefront, workgroup LDS rows, global
    rows by LDS limit) and the out-list probes give the oracle's rows."""
    import paper_1901_10026_amd as tg
    rp, ci = graphgen.gnp(450, 0.75, 31)
    ty = graphgen.types_uniform(450, 8, 31)
    ei, ej = oracle.canonical_edges(rp, ci)
    sample = np.linspace(0, len(ei) - 1, 60).astype(np.int64)
    want_rows, _ = oracle.count_edges(rp, ci, ty, 8, ei[sample], ej[sample], nthreads=8)
    base_g, base_r, _ = gpu_count(rp, ci, ty, 8)
    assert np.array_equal(base_r[sample], want_rows)
    for d in ({"clique_pass": 0}, {"clique_pass_lds_kib": 0}, {"clique_pass_lds_kib": 16, "clique_pass_grid": 3}):
        gg, rr, _ = gpu_count(rp, ci, ty, 8, tuning=tg.Tuning.from_dict(d))
        note(f"G(450, 0.75) with {d}")
        assert np.array_equal(gg, base_g) and np.array_equal(rr, base_r), d


def edge_list(rp, ci, shift=0):
    src = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    keep = src < ci
    return list(zip((src[keep] + shift).tolist(), (ci[keep] + shift).tolist()))


def with_hub(n, edges, leaves=66000, links=10):
    """The graph on nodes 0..n-1 and one more node (id n) joined to nodes
    0..links-1 and to `leaves` new leaves: its degree passes 65535."""
    edges = edges + [(v, n) for v in range(links)] + [(n, n + 1 + v) for v in range(leaves)]
    return csr_from_edges(n + 1 + leaves, edges)


def gnp_with_hub(leaves=66000, links=10):
    """G(450, 0.75) with a hub (id 450) whose wedge work stays below that of
    the densest G(450, 0.75) nodes."""
    rp, ci = graphgen.gnp(450, 0.75, 31)
    return with_hub(450, edge_list(rp, ci), leaves, links)


@pytest.mark.parametrize("which,L,lds_kib", [("cl-2k", 3, 4), ("gnp", 5, 4), ("gnp", 8, 5), ("kab", 2, 4),
                                             ("hub", 5, 4)])
def test_cycle_parts_match_the_grouped_pass(which, L, lds_kib):
    """Middle counts of the dense 4-cycle groups from records bucketed by
    far-end id range and summed in LDS (every heavy node dense, tables small
    enough for several ranges, small walk items) or from global atomics: the
    same rows, and the oracle's on a sample.  With a node of degree 65536 or
    more, only the groups whose nodes all have smaller degrees take the
    bucketed pass (16-bit rows inside 32-bit row space), before and after a
    group of 32-bit rows."""
    import paper_1901_10026_amd as tg
    if which == "hub":
        rp, ci = gnp_with_hub()
        ty = graphgen.types_uniform(len(rp) - 1, L, 31)
        assert np.diff(rp).max() >= 65536
    elif which == "cl-2k":
        g = graphgen.chung_lu_small()
        rp, ci = g.row_ptr, g.col_idx
        ty = graphgen.types_uniform(g.n, L, 5)
    elif which == "gnp":
        rp, ci = graphgen.gnp(450, 0.75, 31)
        ty = graphgen.types_uniform(450, L, 31)
    else:
        rp, ci = complete_bipartite(40, 260)
        ty = (np.arange(300) % L).astype(np.uint8)
    note(f"cycle parts: {which} L={L}")
    ei, ej = oracle.canonical_edges(rp, ci)
    sample = np.linspace(0, len(ei) - 1, 50).astype(np.int64)
    if which == "hub":  # the hub's edges into G(450, 0.75) too
        sample = np.union1d(sample, np.nonzero((ej == 450) & (ei < 450))[0])
    want_rows, _ = oracle.count_edges(rp, ci, ty, L, ei[sample], ej[sample], nthreads=8)
    base_g, base_r, _ = gpu_count(rp, ci, ty, L, tuning=tg.Tuning.from_dict({"c4_parts": 0}))
    assert np.array_equal(base_r[sample], want_rows)
    for d in ({}, {"c4_part_hash_ratio": 0}, {"c4_part_hash_ratio": 0, "c4_part_lds_kib": lds_kib},
              {"c4_part_hash_ratio": 0, "c4_part_lds_kib": lds_kib, "c4_part_chunk": 256},
              {"c4_part_hash_ratio": 0, "c4_slices": 8}):
        gg, rr, _ = gpu_count(rp, ci, ty, L, tuning=tg.Tuning.from_dict(d))
        assert np.array_equal(gg, base_g) and np.array_equal(rr, base_r), d


def test_split_cycle_counters():
    """A graph with a node of degree 66010, so that a 4-cycle count may need
    64 bits: per-slot rows of 32-bit counters, with every edge (a, b) of
    (d_a - 1)(d_b - 1) >= 2^k counted in its 64-bit per-edge counters instead
    (k = 32: none of them; 10 and 1: most edges away from the leaves), give
    the rows of 64-bit slot rows, and so do 64-bit per-edge counters alone
    (split off); also with one node per group and every heavy node dense."""
    import paper_1901_10026_amd as tg
    # G(450, 0.75) (dense groups) and the Chung-Lu graph on 2000 nodes (every
    # node tier) side by side, then the hub
    rg, cg = graphgen.gnp(450, 0.75, 31)
    c = graphgen.chung_lu_small()
    rp, ci = with_hub(450 + c.n, edge_list(rg, cg) + edge_list(c.row_ptr, c.col_idx, shift=450))
    hub = 450 + c.n
    L = 5
    ty = graphgen.types_uniform(len(rp) - 1, L, 31)
    ei, ej = oracle.canonical_edges(rp, ci)
    sample = np.union1d(np.linspace(0, len(ei) - 1, 60).astype(np.int64), np.nonzero((ej == hub) & (ei < hub))[0])
    want_rows, _ = oracle.count_edges(rp, ci, ty, L, ei[sample], ej[sample], nthreads=8)
    base_g, base_r, _ = gpu_count(rp, ci, ty, L)
    assert np.array_equal(base_r[sample], want_rows)
    for k in (32, 10, 1, 0):
        for extra in ({}, {"c4_group_kwedges": 1, "c4_hash_ratio": 0, "c4_part_hash_ratio": 0}):
            d = dict({"c4_slot_budget_mb": 0, "c4_split_log2": k}, **extra)
            note(f"split counters {d}")
            gg, rr, _ = gpu_count(rp, ci, ty, L, tuning=tg.Tuning.from_dict(d))
            assert np.array_equal(gg, base_g) and np.array_equal(rr, base_r), d


def test_release_scratch_between_calls():
    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    g1, r1, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L)
    tg.release_scratch()
    tg.release_scratch()  # nothing held: still fine
    g2, r2, _ = gpu_count(g.row_ptr, g.col_idx, g.types, g.L)
    assert np.array_equal(g1, g2) and np.array_equal(r1, r2)
