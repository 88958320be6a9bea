"""Global counts with every instance counted a fixed number of times
(tg_count_global) against the oracle's global counts (Eq. 17 over its
per-edge rows, or brute force), and against tg_count at full size."""
import numpy as np
import pytest

import graphgen
import oracle
from _gpu import note, to_dev
from _graphs import all_graphs, complete, complete_bipartite, cycle, star

pytestmark = pytest.mark.gpu


def gpu_global(row_ptr, col_idx, types, L, **kw):
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, ty = to_dev(row_ptr, col_idx, types)
    g = tg.count_global(rp, ci, ty, L, **kw)
    torch.cuda.synchronize()
    return g.cpu().numpy().view(np.uint64)


def test_tiny_graphs_match_brute_force():
    for idx in range(200):
        g = graphgen.tiny_graph(idx)
        _, _, want = oracle.brute(g.row_ptr, g.col_idx, g.types, g.L)
        got = gpu_global(g.row_ptr, g.col_idx, g.types, g.L, validate=True)
        assert np.array_equal(got, want), f"tiny{idx} n={g.n} m={g.m} L={g.L}"


def test_every_graph_on_five_nodes():
    ty = np.array([0, 1, 0, 1, 2], np.uint8)
    for q, (rp, ci) in enumerate(all_graphs(5)):
        _, _, want = oracle.brute(rp, ci, ty, 3)
        assert np.array_equal(gpu_global(rp, ci, ty, 3), want), f"5-node graph {q}"


def test_chung_lu_2k():
    g = graphgen.chung_lu_small()
    _, want = oracle.count_all(g.row_ptr, g.col_idx, g.types, g.L, per_edge=False, nthreads=8)
    assert np.array_equal(gpu_global(g.row_ptr, g.col_idx, g.types, g.L), want)


def test_special_graphs():
    cases = [("K7", complete(7), 3), ("K5,6", complete_bipartite(5, 6), 2), ("star9", star(9), 2),
             ("C6", cycle(6), 1)]
    for name, (rp, ci), L in cases:
        n = len(rp) - 1
        ty = (np.arange(n) % L).astype(np.uint8)
        _, _, want = oracle.brute(rp, ci, ty, L)
        assert np.array_equal(gpu_global(rp, ci, ty, L), want), name


@pytest.mark.parametrize("L", [1, 8, 16])
def test_many_types(L):
    # dense random graph: every 4-clique class and (L = 16) key sums outside LDS
    rp, ci = graphgen.gnp(60, 0.4, 9)
    ty = (np.arange(60) % L).astype(np.uint8)
    _, want = oracle.count_all(rp, ci, ty, L, per_edge=False, nthreads=8)
    assert np.array_equal(gpu_global(rp, ci, ty, L), want)


# the per-edge-class 4-clique kernels (no clique pass) with tiny class limits
SMALL_CLASSES = {"clique_pass": 0, "clique_team_max": 2, "clique_wave_max": 6, "clique_lds_ids": 3}


def test_clique_launch_classes_and_overflow():
    """Tiny class limits send most edges through the wavefront and workgroup
    4-clique kernels and most workgroup edges' common neighbours to global
    scratch: still the oracle's counts."""
    import paper_1901_10026_amd as tg
    t = tg.Tuning.from_dict(SMALL_CLASSES)
    g = graphgen.chung_lu_small()
    _, want = oracle.count_all(g.row_ptr, g.col_idx, g.types, g.L, per_edge=False, nthreads=8)
    assert np.array_equal(gpu_global(g.row_ptr, g.col_idx, g.types, g.L, tuning=t), want)
    rp, ci = graphgen.gnp(60, 0.4, 9)
    ty = (np.arange(60) % 8).astype(np.uint8)
    _, want = oracle.count_all(rp, ci, ty, 8, per_edge=False, nthreads=8)
    assert np.array_equal(gpu_global(rp, ci, ty, 8, tuning=t), want)


def test_complete_graph_closed_form():
    """K_n: every 3-set is a triangle and every 4-set a 4-clique, so the
    counts are products of binomials of the type class sizes."""
    import itertools
    import math

    import paper_1901_10026_amd as tg
    n, L = 90, 3
    rp, ci = complete(n)
    ty = (np.arange(n) % L).astype(np.uint8)
    sizes = np.bincount(ty, minlength=L)
    want = np.zeros(oracle.num_keys(L), np.uint64)
    for k, shape in ((3, 1), (4, 7)):
        for ms in itertools.combinations_with_replacement(range(L), k):
            c = 1
            for t in set(ms):
                c *= math.comb(int(sizes[t]), ms.count(t))
            want[oracle.key(L, shape, list(ms))] = c
    for tun in (None, tg.Tuning.from_dict(SMALL_CLASSES)):
        assert np.array_equal(gpu_global(rp, ci, ty, L, tuning=tun), want)
    # K_400: the lowest node has 399 higher neighbours (global-scratch rows)
    n = 400
    rp, ci = complete(n)
    ty = (np.arange(n) % L).astype(np.uint8)
    got = gpu_global(rp, ci, ty, L)
    sizes = np.bincount(ty, minlength=L)
    for ms in itertools.combinations_with_replacement(range(L), 4):
        c = 1
        for t in set(ms):
            c *= math.comb(int(sizes[t]), ms.count(t))
        assert got[oracle.key(L, 7, list(ms))] == c


def test_empty_and_edgeless_graphs():
    got = gpu_global(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8), 3)
    assert got.shape == (oracle.num_keys(3),) and (got == 0).all()
    got = gpu_global(np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(5, np.uint8), 2, validate=True)
    assert (got == 0).all()


def test_full_size_equals_per_edge_path():
    """cl-1m (1M nodes, 9.8M edges, L=5): the same global vector as tg_count,
    also under other 4-cycle launch shapes."""
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_1m()
    note(f"cl-1m n={g.n} m={g.m} L={g.L}")
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    want, _, _ = tg.count(rp, ci, ty, g.L, per_edge=False)
    ph = {}
    got = tg.count_global(rp, ci, ty, g.L, phase_ms=ph)
    torch.cuda.synchronize()
    note("count_global: " + " ".join(f"{k}={v:.1f}ms" for k, v in ph.items()))
    assert torch.equal(got.view(torch.int64), want.view(torch.int64))
    t = tg.Tuning.from_dict({"c4_hash_ratio": 0, "c4_footprint_mb": 32, "c4_group_kwedges": 512,
                             "c4_chunk": 128})
    got2 = tg.count_global(rp, ci, ty, g.L, tuning=t)
    torch.cuda.synchronize()
    assert torch.equal(got2.view(torch.int64), want.view(torch.int64))
    # 4-cliques from the edge classes instead of the clique pass, and the
    # pass with few workgroups for its global-scratch tier
    for d in ({"clique_pass": 0}, {"clique_pass_grid": 5}, {"clique_pass_lds_kib": 0, "clique_pass_grid": 200}):
        got3 = tg.count_global(rp, ci, ty, g.L, tuning=tg.Tuning.from_dict(d))
        torch.cuda.synchronize()
        assert torch.equal(got3.view(torch.int64), want.view(torch.int64)), d
