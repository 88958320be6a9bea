"""Per-edge orbit output (Table 3's g1..g12 per type or type pair) and the
sparse per-edge format (nonzero (key, count) pairs per edge), against the
oracle."""
import numpy as np
import pytest

import graphgen
import oracle
from _gpu import note, to_dev
from _graphs import all_graphs

pytestmark = pytest.mark.gpu


def gpu_orbits(g_rp, g_ci, g_ty, L, **kw):
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, ty = to_dev(g_rp, g_ci, g_ty)
    m = len(g_ci) // 2
    E = kw["edge_ids"].numel() if "edge_ids" in kw else m
    orb = torch.empty((E, tg.edge_orbit_width(L)), dtype=torch.uint64, device=rp.device)
    glob, rows, ends = tg.count(rp, ci, ty, L, out_orbits=orb, endpoints=True, **kw)
    torch.cuda.synchronize()
    as_np = lambda t: t.cpu().numpy().view(np.uint64) if t is not None else None
    return as_np(glob), as_np(rows), as_np(orb), ends.cpu().numpy()


def test_orbit_rows_match_oracle_on_chung_lu_2k():
    g = graphgen.chung_lu_small()
    _, rows, orb, ends = gpu_orbits(g.row_ptr, g.col_idx, g.types, g.L)
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    want_rows, want_orb = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei, ej, orbits=True, nthreads=8)
    assert np.array_equal(rows, want_rows)
    assert np.array_equal(orb, want_orb)


def test_orbit_rows_match_brute_force_on_tiny_graphs():
    for idx in range(0, 200, 7):
        g = graphgen.tiny_graph(idx)
        if len(g.col_idx) == 0:
            continue
        _, rows, orb, _ = gpu_orbits(g.row_ptr, g.col_idx, g.types, g.L)
        want_rows, want_orb, _ = oracle.brute(g.row_ptr, g.col_idx, g.types, g.L, orbits=True)
        assert np.array_equal(rows, want_rows), idx
        assert np.array_equal(orb, want_orb), idx


def test_orbits_for_sampled_edges_and_rows_only():
    import torch
    g = graphgen.chung_lu_small()
    _, rows, orb, _ = gpu_orbits(g.row_ptr, g.col_idx, g.types, g.L)
    ids = np.arange(5, g.m, 41, dtype=np.int64)
    dev_ids = torch.from_numpy(ids).to("cuda:0")
    glob2, rows2, orb2, _ = gpu_orbits(g.row_ptr, g.col_idx, g.types, g.L, edge_ids=dev_ids, global_counts=False)
    assert glob2 is None
    assert np.array_equal(rows2, rows[ids]) and np.array_equal(orb2, orb[ids])


def test_sparse_rows_are_the_nonzero_entries():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    glob, rows, ends = tg.count(rp, ci, ty, g.L, endpoints=True)
    off, keys, cnts = tg.rows_sparse(rows, ends, ty, g.L)
    torch.cuda.synchronize()
    off, keys = off.cpu().numpy(), keys.cpu().numpy().view(np.uint32)
    cnts, dense = cnts.cpu().numpy().view(np.uint64), rows.cpu().numpy().view(np.uint64)
    ends = ends.cpu().numpy()
    assert off[0] == 0 and off[-1] == len(keys) == int((dense != 0).sum())
    R = dense.shape[1]
    for e in range(0, g.m, 3):
        a, b = g.types[ends[e, 0]], g.types[ends[e, 1]]
        cols = np.nonzero(dense[e])[0]
        want = sorted((oracle.row_key(g.L, int(a), int(b), int(c)), int(dense[e, c])) for c in cols)
        got = sorted(zip(keys[off[e]:off[e + 1]].tolist(), cnts[off[e]:off[e + 1]].tolist()))
        assert got == want, e
    # summing the pairs by key gives the global counts times each shape's edge count
    shape_edges = [2, 3, 3, 3, 4, 4, 5, 6]
    sums = np.zeros(len(glob), dtype=np.uint64)
    np.add.at(sums, keys.astype(np.int64), cnts)
    gl = glob.cpu().numpy().view(np.uint64)
    for k in range(len(gl)):
        assert int(sums[k]) == int(gl[k]) * shape_edges[tg.key_decode(g.L, k)[0]]
    note(f"cl-2k: {len(keys)} nonzero pairs over {g.m} edges (R={R}); "
         f"mean {len(keys) / g.m:.1f}, max {int(np.diff(off).max())} per edge")


def test_sparse_rows_of_the_five_node_census():
    import torch

    import paper_1901_10026_amd as tg
    for gi, (rp_np, ci_np) in enumerate(all_graphs(5)):
        if len(ci_np) == 0 or gi % 8:
            continue
        types = np.array([0, 1, 0, 2, 1], dtype=np.uint8)
        rp, ci, ty = to_dev(rp_np, ci_np, types)
        _, rows, ends = tg.count(rp, ci, ty, 3, endpoints=True)
        off, keys, cnts = tg.rows_sparse(rows, ends, ty, 3)
        torch.cuda.synchronize()
        dense = rows.cpu().numpy().view(np.uint64)
        assert int(off[-1]) == int((dense != 0).sum()), gi
        assert int(cnts.cpu().numpy().view(np.uint64).sum()) == int(dense.sum()), gi


def test_sparse_rows_of_an_edgeless_graph():
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, ty = to_dev(np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(3, np.uint8))
    _, rows, ends = tg.count(rp, ci, ty, 2, endpoints=True)
    off, keys, cnts = tg.rows_sparse(rows, ends, ty, 2)
    torch.cuda.synchronize()
    assert rows.shape == (0, tg.edge_row_width(2))
    assert off.cpu().tolist() == [0] and keys.numel() == 0 and cnts.numel() == 0


def _sparse_of_rows(rows, ei, ej, ty, L):
    """Per edge, the oracle row's nonzero entries as (global key, count) in
    column order."""
    out = []
    for q in range(len(rows)):
        cols = np.nonzero(rows[q])[0]
        out.append([(oracle.row_key(L, int(ty[ei[q]]), int(ty[ej[q]]), int(c)), int(rows[q, c])) for c in cols])
    return out


def _pairs(keys, counts, start, length):
    keys = keys.cpu().numpy().view(np.uint32)
    counts = counts.cpu().numpy().view(np.uint64)
    start, length = start.cpu().numpy(), length.cpu().numpy()
    return [list(zip(keys[s:s + n].astype(int).tolist(), counts[s:s + n].astype(int).tolist()))
            for s, n in zip(start, length)]


def test_sparse_output_straight_from_the_row_kernel():
    """tg_count_sparse on the 2000-node graph: every edge's pairs are the
    oracle row's nonzero entries (keys through the oracle's key map), the
    global counts equal tg_count's, and a range and an id list give the same
    pairs as the full call."""
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    glob, keys, counts, start, length = tg.count_sparse(rp, ci, ty, g.L)
    torch.cuda.synchronize()
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    want_rows, want_glob = oracle.count_all(g.row_ptr, g.col_idx, g.types, g.L, nthreads=8)
    want = _sparse_of_rows(want_rows, ei, ej, g.types, g.L)
    got = _pairs(keys, counts, start, length)
    assert got == want
    assert np.array_equal(glob.cpu().numpy().view(np.uint64), want_glob)
    s = start.cpu().numpy()
    ln = length.cpu().numpy()
    spans = sorted(zip(s.tolist(), (s + ln).tolist()))
    assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:])) and spans[-1][1] == keys.numel()
    g2, k2, c2, s2, l2 = tg.count_sparse(rp, ci, ty, g.L, edge_range=(500, 2500), global_counts=False)
    assert g2 is None and _pairs(k2, c2, s2, l2) == want[500:2500]
    ids = np.arange(7, g.m, 29, dtype=np.int64)
    _, k3, c3, s3, l3 = tg.count_sparse(rp, ci, ty, g.L, edge_ids=torch.from_numpy(ids).to(rp.device))
    assert _pairs(k3, c3, s3, l3) == [want[q] for q in ids]


def test_sparse_output_capacity_and_limits():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    _, keys, _, _, _ = tg.count_sparse(rp, ci, ty, g.L, edge_range=(0, 300))
    need = keys.numel()
    with pytest.raises(tg.TGError) as ex:
        tg.count_sparse(rp, ci, ty, g.L, edge_range=(0, 300), capacity=need - 1)
    assert ex.value.name == "TG_ERR_INVALID_ARG" and str(need) in str(ex.value)
    # pairs of different edges land in any order: compare them edge by edge
    _, k0, c0, s0, l0 = tg.count_sparse(rp, ci, ty, g.L, edge_range=(0, 300), capacity=need)
    _, k1, c1, s1, l1 = tg.count_sparse(rp, ci, ty, g.L, edge_range=(0, 300))
    assert k0.numel() == need and _pairs(k0, c0, s0, l0) == _pairs(k1, c1, s1, l1)
    rp2, ci2 = graphgen.gnp(30, 0.3, 5)
    with pytest.raises(tg.TGError) as ex:
        tg.count_sparse(*to_dev(rp2, ci2, np.zeros(30, np.uint8)), 9)
    assert ex.value.name == "TG_ERR_UNSUPPORTED_L"
