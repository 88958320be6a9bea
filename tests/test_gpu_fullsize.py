"""Full-size parity at the benchmark's workload (Chung-Lu, 1M nodes, ~9.8M
edges, L=5) in the benchmark's launch configuration: sampled per-edge rows
against the oracle, plus properties that hold at any size."""
import numpy as np
import pytest

import graphgen
import oracle
from _gpu import note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_1m()
    note(f"cl-1m n={g.n} m={g.m} L={g.L}")
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    glob, rows, _ = tg.count(rp, ci, ty, g.L, per_edge=True, schedule="degree")
    torch.cuda.synchronize()
    return g, rp, ci, ty, glob, rows


def stratified_sample(g, per_decile=12, heaviest=8, seed=7):
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    d = np.diff(g.row_ptr).astype(np.int64)
    cost = d[ei] * d[ej]
    order = np.argsort(cost, kind="stable")
    rng = np.random.default_rng(seed)
    picks = []
    for part in np.array_split(order, 10):
        picks.extend(rng.choice(part, size=per_decile, replace=False))
    picks.extend(order[-heaviest:])
    return np.unique(np.array(picks, dtype=np.int64)), ei, ej


def test_sampled_rows_match_oracle(big):
    g, _, _, _, _, rows = big
    idx, ei, ej = stratified_sample(g)
    note(f"oracle on {len(idx)} sampled edges")
    want, _ = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei[idx], ej[idx], nthreads=16)
    import torch
    got = rows.index_select(0, torch.from_numpy(idx).to(rows.device)).cpu().numpy().view(np.uint64)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} sampled edges differ: {idx[bad][:5]}"


def test_global_equals_row_sums(big):
    import torch

    import paper_1901_10026_amd as tg
    g, _, _, ty, glob, rows = big
    L = g.L
    R = tg.edge_row_width(L)
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    pair = torch.from_numpy((g.types[ei].astype(np.int64) * L + g.types[ej]).astype(np.int64)).to(rows.device)
    r64 = rows.view(torch.int64)
    acc = np.zeros(tg.num_keys(L), dtype=object)
    for c in range(L * L):
        sel = (pair == c).nonzero().flatten()
        if sel.numel() == 0:
            continue
        colsum = r64.index_select(0, sel).sum(0).cpu().numpy()
        a, b = divmod(c, L)
        for col in range(R):
            acc[tg.edge_row_key(L, a, b, col)] += int(colsum[col])
    gl = glob.cpu().numpy().view(np.uint64)
    div = [2, 3, 3, 3, 4, 4, 5, 6]
    for k in range(len(acc)):
        shape = tg.key_decode(L, k)[0]
        assert acc[k] % div[shape] == 0
        assert acc[k] // div[shape] == int(gl[k]), f"key {k}"


def test_typed_counts_partition_untyped_counts(big):
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, glob, _ = big
    zeros = torch.zeros_like(ty)
    g1, _, _ = tg.count(rp, ci, zeros, 1, per_edge=False, schedule="none")
    torch.cuda.synchronize()
    g1 = g1.cpu().numpy().view(np.uint64)
    gl = glob.cpu().numpy().view(np.uint64)
    per_shape = np.zeros(8, dtype=object)
    for k in range(len(gl)):
        per_shape[tg.key_decode(g.L, k)[0]] += int(gl[k])
    assert [int(x) for x in per_shape] == [int(x) for x in g1]


def test_schedules_agree_at_full_size(big):
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, glob, rows = big
    g2, r2, _ = tg.count(rp, ci, ty, g.L, per_edge=True, schedule="none")
    torch.cuda.synchronize()
    assert torch.equal(g2.view(torch.int64), glob.view(torch.int64))
    assert torch.equal(r2.view(torch.int64), rows.view(torch.int64))


def test_launch_shapes_agree_at_full_size(big):
    """Hash tables for the lighter heavy nodes, small node groups and wedge
    chunks, other team thresholds, T_ij by row intersection instead of the
    kept lists, every heavy node in the grouped 4-cycle pass (no id-range
    parts): the same counts."""
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, glob, rows = big
    t = tg.Tuning.from_dict({"c4_hash_ratio": 4, "c4_footprint_mb": 32, "c4_group_kwedges": 512,
                             "c4_chunk": 256, "light_max_degree": 64, "heavy_min_degree": 1024,
                             "combine_grid": 1024, "wg_grid": 300, "c4_slot_budget_mb": 0, "c4_slices": 8,
                             "tlist_budget_mib": 0, "c4_parts": 0})
    g2, r2, _ = tg.count(rp, ci, ty, g.L, per_edge=True, tuning=t)
    torch.cuda.synchronize()
    assert torch.equal(g2.view(torch.int64), glob.view(torch.int64))
    assert torch.equal(r2.view(torch.int64), rows.view(torch.int64))


def test_cycle_parts_at_full_size(big):
    """Middle counts of every heavy node from range-bucketed records summed in
    LDS (all of them in dense groups), the credit walk split into far-end
    slices, small tables (more ranges) and small walk items: the same counts
    as the default."""
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, glob, rows = big
    for d in ({"c4_part_hash_ratio": 0}, {"c4_slices": 8},
              {"c4_part_hash_ratio": 0, "c4_part_lds_kib": 64, "c4_part_chunk": 512}):
        note(f"cl-1m with {d}")
        g2, r2, _ = tg.count(rp, ci, ty, g.L, per_edge=True, tuning=tg.Tuning.from_dict(d))
        torch.cuda.synchronize()
        assert torch.equal(g2.view(torch.int64), glob.view(torch.int64)), d
        assert torch.equal(r2.view(torch.int64), rows.view(torch.int64)), d


def test_clique_pass_equals_out_list_probes_at_full_size(big):
    """4-cliques from the whole-graph pass (each clique once from its lowest
    node, the default) and from the per-edge out-list probes of the gather:
    the same rows; the pass also with few workgroups for its global-scratch
    tier."""
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, glob, rows = big
    for d in ({"clique_pass": 0}, {"clique_pass": 1, "clique_pass_grid": 7},
              {"clique_pass_lds_kib": 0, "clique_pass_grid": 300}, {"clique_pass_lds_kib": 40}):
        g2, r2, _ = tg.count(rp, ci, ty, g.L, per_edge=True, tuning=tg.Tuning.from_dict(d))
        torch.cuda.synchronize()
        note(f"tuning {d}: same rows")
        assert torch.equal(g2.view(torch.int64), glob.view(torch.int64)), d
        assert torch.equal(r2.view(torch.int64), rows.view(torch.int64)), d
