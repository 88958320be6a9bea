"""Skewed giant graph (Chung-Lu, 20M nodes, L=8 Zipf types).  Its dense
per-edge rows do not fit in memory; the call takes the sparse per-edge
output (nonzero (key, count) pairs straight from the row kernel) of an edge
sample only (global_counts=False): the 4-cycle and clique passes cover the
whole graph, the per-edge step only the sample, and every sampled edge's
pairs must be the oracle row's nonzero entries.  The sample is stratified
by degree product and also holds the heaviest edges of the graph (the
largest d_i * d_j): hub-hub edges with the longest common-neighbour sets,
which take the workgroup teams."""
import numpy as np
import pytest

import graphgen
import oracle
from _gpu import note, to_dev

pytestmark = pytest.mark.gpu


def sample_edges(d, s, ei, ej, per_decile=6, heaviest=3, budget=4e8, top=20, top_budget=1.2e9, seed=11):
    """Stratified by degree-product decile, uniform within each decile among
    edges whose oracle cost (s_i + s_j element visits) fits the budget, plus
    the heaviest such edges, plus the `top` edges of largest d_i * d_j whose
    cost fits top_budget."""
    cost = d[ei] * d[ej]
    ocost = s[ei] + s[ej]
    order = np.argsort(cost, kind="stable")
    rng = np.random.default_rng(seed)
    picks = []
    for part in np.array_split(order, 10):
        ok = part[ocost[part] <= budget]
        picks.extend(rng.choice(ok, size=min(per_decile, len(ok)), replace=False))
    ok = order[ocost[order] <= budget]
    picks.extend(ok[-heaviest:])
    ok = order[ocost[order] <= top_budget]
    picks.extend(ok[-top:])
    return np.unique(np.array(picks, dtype=np.int64))


def test_giant_sampled_rows():
    import torch

    import paper_1901_10026_amd as tg
    note("cl-20m: generating")
    g = graphgen.workload("cl-20m")
    d = np.diff(g.row_ptr).astype(np.int64)
    note(f"cl-20m n={g.n} m={g.m} L={g.L} max_deg={d.max()}")
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    note("cl-20m: canonical edges listed")
    cs = np.concatenate([[0], np.cumsum(d[g.col_idx])])
    s = cs[g.row_ptr[1:]] - cs[g.row_ptr[:-1]]  # neighbour degree sums
    del cs
    ids = sample_edges(d, s, ei, ej)
    prod = d[ei[ids]] * d[ej[ids]]
    note(f"sampled {len(ids)} edges, largest d_i*d_j {prod.max():.3e} (graph: {(d[ei] * d[ej]).max():.3e}), "
         f"largest oracle cost {(s[ei[ids]] + s[ej[ids]]).max():.3e}")
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    dev_ids = torch.from_numpy(ids).to(rp.device)
    note("cl-20m: counting the sampled edges, sparse output only (the 4-cycle and clique passes cover the "
         "whole graph)")
    ph = {}
    glob, keys, counts, start, length = tg.count_sparse(rp, ci, ty, g.L, edge_ids=dev_ids, global_counts=False,
                                                        phase_ms=ph)
    torch.cuda.synchronize()
    note("tg_count_sparse done: " + " ".join(f"{k}={v:.0f}ms" for k, v in ph.items()))
    assert glob is None
    del rp, ci, ty
    keys = keys.cpu().numpy().view(np.uint32)
    counts = counts.cpu().numpy().view(np.uint64)
    start, length = start.cpu().numpy(), length.cpu().numpy()
    note("cl-20m: oracle on the sampled edges")
    want, _ = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei[ids], ej[ids], nthreads=16)
    bad = []
    for q in range(len(ids)):
        a, b = int(g.types[ei[ids[q]]]), int(g.types[ej[ids[q]]])
        cols = np.nonzero(want[q])[0]
        exp = [(oracle.row_key(g.L, a, b, int(c)), int(want[q, c])) for c in cols]
        s0, n0 = int(start[q]), int(length[q])
        got = list(zip(keys[s0:s0 + n0].astype(int).tolist(), counts[s0:s0 + n0].astype(int).tolist()))
        if got != exp:
            bad.append(q)
    assert not bad, f"{len(bad)} of {len(ids)} sampled edges differ, first edge {ids[bad[0]]}"
    note(f"{len(ids)} sampled edges' sparse pairs match the oracle's nonzero row entries")


def test_small_call_after_the_giant_one():
    """The call after a 20M-node one: growing the workspace to that call's
    size does not fit next to what the pool caches; the call allocates piece
    by piece instead and is exact."""
    import paper_1901_10026_amd as tg
    g = graphgen.tiny_graph(7)
    rb, _, gb = oracle.brute(g.row_ptr, g.col_idx, g.types, g.L)
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    glob, rows, _ = tg.count(rp, ci, ty, g.L)
    assert np.array_equal(glob.cpu().numpy().view(np.uint64), gb)
    assert np.array_equal(rows.cpu().numpy().view(np.uint64), rb)
    tg.release_scratch()
