"""Skewed giant graph (Chung-Lu, 20M nodes, L=8 Zipf types).  Its per-edge
rows do not fit in memory, so the call counts rows only for an edge sample
(global_counts=False): the 4-cycle pass covers the whole graph, the
per-edge step only the sample, and every sampled row must equal the
oracle's.  The sample is stratified by degree product and also holds the
heaviest edges of the graph (the largest d_i * d_j): hub-hub edges with the
longest common-neighbour sets, which take the workgroup teams and the
global-scratch path of T_ij."""
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
    note("cl-20m: counting the sampled rows (the 4-cycle pass covers the whole graph)")
    ph = {}
    glob, rows, ends = tg.count(rp, ci, ty, g.L, per_edge=True, edge_ids=dev_ids, global_counts=False,
                                endpoints=True, phase_ms=ph)
    torch.cuda.synchronize()
    note("tg_count done: " + " ".join(f"{k}={v:.0f}ms" for k, v in ph.items()))
    assert glob is None
    del rp, ci, ty
    ends = ends.cpu().numpy()
    assert np.array_equal(ends[:, 0], ei[ids]) and np.array_equal(ends[:, 1], ej[ids])
    got = rows.cpu().numpy().view(np.uint64)
    note("cl-20m: oracle on the sampled edges")
    want, _ = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei[ids], ej[ids], nthreads=16)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} of {len(ids)} sampled rows differ, first edge {ids[bad[0]]}"
    note(f"{len(ids)} sampled rows match the oracle")
