"""Bipartite and 3-partite workloads at full size: sampled rows against the
oracle, and the structural zeros that the part structure forces."""
import itertools

import numpy as np
import pytest

import graphgen
import oracle
from _gpu import note, to_dev

pytestmark = pytest.mark.gpu

SHAPE_EDGES = {
    0: [(0, 1), (1, 2)],
    1: [(0, 1), (1, 2), (0, 2)],
    2: [(0, 1), (1, 2), (2, 3)],
    3: [(0, 1), (0, 2), (0, 3)],
    4: [(0, 1), (1, 2), (2, 3), (3, 0)],
    5: [(0, 1), (1, 2), (0, 2), (2, 3)],
    6: [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)],
    7: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
}


def colourable(shape, types):
    """Some placement of the type multiset on the shape's nodes gives every
    edge two different types."""
    for perm in set(itertools.permutations(types)):
        if all(perm[a] != perm[b] for a, b in SHAPE_EDGES[shape]):
            return True
    return False


def run(name):
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.workload(name)
    note(f"{name} n={g.n} m={g.m} L={g.L}")
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    glob, rows, _ = tg.count(rp, ci, ty, g.L)
    # global counts counted once per instance agree at full size
    once = tg.count_global(rp, ci, ty, g.L)
    torch.cuda.synchronize()
    assert torch.equal(once.view(torch.int64), glob.view(torch.int64))
    return g, glob, rows


def check_sample(g, rows, n_per_decile=8, heaviest=6):
    import torch
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    d = np.diff(g.row_ptr).astype(np.int64)
    order = np.argsort(d[ei] * d[ej], kind="stable")
    rng = np.random.default_rng(17)
    picks = [rng.choice(part, n_per_decile, replace=False) for part in np.array_split(order, 10)]
    idx = np.unique(np.concatenate(picks + [order[-heaviest:]]))
    want, _ = oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, ei[idx], ej[idx], nthreads=16)
    got = rows.index_select(0, torch.from_numpy(idx).to(rows.device)).cpu().numpy().view(np.uint64)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} sampled edges differ"


def check_zeros(g, glob, rows):
    import torch

    import paper_1901_10026_amd as tg
    gl = glob.cpu().numpy().view(np.uint64)
    nonzero_colourable = 0
    for k in range(len(gl)):
        shape, types = tg.key_decode(g.L, k)
        if not colourable(shape, types):
            assert gl[k] == 0, (shape, types)
        elif gl[k]:
            nonzero_colourable += 1
    assert nonzero_colourable > 0
    L = g.L
    R = tg.edge_row_width(L)
    r64 = rows.view(torch.int64)
    # rows of edges (i, j): types differ (edges join different parts), so a
    # column is forced to zero when its key is not colourable for (phi_i, phi_j)
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    pair = torch.from_numpy((g.types[ei].astype(np.int64) * L + g.types[ej]).astype(np.int64)).to(rows.device)
    for a in range(L):
        for b in range(L):
            if a == b:
                continue
            sel = (pair == a * L + b).nonzero().flatten()
            if sel.numel() == 0:
                continue
            cols = [c for c in range(R) if not colourable(*tg.key_decode(L, tg.edge_row_key(L, a, b, c)))]
            if cols:
                sub = r64.index_select(0, sel).index_select(1, torch.tensor(cols, device=rows.device))
                assert int(sub.abs().max()) == 0, (a, b)


def test_bipartite_50m():
    g, glob, rows = run("bip-50m")
    assert (np.diff(g.row_ptr) > 0).any()
    check_zeros(g, glob, rows)
    # no triangle-containing graphlet at all
    import paper_1901_10026_amd as tg
    gl = glob.cpu().numpy().view(np.uint64)
    for k in range(len(gl)):
        if tg.key_decode(g.L, k)[0] in (1, 5, 6, 7):
            assert gl[k] == 0
    check_sample(g, rows)


def test_tripartite_30m():
    import paper_1901_10026_amd as tg
    g, glob, rows = run("tri-30m")
    check_zeros(g, glob, rows)
    gl = glob.cpu().numpy().view(np.uint64)
    for k in range(len(gl)):
        shape, types = tg.key_decode(g.L, k)
        if shape == 7:
            assert gl[k] == 0                      # no 4-clique on 3 parts
        if shape == 1 and gl[k]:
            assert sorted(types) == [0, 1, 2]     # triangles use one node of each part
    assert gl[tg.key_encode(3, 1, [0, 1, 2])] > 0
    check_sample(g, rows)
