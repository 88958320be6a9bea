"""Parity of tg_count_directed4 (directed typed 4-node graphlets) with the
directed 4-node oracle: per-edge rows and global counts on tiny digraphs and
an oriented G(60, 0.3), and, on the oriented 2000-node Chung-Lu graph, the
direction-summed global counts against tg_count's undirected 4-node keys."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import directed4 as d4
from _gpu import device, note

pytestmark = pytest.mark.gpu


def run(rp, ci, sd, ty, L, **kw):
    import torch

    import paper_1901_10026_amd as tg
    dev = device()
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    g, rows, inf = tg.count_directed4(t(rp, np.int32), t(ci, np.int32), t(sd, np.uint8), t(ty, np.uint8), L, **kw)
    torch.cuda.synchronize()
    return (g.cpu().numpy().view(np.uint64) if g is not None else None,
            rows.cpu().numpy().view(np.uint64) if rows is not None else None,
            inf.cpu().numpy() if inf is not None else None)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_tiny_digraphs(L):
    T = d4.KeyTable(L)
    for idx in range(40):
        g = graphgen.tiny_graph(idx)
        sd = graphgen.orient(g.row_ptr, g.col_idx, 900 + idx, 0.3)
        ty = (g.types % L).astype(np.uint8)
        note(f"tiny{idx} n={g.n} m={g.m} L={L}")
        want_g = d4.brute_global(g.n, d4.arcs_from_csr(g.row_ptr, g.col_idx, sd), ty, L, table=T)
        want_r, pairs = d4.edge_rows(g.row_ptr, g.col_idx, sd, ty, L, table=T)
        got_g, got_r, inf = run(g.row_ptr, g.col_idx, sd, ty, L, per_edge=True, info=True, validate=True)
        assert np.array_equal(got_g, want_g), idx
        assert np.array_equal(got_r, want_r), idx
        assert [tuple(x[:2]) for x in inf] == [tuple(p) for p in pairs]


@pytest.mark.parametrize("L", [2, 4])
def test_dense_random_digraph(L):
    rp, ci = graphgen.gnp(60, 0.3, 21)
    sd = graphgen.orient(rp, ci, 22, 0.25)
    ty = (np.arange(60) % L).astype(np.uint8)
    T = d4.KeyTable(L)
    want_r, _ = d4.edge_rows(rp, ci, sd, ty, L, table=T)
    got_g, got_r, _ = run(rp, ci, sd, ty, L, per_edge=True)
    assert np.array_equal(got_r, want_r)
    assert np.array_equal(got_g, d4.rows_to_global(want_r, T))


def test_direction_summed_counts_equal_undirected_counts():
    """cl-2k oriented (20% reciprocal), L = 3: summed over the directed keys
    of each (shape, type multiset), the counts equal tg_count's undirected
    4-node global counts, which equal the oracle's."""
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    sd = graphgen.orient(g.row_ptr, g.col_idx, 23, 0.2)
    L = g.L
    got, _, _ = run(g.row_ptr, g.col_idx, sd, g.types, L)
    _, want = oracle.count_all(g.row_ptr, g.col_idx, g.types, L, per_edge=False, nthreads=8)
    summed = np.zeros(oracle.num_keys(L), dtype=np.uint64)
    for q in range(len(got)):
        arcs, ty = tg.directed4_key_decode(L, q)
        deg, ne = [0] * 4, 0
        for x, y in d4.UNORDERED:
            if arcs >> d4._BIT[(x, y)] & 1 or arcs >> d4._BIT[(y, x)] & 1:
                ne += 1
                deg[x] += 1
                deg[y] += 1
        mx = max(deg)
        h = (3 if mx == 3 else 2) if ne == 3 else ((5 if mx == 3 else 4) if ne == 4 else (6 if ne == 5 else 7))
        summed[oracle.key(L, h, list(ty))] += got[q]
    four = slice(oracle.shape_offset(L, 2), oracle.num_keys(L))
    assert np.array_equal(summed[four], want[four])
    note(f"cl-2k: {int(got.sum())} directed typed 4-node sets")


def test_rejections():
    import paper_1901_10026_amd as tg
    rp, ci = graphgen.gnp(20, 0.3, 24)
    sd = graphgen.orient(rp, ci, 25, 0.2)
    ty = np.zeros(20, np.uint8)
    with pytest.raises(tg.TGError) as ex:
        run(rp, ci, sd, ty, 5)
    assert ex.value.name == "TG_ERR_UNSUPPORTED_L"
    bad = sd.copy()
    bad[0] = 0
    with pytest.raises(tg.TGError) as ex:
        run(rp, ci, bad, ty, 2, validate=True)
    assert ex.value.name == "TG_ERR_INVALID_GRAPH"
    from _graphs import star
    rp, ci = star(1100)  # d_i + d_j - 2 = 1099 on every edge
    with pytest.raises(tg.TGError) as ex:
        run(rp, ci, graphgen.orient(rp, ci, 26, 0.2), np.zeros(1101, np.uint8), 1)
    assert ex.value.name == "TG_ERR_INVALID_ARG"
