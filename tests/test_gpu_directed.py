"""Directed typed 3-node graphlets on the GPU (tg_count_directed3) against
the directed oracle: per-edge rows and global counts."""
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import directed as od
from _gpu import note, to_dev
from _graphs import csr_from_arcs

pytestmark = pytest.mark.gpu


def gpu_dir(row_ptr, col_idx, slot_dir, types, L, **kw):
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, ty = to_dev(row_ptr, col_idx, types)
    sd = torch.from_numpy(np.ascontiguousarray(slot_dir, dtype=np.uint8)).to(rp.device)
    g, rows, info = tg.count_directed3(rp, ci, sd, ty, L, info=True, **kw)
    torch.cuda.synchronize()
    return (g.cpu().numpy().view(np.uint64), rows.cpu().numpy().view(np.uint64), info.cpu().numpy())


def test_tiny_digraphs_match_brute_force():
    for idx in range(120):
        g, sd = graphgen.tiny_digraph(idx)
        if g.m == 0:
            continue
        glob, rows, info = gpu_dir(g.row_ptr, g.col_idx, sd, g.types, g.L, validate=True)
        want_rows, codes, ends = od.edge_rows(g.row_ptr, g.col_idx, sd, g.types, g.L)
        assert np.array_equal(rows, want_rows), idx
        assert np.array_equal(info[:, 2], codes) and [tuple(x) for x in info[:, :2]] == ends, idx
        want = od.brute_global(g.n, od.arcs_from_csr(g.row_ptr, g.col_idx, sd), g.types, g.L)
        assert np.array_equal(glob, want), idx


def test_chung_lu_2k_oriented():
    g = graphgen.chung_lu_small()
    for seed, p_both in ((1, 0.2), (2, 0.0), (3, 1.0)):
        sd = graphgen.orient(g.row_ptr, g.col_idx, seed, p_both)
        glob, rows, info = gpu_dir(g.row_ptr, g.col_idx, sd, g.types, g.L)
        want_rows, codes, ends = od.edge_rows(g.row_ptr, g.col_idx, sd, g.types, g.L)
        assert np.array_equal(rows, want_rows), seed
        assert np.array_equal(glob, od.rows_to_global(want_rows, codes, ends, g.types, g.L)), seed


def test_closed_forms():
    import paper_1901_10026_amd as tg
    n = 40
    # transitive tournament, L = 1: every triple is the transitive triad
    rp, ci, sd = csr_from_arcs(n, {(u, v) for u in range(n) for v in range(u + 1, n)})
    glob, _, _ = gpu_dir(rp, ci, sd, np.zeros(n, np.uint8), 1)
    assert glob[tg.directed3_key_encode(1, 0b010101, [0, 0, 0])] == math.comb(n, 3) == glob.sum()
    # all-mutual complete graph with two types
    rp, ci, sd = csr_from_arcs(n, {(u, v) for u in range(n) for v in range(n) if u != v})
    ty = (np.arange(n) % 2).astype(np.uint8)
    glob, _, _ = gpu_dir(rp, ci, sd, ty, 2)
    a, b = 20, 20
    assert glob[tg.directed3_key_encode(2, 63, [0, 0, 0])] == math.comb(a, 3)
    assert glob[tg.directed3_key_encode(2, 63, [0, 0, 1])] == math.comb(a, 2) * b
    assert glob.sum() == math.comb(n, 3)
    # directed cycle 0 -> 1 -> ... -> n-1 -> 0: n directed 2-paths
    rp, ci, sd = csr_from_arcs(n, {(v, (v + 1) % n) for v in range(n)})
    glob, _, _ = gpu_dir(rp, ci, sd, np.zeros(n, np.uint8), 1)
    assert glob[tg.directed3_key_encode(1, 0b010001, [0, 0, 0])] == n == glob.sum()


@pytest.mark.parametrize("L", [8, 16])
def test_many_types(L):
    rp, ci = graphgen.gnp(60, 0.4, 9)
    ty = (np.arange(60) % L).astype(np.uint8)
    sd = graphgen.orient(rp, ci, 11, 0.3)
    glob, rows, _ = gpu_dir(rp, ci, sd, ty, L)
    want_rows, codes, ends = od.edge_rows(rp, ci, sd, ty, L)
    assert np.array_equal(rows, want_rows)
    assert np.array_equal(glob, od.brute_global(60, od.arcs_from_csr(rp, ci, sd), ty, L))


def test_bad_direction_bytes_are_reported():
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, sd = csr_from_arcs(4, {(0, 1), (1, 2), (2, 3)})
    for bad in ("zero", "unmirrored"):
        s2 = sd.copy()
        if bad == "zero":
            s2[0] = 0
        else:
            s2[0] = 3
        d_rp, d_ci, d_ty = to_dev(rp, ci, np.zeros(4, np.uint8))
        with pytest.raises(tg.TGError) as e:
            tg.count_directed3(d_rp, d_ci, torch.from_numpy(s2).to(d_rp.device), d_ty, 1, validate=True)
        assert e.value.name == "TG_ERR_INVALID_GRAPH"


def test_full_size_rows_and_directions():
    """cl-1m oriented (20% reciprocal): sampled rows against the oracle; the
    rows summed over directions equal tg_count's wedge and triangle columns;
    global counts equal the row sums per key divided by support edges."""
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_1m()
    sd = graphgen.orient(g.row_ptr, g.col_idx, 99, 0.2)
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    d_sd = torch.from_numpy(sd).to(rp.device)
    ph = {}
    glob, rows, info = tg.count_directed3(rp, ci, d_sd, ty, g.L, info=True, phase_ms=ph)
    torch.cuda.synchronize()
    note("directed3 cl-1m: " + " ".join(f"{k}={v:.1f}ms" for k, v in ph.items()))
    L = g.L
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    d = np.diff(g.row_ptr).astype(np.int64)
    order = np.argsort(d[ei] * d[ej], kind="stable")
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.choice(p, 4, replace=False) for p in np.array_split(order, 10)] +
                                   [order[-4:]]))
    got = rows.index_select(0, torch.from_numpy(idx).to(rows.device)).cpu().numpy().view(np.uint64)
    want = od.rows_for_edges(g.row_ptr, g.col_idx, sd, g.types, L, list(zip(ei[idx], ej[idx])))
    assert np.array_equal(got, want)
    _, und, _ = tg.count(rp, ci, ty, L, per_edge=True, global_counts=False)
    r = rows.view(torch.int64).view(-1, 15, L)
    pad = torch.zeros((r.shape[0], 1, L), dtype=torch.int64, device=r.device)
    r = torch.cat([pad, r], dim=1).view(-1, 4, 4, L)
    wedge = r[:, 1:, 0, :].sum(dim=1) + r[:, 0, 1:, :].sum(dim=1)
    tri = r[:, 1:, 1:, :].sum(dim=(1, 2))
    u = und.view(torch.int64)
    assert torch.equal(wedge, u[:, :L]) and torch.equal(tri, u[:, L:2 * L])
    # every typed triangle / wedge of the support shows up once per triple
    gl = glob.cpu().numpy().view(np.uint64)
    supp = np.array([od.support_edges(tg.directed3_key_decode(L, k)[0]) for k in range(len(gl))])
    total_rows = int(rows.view(torch.int64).sum().item())
    assert int((gl.astype(object) * supp).sum()) == total_rows


def test_edgeless_and_empty_digraphs():
    import torch

    import paper_1901_10026_amd as tg
    for n in (0, 4):
        rp, ci, ty = to_dev(np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(n, np.uint8))
        sd = torch.zeros(0, dtype=torch.uint8, device=rp.device)
        glob, rows, _ = tg.count_directed3(rp, ci, sd, ty, 3, validate=n > 0)
        torch.cuda.synchronize()
        assert rows.shape == (0, 45) and int(glob.view(torch.int64).abs().sum()) == 0
        assert glob.numel() == tg.directed3_num_keys(3)
