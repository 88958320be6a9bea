"""Parity of tg_count_batch (many small graphs, one call) with the oracle."""
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
from _gpu import device, note

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
from batch_digest import digests  # noqa: E402

pytestmark = pytest.mark.gpu


def run_batch(b, tuning=None):
    import torch

    import paper_1901_10026_amd as tg
    dev = device()
    key_off = tg.key_offsets(b.L)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    out = tg.count_batch(t(b.node_off, np.int64), t(b.slot_off, np.int64), t(b.row_ptr, np.int32),
                         t(b.col_idx, np.int32), t(b.types, np.uint8), t(b.L, np.uint8), t(key_off, np.int64),
                         tuning=tuning)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64), key_off


def check_graphs(b, got, key_off, which):
    for g in which:
        rp, ci, ty, L = b.graph(g)
        if len(rp) - 1 <= 12:
            _, _, want = oracle.brute(rp, ci, ty, L)
        else:
            _, want = oracle.count_all(rp, ci, ty, L, per_edge=False, nthreads=8)
        assert np.array_equal(got[key_off[g]:key_off[g + 1]], want), f"graph {g} (n={len(rp) - 1}, L={L})"


def test_small_mixed_batch_all_graphs():
    b = graphgen.batch_gnp(300, 1, 500, 0.02, 0.5, 1, 8, 41)
    note(f"batch of {b.G} graphs, {int(b.node_off[-1])} nodes, {int(b.slot_off[-1]) // 2} edges")
    got, key_off = run_batch(b)
    check_graphs(b, got, key_off, range(b.G))


def test_every_kernel_variant():
    import paper_1901_10026_amd as tg
    b = graphgen.batch_gnp(120, 1, 500, 0.05, 0.4, 2, 8, 42)
    base, key_off = run_batch(b)
    check_graphs(b, base, key_off, range(0, b.G, 3))
    wmax = {0: 1, 1: 2, 2: 2, 3: 4, 4: 4, 5: 8}
    for v in range(6):
        t = tg.Tuning.default()
        for w in range(9):
            if wmax[v] >= max(1, w):
                t.batch_variant[w] = v
        got, _ = run_batch(b, tuning=t)
        assert np.array_equal(got, base), f"variant {v}"


def test_replayed_graph_is_stable():
    b = graphgen.batch_gnp(200, 5, 300, 0.05, 0.3, 2, 8, 43)
    first, key_off = run_batch(b)
    for _ in range(3):
        again, _ = run_batch(b)
        assert np.array_equal(again, first)
    check_graphs(b, first, key_off, range(0, b.G, 5))


def test_full_size_batch_all_graphs():
    # 100,000 graphs, n log-uniform in [10, 500], density U(0.02, 0.3),
    # L uniform in 2..8, seed 4: every graph's global counts are compared
    # with the oracle's through a per-graph digest and count total written by
    # tests/golden/make_batch_digests.py; a sample is also compared key by
    # key with a fresh oracle count.
    b = graphgen.batch_gnp(100_000, 10, 500, 0.02, 0.3, 2, 8, 4)
    note(f"full batch: {b.G} graphs, {int(b.slot_off[-1]) // 2} edges")
    got, key_off = run_batch(b)
    ref = np.load(os.path.join(GOLDEN, "gnp_batch_100k_digests.npz"))
    assert np.array_equal(ref["L"], b.L) and np.array_equal(ref["edges"], np.diff(b.slot_off) // 2)
    dig, tot = digests(got, key_off)
    bad = np.nonzero((dig != ref["digest"]) | (tot != ref["total"]))[0]
    assert len(bad) == 0, f"{len(bad)} of {b.G} graphs differ from the oracle, first {bad[:5]}"
    note(f"all {b.G} graph digests equal the oracle's")
    n = np.diff(b.node_off)
    rng = np.random.default_rng(3)
    big = np.argsort(n)[-6:]
    sample = np.unique(np.concatenate([rng.choice(b.G, 30, replace=False), big]))
    check_graphs(b, got, key_off, sample)


def test_validate_rejects_bad_graphs():
    import torch

    import paper_1901_10026_amd as tg
    dev = device()
    b = graphgen.batch_gnp(40, 5, 100, 0.1, 0.4, 2, 8, 44)
    key_off = tg.key_offsets(b.L)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

    def call(ci=b.col_idx, ty=b.types):
        return tg.count_batch(t(b.node_off, np.int64), t(b.slot_off, np.int64), t(b.row_ptr, np.int32),
                              t(ci, np.int32), t(ty, np.uint8), t(b.L, np.uint8), t(key_off, np.int64),
                              validate=True)

    good = call().cpu().numpy().view(np.uint64)
    base, _ = run_batch(b)
    assert np.array_equal(good, base)
    g = int(np.argmax(np.diff(b.slot_off)))  # a graph with edges
    n0, s0 = int(b.node_off[g]), int(b.slot_off[g])
    ty = b.types.copy()
    ty[n0] = b.L[g]  # type == L_g
    with pytest.raises(tg.TGError) as ex:
        call(ty=ty)
    assert ex.value.name == "TG_ERR_TYPE_RANGE"
    n_g = int(b.node_off[g + 1] - n0)
    for mutate in ("range", "order", "asym"):
        ci = b.col_idx.copy()
        if mutate == "range":
            ci[s0] = n_g          # column id outside the graph
        elif mutate == "order":
            ci[s0], ci[s0 + 1] = ci[s0 + 1], ci[s0]
        else:
            rp, cig, _, _ = b.graph(g)
            # move the first slot of row u to a node it is not adjacent to
            u = int(np.argmax(np.diff(rp) > 0))
            nbrs = set(cig[rp[u]:rp[u + 1]].tolist()) | {u}
            free = [v for v in range(n_g) if v not in nbrs]
            if not free:
                continue
            row = sorted(set(cig[rp[u]:rp[u + 1]].tolist()[1:]) | {free[0]})
            ci[s0 + rp[u]:s0 + rp[u + 1]] = row
        note(f"batch validation: {mutate} in graph {g}")
        with pytest.raises(tg.TGError) as ex:
            call(ci=ci)
        assert ex.value.name == "TG_ERR_INVALID_GRAPH", mutate
