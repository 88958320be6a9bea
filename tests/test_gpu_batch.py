"""Parity of tg_count_batch (many small graphs, one call) with the oracle."""
import numpy as np
import pytest

import graphgen
import oracle
from _gpu import device, note

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


def test_full_size_batch_sampled():
    # 100,000 graphs, n log-uniform in [10, 500], density U(0.02, 0.3),
    # L uniform in 2..8: every graph is counted; a sample is checked.
    b = graphgen.batch_gnp(100_000, 10, 500, 0.02, 0.3, 2, 8, 4)
    note(f"full batch: {b.G} graphs, {int(b.slot_off[-1]) // 2} edges")
    got, key_off = run_batch(b)
    n = np.diff(b.node_off)
    rng = np.random.default_rng(3)
    big = np.argsort(n)[-6:]
    sample = np.unique(np.concatenate([rng.choice(b.G, 60, replace=False), big]))
    check_graphs(b, got, key_off, sample)
