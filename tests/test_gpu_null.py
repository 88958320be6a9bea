"""Type-permutation null model (the exploratory analysis' randomized typed
motif distributions): global counts of one graph under many type vectors
with shared structure (tg_count_global_types), against the oracle per vector
and against the closed form of the mean over all relabellings."""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from _gpu import note, to_dev
from _graphs import csr_from_edges

pytestmark = pytest.mark.gpu


def gpu_types(row_ptr, col_idx, vectors, L, **kw):
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, _ = to_dev(row_ptr, col_idx, vectors[0])
    tv = torch.from_numpy(np.ascontiguousarray(vectors, dtype=np.uint8)).to(rp.device)
    counts, mean = tg.count_global_types(rp, ci, tv, L, **kw)
    torch.cuda.synchronize()
    return counts.cpu().numpy().view(np.uint64), (mean.cpu().numpy() if mean is not None else None)


def test_each_permutation_matches_the_oracle():
    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    perms = tg.type_permutations(g.types, 4, seed=21)
    counts, mean = gpu_types(g.row_ptr, g.col_idx, perms, g.L, validate=True)
    for b in range(len(perms)):
        _, want = oracle.count_all(g.row_ptr, g.col_idx, perms[b], g.L, per_edge=False, nthreads=8)
        assert np.array_equal(counts[b], want), f"permutation {b}"
    # the mean: exact integer sums over the vectors, one division
    for k in range(len(mean)):
        s = sum(int(counts[b, k]) for b in range(len(perms)))
        assert mean[k] == s / len(perms)


def test_mean_over_all_relabellings_is_hypergeometric():
    """Summed over every distinct assignment of the type multiset to the
    nodes, the count of (shape, multiset M) on k nodes is the untyped count
    times k!/prod m_t! * (n-k)!/prod (n_t - m_t)!."""
    rng = np.random.default_rng(4)
    n = 8
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < 0.5]
    rp, ci = csr_from_edges(n, edges)
    base = [0, 0, 0, 1, 1, 2, 2, 2]
    L = 3
    vectors = np.array(sorted(set(itertools.permutations(base))), dtype=np.uint8)
    note(f"{len(vectors)} distinct relabellings of n={n}, m={len(edges)}")
    counts, mean = gpu_types(rp, ci, vectors, L)
    total = counts.astype(object).sum(axis=0)
    _, _, untyped = oracle.brute(rp, ci, np.zeros(n, np.uint8), 1)
    nt = [base.count(t) for t in range(L)]
    for shape in range(8):
        k = 3 if shape < 2 else 4
        n_h = int(untyped[oracle.key(1, shape, [0] * k)])
        for ms in itertools.combinations_with_replacement(range(L), k):
            mt = [ms.count(t) for t in range(L)]
            if any(mt[t] > nt[t] for t in range(L)):
                ways = 0
            else:
                ways = math.factorial(k) * math.factorial(n - k)
                for t in range(L):
                    ways //= math.factorial(mt[t]) * math.factorial(nt[t] - mt[t])
            assert total[oracle.key(L, shape, list(ms))] == n_h * ways, (shape, ms)
    assert np.allclose(mean, total.astype(np.float64) / len(vectors), rtol=1e-15)


def test_full_size_permutations_equal_single_counts():
    """cl-1m: two permutations through the shared path equal separate
    tg_count_global calls."""
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_1m()
    perms = tg.type_permutations(g.types, 2, seed=3)
    rp, ci, _ = to_dev(g.row_ptr, g.col_idx, g.types)
    tv = torch.from_numpy(perms).to(rp.device)
    ph = {}
    counts, _ = tg.count_global_types(rp, ci, tv, g.L, phase_ms=ph)
    note("2 permutations: " + " ".join(f"{k}={v:.1f}ms" for k, v in ph.items()))
    for b in range(2):
        single = tg.count_global(rp, ci, tv[b].contiguous(), g.L)
        torch.cuda.synchronize()
        assert torch.equal(counts[b].view(torch.int64), single.view(torch.int64)), b


def test_one_type_vector_and_an_edgeless_graph():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.tiny_graph(17)
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    counts, mean = tg.count_global_types(rp, ci, ty.view(1, -1).contiguous(), g.L)
    single = tg.count_global(rp, ci, ty, g.L)
    torch.cuda.synchronize()
    assert torch.equal(counts[0].view(torch.int64), single.view(torch.int64))
    assert np.array_equal(mean.cpu().numpy(), single.cpu().numpy().view(np.uint64).astype(np.float64))
    rp0, ci0, _ = to_dev(np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(5, np.uint8))
    tv = torch.zeros((3, 5), dtype=torch.uint8, device=rp0.device)
    counts, mean = tg.count_global_types(rp0, ci0, tv, 2)
    torch.cuda.synchronize()
    assert int(counts.view(torch.int64).abs().sum()) == 0 and float(mean.abs().sum()) == 0.0
