"""The stored per-graph digests of the 100,000-graph batch (written by
tests/golden/make_batch_digests.py from the oracle) against fresh oracle
counts of a sample of its graphs, and the digest's sensitivity (CPU)."""
import os
import sys

import numpy as np

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
from batch_digest import digests  # noqa: E402


def test_stored_digests_match_fresh_oracle_counts():
    b = graphgen.batch_gnp(100_000, 10, 500, 0.02, 0.3, 2, 8, 4)
    ref = np.load(os.path.join(GOLDEN, "gnp_batch_100k_digests.npz"))
    assert len(ref["digest"]) == b.G and np.array_equal(ref["L"], b.L)
    rng = np.random.default_rng(17)
    n = np.diff(b.node_off)
    pick = np.unique(np.concatenate([rng.choice(b.G, 25, replace=False), np.argsort(n)[:3]]))
    for g in pick:
        rp, ci, ty, L = b.graph(int(g))
        _, glob = oracle.count_all(rp, ci, ty, L, per_edge=False, nthreads=8)
        d, t = digests(glob, np.array([0, len(glob)]))
        assert d[0] == ref["digest"][g] and t[0] == ref["total"][g], int(g)


def test_digest_sees_changed_swapped_and_shifted_counts():
    c = np.arange(1, 39, dtype=np.uint64)
    ko = np.array([0, 38])
    base = digests(c, ko)[0][0]
    c2 = c.copy()
    c2[5] += 1
    assert digests(c2, ko)[0][0] != base
    c3 = c.copy()
    c3[[3, 9]] = c3[[9, 3]]
    assert digests(c3, ko)[0][0] != base
    two = np.concatenate([c, c])
    d2, _ = digests(two, np.array([0, 37, 76]))  # offsets shifted by one
    assert d2[0] != base
