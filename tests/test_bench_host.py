"""Host-side checks of the benchmark script: its byte model on graphs small
enough to count by hand, the one-GPU guard, and that the committed counter
summary belongs to the committed combine sources."""
import subprocess
import sys

import numpy as np

import bench
from _graphs import complete


class _G:
    def __init__(self, rp, ci):
        self.row_ptr, self.col_idx, self.n = rp, ci, len(rp) - 1


def test_combine_bytes_on_a_triangle():
    # K3, L = 1: m = 3, every degree 2, |T_ij| = 1 per edge (tau_sum = 3);
    # P = 1, R = 2L + 6P = 8
    st = bench.graph_stats(_G(*complete(3)))
    assert st["m"] == 3
    fixed = 8 + 16 + 2 * (4 + 16) + 4 + 8 + 8 * 8
    member = 1 + 12
    # 4-cliques from the clique pass's 32-bit counters (one type pair)
    assert bench.combine_bytes(st, 1, 3, lists=True, k4_width=4) == 3 * fixed + (8 * 3 + 12 * 3) + 3 * member + 3 * 4
    assert bench.combine_bytes(st, 1, 3, lists=False, k4_width=4) == 3 * fixed + 4 * 3 * (2 + 2) + 3 * member + 3 * 4
    # ... or from out-list probes: 8 B of offsets per member, 4 B per probe
    assert bench.combine_bytes(st, 1, 3, lists=True, probes=5) == 3 * fixed + (8 * 3 + 12 * 3) + 3 * member + 8 * 3 + 20
    assert bench.keeps_lists(st)


def test_combine_bytes_grow_with_types():
    # K6: the per-edge part grows with L as 2(4L + 16L^2) + 4L + 8P + 8R
    st = bench.graph_stats(_G(*complete(6)))
    tau_sum = 3 * 20
    per = [bench.combine_bytes(st, L, tau_sum, lists=True, k4_width=8) for L in (1, 2, 3)]
    for L, b in zip((1, 2, 3), per):
        P = L * (L + 1) // 2
        R = 2 * L + 6 * P
        fixed = 8 + 16 + 2 * (4 * L + 16 * L * L) + 4 * L + 8 * P + 8 * R
        assert b == 15 * fixed + 8 * 15 + 12 * tau_sum + tau_sum * (1 + 12 * L) + 15 * P * 8


def test_degree_order_and_wedges_of_k4():
    # K4: equal degrees, so the order is by id: out-degrees 3, 2, 1, 0.
    # Scanned wedges sum d_u d+_u = 3 (3 + 2 + 1) = 18; oriented wedges x-u-w
    # with both u and w below x: u=0: x=1 none, x=2 {1}, x=3 {1,2}; u=1: x=2
    # {0}, x=3 {0,2}; u=2: x=3 {0,1}: 0+1+2+1+2+2 = 8
    st = bench.graph_stats(_G(*complete(4)))
    assert list(st["dplus"]) == [3, 2, 1, 0]
    assert bench.cycle_wedges(st) == (18, 8)
    L, P = 2, 3
    assert bench.cycles_bytes(st, L, 18, 8, 4) == 16 * 18 + 8 * (4 + 2 * L + 1) + 3 * 6 * P * 4
    # clique pass: lower neighbours d- = 0, 1, 2, 3, so the out-list reads are
    # 1 (8 + 8*2) + 2 (8 + 8*1) + 3 (8 + 0) = 80 B, plus 5 B per edge and the
    # counters cleared and flushed
    assert bench.clique_bytes(st, L, 4) == 5 * 6 + 80 + 2 * 6 * P * 4


def test_clique_probes_by_definition():
    # the probe count of the out-list path is the sum over edges of the
    # out-degrees of T_ij's members; on K5 every T_ij has 3 members and the
    # formula over nodes (d+_k times the triangles at k) must agree
    rp, ci = complete(5)
    st = bench.graph_stats(_G(rp, ci))
    adj = [set(ci[rp[v]:rp[v + 1]].tolist()) for v in range(5)]
    by_edges = sum(int(st["dplus"][k]) for i, j in zip(st["ei"], st["ej"]) for k in adj[i] & adj[j])
    tri = np.array([sum(1 for a in adj[k] for b in adj[k] if a < b and b in adj[a]) for k in range(5)])
    assert by_edges == bench.clique_probes(st, tri) == int((st["dplus"] * tri).sum())


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "--gpus 1" in r.stderr


def test_committed_traffic_matches_the_kernel_sources():
    # the counter summary records a hash of the sources it was taken on;
    # a kernel change without new counters makes bench.py report null
    t = bench.stored_traffic("cl-1m")
    assert t is not None and all(t.get(ph, 0) > 0 for ph in ("cycles", "cliques", "combine"))
    assert bench.stored_traffic("cl-2k") is None
