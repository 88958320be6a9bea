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
    assert bench.combine_bytes(st, 1, 3, lists=True) == 3 * fixed + (8 * 3 + 12 * 3) + 3 * member
    assert bench.combine_bytes(st, 1, 3, lists=False) == 3 * fixed + 4 * 3 * (2 + 2) + 3 * member
    assert bench.keeps_lists(st)


def test_combine_bytes_grow_with_types():
    # K6: the per-edge part grows with L as 2(4L + 16L^2) + 4L + 8P + 8R
    st = bench.graph_stats(_G(*complete(6)))
    tau_sum = 3 * 20
    per = [bench.combine_bytes(st, L, tau_sum, lists=True) for L in (1, 2, 3)]
    for L, b in zip((1, 2, 3), per):
        P = L * (L + 1) // 2
        R = 2 * L + 6 * P
        fixed = 8 + 16 + 2 * (4 * L + 16 * L * L) + 4 * L + 8 * P + 8 * R
        assert b == 15 * fixed + 8 * 15 + 12 * tau_sum + tau_sum * (1 + 12 * L)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "--gpus 1" in r.stderr


def test_committed_traffic_matches_the_combine_sources():
    # the counter summary records a hash of the sources it was taken on;
    # a kernel change without new counters makes bench.py report null
    t = bench.stored_traffic("cl-1m")
    assert t is not None and t > 0
    assert bench.stored_traffic("cl-2k") is None
