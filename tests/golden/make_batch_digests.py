"""Writes gnp_batch_100k_digests.npz: the oracle's global counts of every
graph of the 100,000-graph batch workload (n log-uniform in [10, 500],
density uniform in [0.02, 0.3], L uniform in 2..8, seed 4), reduced to one
digest and one count total per graph.  Calls only the oracle and the input
generator.  Run from the repository root:
    python tests/golden/make_batch_digests.py [threads]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import graphgen  # noqa: E402
import oracle  # noqa: E402
from batch_digest import digests  # noqa: E402

BATCH = dict(G=100_000, nmin=10, nmax=500, rmin=0.02, rmax=0.3, lmin=2, lmax=8, seed=4)
OUT = os.path.join(HERE, "gnp_batch_100k_digests.npz")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    b = graphgen.batch_gnp(BATCH["G"], BATCH["nmin"], BATCH["nmax"], BATCH["rmin"], BATCH["rmax"], BATCH["lmin"],
                           BATCH["lmax"], BATCH["seed"])
    t0 = time.time()
    counts, key_off = oracle.count_batch(b.node_off, b.slot_off, b.row_ptr, b.col_idx, b.types, b.L,
                                         nthreads=threads)
    dig, tot = digests(counts, key_off)
    np.savez(OUT, digest=dig, total=tot, L=np.asarray(b.L, dtype=np.uint8),
             edges=(np.diff(b.slot_off) // 2).astype(np.int64))
    print(f"{b.G} graphs counted by the oracle in {time.time() - t0:.0f} s on {threads} threads -> {OUT}")


if __name__ == "__main__":
    main()
