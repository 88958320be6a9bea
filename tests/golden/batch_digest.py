"""Per-graph 64-bit digests of batch global counts (test infrastructure).

A digest is a weighted sum, modulo 2^64, of one graph's K(L_g) global counts
with fixed odd 64-bit weights (the SplitMix64 output function, Steele, Lea,
Flood 2014, applied to the key index), so a changed count, a swapped pair of
keys or a shifted graph offset all change it.  The stored digests of the
100,000-graph batch are written by ``make_batch_digests.py`` from the
oracle's counts; tests recompute digests of the library's output with the
same function and compare every graph.
"""
import numpy as np

_M64 = (1 << 64) - 1


def _mix(x):
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return (z ^ (z >> 31)) | 1


def weights(kmax):
    return np.array([_mix(k) for k in range(kmax)], dtype=np.uint64)


def digests(counts, key_off):
    """(digest, total) per graph: counts is uint64[key_off[-1]], graph g's
    counts are counts[key_off[g]:key_off[g+1]] (every graph has keys)."""
    counts = np.asarray(counts, dtype=np.uint64)
    key_off = np.asarray(key_off, dtype=np.int64)
    sizes = np.diff(key_off)
    w = weights(int(sizes.max()) if len(sizes) else 0)
    local = np.arange(len(counts), dtype=np.int64) - np.repeat(key_off[:-1], sizes)
    with np.errstate(over="ignore"):
        prod = counts * w[local]
        dig = np.add.reduceat(prod, key_off[:-1]) if len(sizes) else np.zeros(0, np.uint64)
        tot = np.add.reduceat(counts, key_off[:-1]) if len(sizes) else np.zeros(0, np.uint64)
    return dig.astype(np.uint64), tot.astype(np.uint64)
