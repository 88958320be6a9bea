// Sparse per-edge output: the nonzero entries of dense per-edge rows as
// (global typed-graphlet key, count) pairs, edge by edge in row order, the
// compact per-edge form the paper stores instead of dense vectors.
//
// Column c of the row of an edge with endpoint types (a, b): c < L is the
// wedge with third type c, L <= c < 2L the triangle with third type c - L,
// and 2L + s P + p the 4-node shape 2 + s with other types (t, u), t <= u,
// p = u (u + 1) / 2 + t.

#include "tg_internal.h"

namespace tg {

__device__ __forceinline__ int64_t row_column_key(int L, int P, int a, int b, int c) {
  if (c < L) return key_of(L, 0, a, b, c, 0);
  if (c < 2 * L) return key_of(L, 1, a, b, c - L, 0);
  const int q = c - 2 * L, s = q / P, p = q - s * P;
  int u = 0;
  while ((u + 1) * (u + 2) / 2 <= p) ++u;
  return key_of(L, 2 + s, a, b, p - u * (u + 1) / 2, u);
}

// One wavefront per edge: nonzero count of its row.
__global__ void __launch_bounds__(256) k_sparse_count(int64_t E, int R, const uint64_t* __restrict__ rows,
                                                      int64_t* __restrict__ cnt) {
  const int ln = lane();
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + threadIdx.x / TG_WAVE; e < E;
       e += (int64_t)gridDim.x * (blockDim.x / TG_WAVE)) {
    int c = 0;
    for (int q = ln; q < R; q += TG_WAVE) c += rows[e * R + q] != 0 ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, TG_WAVE);
    if (ln == 0) cnt[e] = c;
  }
}

// One wavefront per edge: its nonzero entries, in column order, at offset[e].
__global__ void __launch_bounds__(256) k_sparse_fill(int64_t E, int L, const uint64_t* __restrict__ rows,
                                                     const int32_t* __restrict__ ends,
                                                     const uint8_t* __restrict__ types,
                                                     const int64_t* __restrict__ offset, uint32_t* __restrict__ keys,
                                                     uint64_t* __restrict__ counts) {
  const int P = L * (L + 1) / 2, R = 2 * L + 6 * P;
  const int ln = lane();
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + threadIdx.x / TG_WAVE; e < E;
       e += (int64_t)gridDim.x * (blockDim.x / TG_WAVE)) {
    const int a = types[ends[2 * e]], b = types[ends[2 * e + 1]];
    int64_t pos = offset[e];
    for (int q0 = 0; q0 < R; q0 += TG_WAVE) {
      const int q = q0 + ln;
      const uint64_t v = q < R ? rows[e * R + q] : 0ull;
      const uint64_t mask = ballot(v != 0);
      if (v != 0) {
        const int64_t at = pos + lanes_below(mask);
        keys[at] = (uint32_t)row_column_key(L, P, a, b, q);
        counts[at] = v;
      }
      pos += __popcll(mask);
    }
  }
}

}  // namespace tg
