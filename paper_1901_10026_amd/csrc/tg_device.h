// Device-side helpers shared by the gfx950 kernels: wavefront primitives,
// degree order, type-pair indexing and the dense key rank.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TG_WAVE 64

namespace tg {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders LDS traffic between lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, TG_WAVE);
  return v;
}

// Degree order: u precedes v when (d_u, u) < (d_v, v).
__device__ __forceinline__ bool precedes(int32_t du, int32_t u, int32_t dv, int32_t v) {
  return du < dv || (du == dv && u < v);
}

// First index in sorted a[0, len) whose value is >= key (len if none).
__device__ __forceinline__ int32_t lower_bound(const int32_t* a, int32_t len, int32_t key) {
  int32_t lo = 0, hi = len;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Unordered type pair {t, u} -> u(u+1)/2 + t with t <= u.
__device__ __forceinline__ int pair_index(int t, int u) {
  if (t > u) { int s = t; t = u; u = s; }
  return u * (u + 1) / 2 + t;
}

__device__ __forceinline__ int64_t c2(int64_t x) { return x * (x - 1) / 2; }
__device__ __forceinline__ int64_t c3(int64_t x) { return x * (x - 1) * (x - 2) / 6; }
__device__ __forceinline__ int64_t c4(int64_t x) { return x * (x - 1) * (x - 2) * (x - 3) / 24; }

// Global key of (shape h, types a, b, c[, d]) for L types; 4-node shapes use d.
__device__ __forceinline__ int64_t key_of(int L, int h, int a, int b, int c, int d) {
  const int64_t C3 = c3(L + 2), C4 = c4(L + 3);
  if (h < 2) {
    int x0 = min(a, min(b, c)), x2 = max(a, max(b, c)), x1 = a + b + c - x0 - x2;
    return (int64_t)h * C3 + x0 + c2(x1 + 1) + c3(x2 + 2);
  }
  // sorting network on four values
  int v0 = a, v1 = b, v2 = c, v3 = d, s;
#define TG_CS(x, y) if (x > y) { s = x; x = y; y = s; }
  TG_CS(v0, v1) TG_CS(v2, v3) TG_CS(v0, v2) TG_CS(v1, v3) TG_CS(v1, v2)
#undef TG_CS
  return 2 * C3 + (int64_t)(h - 2) * C4 + v0 + c2(v1 + 1) + c3(v2 + 2) + c4(v3 + 3);
}

}  // namespace tg
