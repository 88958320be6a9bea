// gfx950 kernel for many small typed graphs in one launch per size bucket.
//
// One team (a wavefront, or a workgroup of four) owns one graph at a time and
// pulls the next graph from a per-bucket queue (graphs are queued largest
// first).  The graph is relabelled so that nodes of each type are contiguous,
// and its adjacency is held as bit rows in LDS (at most 64 * W_MAX nodes).
// Every edge (i, j) is handled by one lane with the sets of Section 4 as bit
// masks: T = A_i & A_j, S_i = A_i & ~A_j minus j, S_j = A_j & ~A_i minus i.
// For every node k of T, S_i, S_j the lane counts, per type u, k's neighbours
// in T, S_i, S_j (popcounts over the type's bit range) and in I (from k's typed
// degree), which are exactly the explicit orbits of Algorithms 2-3:
//   k in T:   g12 += |A_k & T|,  g10 += |A_k & (S_i|S_j)|,  g8 += |A_k & I|
//   k in S_i: g7  += |A_k & S_i|,                          g3 += |A_k & I|
//   k in S_j: g7  += |A_k & S_j|, g6 += |A_k & S_i|,       g3 += |A_k & I|
// (g7, g12 as ordered pairs, i.e. twice).  The graph's global counts are then
// sums over edges of Eqs. 7-16 mapped to keys, divided by the shape's edge
// count (Eq. 17).  All key sums are kept doubled so that the ordered
// within-class pairs stay integral; the final division removes the factor.

#include "tg_device.h"

namespace tg {

struct BatchArgs {
  const int64_t* node_off;   // [G+1]
  const int64_t* slot_off;   // [G+1]
  const int32_t* row_ptr;    // local row pointers, graph g at node_off[g] + g
  const int32_t* col_idx;    // local ids
  const uint8_t* types;      // [node_off[G]]
  const uint8_t* Lg;         // [G]
  const int64_t* key_off;    // [G+1]
  uint64_t* out;             // [key_off[G]]
  int32_t* flag;             // set when a key sum is not divisible
};

#define TG_BATCH_LMAX 8

template <int W_MAX>
struct BatchLds {
  uint64_t adj[64 * W_MAX][W_MAX];     // bit rows, relabelled ids
  uint16_t deg_t[64 * W_MAX][TG_BATCH_LMAX];
  uint16_t new_id[64 * W_MAX];
  int32_t rp[64 * W_MAX + 1];
  int32_t type_cnt[TG_BATCH_LMAX + 1];
  int32_t type_start[TG_BATCH_LMAX + 1];
  int32_t item;
};

template <int NWAVES>
__device__ __forceinline__ void bteam_sync() {
  if (NWAVES == 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

__device__ __forceinline__ void acc_add(uint64_t* acc, int64_t key, int64_t v) {
  if (v) atomicAdd((unsigned long long*)&acc[key], (unsigned long long)v);
}

// Bits [lo, hi) of a 64-bit word (0 <= lo, hi <= 64).
__device__ __forceinline__ uint64_t range_mask(int lo, int hi) {
  if (hi <= lo) return 0ull;
  const uint64_t upto_hi = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
  const uint64_t below_lo = lo >= 64 ? ~0ull : ((1ull << lo) - 1ull);
  return upto_hi & ~below_lo;
}

// Bits of word w that belong to type u: nodes are relabelled so that type u
// holds ids [ts[u], ts[u+1]).
__device__ __forceinline__ uint64_t type_word_mask(const int32_t (&ts)[TG_BATCH_LMAX + 1], int u, int w) {
  const int base = 64 * w;
  const int lo = min(max(ts[u] - base, 0), 64), hi = min(max(ts[u + 1] - base, 0), 64);
  return range_mask(lo, hi);
}

// Counts per type u of the set bits of a[0..W), b[0..W), c[0..W).
template <int W_MAX>
__device__ __forceinline__ void typed_popc3(const uint64_t (&a)[W_MAX], const uint64_t (&b)[W_MAX],
                                            const uint64_t (&c)[W_MAX], const int32_t (&ts)[TG_BATCH_LMAX + 1],
                                            int L, int32_t (&ca)[TG_BATCH_LMAX], int32_t (&cb)[TG_BATCH_LMAX],
                                            int32_t (&cc)[TG_BATCH_LMAX]) {
#pragma unroll
  for (int u = 0; u < TG_BATCH_LMAX; ++u) {
    int32_t sa = 0, sb = 0, sc = 0;
    if (u < L) {
#pragma unroll
      for (int w = 0; w < W_MAX; ++w) {
        const uint64_t m = type_word_mask(ts, u, w);
        if (m) {
          sa += __popcll(a[w] & m);
          sb += __popcll(b[w] & m);
          sc += __popcll(c[w] & m);
        }
      }
    }
    ca[u] = sa;
    cb[u] = sb;
    cc[u] = sc;
  }
}

template <int W_MAX, int NWAVES, bool LDS_ACC>
__global__ void __launch_bounds__(256) k_batch(BatchArgs A, int64_t count, const int32_t* __restrict__ list,
                                               int32_t* __restrict__ queue) {
  constexpr int TEAMS = 4 / NWAVES;
  constexpr int TSIZE = NWAVES * TG_WAVE;
  constexpr int NMAX = 64 * W_MAX;
  static_assert(!LDS_ACC || TEAMS == 1, "an LDS key accumulator is shared by the whole workgroup");
  __shared__ BatchLds<W_MAX> lds_all[TEAMS];
  __shared__ uint64_t keyacc_lds[LDS_ACC ? 2220 : 1];
  const int team = threadIdx.x / TSIZE;
  const int tid = threadIdx.x % TSIZE;
  BatchLds<W_MAX>& S = lds_all[team];
  const int shape_edges[8] = {2, 3, 3, 3, 4, 4, 5, 6};

  for (;;) {
    if (tid == 0) S.item = atomicAdd(queue, 1);
    bteam_sync<NWAVES>();
    const int64_t item = S.item;
    bteam_sync<NWAVES>();
    if (item >= count) break;
    const int32_t g = list[item];
    const int64_t n0 = A.node_off[g];
    const int n = (int)(A.node_off[g + 1] - n0);
    const int64_t s0 = A.slot_off[g];
    const int nslots = (int)(A.slot_off[g + 1] - s0);
    const int32_t* grp = A.row_ptr + n0 + g;
    const int32_t* gci = A.col_idx + s0;
    const uint8_t* gty = A.types + n0;
    const int L = A.Lg[g];
    const int W = (n + 63) / 64;
    const int64_t C3 = c3(L + 2), C4n = c4(L + 3), K = 2 * C3 + 6 * C4n;
    uint64_t* acc = LDS_ACC ? keyacc_lds : A.out + A.key_off[g];
    (void)NMAX;

    // ---- load: type histogram, relabel by type, bit rows, typed degrees
    for (int q = tid; q <= TG_BATCH_LMAX; q += TSIZE) S.type_cnt[q] = 0;
    for (int64_t q = tid; q < K; q += TSIZE) acc[q] = 0;
    for (int v = tid; v <= n; v += TSIZE) S.rp[v] = grp[v];
    for (int v = tid; v < n; v += TSIZE)
      for (int w = 0; w < W_MAX; ++w) S.adj[v][w] = 0;
    bteam_sync<NWAVES>();
    for (int v = tid; v < n; v += TSIZE) S.new_id[v] = (uint16_t)atomicAdd(&S.type_cnt[gty[v]], 1);
    bteam_sync<NWAVES>();
    if (tid == 0) {
      int a = 0;
      for (int t = 0; t <= TG_BATCH_LMAX; ++t) {
        S.type_start[t] = a;
        a += (t < L) ? S.type_cnt[t] : 0;
      }
    }
    bteam_sync<NWAVES>();
    for (int v = tid; v < n; v += TSIZE) S.new_id[v] = (uint16_t)(S.new_id[v] + S.type_start[gty[v]]);
    bteam_sync<NWAVES>();
    for (int s = tid; s < nslots; s += TSIZE) {
      const int v = lower_bound(S.rp, n + 1, s + 1) - 1;  // row holding slot s
      const int a = S.new_id[v], b = S.new_id[gci[s]];
      atomicOr((unsigned long long*)&S.adj[a][b >> 6], (unsigned long long)(1ull << (b & 63)));
    }
    bteam_sync<NWAVES>();
    int32_t ts[TG_BATCH_LMAX + 1];
#pragma unroll
    for (int t = 0; t <= TG_BATCH_LMAX; ++t) ts[t] = S.type_start[t];
    for (int v = tid; v < n; v += TSIZE) {
      uint64_t x[W_MAX];
#pragma unroll
      for (int w = 0; w < W_MAX; ++w) x[w] = (w < W) ? S.adj[v][w] : 0ull;
      int32_t c[TG_BATCH_LMAX], c1[TG_BATCH_LMAX], c2[TG_BATCH_LMAX];
      typed_popc3<W_MAX>(x, x, x, ts, L, c, c1, c2);
#pragma unroll
      for (int u = 0; u < TG_BATCH_LMAX; ++u) S.deg_t[v][u] = (uint16_t)c[u];
    }
    bteam_sync<NWAVES>();

    // ---- one lane per edge (i < j in the original ids)
    for (int s = tid; s < nslots; s += TSIZE) {
      const int v = lower_bound(S.rp, n + 1, s + 1) - 1;
      const int ov = gci[s];
      if (ov <= v) continue;
      const int i = S.new_id[v], j = S.new_id[ov];
      const int pi = gty[v], pj = gty[ov];
      uint64_t T[W_MAX], Si[W_MAX], Sj[W_MAX];
#pragma unroll
      for (int w = 0; w < W_MAX; ++w) {
        const uint64_t ai = (w < W) ? S.adj[i][w] : 0ull, aj = (w < W) ? S.adj[j][w] : 0ull;
        const uint64_t bi = ((i >> 6) == w) ? (1ull << (i & 63)) : 0ull;
        const uint64_t bj = ((j >> 6) == w) ? (1ull << (j & 63)) : 0ull;
        T[w] = ai & aj;
        Si[w] = ai & ~aj & ~bj;
        Sj[w] = aj & ~ai & ~bi;
      }
      int32_t nT[TG_BATCH_LMAX], nSi[TG_BATCH_LMAX], nSj[TG_BATCH_LMAX];
      typed_popc3<W_MAX>(T, Si, Sj, ts, L, nT, nSi, nSj);
      // 3-node graphlets and the product terms of Eqs. 7-10, doubled
#pragma unroll
      for (int u = 0; u < TG_BATCH_LMAX; ++u) {
        if (u >= L) continue;
        acc_add(acc, key_of(L, 0, pi, pj, u, 0), 2 * (int64_t)(nSi[u] + nSj[u]));
        acc_add(acc, key_of(L, 1, pi, pj, u, 0), 2 * (int64_t)nT[u]);
#pragma unroll
        for (int t = 0; t <= u; ++t) {
          // every per-edge quantity of a graph of at most 512 nodes fits 32 bits
          const int32_t Sit = nSi[t], Siu = nSi[u], Sjt = nSj[t], Sju = nSj[u], Tt = nT[t], Tu = nT[u];
          int32_t p4, p5, p9, p11;
          if (t == u) {
            p4 = Sit * Sjt;
            p5 = Sit * (Sit - 1) / 2 + Sjt * (Sjt - 1) / 2;
            p9 = Tt * (Sit + Sjt);
            p11 = Tt * (Tt - 1) / 2;
          } else {
            p4 = Sit * Sju + Siu * Sjt;
            p5 = Sit * Siu + Sjt * Sju;
            p9 = Tt * (Siu + Sju) + Tu * (Sit + Sjt);
            p11 = Tt * Tu;
          }
          acc_add(acc, key_of(L, 2, pi, pj, t, u), 2 * (int64_t)p4);
          acc_add(acc, key_of(L, 3, pi, pj, t, u), 2 * (int64_t)p5);
          acc_add(acc, key_of(L, 5, pi, pj, t, u), 2 * (int64_t)p9);
          acc_add(acc, key_of(L, 6, pi, pj, t, u), 2 * (int64_t)p11);
        }
      }
      // explicit orbits, one type t of k at a time
#pragma unroll 1
      for (int t = 0; t < L; ++t) {
        int32_t r3[TG_BATCH_LMAX], r6[TG_BATCH_LMAX], r7[TG_BATCH_LMAX], r8[TG_BATCH_LMAX], r10[TG_BATCH_LMAX],
            r12[TG_BATCH_LMAX];
#pragma unroll
        for (int u = 0; u < TG_BATCH_LMAX; ++u) r3[u] = r6[u] = r7[u] = r8[u] = r10[u] = r12[u] = 0;
        bool any = false;
#pragma unroll
        for (int w = 0; w < W_MAX; ++w) {
          const uint64_t m = type_word_mask(ts, t, w);
          uint64_t bits = (T[w] | Si[w] | Sj[w]) & m;
          while (bits) {
            const int b = __builtin_ctzll(bits);
            bits &= bits - 1;
            const int k = w * 64 + b;
            const uint64_t kb = 1ull << b;
            const int cls = (T[w] & kb) ? 0 : ((Si[w] & kb) ? 1 : 2);
            uint64_t ak[W_MAX];
#pragma unroll
            for (int q = 0; q < W_MAX; ++q) ak[q] = (q < W) ? S.adj[k][q] : 0ull;
#pragma unroll
            for (int u = 0; u < TG_BATCH_LMAX; ++u) {
              if (u >= L) continue;
              // k's neighbours of type u in T, S_i and S_j
              int32_t cT = 0, cSi = 0, cSj = 0;
#pragma unroll
              for (int q = 0; q < W_MAX; ++q) {
                const uint64_t mq = type_word_mask(ts, u, q);
                if (mq) {
                  const uint64_t a = ak[q] & mq;
                  cT += __popcll(a & T[q]);
                  cSi += __popcll(a & Si[q]);
                  cSj += __popcll(a & Sj[q]);
                }
              }
              const int32_t dku = S.deg_t[k][u];
              if (cls == 0) {
                const int32_t cI = dku - (pi == u) - (pj == u) - cT - cSi - cSj;
                r12[u] += cT;
                r10[u] += cSi + cSj;
                r8[u] += cI;
              } else if (cls == 1) {
                const int32_t cI = dku - (pi == u) - cT - cSi - cSj;
                r7[u] += cSi;
                r3[u] += cI;
              } else {
                const int32_t cI = dku - (pj == u) - cT - cSi - cSj;
                r7[u] += cSj;
                r6[u] += cSi;
                r3[u] += cI;
              }
            }
            any = true;
          }
        }
        if (!any) continue;
#pragma unroll
        for (int u = 0; u < TG_BATCH_LMAX; ++u) {
          if (u >= L) continue;
          // h3 = g3 + g4, g4 = p4 - g6; h4 = g5 = p5 - g7; h5 = g6;
          // h6 = g7 + g8 + g9, g9 = p9 - g10; h7 = g10 + g11, g11 = p11 - g12; h8 = g12
          acc_add(acc, key_of(L, 2, pi, pj, t, u), 2 * (int64_t)(r3[u] - r6[u]));
          acc_add(acc, key_of(L, 3, pi, pj, t, u), -(int64_t)r7[u]);
          acc_add(acc, key_of(L, 4, pi, pj, t, u), 2 * (int64_t)r6[u]);
          acc_add(acc, key_of(L, 5, pi, pj, t, u), (int64_t)r7[u] + 2 * (int64_t)(r8[u] - r10[u]));
          acc_add(acc, key_of(L, 6, pi, pj, t, u), 2 * (int64_t)r10[u] - r12[u]);
          acc_add(acc, key_of(L, 7, pi, pj, t, u), (int64_t)r12[u]);
        }
      }
    }
    bteam_sync<NWAVES>();
    // ---- Eq. 17 on the doubled sums
    uint64_t* out = A.out + A.key_off[g];
    for (int64_t k = tid; k < K; k += TSIZE) {
      const int h = k < 2 * C3 ? (int)(k / C3) : 2 + (int)((k - 2 * C3) / C4n);
      const uint64_t d = 2ull * (uint64_t)shape_edges[h];
      const uint64_t v = acc[k];
      if (v % d) atomicOr(A.flag, 1);
      out[k] = v / d;
    }
    bteam_sync<NWAVES>();
  }
}

// Size class of a graph: words per bit row.
// Argument checks per graph: size, L, key range.
__global__ void k_batch_classify(int64_t G, const int64_t* __restrict__ node_off, const uint8_t* __restrict__ Lg,
                                 const int64_t* __restrict__ key_off, int32_t* __restrict__ bad) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = node_off[g + 1] - node_off[g];
    const int L = Lg[g];
    if (n < 0 || n > 512) atomicOr(bad, 1);
    if (L < 1 || L > TG_BATCH_LMAX) { atomicOr(bad, 2); continue; }
    if (key_off[g + 1] - key_off[g] != 2 * c3(L + 2) + 6 * c4(L + 3)) atomicOr(bad, 4);
  }
}

// Queue order: largest graphs first inside each size class (coarse: by n / 8).
__global__ void k_batch_scatter(int64_t G, const int64_t* __restrict__ node_off, int32_t* __restrict__ cursor,
                                int32_t* __restrict__ list) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = min(max(node_off[g + 1] - node_off[g], (int64_t)0), (int64_t)512);
    const int W = (int)((n + 63) / 64);
    const int sub = 7 - (int)((n - 1 - (int64_t)(W > 0 ? (W - 1) * 64 : 0)) / 8);  // 0 = largest within the class
    list[atomicAdd(&cursor[W * 8 + (sub < 0 ? 0 : (sub > 7 ? 7 : sub))], 1)] = (int32_t)g;
  }
}

__global__ void k_batch_subcount(int64_t G, const int64_t* __restrict__ node_off, int32_t* __restrict__ counts) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = min(max(node_off[g + 1] - node_off[g], (int64_t)0), (int64_t)512);
    const int W = (int)((n + 63) / 64);
    const int sub = 7 - (int)((n - 1 - (int64_t)(W > 0 ? (W - 1) * 64 : 0)) / 8);
    atomicAdd(&counts[W * 8 + (sub < 0 ? 0 : (sub > 7 ? 7 : sub))], 1);
  }
}

// Optional input check (tg_options.validate), one wavefront per graph: row
// pointers from 0 to the graph's slot count and non-decreasing, types below
// L_g, column ids in [0, n_g) without self loops, rows strictly increasing,
// and every slot (u, v) mirrored by (v, u).  bad: bit 8 = a type >= L_g,
// bit 16 = a CSR violation.  Slots are only examined once the graph's row
// pointers have passed, so that every read stays inside the graph.
__global__ void __launch_bounds__(256) k_batch_validate(int64_t G, const int64_t* __restrict__ node_off,
                                                        const int64_t* __restrict__ slot_off,
                                                        const int32_t* __restrict__ rp_all,
                                                        const int32_t* __restrict__ ci_all,
                                                        const uint8_t* __restrict__ ty_all,
                                                        const uint8_t* __restrict__ Lg, int32_t* __restrict__ bad) {
  const int ln = lane();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TG_WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / TG_WAVE;
  for (int64_t g = wid; g < G; g += nw) {
    const int64_t n0 = node_off[g];
    const int64_t n = node_off[g + 1] - n0;
    const int64_t nnz = slot_off[g + 1] - slot_off[g];
    if (n < 0 || n > 512 || nnz < 0) continue;  // reported by k_batch_classify
    const int32_t* rp = rp_all + n0 + g;
    const int32_t* ci = ci_all + slot_off[g];
    const int L = Lg[g];
    bool rbad = false, tbad = false;
    for (int64_t v = ln; v <= n; v += TG_WAVE) {
      const int32_t r = rp[v];
      if (r < 0 || r > nnz || (v == 0 && r != 0) || (v == n && r != nnz) || (v > 0 && rp[v - 1] > r)) rbad = true;
      if (v < n && ty_all[n0 + v] >= L) tbad = true;
    }
    if (ballot(tbad) && ln == 0) atomicOr(bad, 8);
    if (ballot(rbad)) {
      if (ln == 0) atomicOr(bad, 16);
      continue;
    }
    bool sbad = false;
    for (int64_t q = ln; q < nnz; q += TG_WAVE) {
      int32_t lo = 0, hi = (int32_t)n;  // row u: the largest u with rp[u] <= q
      while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (rp[mid] <= q) lo = mid; else hi = mid;
      }
      const int32_t u = lo, v = ci[q];
      if (v < 0 || v >= n || v == u || (q > rp[u] && ci[q - 1] >= v)) { sbad = true; continue; }
      const int32_t p = lower_bound(ci + rp[v], rp[v + 1] - rp[v], u);
      if (p >= rp[v + 1] - rp[v] || ci[rp[v] + p] != u) sbad = true;
    }
    if (ballot(sbad) && ln == 0) atomicOr(bad, 16);
  }
}

__global__ void k_zero_i32(int32_t* p, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) p[q] = 0;
}

}  // namespace tg
