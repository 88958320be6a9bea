// gfx950 kernels for per-edge typed 3/4-node graphlet counting.
//
// Pipeline for one graph (see tg_api.hip for the host side):
//   prep     degree, typed degree D[v][t], canonical edge ids, slot->edge map,
//            degree-ordered out-lists (each edge kept at its lower endpoint)
//   tau      typed triangle counts per edge: tau_e[t] = |T_ij^t|
//   tables   per-node sums P[i][t][u] = sum_{k in Gamma_i^t} D[k][u] and
//            U[i][t][u] = sum_{k in Gamma_i^t} tau_(i,k)[u]
//   c4       non-induced typed 4-cycles through every edge, by degree-ordered
//            wedges (each 4-cycle found once, from its highest-ranked node)
//   combine  per edge: T_ij, sums over T of tau and D, typed edges inside T
//            (4-cliques), then every 4-node orbit by the identities recorded
//            in combine_edge(), Eqs. 7-10 and Eqs. 11-16; per-edge row and
//            global key accumulation
//   finalize divide global sums by the shape's edge count (Eq. 17)
//
// All counting is exact integer arithmetic; the order in which work items run
// never changes a result.

#include "tg_internal.h"

using namespace tg;

// ------------------------------------------------------------------ fills --

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = v;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = v;
}

// --------------------------------------------------------------- validate --

// Row pointers: rp[0] == 0, rp[n] == nnz, non-decreasing; types < L.
__global__ void k_validate_rows(int64_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                const uint8_t* __restrict__ ty, int L, int32_t* __restrict__ flags) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = rp[v];
    if (v == 0 && a != 0) atomicOr(&flags[0], TG_VFLAG_ROWPTR);
    if (v == n && (int64_t)a != nnz) atomicOr(&flags[0], TG_VFLAG_ROWPTR);
    if (v < n) {
      int32_t b = rp[v + 1];
      if (b < a || a < 0 || (int64_t)b > nnz) atomicOr(&flags[0], TG_VFLAG_ROWPTR);
      if (ty[v] >= L) atomicOr(&flags[0], TG_VFLAG_TYPE);
    }
  }
}

// Slots (row pointers already valid): ids in range, no self loop, strictly
// increasing rows.
__global__ void k_validate_slots(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 int32_t* __restrict__ flags) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t prev = -1;
    for (int32_t s = rp[v]; s < rp[v + 1]; ++s) {
      int32_t k = ci[s];
      if (k < 0 || (int64_t)k >= n) { atomicOr(&flags[0], TG_VFLAG_RANGE); break; }
      if (k == v) atomicOr(&flags[0], TG_VFLAG_SELFLOOP);
      if (k <= prev) atomicOr(&flags[0], TG_VFLAG_ORDER);
      prev = k;
    }
  }
}

// Symmetry (rows valid and sorted): (v, k) stored implies (k, v) stored.
__global__ void k_validate_symmetry(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    int32_t* __restrict__ flags) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    for (int32_t s = rp[v]; s < rp[v + 1]; ++s) {
      int32_t k = ci[s];
      int32_t len = rp[k + 1] - rp[k];
      int32_t p = lower_bound(ci + rp[k], len, (int32_t)v);
      if (p >= len || ci[rp[k] + p] != (int32_t)v) { atomicOr(&flags[0], TG_VFLAG_ASYMMETRIC); break; }
    }
  }
}

// ------------------------------------------------------------------- prep --

__global__ void k_degree(int64_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ deg) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    deg[v] = rp[v + 1] - rp[v];
}

// One wavefront per node v: typed degree, number of upper slots (k > v),
// out-degree in the degree order, wedge work W(v) = sum of d_u over
// neighbours u preceding v, and s(v) = sum of neighbour degrees.
__global__ void k_node_stats(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const int32_t* __restrict__ deg, const uint8_t* __restrict__ ty, int L,
                             uint32_t* __restrict__ D, int32_t* __restrict__ n_upper, int32_t* __restrict__ n_out,
                             uint64_t* __restrict__ wedge_work, uint64_t* __restrict__ nbr_deg_sum) {
  const int64_t v = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + threadIdx.x / TG_WAVE;
  if (v >= n) return;
  const int ln = lane();
  const int32_t dv = deg[v], base = rp[v];
  uint32_t my_t = 0;
  int32_t up = 0, out = 0;
  uint64_t wsum = 0, ssum = 0;
  for (int32_t b0 = 0; b0 < dv; b0 += TG_WAVE) {
    const bool valid = b0 + ln < dv;
    const int32_t k = valid ? ci[base + b0 + ln] : -1;
    const int32_t dk = valid ? deg[k] : 0;
    const int t = valid ? (int)ty[k] : -1;
    for (int tt = 0; tt < L; ++tt) {
      uint32_t c = (uint32_t)__popcll(ballot(t == tt));
      if (ln == tt) my_t += c;
    }
    up += __popcll(ballot(valid && k > (int32_t)v));
    out += __popcll(ballot(valid && precedes(dv, (int32_t)v, dk, k)));
    wsum += (valid && precedes(dk, k, dv, (int32_t)v)) ? (uint64_t)dk : 0ull;
    ssum += (uint64_t)dk;
  }
  wsum = wave_sum_u64(wsum);
  ssum = wave_sum_u64(ssum);
  if (ln < L) D[v * L + ln] = my_t;
  if (ln == 0) {
    n_upper[v] = up;
    n_out[v] = out;
    wedge_work[v] = wsum;
    nbr_deg_sum[v] = ssum;
  }
}

// Exclusive scan of int32 counts into int32 offsets (offsets[n] = total), in
// three passes over blocks of 1024.
__global__ void k_scan_blocks(int64_t n, const int32_t* __restrict__ in, int32_t* __restrict__ out,
                              int32_t* __restrict__ block_sums) {
  __shared__ int32_t s[1024];
  const int64_t base = (int64_t)blockIdx.x * 1024;
  for (int q = threadIdx.x; q < 1024; q += blockDim.x) s[q] = (base + q < n) ? in[base + q] : 0;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t add[4];
    for (int r = 0; r < 4; ++r) {
      int q = threadIdx.x + r * 256;
      add[r] = (q >= off) ? s[q - off] : 0;
    }
    __syncthreads();
    for (int r = 0; r < 4; ++r) s[threadIdx.x + r * 256] += add[r];
    __syncthreads();
  }
  for (int q = threadIdx.x; q < 1024; q += blockDim.x)
    if (base + q < n) out[base + q] = (q > 0) ? s[q - 1] : 0;
  if (threadIdx.x == 0) block_sums[blockIdx.x] = s[1023];
}

__global__ void k_scan_sums(int64_t nblocks, int32_t* __restrict__ block_sums, int32_t* __restrict__ total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t acc = 0;
  for (int64_t b = 0; b < nblocks; ++b) {
    int32_t x = block_sums[b];
    block_sums[b] = acc;
    acc += x;
  }
  *total = acc;
}

__global__ void k_scan_add(int64_t n, int32_t* __restrict__ out, const int32_t* __restrict__ block_sums,
                           const int32_t* __restrict__ total) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (int64_t)gridDim.x * blockDim.x) {
    if (x == n) out[n] = *total;
    else out[x] += block_sums[x / 1024];
  }
}

// One wavefront per node v: canonical edge ids of its upper slots, the
// slot->edge map for every slot, and the degree-ordered out-list.
__global__ void k_fill_edges(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const int32_t* __restrict__ deg, const int32_t* __restrict__ n_upper,
                             const int32_t* __restrict__ upper_off, const int32_t* __restrict__ out_off,
                             int32_t* __restrict__ ei, int32_t* __restrict__ ej, int32_t* __restrict__ s2e,
                             int32_t* __restrict__ out_col) {
  const int64_t v = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + threadIdx.x / TG_WAVE;
  if (v >= n) return;
  const int ln = lane();
  const int32_t dv = deg[v], base = rp[v];
  const int32_t first_up = rp[v + 1] - n_upper[v];
  int32_t acc = 0;
  for (int32_t b0 = 0; b0 < dv; b0 += TG_WAVE) {
    const bool valid = b0 + ln < dv;
    const int32_t s = base + b0 + ln;
    const int32_t k = valid ? ci[s] : -1;
    const int32_t dk = valid ? deg[k] : 0;
    if (valid) {
      if (k > (int32_t)v) {
        const int32_t e = upper_off[v] + (s - first_up);
        ei[e] = (int32_t)v;
        ej[e] = k;
        s2e[s] = e;
      } else {
        const int32_t p = rp[k] + lower_bound(ci + rp[k], dk, (int32_t)v);
        s2e[s] = upper_off[k] + (p - (rp[k + 1] - n_upper[k]));
      }
    }
    const bool hi = valid && precedes(dv, (int32_t)v, dk, k);
    const uint64_t mask = ballot(hi);
    if (hi) out_col[out_off[v] + acc + lanes_below(mask)] = k;
    acc += __popcll(mask);
  }
}

// -------------------------------------------------------------------- tau --

// One wavefront per edge: tau_e[t] = |Gamma_i^t intersect Gamma_j^t| by
// binary search of the shorter row's ids in the longer row.
__global__ void k_tau(int64_t count, const int32_t* __restrict__ list, const int32_t* __restrict__ ei,
                      const int32_t* __restrict__ ej, const int32_t* __restrict__ rp,
                      const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                      const uint8_t* __restrict__ ty, int L, uint32_t* __restrict__ tau) {
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + threadIdx.x / TG_WAVE;
  if (w >= count) return;
  const int ln = lane();
  const int32_t e = list ? list[w] : (int32_t)w;
  const int32_t i = ei[e], j = ej[e];
  const bool ia = deg[i] <= deg[j];
  const int32_t a = ia ? i : j, b = ia ? j : i;
  const int32_t la = deg[a], lb = deg[b];
  const int32_t* pa = ci + rp[a];
  const int32_t* pb = ci + rp[b];
  uint32_t my_t = 0;
  for (int32_t b0 = 0; b0 < la; b0 += TG_WAVE) {
    const bool valid = b0 + ln < la;
    int t = -1;
    if (valid) {
      const int32_t k = pa[b0 + ln];
      const int32_t p = lower_bound(pb, lb, k);
      if (p < lb && pb[p] == k) t = ty[k];
    }
    for (int tt = 0; tt < L; ++tt) {
      uint32_t c = (uint32_t)__popcll(ballot(t == tt));
      if (ln == tt) my_t += c;
    }
  }
  if (ln < L) tau[(int64_t)e * L + ln] = my_t;
}

// ----------------------------------------------------------------- tables --

// One wavefront per node i: P[i][t][u] and U[i][t][u].
__global__ void k_node_tables(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const uint8_t* __restrict__ ty, int L, const uint32_t* __restrict__ D,
                              const uint32_t* __restrict__ tau, const int32_t* __restrict__ s2e,
                              uint64_t* __restrict__ Pn, uint64_t* __restrict__ Un) {
  extern __shared__ uint64_t lds_tables[];
  const int wv = threadIdx.x / TG_WAVE;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + wv;
  const int ln = lane();
  const int LL = L * L;
  uint64_t* Pa = lds_tables + (int64_t)wv * 2 * LL;
  uint64_t* Ua = Pa + LL;
  for (int x = ln; x < 2 * LL; x += TG_WAVE) Pa[x] = 0;
  wave_sync();
  if (i >= n) return;
  const int32_t base = rp[i], d = rp[i + 1] - base;
  for (int32_t b0 = 0; b0 < d; b0 += TG_WAVE) {
    if (b0 + ln < d) {
      const int32_t s = base + b0 + ln;
      const int32_t k = ci[s];
      const int t = ty[k];
      const int64_t e = s2e[s];
      for (int u = 0; u < L; ++u) {
        const uint32_t dv = D[(int64_t)k * L + u];
        if (dv) atomicAdd((unsigned long long*)&Pa[t * L + u], (unsigned long long)dv);
        const uint32_t tv = tau[e * L + u];
        if (tv) atomicAdd((unsigned long long*)&Ua[t * L + u], (unsigned long long)tv);
      }
    }
  }
  wave_sync();
  for (int x = ln; x < LL; x += TG_WAVE) {
    Pn[i * LL + x] = Pa[x];
    Un[i * LL + x] = Ua[x];
  }
}

// ------------------------------------------------------------- 4-cycles --
//
// A 4-cycle x-u-w-u'-x is found once: from its highest-ranked node x (degree
// order), as two wedges x-u-w and x-u'-w whose middles u, u' and far end w all
// precede x.  With c_t(x, w) = number of middles of type t between x and w,
// the wedge x-u-w lies on c_t - [phi_u = t] cycles whose fourth node has type
// t; each such cycle is credited to edge (x, u) with other-node types
// {phi_w, t} and to edge (u, w) with {phi_x, t}.  Every edge of every 4-cycle
// is credited exactly once.  The counts are non-induced: a diamond adds one
// cycle to each rim edge and a 4-clique two to each edge.

__device__ __forceinline__ uint32_t hash_home(int32_t key, int log2cap) {
  return ((uint32_t)key * 2654435761u) >> (32 - log2cap);
}

__device__ __forceinline__ int hash_insert(int32_t* keys, int log2cap, int32_t key) {
  const uint32_t mask = (1u << log2cap) - 1;
  uint32_t h = hash_home(key, log2cap);
  for (;;) {
    const int32_t old = atomicCAS(&keys[h], -1, key);
    if (old == -1 || old == key) return (int)h;
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int hash_find(const int32_t* keys, int log2cap, int32_t key) {
  const uint32_t mask = (1u << log2cap) - 1;
  uint32_t h = hash_home(key, log2cap);
  for (;;) {
    const int32_t k = keys[h];
    if (k == key) return (int)h;
    if (k == -1) return -1;
    h = (h + 1) & mask;
  }
}

template <int NWAVES>
__device__ __forceinline__ void team_sync() {
  if (NWAVES == 1) wave_sync();
  else __syncthreads();
}

// Credits the cycles through wedge x-u-w (slots sxu of x's row and suw of
// u's row) given the typed middle counts between x and w.
__device__ __forceinline__ void credit_wedge(uint64_t* __restrict__ C4, int L, int P, int32_t e_xu, int32_t e_uw,
                                             int phx, int phu, int phw, int t, uint32_t cnt_t) {
  const int64_t c = (int64_t)cnt_t - (t == phu ? 1 : 0);
  if (c > 0) {
    atomicAdd((unsigned long long*)&C4[(int64_t)e_xu * P + pair_index(phw, t)], (unsigned long long)c);
    atomicAdd((unsigned long long*)&C4[(int64_t)e_uw * P + pair_index(phx, t)], (unsigned long long)c);
  }
}

// One team (NWAVES wavefronts) per node x, middle counts in LDS hash tables:
// kw/tw keyed by w (totals), kt/ct keyed by w*L+t (typed counts).
template <int NWAVES, int LOG2CAP>
__global__ void __launch_bounds__(256) k_c4_hash(int64_t count, const int32_t* __restrict__ list,
                                                 const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const int32_t* __restrict__ deg, const uint8_t* __restrict__ ty,
                                                 int L, const int32_t* __restrict__ s2e,
                                                 uint64_t* __restrict__ C4) {
  constexpr int CAP = 1 << LOG2CAP;
  constexpr int TEAMS = 4 / NWAVES;
  __shared__ int32_t kw_all[TEAMS][CAP];
  __shared__ uint32_t tw_all[TEAMS][CAP];
  __shared__ int32_t kt_all[TEAMS][CAP];
  __shared__ uint32_t ct_all[TEAMS][CAP];
  const int team = threadIdx.x / (NWAVES * TG_WAVE);
  const int tid = threadIdx.x % (NWAVES * TG_WAVE);
  const int wv = tid / TG_WAVE, ln = lane();
  int32_t* kw = kw_all[team];
  uint32_t* tw = tw_all[team];
  int32_t* kt = kt_all[team];
  uint32_t* ct = ct_all[team];
  const int P = L * (L + 1) / 2;
  for (int64_t item = (int64_t)blockIdx.x * TEAMS + team; item < count; item += (int64_t)gridDim.x * TEAMS) {
    for (int q = tid; q < CAP; q += NWAVES * TG_WAVE) { kw[q] = -1; tw[q] = 0; kt[q] = -1; ct[q] = 0; }
    team_sync<NWAVES>();
    const int32_t x = list[item];
    const int32_t dx = deg[x], bx = rp[x];
    const int phx = ty[x];
    for (int pass = 0; pass < 2; ++pass) {
      for (int32_t q = wv; q < dx; q += NWAVES) {
        const int32_t u = ci[bx + q];
        const int32_t du = deg[u];
        if (!precedes(du, u, dx, x)) continue;
        const int phu = ty[u];
        const int32_t bu = rp[u];
        for (int32_t b0 = 0; b0 < du; b0 += TG_WAVE) {
          if (b0 + ln >= du) continue;
          const int32_t w = ci[bu + b0 + ln];
          if (!precedes(deg[w], w, dx, x)) continue;
          if (pass == 0) {
            const int h = hash_insert(kw, LOG2CAP, w);
            atomicAdd(&tw[h], 1u);
            const int g = hash_insert(kt, LOG2CAP, w * L + phu);
            atomicAdd(&ct[g], 1u);
          } else {
            const int h = hash_find(kw, LOG2CAP, w);
            if (tw[h] < 2) continue;
            const int32_t e_xu = s2e[bx + q], e_uw = s2e[bu + b0 + ln];
            const int phw = ty[w];
            for (int t = 0; t < L; ++t) {
              const int g = hash_find(kt, LOG2CAP, w * L + t);
              credit_wedge(C4, L, P, e_xu, e_uw, phx, phu, phw, t, g >= 0 ? ct[g] : 0u);
            }
          }
        }
      }
      team_sync<NWAVES>();
    }
  }
}

// Nodes with large wedge work: a group of nodes at a time, each with a dense
// per-node array of typed middle counts cnt[w * CS + t] (CS = 8 for L <= 8,
// else 16: one aligned row per far end w) in global memory.  Phase 0 counts,
// phase 1 credits, phase 2 clears; kernel boundaries order the phases.
//
// Work mapping: wavefront q takes 64 consecutive (node, slot) pairs of the
// group's rows; the pairs whose middle u precedes x contribute d_u wedges,
// and the wavefront's wedges are dealt to lanes 64 at a time through a
// wavefront prefix sum, so that lanes stay busy whatever the degrees.
__device__ __forceinline__ int32_t wave_excl_scan(int32_t v, int32_t* total) {
  const int ln = lane();
  int32_t x = v;
  for (int off = 1; off < TG_WAVE; off <<= 1) {
    const int32_t y = __shfl_up(x, off, TG_WAVE);
    if (ln >= off) x += y;
  }
  *total = __shfl(x, TG_WAVE - 1, TG_WAVE);
  return x - v;
}

__global__ void __launch_bounds__(256) k_c4_group(int phase, int G, const int32_t* __restrict__ gx,
                                                  const int64_t* __restrict__ gpref, uint32_t* __restrict__ dense,
                                                  int64_t stride, int CS, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                                                  const uint8_t* __restrict__ ty, int L,
                                                  const int32_t* __restrict__ s2e, uint64_t* __restrict__ C4) {
  const int64_t wq = (int64_t)blockIdx.x * (blockDim.x / TG_WAVE) + threadIdx.x / TG_WAVE;
  const int64_t total_slots = gpref[G];
  const int64_t s0 = wq * TG_WAVE;
  if (s0 >= total_slots) return;
  const int ln = lane();
  const int P = L * (L + 1) / 2;
  // this lane's (node, slot) pair
  const int64_t sl = s0 + ln;
  int g = 0;
  int32_t x = 0, dx = 0, u = 0, bu = 0, cu = 0, e_xu = 0;
  int phx = 0, phu = 0;
  if (sl < total_slots) {
    int lo = 0, hi = G;  // largest g with gpref[g] <= sl
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (gpref[mid] <= sl) lo = mid; else hi = mid;
    }
    g = lo;
    x = gx[g];
    dx = deg[x];
    const int32_t sx = rp[x] + (int32_t)(sl - gpref[g]);
    u = ci[sx];
    const int32_t du = deg[u];
    if (precedes(du, u, dx, x)) {
      cu = du;
      bu = rp[u];
      phx = ty[x];
      phu = ty[u];
      e_xu = s2e[sx];
    }
  }
  int32_t tot = 0;
  const int32_t excl = wave_excl_scan(cu, &tot);
  for (int32_t c0 = 0; c0 < tot; c0 += TG_WAVE) {
    const int32_t v = c0 + ln;
    // owner lane: the largest l with excl[l] <= v (excl is non-decreasing)
    int o = 0;
    for (int step = 32; step > 0; step >>= 1) {
      const int32_t ex = __shfl(excl, o + step, TG_WAVE);
      if (o + step < TG_WAVE && ex <= v) o += step;
    }
    const int32_t o_excl = __shfl(excl, o, TG_WAVE);
    const int32_t o_bu = __shfl(bu, o, TG_WAVE);
    const int32_t o_x = __shfl(x, o, TG_WAVE);
    const int32_t o_dx = __shfl(dx, o, TG_WAVE);
    const int o_g = __shfl(g, o, TG_WAVE);
    const int o_phx = __shfl(phx, o, TG_WAVE);
    const int o_phu = __shfl(phu, o, TG_WAVE);
    const int32_t o_exu = __shfl(e_xu, o, TG_WAVE);
    if (v >= tot) continue;
    const int32_t suw = o_bu + (v - o_excl);
    const int32_t w = ci[suw];
    if (!precedes(deg[w], w, o_dx, o_x)) continue;
    uint32_t* row = dense + (int64_t)o_g * stride + (int64_t)w * CS;
    if (phase == 0) {
      atomicAdd(&row[o_phu], 1u);
    } else if (phase == 1) {
      uint32_t c[16];
      uint32_t sum = 0;
      for (int t = 0; t < L; ++t) { c[t] = row[t]; sum += c[t]; }
      if (sum < 2) continue;
      const int32_t e_uw = s2e[suw];
      const int phw = ty[w];
      for (int t = 0; t < L; ++t) credit_wedge(C4, L, P, o_exu, e_uw, o_phx, o_phu, phw, t, c[t]);
    } else {
      for (int t = 0; t < L; ++t) row[t] = 0u;
    }
  }
}

// ------------------------------------------------------------- combine --
//
// Per edge (i, j), with T = T_ij, S_i, S_j, I as in Section 4 and ordered
// typed pair counts E(X^t, Y^u) = #{(k, r): k in X of type t, r in Y of type
// u, k ~ r}:
//   A_i[t][u] = sum_{k in T^t} tau_(i,k)[u],  A_j likewise,
//   Q[t][u]   = sum_{k in T^t} D[k][u],
//   Mu[t][u]  = edges {k, r} inside T with k preceding r, typed (phi_k, phi_r),
//   M(t,u)    = Mu[t][u] + Mu[u][t] = E(T^t, T^u).
// Every neighbour of k in T is i, j, or in T, S_i, S_j or I, and every
// neighbour of k in S_i is i or in T, S_i, S_j or I.  Hence
//   E(T^t, S_i^u) = A_i[t][u] - |T^t| [phi_j = u] - M(t,u)
//   E(T^t, I^u)   = Q[t][u] - |T^t| ([phi_i=u] + [phi_j=u]) - M - E(T,S_i) - E(T,S_j)
//   E(S_i^t, S_i^u) = U[i][t][u] - [phi_j=t] |T^u| - A_i[t][u] - E(T^u, S_i^t)
//   E(S_i^t, I^u) = P[i][t][u] - [phi_j=t] D[j][u] - Q[t][u] - |S_i^t| [phi_i=u]
//                   - E(T^u, S_i^t) - E(S_i^t, S_i^u) - E(S_i^t, S_j^u)
// and the non-induced 4-cycle count through (i, j) is g6 + g10 + 2 g12.  With
// sym(X){t,u} = X[t][u] + X[u][t] (t != u) or X[t][t], the explicit orbits of
// Algorithms 2-3 are
//   g12 = sym(Mu), g10 = sym(E(T,S_i) + E(T,S_j)), g8 = sym(E(T,I)),
//   g7 = (sym(E(S_i,S_i)) + sym(E(S_j,S_j))) / 2, g6 = C4 - g10 - 2 g12,
//   g3 = sym(E(S_i,I) + E(S_j,I)),
// then g4, g5, g9, g11 follow from Eqs. 7-10 and the graphlets from Eqs. 11-16.

template <int NWAVES>
__device__ __forceinline__ void combine_edge(const EdgeArgs& A, int32_t e, int32_t* Tid, uint8_t* Tty,
                                             uint64_t* __restrict__ acc, uint64_t* gacc, int32_t* s_cnt, int tid) {
  const int L = A.L, LL = L * L, P = L * (L + 1) / 2;
  const int R = 2 * L + 6 * P;
  uint64_t* Aa = acc;
  uint64_t* Ab = acc + LL;
  uint64_t* Q = acc + 2 * LL;
  uint64_t* Mu = acc + 3 * LL;
  for (int x = tid; x < 4 * LL; x += NWAVES * TG_WAVE) acc[x] = 0;
  team_sync<NWAVES>();
  const int32_t i = A.ei[e], j = A.ej[e];
  const int32_t di = A.deg[i], dj = A.deg[j];
  const bool a_is_i = di <= dj;
  const int32_t a = a_is_i ? i : j, b = a_is_i ? j : i;
  const int32_t la = a_is_i ? di : dj, lb = a_is_i ? dj : di;
  const int32_t ra = A.rp[a], rb = A.rp[b];
  const int wv = tid / TG_WAVE, ln = lane();

  // T_ij with the sums of tau and D over its members
  int32_t nT = 0;
  for (int32_t b0 = 0; b0 < la; b0 += NWAVES * TG_WAVE) {
    const int32_t idx = b0 + tid;
    bool found = false;
    int32_t k = 0, p = 0;
    if (idx < la) {
      k = A.ci[ra + idx];
      p = lower_bound(A.ci + rb, lb, k);
      found = p < lb && A.ci[rb + p] == k;
    }
    int t = 0;
    if (found) {
      t = A.ty[k];
      const int64_t ea = A.s2e[ra + idx], eb = A.s2e[rb + p];
      for (int u = 0; u < L; ++u) {
        const uint32_t va = A.tau[ea * L + u];
        if (va) atomicAdd((unsigned long long*)&Aa[t * L + u], (unsigned long long)va);
        const uint32_t vb = A.tau[eb * L + u];
        if (vb) atomicAdd((unsigned long long*)&Ab[t * L + u], (unsigned long long)vb);
        const uint32_t vd = A.D[(int64_t)k * L + u];
        if (vd) atomicAdd((unsigned long long*)&Q[t * L + u], (unsigned long long)vd);
      }
    }
    const uint64_t mask = ballot(found);
    int32_t before = 0, total = __popcll(mask);
    if (NWAVES > 1) {
      if (ln == 0) s_cnt[wv] = total;
      __syncthreads();
      total = 0;
      for (int q = 0; q < NWAVES; ++q) {
        const int32_t c = s_cnt[q];
        if (q < wv) before += c;
        total += c;
      }
      __syncthreads();
    }
    if (found) {
      const int32_t pos = nT + before + lanes_below(mask);
      Tid[pos] = k;
      Tty[pos] = (uint8_t)t;
    }
    nT += total;
  }
  team_sync<NWAVES>();

  // instrumented work: probes of the intersection, gathers per member of T,
  // out-list elements scanned, epilogue entries
  uint64_t my_work = 0;
  if (A.work && wv == 0)
    my_work = (uint64_t)la * (uint64_t)(1 + (lb > 0 ? 32 - __clz(lb) : 0)) + (uint64_t)nT * 3u * (uint64_t)L +
              (uint64_t)(P + L);

  // typed edges inside T (4-cliques through (i, j)), each from its lower end
  for (int32_t q = wv; q < nT; q += NWAVES) {
    const int32_t k = Tid[q];
    const int tk = Tty[q];
    const int32_t o0 = A.out_off[k], o1 = A.out_off[k + 1];
    my_work += (uint64_t)(1 + o1 - o0);
    for (int32_t c0 = o0; c0 < o1; c0 += TG_WAVE) {
      if (c0 + ln < o1) {
        const int32_t r = A.out_col[c0 + ln];
        const int32_t pp = lower_bound(Tid, nT, r);
        if (pp < nT && Tid[pp] == r) atomicAdd((unsigned long long*)&Mu[tk * L + Tty[pp]], 1ull);
      }
    }
  }
  if (A.work && ln == 0 && my_work) atomicAdd((unsigned long long*)&A.work[e], (unsigned long long)my_work);
  team_sync<NWAVES>();

  // per type pair: every orbit, then every graphlet
  const int pi = A.ty[i], pj = A.ty[j];
  const uint64_t* Ai = a_is_i ? Aa : Ab;
  const uint64_t* Aj = a_is_i ? Ab : Aa;
  const uint32_t* tau_e = A.tau + (int64_t)e * L;
  const uint32_t* Di = A.D + (int64_t)i * L;
  const uint32_t* Dj = A.D + (int64_t)j * L;
  const uint64_t* Ui = A.Un + (int64_t)i * LL;
  const uint64_t* Uj = A.Un + (int64_t)j * LL;
  const uint64_t* Pi = A.Pn + (int64_t)i * LL;
  const uint64_t* Pj = A.Pn + (int64_t)j * LL;
  uint64_t* row = (A.edge_counts && e >= A.edge_begin && e < A.edge_end)
                      ? A.edge_counts + (int64_t)(e - A.edge_begin) * R : nullptr;
  auto gadd = [&](int64_t key, int64_t v) {
    if (v == 0) return;
    if (gacc) atomicAdd((unsigned long long*)&gacc[key], (unsigned long long)v);
    else atomicAdd((unsigned long long*)&A.global_sums[key], (unsigned long long)v);
  };
  auto Tn = [&](int x) -> int64_t { return (int64_t)tau_e[x]; };
  auto Si = [&](int x) -> int64_t { return (int64_t)Di[x] - tau_e[x] - (pj == x ? 1 : 0); };
  auto Sj = [&](int x) -> int64_t { return (int64_t)Dj[x] - tau_e[x] - (pi == x ? 1 : 0); };
  for (int c = tid; c < L; c += NWAVES * TG_WAVE) {
    const int64_t wedge = Si(c) + Sj(c), tri = Tn(c);
    if (row) { row[c] = (uint64_t)wedge; row[L + c] = (uint64_t)tri; }
    gadd(key_of(L, 0, pi, pj, c, 0), wedge);
    gadd(key_of(L, 1, pi, pj, c, 0), tri);
  }
  for (int p = tid; p < P; p += NWAVES * TG_WAVE) {
    int u = 0;
    while ((u + 1) * (u + 2) / 2 <= p) ++u;
    const int t = p - u * (u + 1) / 2;
    auto sym = [&](auto f) -> int64_t { return t == u ? f(t, t) : f(t, u) + f(u, t); };
    auto M = [&](int x, int y) -> int64_t { return (int64_t)(Mu[x * L + y] + Mu[y * L + x]); };
    auto ETSi = [&](int x, int y) -> int64_t { return (int64_t)Ai[x * L + y] - Tn(x) * (pj == y) - M(x, y); };
    auto ETSj = [&](int x, int y) -> int64_t { return (int64_t)Aj[x * L + y] - Tn(x) * (pi == y) - M(x, y); };
    auto ETI = [&](int x, int y) -> int64_t {
      return (int64_t)Q[x * L + y] - Tn(x) * ((pi == y) + (pj == y)) - M(x, y) - ETSi(x, y) - ETSj(x, y);
    };
    const int64_t g12 = sym([&](int x, int y) -> int64_t { return (int64_t)Mu[x * L + y]; });
    const int64_t g10 = sym(ETSi) + sym(ETSj);
    const int64_t g8 = sym(ETI);
    const int64_t sSiSi = sym([&](int x, int y) -> int64_t { return (int64_t)Ui[x * L + y]; })
                        - sym([&](int x, int y) -> int64_t { return (pj == x) ? Tn(y) : 0; })
                        - sym([&](int x, int y) -> int64_t { return (int64_t)Ai[x * L + y]; }) - sym(ETSi);
    const int64_t sSjSj = sym([&](int x, int y) -> int64_t { return (int64_t)Uj[x * L + y]; })
                        - sym([&](int x, int y) -> int64_t { return (pi == x) ? Tn(y) : 0; })
                        - sym([&](int x, int y) -> int64_t { return (int64_t)Aj[x * L + y]; }) - sym(ETSj);
    const int64_t g7 = (sSiSi + sSjSj) / 2;
    const int64_t g6 = (int64_t)A.C4[(int64_t)e * P + p] - g10 - 2 * g12;
    const int64_t g3 = sym([&](int x, int y) -> int64_t { return (int64_t)Pi[x * L + y]; })
                     + sym([&](int x, int y) -> int64_t { return (int64_t)Pj[x * L + y]; })
                     - sym([&](int x, int y) -> int64_t { return (pj == x) ? (int64_t)Dj[y] : 0; })
                     - sym([&](int x, int y) -> int64_t { return (pi == x) ? (int64_t)Di[y] : 0; })
                     - 2 * sym([&](int x, int y) -> int64_t { return (int64_t)Q[x * L + y]; })
                     - sym([&](int x, int y) -> int64_t { return (pi == y) ? Si(x) : 0; })
                     - sym([&](int x, int y) -> int64_t { return (pj == y) ? Sj(x) : 0; })
                     - g10 - sSiSi - sSjSj - 2 * g6;
    int64_t g4, g5, g9, g11;
    if (t == u) {
      g4 = Si(t) * Sj(t) - g6;                         // Eq. 7
      g5 = c2(Si(t)) + c2(Sj(t)) - g7;                 // Eq. 8
      g9 = Tn(t) * (Si(t) + Sj(t)) - g10;              // Eq. 9
      g11 = c2(Tn(t)) - g12;                           // Eq. 10
    } else {
      g4 = Si(t) * Sj(u) + Si(u) * Sj(t) - g6;
      g5 = Si(t) * Si(u) + Sj(t) * Sj(u) - g7;
      g9 = Tn(t) * (Si(u) + Sj(u)) + Tn(u) * (Si(t) + Sj(t)) - g10;
      g11 = Tn(t) * Tn(u) - g12;
    }
    const int64_t h[6] = {g3 + g4, g5, g6, g7 + g8 + g9, g10 + g11, g12};  // Eqs. 11-16
    for (int s = 0; s < 6; ++s) {
      if (row) row[2 * L + s * P + p] = (uint64_t)h[s];
      gadd(key_of(L, 2 + s, pi, pj, t, u), h[s]);
    }
  }
  team_sync<NWAVES>();
}

// One wavefront per edge (|T_ij| <= TG_T_WAVE_CAP), grid-stride over a list.
__global__ void __launch_bounds__(256) k_combine_wave(EdgeArgs A, int64_t count, const int32_t* __restrict__ list,
                                                      int nkeys) {
  extern __shared__ uint64_t smem_cw[];
  const int LL = A.L * A.L;
  uint64_t* gacc = A.gacc_in_lds ? smem_cw : nullptr;
  const int koff = A.gacc_in_lds ? nkeys : 0;
  const int wv = threadIdx.x / TG_WAVE;
  uint64_t* acc = smem_cw + koff + (int64_t)wv * 4 * LL;
  int32_t* Tid = (int32_t*)(smem_cw + koff + 4 * 4 * LL) + wv * TG_T_WAVE_CAP;
  uint8_t* Tty = (uint8_t*)((int32_t*)(smem_cw + koff + 4 * 4 * LL) + 4 * TG_T_WAVE_CAP) + wv * TG_T_WAVE_CAP;
  if (gacc) {
    for (int x = threadIdx.x; x < nkeys; x += blockDim.x) gacc[x] = 0;
  }
  __syncthreads();
  for (int64_t w = (int64_t)blockIdx.x * 4 + wv; w < count; w += (int64_t)gridDim.x * 4)
    combine_edge<1>(A, list[w], Tid, Tty, acc, gacc, nullptr, threadIdx.x % TG_WAVE);
  __syncthreads();
  if (gacc) {
    for (int x = threadIdx.x; x < nkeys; x += blockDim.x)
      if (gacc[x]) atomicAdd((unsigned long long*)&A.global_sums[x], (unsigned long long)gacc[x]);
  }
}

// One workgroup per edge, grid-stride over a list; T_ij in LDS when it fits,
// else in this workgroup's slice of a global scratch.
__global__ void __launch_bounds__(256) k_combine_wg(EdgeArgs A, int64_t count, const int32_t* __restrict__ list,
                                                    int nkeys, int32_t* __restrict__ t_over, int64_t t_over_cap) {
  extern __shared__ uint64_t smem_cg[];
  const int LL = A.L * A.L;
  uint64_t* gacc = A.gacc_in_lds ? smem_cg : nullptr;
  const int koff = A.gacc_in_lds ? nkeys : 0;
  uint64_t* acc = smem_cg + koff;
  int32_t* s_cnt = (int32_t*)(smem_cg + koff + 4 * LL);
  int32_t* Tid_l = s_cnt + 4;
  uint8_t* Tty_l = (uint8_t*)(Tid_l + TG_T_WG_CAP);
  int32_t* Tid_g = t_over ? t_over + (int64_t)blockIdx.x * t_over_cap : nullptr;
  uint8_t* Tty_g = t_over ? (uint8_t*)(t_over + (int64_t)gridDim.x * t_over_cap) + (int64_t)blockIdx.x * t_over_cap
                          : nullptr;
  if (gacc) {
    for (int x = threadIdx.x; x < nkeys; x += blockDim.x) gacc[x] = 0;
  }
  __syncthreads();
  for (int64_t w = blockIdx.x; w < count; w += gridDim.x) {
    const int32_t e = list[w];
    uint32_t tsum = 0;
    for (int t = 0; t < A.L; ++t) tsum += A.tau[(int64_t)e * A.L + t];
    const bool big = tsum > TG_T_WG_CAP;
    combine_edge<4>(A, e, big ? Tid_g : Tid_l, big ? Tty_g : Tty_l, acc, gacc, s_cnt, threadIdx.x);
  }
  __syncthreads();
  if (gacc) {
    for (int x = threadIdx.x; x < nkeys; x += blockDim.x)
      if (gacc[x]) atomicAdd((unsigned long long*)&A.global_sums[x], (unsigned long long)gacc[x]);
  }
}

// ------------------------------------------------------------- schedule --

// Edge class (0: one wavefront, 1: one workgroup) and cost bucket (0 = most
// expensive).  cost: 0 none, 1 degree product, 2 given per-edge cost.
struct BinParams {
  int mode;              // 0 none, 1 degree product, 2 predicted log2 cost
  int heavy_min_degree;  // min(d_i, d_j) above this: workgroup
  int heavy_log2_cost;   // floor(log2 cost) above this: workgroup
};

__device__ __forceinline__ void edge_bin(int32_t e, const int32_t* ei, const int32_t* ej, const int32_t* deg,
                                         const uint32_t* tau, int L, BinParams bp, const float* pred, int* cls,
                                         int* bucket, uint32_t* tsum_out) {
  const int32_t i = ei[e], j = ej[e];
  const int32_t di = deg[i], dj = deg[j];
  uint32_t tsum = 0;
  for (int t = 0; t < L; ++t) tsum += tau[(int64_t)e * L + t];
  *tsum_out = tsum;
  int heavy = (tsum > TG_T_WAVE_CAP || min(di, dj) > bp.heavy_min_degree) ? 1 : 0;
  if (bp.mode == 0) { *cls = heavy; *bucket = 0; return; }
  double c;
  if (bp.mode == 1) c = (double)di * (double)dj;
  else c = exp2((double)pred[e]);
  int lg = (int)floor(log2(c + 1.0));
  lg = lg < 0 ? 0 : (lg > 63 ? 63 : lg);
  if (lg > bp.heavy_log2_cost) heavy = 1;
  *cls = heavy;
  *bucket = 63 - lg;
}

// Bin counts and scatter use a per-workgroup LDS histogram so that global
// atomics are one per (workgroup tile, bin) rather than one per item.
__global__ void __launch_bounds__(256) k_edge_bin_count(int64_t m, const int32_t* __restrict__ ei,
                                                        const int32_t* __restrict__ ej,
                                                        const int32_t* __restrict__ deg,
                                                        const uint32_t* __restrict__ tau, int L, BinParams bp,
                                                        const float* __restrict__ pred, int32_t* __restrict__ counts,
                                                        uint32_t* __restrict__ max_t_heavy) {
  __shared__ int32_t h[128];
  __shared__ uint32_t tmax;
  for (int q = threadIdx.x; q < 128; q += blockDim.x) h[q] = 0;
  if (threadIdx.x == 0) tmax = 0;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int cls, bucket;
    uint32_t tsum;
    edge_bin((int32_t)e, ei, ej, deg, tau, L, bp, pred, &cls, &bucket, &tsum);
    atomicAdd(&h[cls * 64 + bucket], 1);
    if (cls == 1) atomicMax(&tmax, tsum);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 128; q += blockDim.x)
    if (h[q]) atomicAdd(&counts[q], h[q]);
  if (threadIdx.x == 0 && tmax) atomicMax(max_t_heavy, tmax);
}

__global__ void __launch_bounds__(256) k_edge_bin_scatter(int64_t m, const int32_t* __restrict__ ei,
                                                          const int32_t* __restrict__ ej,
                                                          const int32_t* __restrict__ deg,
                                                          const uint32_t* __restrict__ tau, int L, BinParams bp,
                                                          const float* __restrict__ pred,
                                                          int32_t* __restrict__ cursor, int32_t* __restrict__ list) {
  __shared__ int32_t h[128];
  __shared__ int32_t base[128];
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < m; t0 += (int64_t)gridDim.x * blockDim.x) {
    for (int q = threadIdx.x; q < 128; q += blockDim.x) h[q] = 0;
    __syncthreads();
    const int64_t e = t0 + threadIdx.x;
    int bin = -1, local = 0;
    if (e < m) {
      int cls, bucket;
      uint32_t tsum;
      edge_bin((int32_t)e, ei, ej, deg, tau, L, bp, pred, &cls, &bucket, &tsum);
      bin = cls * 64 + bucket;
      local = atomicAdd(&h[bin], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 128; q += blockDim.x)
      base[q] = h[q] ? atomicAdd(&cursor[q], h[q]) : 0;
    __syncthreads();
    if (bin >= 0) list[base[bin] + local] = (int32_t)e;
    __syncthreads();
  }
}

// Node tiers for the 4-cycle pass by wedge work W(x): 0 none, 1 wavefront,
// 2 workgroup, 3 grouped dense.
__device__ __forceinline__ int node_tier(uint64_t W) {
  return W == 0 ? 0 : (W <= TG_C4_LIGHT_W ? 1 : (W <= TG_C4_MED_W ? 2 : 3));
}

__global__ void __launch_bounds__(256) k_node_tier_count(int64_t n, const uint64_t* __restrict__ W,
                                                         int32_t* __restrict__ counts) {
  __shared__ int32_t h[4];
  if (threadIdx.x < 4) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[node_tier(W[v])], 1);
  __syncthreads();
  if (threadIdx.x < 4 && h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_node_tier_scatter(int64_t n, const uint64_t* __restrict__ W,
                                                           int32_t* __restrict__ cursor, int32_t* __restrict__ list) {
  __shared__ int32_t h[4];
  __shared__ int32_t base[4];
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < n; t0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < 4) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t v = t0 + threadIdx.x;
    int tier = -1, local = 0;
    if (v < n) {
      tier = node_tier(W[v]);
      local = atomicAdd(&h[tier], 1);
    }
    __syncthreads();
    if (threadIdx.x < 4) base[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0;
    __syncthreads();
    if (tier >= 0) list[base[tier] + local] = (int32_t)v;
    __syncthreads();
  }
}

__global__ void k_gather_node_info(int64_t count, const int32_t* __restrict__ list, const uint64_t* __restrict__ W,
                                   const int32_t* __restrict__ deg, uint64_t* __restrict__ w_out,
                                   int32_t* __restrict__ d_out) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    w_out[q] = W[list[q]];
    d_out[q] = deg[list[q]];
  }
}

// -------------------------------------------------------------- finalize --

// Eq. 17: divide each key's per-edge sum by the edge count of its shape.
__global__ void k_finalize(uint64_t* __restrict__ g, int L, int32_t* __restrict__ flag) {
  const int64_t C3 = c3(L + 2), C4n = c4(L + 3), K = 2 * C3 + 6 * C4n;
  const int shape_edges[8] = {2, 3, 3, 3, 4, 4, 5, 6};
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
    const int h = k < 2 * C3 ? (int)(k / C3) : 2 + (int)((k - 2 * C3) / C4n);
    const uint64_t d = (uint64_t)shape_edges[h];
    const uint64_t v = g[k];
    if (v % d) atomicOr(flag, 1);
    g[k] = v / d;
  }
}

__global__ void k_copy_endpoints(int64_t e0, int64_t e1, const int32_t* __restrict__ ei,
                                 const int32_t* __restrict__ ej, int32_t* __restrict__ out) {
  for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
    out[2 * (e - e0)] = ei[e];
    out[2 * (e - e0) + 1] = ej[e];
  }
}
