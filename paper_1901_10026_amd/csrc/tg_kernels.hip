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

// Exclusive scan of counts into offsets (offsets[n] = total), in three
// passes over blocks of 1024; T is int32_t or int64_t.
template <class T>
__global__ void __launch_bounds__(256) k_scan_blocks(int64_t n, const T* __restrict__ in, T* __restrict__ out,
                                                     T* __restrict__ block_sums) {
  __shared__ T s[1024];
  const int64_t base = (int64_t)blockIdx.x * 1024;
  for (int q = threadIdx.x; q < 1024; q += blockDim.x) s[q] = (base + q < n) ? in[base + q] : (T)0;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    T add[4];
    for (int r = 0; r < 4; ++r) {
      int q = threadIdx.x + r * 256;
      add[r] = (q >= off) ? s[q - off] : (T)0;
    }
    __syncthreads();
    for (int r = 0; r < 4; ++r) s[threadIdx.x + r * 256] += add[r];
    __syncthreads();
  }
  for (int q = threadIdx.x; q < 1024; q += blockDim.x)
    if (base + q < n) out[base + q] = (q > 0) ? s[q - 1] : (T)0;
  if (threadIdx.x == 0) block_sums[blockIdx.x] = s[1023];
}

// Exclusive scan of the block sums in place (one workgroup of 256), total
// into *total.
template <class T>
__global__ void __launch_bounds__(256) k_scan_sums(int64_t nblocks, T* __restrict__ block_sums,
                                                   T* __restrict__ total) {
  __shared__ T part[256];
  const int64_t per = (nblocks + 255) / 256;
  const int64_t b0 = min((int64_t)threadIdx.x * per, nblocks), b1 = min(b0 + per, nblocks);
  T acc = 0;
  for (int64_t b = b0; b < b1; ++b) acc += block_sums[b];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int q = 0; q < 256; ++q) {
      const T v = part[q];
      part[q] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  T run = part[threadIdx.x];
  for (int64_t b = b0; b < b1; ++b) {
    const T v = block_sums[b];
    block_sums[b] = run;
    run += v;
  }
}

template <class T>
__global__ void k_scan_add(int64_t n, T* __restrict__ out, const T* __restrict__ block_sums,
                           const T* __restrict__ total) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (int64_t)gridDim.x * blockDim.x) {
    if (x == n) out[n] = *total;
    else out[x] += block_sums[x / 1024];
  }
}

// One wavefront per node v: canonical edge ids of its upper slots, the
// slot->edge map for every slot, both slots of every edge (es_lo in the row
// of its lower end, es_hi in the other) and the degree-ordered out-list.
__global__ void k_fill_edges(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const int32_t* __restrict__ deg, const int32_t* __restrict__ n_upper,
                             const int32_t* __restrict__ upper_off, const int32_t* __restrict__ out_off,
                             int32_t* __restrict__ ei, int32_t* __restrict__ ej, int32_t* __restrict__ s2e,
                             int32_t* __restrict__ es_lo, int32_t* __restrict__ es_hi,
                             int32_t* __restrict__ out_col, int32_t* __restrict__ out_eid) {
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
    int32_t e = 0;
    if (valid) {
      if (k > (int32_t)v) {
        e = upper_off[v] + (s - first_up);
        ei[e] = (int32_t)v;
        ej[e] = k;
        s2e[s] = e;
        es_lo[e] = s;
      } else {
        const int32_t p = rp[k] + lower_bound(ci + rp[k], dk, (int32_t)v);
        e = upper_off[k] + (p - (rp[k + 1] - n_upper[k]));
        s2e[s] = e;
        es_hi[e] = s;
      }
    }
    const bool hi = valid && precedes(dv, (int32_t)v, dk, k);
    const uint64_t mask = ballot(hi);
    if (hi) {
      out_col[out_off[v] + acc + lanes_below(mask)] = k;
      if (out_eid) out_eid[out_off[v] + acc + lanes_below(mask)] = e;
    }
    acc += __popcll(mask);
  }
}

// -------------------------------------------------------------------- tau --

// tau_e[t] = |Gamma_i^t intersect Gamma_j^t| by binary search of the shorter
// row's ids in the longer row.  One team of TSIZE lanes (16 or 64) per edge;
// a launch takes the edges whose shorter row length lies in (dlo, dhi], so
// short rows do not leave most of a wavefront idle.
template <int TSIZE>
__global__ void __launch_bounds__(256) k_tau(int64_t m, int32_t dlo, int32_t dhi, const int32_t* __restrict__ ei,
                                             const int32_t* __restrict__ ej, const int32_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                                             const uint8_t* __restrict__ ty, int L, uint32_t* __restrict__ tau,
                                             const int32_t* __restrict__ es_lo, const int32_t* __restrict__ es_hi,
                                             uint32_t* __restrict__ tau_s, const int64_t* __restrict__ tl_off,
                                             int32_t* __restrict__ tl_k, int32_t* __restrict__ tl_e,
                                             int tl_packed, int32_t hub_min) {
  constexpr int TEAMS = 256 / TSIZE;
  // wavefront teams copy a longer row of at most STAGE ids to LDS and
  // search it there (16 KB per workgroup; 2048 ids measured slower, the
  // workgroups per CU halving)
  constexpr int STAGE = TSIZE == TG_WAVE ? 1024 : 0;
  __shared__ int32_t stage[STAGE ? TEAMS * STAGE : 1];
  const int team = threadIdx.x / TSIZE, tl = threadIdx.x % TSIZE;
  for (int64_t e = (int64_t)blockIdx.x * TEAMS + team; e < m; e += (int64_t)gridDim.x * TEAMS) {
    const int32_t i = ei[e], j = ej[e];
    const int32_t di = deg[i], dj = deg[j];
    const bool ia = di <= dj;
    const int32_t la = ia ? di : dj, lb = ia ? dj : di;
    if (la <= dlo || la > dhi || lb > hub_min) continue;  // hub rows: k_tau_hub
    const int32_t ra = rp[ia ? i : j], rb = rp[ia ? j : i];
    const int32_t* pa = ci + ra;
    const int32_t* pb = ci + rb;
    if (STAGE && lb <= STAGE) {  // the team is one wavefront
      int32_t* sb = stage + team * STAGE;
      wave_sync();  // the previous edge's searches are done
      for (int32_t x = tl; x < lb; x += TSIZE) sb[x] = pb[x];
      wave_sync();
      pb = sb;
    }
    // with lists, the edge keeps its common neighbours in id order, with
    // their CSR slots in the rows of both ends (ids as id << 4 | type when
    // tl_packed, so that the gather reads no type by id)
    const bool keep = tl_off != nullptr;
    const int64_t lbase = keep ? tl_off[e] : 0;
    int32_t nkept = 0;
    uint32_t my_t = 0;
    for (int32_t b0 = 0; b0 < la; b0 += TSIZE) {
      int t = -1;
      int32_t k = 0, p = 0;
      if (b0 + tl < la) {
        k = pa[b0 + tl];
        p = lower_bound(pb, lb, k);
        if (p < lb && pb[p] == k) t = ty[k];
      }
      const uint64_t wm = ballot(t >= 0);
      const uint64_t tm = (TSIZE >= TG_WAVE) ? wm : ((wm >> ((lane() / TSIZE) * TSIZE)) & ((1ull << TSIZE) - 1ull));
      if (keep) {
        if (t >= 0) {
          const int64_t pos = lbase + nkept + __popcll(tm & ((1ull << tl) - 1ull));
          tl_k[pos] = tl_packed ? ((k << 4) | t) : k;
          tl_e[2 * pos] = ra + b0 + tl;
          tl_e[2 * pos + 1] = rb + p;
        }
        nkept += __popcll(tm);
      }
      if (tm) {
        for (int tt = 0; tt < L; ++tt) {
          const uint64_t b = ballot(t == tt);
          const uint64_t bt = (TSIZE >= TG_WAVE) ? b : ((b >> ((lane() / TSIZE) * TSIZE)) & ((1ull << TSIZE) - 1ull));
          if (tl == tt) my_t += (uint32_t)__popcll(bt);
        }
      }
    }
    if (tl < L) {  // TSIZE >= 16 >= L
      tau[e * L + tl] = my_t;
      if (tau_s) {
        tau_s[(int64_t)es_lo[e] * L + tl] = my_t;
        tau_s[(int64_t)es_hi[e] * L + tl] = my_t;
      }
    }
  }
}

// Hub rows as bitmaps: for each hub (a node whose row is longer than the
// tau pass's hub threshold) one bit per node id over nw = ceil(n / 64) words
// and, per word, the number of set bits before it (its row position), so
// that an edge whose longer row is a hub finds each id of its shorter row
// with two loads instead of a binary search.  bits must be zero on entry.
__global__ void k_hub_bits(int64_t nslots, int64_t nh, const int32_t* __restrict__ hubs,
                           const int64_t* __restrict__ hoff, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, int64_t nw, uint64_t* __restrict__ bits) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nslots; f += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nh;  // the largest h with hoff[h] <= f
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (hoff[mid] <= f) lo = mid; else hi = mid;
    }
    const int32_t k = ci[rp[hubs[lo]] + (f - hoff[lo])];
    atomicOr((unsigned long long*)&bits[lo * nw + (k >> 6)], 1ull << (k & 63));
  }
}

// Nodes whose degree exceeds hmin: their number (count_only) or their list
// and degrees (at cursor[0], any order).
__global__ void __launch_bounds__(256) k_hubs_above(int64_t n, const int32_t* __restrict__ deg, int32_t hmin,
                                                    int count_only, int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ hubs, int64_t* __restrict__ hdeg) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (deg[v] <= hmin) continue;
    const int32_t q = atomicAdd(cursor, 1);
    if (!count_only) {
      hubs[q] = (int32_t)v;
      hdeg[q] = deg[v];
    }
  }
}

__global__ void k_hub_index(int64_t nh, const int32_t* __restrict__ hubs, int32_t* __restrict__ hub_of) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nh; q += (int64_t)gridDim.x * blockDim.x)
    hub_of[hubs[q]] = (int32_t)q;
}

// One workgroup per hub: rank[h][w] = set bits of hub h's words before w.
__global__ void __launch_bounds__(256) k_hub_rank(int64_t nw, const uint64_t* __restrict__ bits,
                                                  int32_t* __restrict__ rank) {
  __shared__ int32_t part[256];
  const int64_t h = blockIdx.x;
  const uint64_t* b = bits + h * nw;
  int32_t* r = rank + h * nw;
  const int64_t per = (nw + 255) / 256;
  const int64_t w0 = min(nw, (int64_t)threadIdx.x * per), w1 = min(nw, w0 + per);
  int32_t c = 0;
  for (int64_t w = w0; w < w1; ++w) c += __popcll(b[w]);
  part[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int q = 0; q < 256; ++q) {
      const int32_t v = part[q];
      part[q] = s;
      s += v;
    }
  }
  __syncthreads();
  int32_t s = part[threadIdx.x];
  for (int64_t w = w0; w < w1; ++w) {
    r[w] = s;
    s += __popcll(b[w]);
  }
}

// tau of the edges whose longer row is a hub's, hub by hub (consecutive
// teams take consecutive slots of one hub's row, so its bitmap stays in
// cache): one 64-lane team per slot s of hub b's row, for the edge (a, b)
// with a = ci[rp[b] + s] when b is that edge's longer side (the side the
// tau kernel searches); the same outputs as k_tau (tau, tau by slot, the
// kept list in id order of the shorter row).
__global__ void __launch_bounds__(256) k_tau_hub(int64_t nslots, int64_t nh, const int32_t* __restrict__ hubs,
                                                 const int64_t* __restrict__ hoff, int64_t nw,
                                                 const uint64_t* __restrict__ bits, const int32_t* __restrict__ rank,
                                                 const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const int32_t* __restrict__ deg, const int32_t* __restrict__ s2e,
                                                 const uint8_t* __restrict__ ty, int L, uint32_t* __restrict__ tau,
                                                 const int32_t* __restrict__ es_lo, const int32_t* __restrict__ es_hi,
                                                 uint32_t* __restrict__ tau_s, const int64_t* __restrict__ tl_off,
                                                 int32_t* __restrict__ tl_k, int32_t* __restrict__ tl_e, int tl_packed) {
  constexpr int TSIZE = TG_WAVE, TEAMS = 256 / TSIZE;
  const int team = threadIdx.x / TSIZE, tl = threadIdx.x % TSIZE;
  for (int64_t f = (int64_t)blockIdx.x * TEAMS + team; f < nslots; f += (int64_t)gridDim.x * TEAMS) {
    int64_t lo = 0, hi = nh;  // the largest h with hoff[h] <= f
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (hoff[mid] <= f) lo = mid; else hi = mid;
    }
    const int32_t b = hubs[lo];
    const int32_t rb = rp[b];
    const int32_t a = ci[rb + (f - hoff[lo])];
    const int32_t da = deg[a], db = deg[b];
    // b is the longer side: i = min(a, b), j = max(a, b), the longer is j
    // when d_i <= d_j, else i (the tau kernel's rule)
    const bool b_is_j = b > a;
    const bool b_longer = b_is_j ? (da <= db) : (db > da);
    if (!b_longer) continue;
    const int32_t e = s2e[rb + (f - hoff[lo])];
    const int32_t ra = rp[a], la = da;
    const uint64_t* hb = bits + lo * nw;
    const int32_t* hr = rank + lo * nw;
    const bool keep = tl_off != nullptr;
    const int64_t lbase = keep ? tl_off[e] : 0;
    int32_t nkept = 0;
    uint32_t my_t = 0;
    for (int32_t b0 = 0; b0 < la; b0 += TSIZE) {
      int t = -1;
      int32_t k = 0, p = 0;
      if (b0 + tl < la) {
        k = ci[ra + b0 + tl];
        const uint64_t w = hb[k >> 6];
        const uint64_t below = w & ((1ull << (k & 63)) - 1ull);
        if ((w >> (k & 63)) & 1ull) {
          p = hr[k >> 6] + __popcll(below);
          t = ty[k];
        }
      }
      const uint64_t tm = ballot(t >= 0);
      if (keep) {
        if (t >= 0) {
          const int64_t pos = lbase + nkept + __popcll(tm & ((1ull << tl) - 1ull));
          tl_k[pos] = tl_packed ? ((k << 4) | t) : k;
          tl_e[2 * pos] = ra + b0 + tl;
          tl_e[2 * pos + 1] = rb + p;
        }
        nkept += __popcll(tm);
      }
      if (tm) {
        for (int tt = 0; tt < L; ++tt) {
          const uint64_t bt = ballot(t == tt);
          if (tl == tt) my_t += (uint32_t)__popcll(bt);
        }
      }
    }
    if (tl < L) {
      tau[(int64_t)e * L + tl] = my_t;
      if (tau_s) {
        tau_s[(int64_t)es_lo[e] * L + tl] = my_t;
        tau_s[(int64_t)es_hi[e] * L + tl] = my_t;
      }
    }
  }
}

// Sum over the edges of the bound below, added to *total.
__global__ void __launch_bounds__(256) k_tl_total(int64_t m, const int32_t* __restrict__ ei,
                                                  const int32_t* __restrict__ ej, const int32_t* __restrict__ deg,
                                                  uint64_t* __restrict__ total) {
  uint64_t s = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    s += (uint64_t)min(deg[ei[e]], deg[ej[e]]);
  s = wave_sum_u64(s);
  if (lane() == 0 && s) atomicAdd((unsigned long long*)total, (unsigned long long)s);
}

// Upper bound on the common-neighbour list of each edge: its shorter row's
// length.
__global__ void k_tl_bound(int64_t m, const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
                           const int32_t* __restrict__ deg, int64_t* __restrict__ bound) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    bound[e] = min(deg[ei[e]], deg[ej[e]]);
  }
}

// ----------------------------------------------------------------- tables --

// One wavefront per node i: P[i][t][u] and U[i][t][u].
__global__ void k_node_tables(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const uint8_t* __restrict__ ty, int L, const uint32_t* __restrict__ D,
                              const uint32_t* __restrict__ tau_s, uint64_t* __restrict__ Pn,
                              uint64_t* __restrict__ Un) {
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
      for (int u = 0; u < L; ++u) {
        const uint32_t dv = D[(int64_t)k * L + u];
        if (dv) atomicAdd((unsigned long long*)&Pa[t * L + u], (unsigned long long)dv);
        const uint32_t tv = tau_s[(int64_t)s * L + u];
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

// Credits go to per-edge rows (s2e given: row = s2e[slot]) or to per-slot
// rows (s2e null: row = slot; consecutive wedges then credit consecutive
// rows, and k_c4_fold adds an edge's two slot rows afterwards).  The counters
// are stored type-pair major, C4[p * crows + row] (crows = number of rows),
// so that the lanes of a wavefront crediting consecutive rows with one type
// pair write consecutive words.
// Credits the cycles through wedge x-u-w (slots sxu of x's row and suw of
// u's row) given the typed middle counts between x and w.
// Per-edge 4-cycle counters are 32 bits when every count fits (the count on
// edge (i, j) is at most (d_i - 1)(d_j - 1)), else 64 bits.
__device__ __forceinline__ void c4_add(uint32_t* C4, int64_t idx, uint64_t v) { atomicAdd(&C4[idx], (uint32_t)v); }
__device__ __forceinline__ void c4_add(uint64_t* C4, int64_t idx, uint64_t v) {
  atomicAdd((unsigned long long*)&C4[idx], (unsigned long long)v);
}

// Split counters: where per-slot 64-bit rows would not fit, the slot rows
// are kept in 32 bits and the few edges whose count may reach lim (an edge
// (a, b) lies on at most (d_a - 1)(d_b - 1) 4-cycles) are credited in 64-bit
// per-edge counters C4e[e * P + p] instead; k_c4_fold_add then adds the slot
// rows of every edge to them.  C4e null: no split.
struct C4Split {
  uint64_t* C4e;
  const int32_t* s2e;  // slot -> canonical edge id
  uint64_t lim;
  int P;
};

// Credit v cycles of type pair p to row `row` (a slot or an edge id) of the
// edge (a, b) of degrees da, db.
template <class C4T>
__device__ __forceinline__ void c4_credit(C4T* __restrict__ C4, int64_t crows, int p, int32_t row, uint64_t v,
                                          const C4Split& X, int32_t da, int32_t db) {
  if (X.C4e && (uint64_t)(da - 1) * (uint64_t)(db - 1) >= X.lim)
    atomicAdd((unsigned long long*)&X.C4e[(int64_t)X.s2e[row] * X.P + p], (unsigned long long)v);
  else
    c4_add(C4, (int64_t)p * crows + row, v);
}

template <class C4T>
__device__ __forceinline__ void credit_wedge(C4T* __restrict__ C4, int64_t crows, int32_t e_xu, int32_t e_uw,
                                             int phx, int phu, int phw, int t, uint32_t cnt_t, const C4Split& X,
                                             int32_t dx, int32_t du, int32_t dw) {
  const int64_t c = (int64_t)cnt_t - (t == phu ? 1 : 0);
  if (c > 0) {
    c4_credit(C4, crows, pair_index(phw, t), e_xu, (uint64_t)c, X, dx, du);
    c4_credit(C4, crows, pair_index(phx, t), e_uw, (uint64_t)c, X, du, dw);
  }
}

// One team (NWAVES wavefronts) per node x, middle counts in LDS hash tables:
// kw/tw keyed by w (totals), kt/ct keyed by w*L+t (typed counts).
// GLOB: instead of crediting edges, every cycle x-u-w-u' adds its count to the
// global 4-cycle key of {phi_x, phi_u, phi_w, phi_u'}; each cycle is reached
// through both of its wedges at x, so the key sums are twice the counts.
template <int NWAVES, int LOG2CAP, class C4T, bool GLOB = false>
__global__ void __launch_bounds__(256) k_c4_hash(int64_t count, const int32_t* __restrict__ list,
                                                 const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const int32_t* __restrict__ deg, const uint8_t* __restrict__ ty,
                                                 int L, const int32_t* __restrict__ s2e,
                                                 C4T* __restrict__ C4, int64_t crows, GAcc ga,
                                                 const uint32_t* __restrict__ cdt, C4Split X) {
  extern __shared__ uint64_t hash_gacc[];
  if (GLOB) gacc_init(ga, hash_gacc);
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
          // degree and type of w: packed per slot when cdt is given (read in
          // row order), else gathered by node id
          const uint32_t dtw = cdt ? cdt[bu + b0 + ln] : 0u;
          const int32_t dw = cdt ? (int32_t)(dtw >> 4) : deg[w];
          if (!precedes(dw, w, dx, x)) continue;
          if (pass == 0) {
            const int h = hash_insert(kw, LOG2CAP, w);
            atomicAdd(&tw[h], 1u);
            const int g = hash_insert(kt, LOG2CAP, w * L + phu);
            atomicAdd(&ct[g], 1u);
          } else {
            const int h = hash_find(kw, LOG2CAP, w);
            if (tw[h] < 2) continue;
            const int32_t e_xu = s2e ? s2e[bx + q] : bx + q;
            const int32_t e_uw = s2e ? s2e[bu + b0 + ln] : bu + b0 + ln;
            const int phw = cdt ? (int)(dtw & 15u) : ty[w];
            for (int t = 0; t < L; ++t) {
              const int g = hash_find(kt, LOG2CAP, w * L + t);
              if (GLOB) {
                const int64_t c = (int64_t)(g >= 0 ? ct[g] : 0u) - (t == phu ? 1 : 0);
                if (c > 0) gacc_add(ga, hash_gacc, key_of(L, 4, phx, phu, phw, t), (uint64_t)c);
              } else {
                credit_wedge(C4, crows, e_xu, e_uw, phx, phu, phw, t, g >= 0 ? ct[g] : 0u, X, dx, du, dw);
              }
            }
          }
        }
      }
      team_sync<NWAVES>();
    }
  }
  if (GLOB) gacc_flush(ga, hash_gacc);
}

// Nodes with large wedge work: a group of nodes at a time, each with a dense
// per-node array of typed middle counts in global memory, one row of RW
// 32-bit words per far end w (RW = CS words of 32-bit counts, or CS / 2
// words holding two 16-bit counts when no count can exceed 65535, i.e. the
// maximum degree is below 65536).  Phase 0 counts, phase 1 credits (phase 3
// instead adds each cycle to its global 4-cycle key, as k_c4_hash does with
// GLOB), phase 2
// clears; kernel boundaries order the phases.
//
// Work mapping: the group's wedges x-u-w, in (node, slot of x's row,
// position in u's row) order, are numbered through wp, the prefix over the
// group's slots of their wedge counts (d_u when u precedes x, else 0).
// Wavefront c takes wedges [c * CH, (c + 1) * CH) whatever the degrees, and
// walks them 64 slots at a time: lane l owns one slot, its clipped wedge
// count goes through a wavefront prefix sum, and the window's wedges are
// dealt to lanes 64 at a time.
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

// Wedge count of each slot of the heavy nodes (listed in processing order,
// hs = prefix of their degrees): d_u when the middle u precedes x, else 0.
__global__ void k_c4_slot_wedges(int64_t nslots, int64_t nnodes, const int32_t* __restrict__ hx,
                                 const int64_t* __restrict__ hs, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                                 int64_t* __restrict__ cnt) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnodes;  // largest q with hs[q] <= s
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (hs[mid] <= s) lo = mid; else hi = mid;
    }
    const int32_t x = hx[lo];
    const int32_t u = ci[rp[x] + (s - hs[lo])];
    const int32_t du = deg[u];
    cnt[s] = precedes(du, u, deg[x], x) ? (int64_t)du : 0;
  }
}

// Far-end slices: slice k holds node ids [k n / nsl, (k+1) n / nsl).  Rows
// are sorted, so slice k of u's row is the contiguous part [bnd[u][k],
// bnd[u][k+1]) (offsets inside the row).
__global__ void k_slice_bounds(int64_t n, int nsl, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               int32_t* __restrict__ bnd) {
  const int64_t total = n * (nsl + 1);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = q / (nsl + 1);
    const int k = (int)(q - u * (nsl + 1));
    const int32_t key = (int32_t)(((int64_t)k * n) / nsl);
    bnd[q] = lower_bound(ci + rp[u], rp[u + 1] - rp[u], key);
  }
}

// Per-slice wedge counts of the first nslots heavy slots:
// cnt[k * nslots + s] = size of slice k of u's row when u precedes x, else 0.
__global__ void k_c4_slot_wedges_sliced(int64_t nslots, int64_t nnodes, int nsl, const int32_t* __restrict__ hx,
                                        const int64_t* __restrict__ hs, const int32_t* __restrict__ rp,
                                        const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                                        const int32_t* __restrict__ bnd, int64_t* __restrict__ cnt) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnodes;  // largest q with hs[q] <= s
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (hs[mid] <= s) lo = mid; else hi = mid;
    }
    const int32_t x = hx[lo];
    const int32_t u = ci[rp[x] + (s - hs[lo])];
    const bool ok = precedes(deg[u], u, deg[x], x);
    const int32_t* b = bnd + (int64_t)u * (nsl + 1);
    for (int k = 0; k < nsl; ++k) cnt[(int64_t)k * nslots + s] = ok ? (int64_t)(b[k + 1] - b[k]) : 0;
  }
}

// HASH: instead of a dense array per node, node gi of the group has an
// open-addressing table of 2^hlog[gi] rows starting at row hoff[gi], keyed by
// w in hkeys (-1 = empty), for nodes whose far ends are few compared with n.
//
// Slices (nsl > 1): workgroup b takes the far ends of slice b % nsl, so that
// with workgroups dealt round-robin to the XCDs and nsl = 8 each XCD's L2
// holds one eighth of a node's count rows.  wp is the group's part of the
// slot prefix of slice k at wp + k * wstride; workgroups stride over the
// chunks of their slice.
template <int PHASE, class C4T, bool HALF, bool HASH>
__global__ void __launch_bounds__(256) k_c4_group(int G, const int32_t* __restrict__ gx,
                                                  const int64_t* __restrict__ gslot, const int64_t* __restrict__ wp,
                                                  int64_t wstride, int nsl, const int32_t* __restrict__ bnd,
                                                  int CH, uint32_t* __restrict__ dense,
                                                  int64_t stride, int RW, const int64_t* __restrict__ hoff,
                                                  const uint8_t* __restrict__ hlog, int32_t* __restrict__ hkeys,
                                                  const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                                                  const uint8_t* __restrict__ ty, int L,
                                                  const int32_t* __restrict__ s2e, C4T* __restrict__ C4,
                                                  int64_t crows, int stage_xu, GAcc ga,
                                                  const uint32_t* __restrict__ cdt, C4Split X) {
  // credits to the edges (x, u) of the window's 64 slots are summed in LDS
  // first (stage_xu: L <= 8 and every sum fits 32 bits); dynamic LDS of
  // 4 * 64 * P words in phase 1 with stage_xu, the key copies of ga in
  // phase 3, else none
  extern __shared__ uint32_t xu_acc[];
  uint64_t* gsm = reinterpret_cast<uint64_t*>(xu_acc);
  if (PHASE == 3) gacc_init(ga, gsm);
  const int wib = threadIdx.x / TG_WAVE;
  const int ln = lane();
  const int P = L * (L + 1) / 2;
  const int ksl = (int)(blockIdx.x % nsl);
  const int64_t cb = blockIdx.x / nsl, nblk = gridDim.x / nsl;
  // gslot holds the group's slot prefix with an arbitrary base
  const int64_t sbase = gslot[0];
  const int64_t S = gslot[G] - sbase;
  const int64_t* wpk = wp + ksl * wstride;
  const int64_t W0 = wpk[0], Wn = wpk[S] - W0;
  uint32_t* xacc = xu_acc + wib * TG_WAVE * P;
  for (int64_t chunk = cb * (blockDim.x / TG_WAVE) + wib; chunk * CH < Wn;
       chunk += nblk * (blockDim.x / TG_WAVE)) {
  const int64_t wbeg = chunk * CH;
  const int64_t wend = min(wbeg + (int64_t)CH, Wn);
  // first slot: the largest s < S with wp[s] - W0 <= wbeg
  int64_t sa;
  {
    int64_t lo = 0, hi = S;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (wpk[mid] - W0 <= wbeg) lo = mid; else hi = mid;
    }
    sa = lo;
  }
  for (;;) {
    if (PHASE == 1 && stage_xu) {
      for (int q = ln; q < TG_WAVE * P; q += TG_WAVE) xacc[q] = 0u;
      wave_sync();
    }
    // this lane's slot and the part of its wedges inside [wbeg, wend)
    const int64_t sl = sa + ln;
    int32_t x = 0, dx = 0, du = 0, bu = 0, cu = 0, off = 0, e_xu = 0, gi = 0;
    int phx = 0, phu = 0;
    if (sl < S) {
      const int64_t ws = wpk[sl] - W0, we = wpk[sl + 1] - W0;
      const int64_t lo = max(ws, wbeg), hi = min(we, wend);
      if (hi > lo) {
        int a = 0, b = G;  // largest g with gslot[g] <= sl
        while (b - a > 1) {
          const int mid = (a + b) >> 1;
          if (gslot[mid] - sbase <= sl) a = mid; else b = mid;
        }
        gi = a;
        x = gx[a];
        dx = deg[x];
        const int32_t sx = rp[x] + (int32_t)(sl - (gslot[a] - sbase));
        const int32_t u = ci[sx];
        if (PHASE == 1) du = cdt ? (int32_t)(cdt[sx] >> 4) : deg[u];
        cu = (int32_t)(hi - lo);
        off = (int32_t)(lo - ws);
        bu = rp[u] + (nsl > 1 ? bnd[(int64_t)u * (nsl + 1) + ksl] : 0);
        phx = ty[x];
        phu = ty[u];
        e_xu = s2e ? s2e[sx] : sx;
      }
    }
    int32_t tot = 0;
    const int32_t excl = wave_excl_scan(cu, &tot);
    // U batches of 64 wedges per step: their row and degree loads are
    // issued before any of them is used
    constexpr int U = 2;
    for (int32_t c0 = 0; c0 < tot; c0 += TG_WAVE * U) {
      int32_t wv[U], sv[U], ov[U];
      bool ok[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int32_t v = c0 + k * TG_WAVE + ln;
        // owner lane: the largest l with excl[l] <= v (excl is non-decreasing)
        int o = 0;
        for (int step = 32; step > 0; step >>= 1) {
          const int32_t ex = __shfl(excl, o + step, TG_WAVE);
          if (o + step < TG_WAVE && ex <= v) o += step;
        }
        const int32_t o_excl = __shfl(excl, o, TG_WAVE);
        const int32_t o_bu = __shfl(bu, o, TG_WAVE);
        const int32_t o_off = __shfl(off, o, TG_WAVE);
        ov[k] = o;
        ok[k] = v < tot;
        sv[k] = o_bu + o_off + (v - o_excl);
        wv[k] = ok[k] ? ci[sv[k]] : 0;
      }
      // degree and type of w: packed per slot when cdt is given (read in row
      // order, next to the ids), else gathered by node id
      int32_t dw[U];
      int tw[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint32_t dt = (ok[k] && cdt) ? cdt[sv[k]] : 0u;
        dw[k] = ok[k] ? (cdt ? (int32_t)(dt >> 4) : deg[wv[k]]) : 0;
        tw[k] = (int)(dt & 15u);
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int o = ov[k];
        const int32_t o_x = __shfl(x, o, TG_WAVE);
        const int32_t o_dx = __shfl(dx, o, TG_WAVE);
        const int32_t o_gi = __shfl(gi, o, TG_WAVE);
        const int o_phx = __shfl(phx, o, TG_WAVE);
        const int o_phu = __shfl(phu, o, TG_WAVE);
        const int32_t o_exu = __shfl(e_xu, o, TG_WAVE);
        const int32_t o_du = PHASE == 1 ? __shfl(du, o, TG_WAVE) : 0;
        const int32_t w = wv[k], suw = sv[k];
        if (!ok[k] || !precedes(dw[k], w, o_dx, o_x)) continue;
        uint32_t* row;
        if (HASH) {
          const int64_t hb = hoff[o_gi];
          const int hl = hlog[o_gi];
          int32_t* keys = hkeys + hb;
          const uint32_t mask = (1u << hl) - 1u;
          uint32_t h = ((uint32_t)w * 2654435761u) >> (32 - hl);
          if (PHASE == 0) {
            for (;;) {
              const int32_t old = atomicCAS(&keys[h], -1, w);
              if (old == -1 || old == w) break;
              h = (h + 1) & mask;
            }
          } else {
            int32_t kk;
            while ((kk = keys[h]) != w && kk != -1) h = (h + 1) & mask;
            if (kk != w) continue;  // not reached: phase 0 inserted every far end
          }
          row = dense + (hb + h) * RW;
        } else {
          row = dense + (int64_t)o_gi * stride + (int64_t)w * RW;
        }
        if (PHASE == 0) {
          if (HALF) atomicAdd(&row[o_phu >> 1], 1u << ((o_phu & 1) << 4));
          else atomicAdd(&row[o_phu], 1u);
        } else if (PHASE == 1 || PHASE == 3) {
          // rows are 16-byte aligned and RW is a multiple of 4 words
          uint32_t c[16];
          uint32_t sum = 0;
          for (int q4 = 0; q4 < RW / 4; ++q4) {
            const uint4 v4 = reinterpret_cast<const uint4*>(row)[q4];
            const uint32_t wd[4] = {v4.x, v4.y, v4.z, v4.w};
            for (int r = 0; r < 4; ++r) {
              if (HALF) {
                c[8 * q4 + 2 * r] = wd[r] & 0xffffu;
                c[8 * q4 + 2 * r + 1] = wd[r] >> 16;
              } else {
                c[4 * q4 + r] = wd[r];
              }
            }
          }
          for (int t = 0; t < L; ++t) sum += c[t];
          if (sum < 2) continue;
          const int phw = cdt ? tw[k] : ty[w];
          if (PHASE == 3) {
            for (int t = 0; t < L; ++t) {
              const int64_t cc = (int64_t)c[t] - (t == o_phu ? 1 : 0);
              if (cc > 0) gacc_add(ga, gsm, key_of(L, 4, o_phx, o_phu, phw, t), (uint64_t)cc);
            }
            continue;
          }
          const int32_t e_uw = s2e ? s2e[suw] : suw;
          for (int t = 0; t < L; ++t) {
            const int64_t cc = (int64_t)c[t] - (t == o_phu ? 1 : 0);
            if (cc <= 0) continue;
            c4_credit(C4, crows, pair_index(o_phx, t), e_uw, (uint64_t)cc, X, o_du, dw[k]);
            if (stage_xu) atomicAdd(&xacc[o * P + pair_index(phw, t)], (uint32_t)cc);
            else c4_credit(C4, crows, pair_index(phw, t), o_exu, (uint64_t)cc, X, o_dx, o_du);
          }
        } else {
          for (int q4 = 0; q4 < RW / 4; ++q4) reinterpret_cast<uint4*>(row)[q4] = make_uint4(0u, 0u, 0u, 0u);
        }
      }
    }
    if (PHASE == 1 && stage_xu) {
      // each lane flushes the sums of its own slot, one type pair at a time
      wave_sync();
      for (int p = 0; p < P; ++p) {
        const uint32_t val = xacc[ln * P + p];
        if (val) c4_credit(C4, crows, p, e_xu, (uint64_t)val, X, dx, du);
      }
      wave_sync();
    }
    // next window, unless it starts at or past this wavefront's last wedge
    sa += TG_WAVE;
    if (sa >= S || wpk[sa] - W0 >= wend) break;
  }
  }
  if (PHASE == 3) gacc_flush(ga, gsm);
}

// Degree and type of every slot's column node, packed as deg << 4 | type
// (degrees below 2^28, types below 16), so that wedge walks read them in row
// order instead of gathering them by node id.
__global__ void k_slot_dt(int64_t nnz, const int32_t* __restrict__ ci, const int32_t* __restrict__ deg,
                          const uint8_t* __restrict__ ty, uint32_t* __restrict__ cdt) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nnz; s += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = ci[s];
    cdt[s] = ((uint32_t)deg[w] << 4) | (uint32_t)ty[w];
  }
}

// Per-edge 4-cycle rows (edge-major, P per edge) from type-pair-major
// per-slot counters: C4e[e][p] = C4s[p][es_lo[e]] + C4s[p][es_hi[e]].
template <class C4T>
__global__ void k_c4_fold(int64_t m, int P, int64_t nslots, const int32_t* __restrict__ es_lo,
                          const int32_t* __restrict__ es_hi, const C4T* __restrict__ C4s, C4T* __restrict__ C4e) {
  const int64_t total = m * P;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = x / P, p = x - e * P;
    C4e[x] = C4s[p * nslots + es_lo[e]] + C4s[p * nslots + es_hi[e]];
  }
}

// Split counters: adds the two 32-bit slot rows of every edge to its 64-bit
// counters (which hold the credits of the edges counted there directly).
__global__ void k_c4_fold_add(int64_t m, int P, int64_t nslots, const int32_t* __restrict__ es_lo,
                              const int32_t* __restrict__ es_hi, const uint32_t* __restrict__ C4s,
                              uint64_t* __restrict__ C4e) {
  const int64_t total = m * P;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = x / P, p = x - e * P;
    C4e[x] += (uint64_t)C4s[p * nslots + es_lo[e]] + (uint64_t)C4s[p * nslots + es_hi[e]];
  }
}

#include "tg_c4part.hip"
#include "tg_combine.hip"
#include "tg_clique.hip"

// ------------------------------------------------------------- schedule --

// Edge class (0: one wavefront, 1: one workgroup) and cost bucket (0 = most
// expensive).  cost: 0 none, 1 degree product, 2 given per-edge cost.
struct BinParams {
  int mode;               // 0 none, 1 degree product, 2 predicted log2 cost
  int light_max_degree;   // class 0 (16-lane team) needs min(d_i, d_j) <= this and |T| <= 64
  int heavy_min_degree;   // min(d_i, d_j) above this: class 2 (workgroup)
  int mid_log2_cost;      // floor(log2 cost) above this: at least class 1 (wavefront)
  int heavy_log2_cost;    // floor(log2 cost) above this: class 2
  int teams16;            // 0: class 0 is folded into class 1 (large L)
};

// Edge class (0: 16-lane team, 1: wavefront, 2: workgroup) and cost bucket
// (0 = most expensive).
__device__ __forceinline__ void edge_bin(int32_t e, const int32_t* ei, const int32_t* ej, const int32_t* deg,
                                         const uint32_t* tau, int L, BinParams bp, const float* pred, int* cls,
                                         int* bucket, uint32_t* tsum_out) {
  const int32_t i = ei[e], j = ej[e];
  const int32_t di = deg[i], dj = deg[j];
  const int32_t dmin = min(di, dj);
  uint32_t tsum = 0;
  for (int t = 0; t < L; ++t) tsum += tau[(int64_t)e * L + t];
  *tsum_out = tsum;
  int c = 0;
  if (tsum > 256 || dmin > bp.heavy_min_degree) c = 2;
  else if (tsum > 64 || dmin > bp.light_max_degree || !bp.teams16) c = 1;
  int fine = 0;
  if (bp.mode != 0) {
    double l2;
    if (bp.mode == 1) l2 = log2((double)di * (double)dj + 1.0);
    else l2 = log2(exp2((double)pred[e]) + 1.0);
    l2 = l2 < 0.0 ? 0.0 : l2;
    const int lg = (int)fmin(floor(l2), 63.0);
    if (lg > bp.heavy_log2_cost) c = 2;
    else if (lg > bp.mid_log2_cost && c == 0) c = 1;
    // buckets of one octave of cost, so that edges of alike cost share
    // wavefronts (teams of 16 lanes run four to a wavefront in lockstep);
    // half octaves and two octaves measured slower
    fine = (int)fmin(floor(l2), 63.0);
  }
  *cls = c;
  *bucket = bp.mode == 0 ? 0 : 63 - fine;
}

// Bin counts and scatter use a per-workgroup LDS histogram so that global
// atomics are one per (workgroup tile, bin) rather than one per item.
// Both passes bin the edges e = sel[q] (sel given) or e = e0 + q, q < count.
__global__ void __launch_bounds__(256) k_edge_bin_count(int64_t count, const int64_t* __restrict__ sel, int64_t e0,
                                                        const int32_t* __restrict__ ei,
                                                        const int32_t* __restrict__ ej,
                                                        const int32_t* __restrict__ deg,
                                                        const uint32_t* __restrict__ tau, int L, BinParams bp,
                                                        const float* __restrict__ pred, int32_t* __restrict__ counts,
                                                        uint32_t* __restrict__ max_t_heavy) {
  __shared__ int32_t h[192];
  __shared__ uint32_t tmax;
  for (int q = threadIdx.x; q < 192; q += blockDim.x) h[q] = 0;
  if (threadIdx.x == 0) tmax = 0;
  __syncthreads();
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = sel ? sel[q] : e0 + q;
    int cls, bucket;
    uint32_t tsum;
    edge_bin((int32_t)e, ei, ej, deg, tau, L, bp, pred, &cls, &bucket, &tsum);
    atomicAdd(&h[cls * 64 + bucket], 1);
    if (cls == 2) atomicMax(&tmax, tsum);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 192; q += blockDim.x)
    if (h[q]) atomicAdd(&counts[q], h[q]);
  if (threadIdx.x == 0 && tmax) atomicMax(max_t_heavy, tmax);
}

__global__ void __launch_bounds__(256) k_edge_bin_scatter(int64_t count, const int64_t* __restrict__ sel,
                                                          int64_t e0, const int32_t* __restrict__ ei,
                                                          const int32_t* __restrict__ ej,
                                                          const int32_t* __restrict__ deg,
                                                          const uint32_t* __restrict__ tau, int L, BinParams bp,
                                                          const float* __restrict__ pred,
                                                          int32_t* __restrict__ cursor, int32_t* __restrict__ list) {
  __shared__ int32_t h[192];
  __shared__ int32_t base[192];
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < count; t0 += (int64_t)gridDim.x * blockDim.x) {
    for (int q = threadIdx.x; q < 192; q += blockDim.x) h[q] = 0;
    __syncthreads();
    const int64_t qe = t0 + threadIdx.x;
    const int64_t e = qe < count ? (sel ? sel[qe] : e0 + qe) : 0;
    int bin = -1, local = 0;
    if (qe < count) {
      int cls, bucket;
      uint32_t tsum;
      edge_bin((int32_t)e, ei, ej, deg, tau, L, bp, pred, &cls, &bucket, &tsum);
      bin = cls * 64 + bucket;
      local = atomicAdd(&h[bin], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 192; q += blockDim.x)
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

__global__ void __launch_bounds__(256) k_max_degree(int64_t n, const int32_t* __restrict__ deg,
                                                    int32_t* __restrict__ out) {
  __shared__ int32_t mx;
  if (threadIdx.x == 0) mx = 0;
  __syncthreads();
  int32_t local = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    local = max(local, deg[v]);
  atomicMax(&mx, local);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, mx);
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

// Listed edges: strictly increasing ids inside [0, m), else *bad = 1.
__global__ void k_check_ids(const int64_t* __restrict__ ids, int64_t k, int64_t m, int32_t* __restrict__ bad) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < k; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = ids[q];
    if (e < 0 || e >= m || (q > 0 && ids[q - 1] >= e)) *bad = 1;
  }
}

__global__ void k_copy_endpoints_ids(const int64_t* __restrict__ ids, int64_t k, const int32_t* __restrict__ ei,
                                     const int32_t* __restrict__ ej, int32_t* __restrict__ out) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < k; q += (int64_t)gridDim.x * blockDim.x) {
    out[2 * q] = ei[ids[q]];
    out[2 * q + 1] = ej[ids[q]];
  }
}

__global__ void k_copy_endpoints(int64_t e0, int64_t e1, const int32_t* __restrict__ ei,
                                 const int32_t* __restrict__ ej, int32_t* __restrict__ out) {
  for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
    out[2 * (e - e0)] = ei[e];
    out[2 * (e - e0) + 1] = ej[e];
  }
}
