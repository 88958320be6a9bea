// ------------------------------------------------------------- 4-cliques --
//
// Typed 4-cliques, each enumerated once from its lowest node a in degree
// order.  The other three nodes of a clique lie in O = out(a), the
// higher-ranked neighbours of a, and form a triangle of the subgraph G_a
// that O induces.  Per node a, one team:
//   1. places O in positions sorted by node type, so that each type owns a
//      contiguous range of positions;
//   2. builds G_a as symmetric adjacency bit rows over those positions, from
//      the out-lists of O's members (an edge (b, c) of G_a with c higher
//      than b is found in out(b));
//   3. for every edge (b, c) of G_a takes the typed popcounts
//      n_t = |row(b) & row(c)| restricted to type t: the nodes d of type t
//      with {a, b, c, d} a 4-clique.
// Per-edge counts (Algorithm 3's orbit g12: the typed edges inside T_ij, per
// unordered type pair of the two other nodes): the clique {a, b, c, d}
// contains six edges, and
//   - edge (b, c) is credited n_t cliques of pair {phi_a, t} directly (once,
//     from its own G_a edge);
//   - edge (a, b) collects, over the G_a edges (b, c) at b, n_t cliques of
//     pair {phi_c, t}.  Every clique reaches (a, b) through both of its G_a
//     edges at b, so the sum is twice the count and is halved when flushed.
// The three edges at a are credited by the second rule, the three others by
// the first, so every clique through every edge is counted exactly once per
// edge.  Counters are edge major, K4[e * P + p], so that the row kernel reads
// an edge's counters from one cache line.
// Global counts (GLOB): each triangle {b, c, d} of G_a is counted once, from
// the edge of its two lowest positions, by restricting the popcounts to the
// positions above both ends; its clique adds one to the 4-clique key of
// {phi_a, phi_b, phi_c, phi_d}.
//
// Teams: a wavefront per node for |O| <= 64 (rows of one word, in LDS), a
// workgroup per node for |O| <= 256 (rows in LDS), and a workgroup per node
// with rows and accumulators in a global scratch slice of its own beyond
// that (read at device scope, past the CU's cache, since other lanes write
// them with atomics).  The ids of O are always searched in LDS, which bounds
// |O| by TG_K4_LDS_IDS; graphs with a larger out-degree count their
// 4-cliques per edge instead (the gather's out-list probes).  In degree
// order |O| <= sqrt(2m), so every graph of up to 8.4M edges qualifies.

namespace tg {

struct K4Args {
  const int32_t* deg;
  const uint8_t* ty;
  int L;
  const int32_t* out_off;  // n + 1
  const int32_t* out_col;  // degree-ordered out-lists, ids increasing inside each
  const int32_t* out_eid;  // canonical edge id of each out-list slot
  int64_t m;
  uint32_t* K4n;           // per-edge counters, 32-bit ...
  uint64_t* K4w;           // ... or 64-bit (one of the two is set), K4[e * P + p]
};

#define TG_K4_LDS_IDS 4096  // largest |O| of the pass (ids of O are kept in LDS)

__device__ __forceinline__ void k4_credit(const K4Args& A, int p, int32_t e, uint32_t v) {
  const int64_t q = (int64_t)e * (A.L * (A.L + 1) / 2) + p;
  if (A.K4w) atomicAdd((unsigned long long*)&A.K4w[q], (unsigned long long)v);
  else atomicAdd(&A.K4n[q], v);
}

template <bool DEV>
__device__ __forceinline__ uint64_t k4_load64(const uint64_t* p) {
  if (DEV) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

template <bool DEV>
__device__ __forceinline__ uint32_t k4_load32(const uint32_t* p) {
  if (DEV) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

template <int TSIZE>
__device__ __forceinline__ void k4_sync() {
  if (TSIZE <= TG_WAVE) wave_sync();
  else __syncthreads();
}

// Exclusive prefix over the team (TSIZE 64 or 256); scan holds TSIZE / 64
// ints of LDS for workgroup teams.
template <int TSIZE>
__device__ __forceinline__ int32_t k4_scan(int32_t v, int32_t* total, int32_t* scan, int tid) {
  const int ln = lane();
  int32_t x = v;
  for (int off = 1; off < TG_WAVE; off <<= 1) {
    const int32_t y = __shfl_up(x, off, TG_WAVE);
    if (ln >= off) x += y;
  }
  if (TSIZE <= TG_WAVE) {
    *total = __shfl(x, TG_WAVE - 1, TG_WAVE);
    return x - v;
  }
  const int wv = tid / TG_WAVE;
  if (ln == TG_WAVE - 1) scan[wv] = x;
  __syncthreads();
  int32_t before = 0, tot = 0;
  for (int q = 0; q < TSIZE / TG_WAVE; ++q) {
    const int32_t c = scan[q];
    if (q < wv) before += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

// Bytes of LDS per team.
//   ids[dcap] i32, pos[dcap] i32, tq[dcap] u8, tstart/fill 2 x 17 i32,
//   scan 4 + 3 * TSIZE i32 (workgroup teams), then rows dcap * NW u64,
//   acc dcap * P u32 and the position -> index map qpos[dcap] i32 (LDS
//   teams), or (GSCR) qpos[dcap] i32, the type by position ptype[dcap] u8
//   and one P-counter accumulator per wavefront
template <int TSIZE, bool GSCR>
__host__ __device__ inline int k4_team_lds(int dcap, int L) {
  const int P = L * (L + 1) / 2, NW = (dcap + 63) / 64;
  int b = 9 * dcap;
  b = (b + 7) & ~7;
  b += 4 * 34;
  if (TSIZE > TG_WAVE) b += 4 * (4 + 3 * TSIZE);
  b = (b + 7) & ~7;
  if (!GSCR) b += 8 * dcap * NW + 4 * dcap * P + 4 * dcap;
  else b += ((5 * dcap + 3) & ~3) + 4 * (TSIZE / TG_WAVE) * P;
  return (b + 15) & ~15;
}

// Global scratch bytes per workgroup for GSCR teams (the bit rows).
__host__ __device__ inline int64_t k4_gscr_bytes(int dcap, int L) {
  const int64_t NW = (dcap + 63) / 64;
  const int64_t b = 8 * (int64_t)dcap * NW;
  (void)L;
  return (b + 255) & ~(int64_t)255;
}

// One team per node of list[0, count) (each with |O| <= dcap).
template <int TSIZE, bool GSCR, bool GLOB>
__global__ void __launch_bounds__(256) k_k4_low(K4Args A, int64_t count, const int32_t* __restrict__ list, int dcap,
                                                char* __restrict__ gscr, int64_t gscr_stride, GAcc ga) {
  extern __shared__ uint64_t smem_k4[];
  constexpr int TEAMS = 256 / TSIZE;
  const int L = A.L, P = L * (L + 1) / 2, NW = (dcap + 63) / 64;
  const int team = threadIdx.x / TSIZE, tid = threadIdx.x % TSIZE;
  const int region = k4_team_lds<TSIZE, GSCR>(dcap, L);
  // global key sums share the dynamic LDS after the teams' regions
  uint64_t* gsm = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(smem_k4) + TEAMS * region);
  if (GLOB) gacc_init(ga, gsm);
  char* base = reinterpret_cast<char*>(smem_k4) + team * region;
  int32_t* ids = reinterpret_cast<int32_t*>(base);  // O, ids increasing
  int32_t* pos = ids + dcap;                         // position of O[q]
  uint8_t* tq = reinterpret_cast<uint8_t*>(pos + dcap);  // type of O[q]
  base = reinterpret_cast<char*>(((uintptr_t)(tq + dcap) + 7) & ~(uintptr_t)7);
  int32_t* tstart = reinterpret_cast<int32_t*>(base);  // [17]
  int32_t* fill = tstart + 17;                         // [17]
  int32_t* scan = fill + 17;                           // workgroup teams: 4 + 3 * TSIZE
  char* after = reinterpret_cast<char*>(scan) + (TSIZE > TG_WAVE ? 4 * (4 + 3 * TSIZE) : 0);
  after = reinterpret_cast<char*>(((uintptr_t)after + 7) & ~(uintptr_t)7);
  uint64_t* rows;
  uint32_t* acc = nullptr;
  int32_t* qpos = nullptr;
  uint8_t* ptype = nullptr;
  uint32_t* accw = nullptr;
  if (GSCR) {
    rows = reinterpret_cast<uint64_t*>(gscr + (int64_t)blockIdx.x * gscr_stride);
    qpos = reinterpret_cast<int32_t*>(after);
    ptype = reinterpret_cast<uint8_t*>(qpos + dcap);
    accw = reinterpret_cast<uint32_t*>(after + ((5 * dcap + 3) & ~3)) + (tid / TG_WAVE) * P;
  } else {
    rows = reinterpret_cast<uint64_t*>(after);
    acc = reinterpret_cast<uint32_t*>(after + 8 * dcap * NW);
    qpos = reinterpret_cast<int32_t*>(acc + dcap * P);
  }
  int32_t* s_excl = scan + 4;  // workgroup teams: excl, out start, owner index

  for (int64_t item = (int64_t)blockIdx.x * TEAMS + team; item < count; item += (int64_t)gridDim.x * TEAMS) {
    const int32_t a = list[item];
    const int32_t oa = A.out_off[a];
    const int32_t D = A.out_off[a + 1] - oa;
    const int phia = A.ty[a];
    const int32_t* O = ids;
    // ---- 1. positions sorted by type
    for (int x = tid; x < 2 * 17; x += TSIZE) tstart[x] = 0;
    k4_sync<TSIZE>();
    for (int32_t q = tid; q < D; q += TSIZE) {
      const int32_t b = A.out_col[oa + q];
      ids[q] = b;
      const int t = A.ty[b];
      tq[q] = (uint8_t)t;
      atomicAdd(&fill[t], 1);
    }
    k4_sync<TSIZE>();
    if (tid == 0) {
      int32_t s = 0;
      for (int t = 0; t < L; ++t) {
        tstart[t] = s;
        s += fill[t];
        fill[t] = 0;
      }
      tstart[L] = s;
    }
    k4_sync<TSIZE>();
    for (int32_t q = tid; q < D; q += TSIZE) {
      const int t = tq[q];
      const int32_t pq = tstart[t] + atomicAdd(&fill[t], 1);
      pos[q] = pq;
      qpos[pq] = q;
      if (GSCR) ptype[pq] = (uint8_t)t;
    }
    // clear rows and accumulators
    for (int64_t x = tid; x < (int64_t)D * NW; x += TSIZE) rows[x] = 0;
    if (!GLOB && !GSCR)
      for (int64_t x = tid; x < (int64_t)D * P; x += TSIZE) acc[x] = 0;
    k4_sync<TSIZE>();
    const int NWa = (D + 63) / 64;  // words per row for this node
    // ---- 2 and 3: passes over the pairs (b, c), b in O, c in out(b): the
    // first sets the bit rows; the second (GSCR teams only: the LDS teams
    // take the edges of G_a from the rows, below) credits the cliques
    for (int pass = 0; pass < (GSCR ? 2 : 1); ++pass) {
      for (int32_t q0 = 0; q0 < D; q0 += TSIZE) {
        const int32_t q = q0 + tid;
        int32_t ostart = 0, ocnt = 0;
        if (q < D) {
          const int32_t b = O[q];
          ostart = A.out_off[b];
          ocnt = A.out_off[b + 1] - ostart;
        }
        int32_t tot;
        const int32_t excl = k4_scan<TSIZE>(ocnt, &tot, scan, tid);
        if (TSIZE > TG_WAVE) {
          s_excl[tid] = excl;
          s_excl[TSIZE + tid] = ostart;
          __syncthreads();
        }
        for (int32_t v = tid; v - tid < tot; v += TSIZE) {
          // owner: the largest lane o with excl[o] <= v
          int o = 0;
#pragma unroll
          for (int step = TSIZE / 2; step > 0; step >>= 1) {
            const int32_t ex = TSIZE <= TG_WAVE ? __shfl(excl, o + step, TSIZE) : s_excl[o + step];
            if (ex <= v) o += step;
          }
          const int32_t o_excl = TSIZE <= TG_WAVE ? __shfl(excl, o, TSIZE) : s_excl[o];
          const int32_t o_start = TSIZE <= TG_WAVE ? __shfl(ostart, o, TSIZE) : s_excl[TSIZE + o];
          if (v >= tot) continue;
          const int32_t slot = o_start + (v - o_excl);
          const int32_t c = A.out_col[slot];
          // c in O?
          const int32_t r = lower_bound(O, D, c);
          if (r >= D || O[r] != c) continue;
          const int32_t qb = q0 + o;
          const int pb = pos[qb], pc = pos[r];
          if (pass == 0) {
            atomicOr((unsigned long long*)&rows[(int64_t)pb * NW + (pc >> 6)], 1ull << (pc & 63));
            atomicOr((unsigned long long*)&rows[(int64_t)pc * NW + (pb >> 6)], 1ull << (pb & 63));
            continue;
          }
          const uint64_t* rb = rows + (int64_t)pb * NW;
          const uint64_t* rc = rows + (int64_t)pc * NW;
          const int tb = tq[qb], tc = tq[r];
          const int32_t e_bc = GLOB ? 0 : A.out_eid[slot];
          // typed popcounts of row(b) & row(c), one type range at a time
          // (GLOB: positions above both ends only)
          const int32_t lo_all = GLOB ? max(pb, pc) + 1 : 0;
          for (int u = 0; u < L; ++u) {
            const int32_t s0 = max(tstart[u], lo_all), s1 = tstart[u + 1];
            if (s0 >= s1) continue;
            uint32_t nv = 0;
            for (int32_t k = s0 >> 6; k <= (s1 - 1) >> 6; ++k) {
              const int32_t b0 = max(s0 - (k << 6), 0), b1 = min(s1 - (k << 6), 64);
              const uint64_t msk = (b1 >= 64 ? ~0ull : ((1ull << b1) - 1ull)) & ~((1ull << b0) - 1ull);
              nv += (uint32_t)__popcll(k4_load64<GSCR>(rb + k) & k4_load64<GSCR>(rc + k) & msk);
            }
            if (!nv) continue;
            if (GLOB) {
              gacc_add(ga, gsm, key_of(L, 7, phia, tb, tc, u), (uint64_t)nv);
              continue;
            }
            k4_credit(A, pair_index(phia, u), e_bc, nv);
            if (!GSCR) {
              atomicAdd(&acc[(int64_t)pb * P + pair_index(tc, u)], nv);
              atomicAdd(&acc[(int64_t)pc * P + pair_index(tb, u)], nv);
            }
          }
        }
        if (TSIZE > TG_WAVE) __syncthreads();
      }
      k4_sync<TSIZE>();
    }
    // ---- 3 (LDS teams): every edge (b, c) of G_a once, from the rows:
    // position pb takes the set bits pc > pb of its row, dealt to lanes
    // through a team prefix sum of their numbers
    if (!GSCR) {
      for (int32_t p0 = 0; p0 < D; p0 += TSIZE) {
        const int32_t pbl = p0 + tid;
        int32_t cnt = 0;
        if (pbl < D) {
          const uint64_t* rw = rows + (int64_t)pbl * NW;
          for (int k = pbl >> 6; k < NWa; ++k) {
            uint64_t w = rw[k];
            if (k == (pbl >> 6)) w &= ((pbl & 63) == 63) ? 0ull : (~0ull << ((pbl & 63) + 1));
            cnt += __popcll(w);
          }
        }
        int32_t tot;
        const int32_t excl = k4_scan<TSIZE>(cnt, &tot, scan, tid);
        if (TSIZE > TG_WAVE) {
          s_excl[tid] = excl;
          __syncthreads();
        }
        for (int32_t v = tid; v - tid < tot; v += TSIZE) {
          // owner: the largest lane o with excl[o] <= v
          int o = 0;
#pragma unroll
          for (int step = TSIZE / 2; step > 0; step >>= 1) {
            const int32_t ex = TSIZE <= TG_WAVE ? __shfl(excl, o + step, TSIZE) : s_excl[o + step];
            if (ex <= v) o += step;
          }
          const int32_t o_excl = TSIZE <= TG_WAVE ? __shfl(excl, o, TSIZE) : s_excl[o];
          if (v >= tot) continue;
          const int32_t pb = p0 + o;
          // pc: the (v - o_excl)-th set bit above pb in row(pb)
          int32_t kth = v - o_excl, pc = -1;
          const uint64_t* rb = rows + (int64_t)pb * NW;
          for (int k = pb >> 6; k < NWa && pc < 0; ++k) {
            uint64_t w = rb[k];
            if (k == (pb >> 6)) w &= ((pb & 63) == 63) ? 0ull : (~0ull << ((pb & 63) + 1));
            const int c = __popcll(w);
            if (kth >= c) {
              kth -= c;
              continue;
            }
            int base = 0;
            for (int sh = 32; sh > 0; sh >>= 1) {  // select the kth set bit
              const uint64_t low = w & ((1ull << sh) - 1ull);
              const int cl = __popcll(low);
              if (kth >= cl) {
                kth -= cl;
                w >>= sh;
                base += sh;
              } else {
                w = low;
              }
            }
            pc = (k << 6) + base;
          }
          const int32_t qb = qpos[pb], qc = qpos[pc];
          const int tb = tq[qb], tc = tq[qc];
          const uint64_t* rc = rows + (int64_t)pc * NW;
          int32_t e_bc = 0;
          if (!GLOB) {
            // the edge (b, c) sits in the out-list of its lower end
            const int32_t b = O[qb], c = O[qc];
            const bool b_low = precedes(A.deg[b], b, A.deg[c], c);
            const int32_t lo_n = b_low ? b : c, hi_n = b_low ? c : b;
            const int32_t s0 = A.out_off[lo_n];
            const int32_t r = lower_bound(A.out_col + s0, A.out_off[lo_n + 1] - s0, hi_n);
            e_bc = A.out_eid[s0 + r];
          }
          // typed popcounts of row(b) & row(c), one type range at a time
          // (GLOB: positions above both ends only)
          const int32_t lo_all = GLOB ? pc + 1 : 0;
          for (int u = 0; u < L; ++u) {
            const int32_t s0 = max(tstart[u], lo_all), s1 = tstart[u + 1];
            if (s0 >= s1) continue;
            uint32_t nv = 0;
            for (int32_t k = s0 >> 6; k <= (s1 - 1) >> 6; ++k) {
              const int32_t b0 = max(s0 - (k << 6), 0), b1 = min(s1 - (k << 6), 64);
              const uint64_t msk = (b1 >= 64 ? ~0ull : ((1ull << b1) - 1ull)) & ~((1ull << b0) - 1ull);
              nv += (uint32_t)__popcll(rb[k] & rc[k] & msk);
            }
            if (!nv) continue;
            if (GLOB) {
              gacc_add(ga, gsm, key_of(L, 7, phia, tb, tc, u), (uint64_t)nv);
              continue;
            }
            k4_credit(A, pair_index(phia, u), e_bc, nv);
            atomicAdd(&acc[(int64_t)pb * P + pair_index(tc, u)], nv);
            atomicAdd(&acc[(int64_t)pc * P + pair_index(tb, u)], nv);
          }
        }
        if (TSIZE > TG_WAVE) __syncthreads();
      }
      k4_sync<TSIZE>();
    }
    // ---- the edges at a (sums are twice the counts)
    if (!GLOB && !GSCR) {
      for (int64_t x = tid; x < (int64_t)D * P; x += TSIZE) {
        const int32_t q = (int32_t)(x / P);
        const int p = (int)(x - (int64_t)q * P);
        const uint32_t v = acc[(int64_t)pos[q] * P + p];
        if (v) k4_credit(A, p, A.out_eid[oa + q], v >> 1);
      }
    }
    if (!GLOB && GSCR) {
      // rows in global memory: instead of two global atomics per G_a edge,
      // each wavefront takes whole rows b and sums, over every neighbour c
      // of b in G_a, the typed popcounts of row(b) & row(c) in its own LDS
      // counters, then credits edge (a, b) once per type pair
      const int wv = tid / TG_WAVE, ln = lane();
      for (int32_t pb = wv; pb < D; pb += TSIZE / TG_WAVE) {
        for (int p = ln; p < P; p += TG_WAVE) accw[p] = 0u;
        wave_sync();
        const uint64_t* rb = rows + (int64_t)pb * NW;
        for (int32_t k = ln; k < NWa; k += TG_WAVE) {
          uint64_t bits = k4_load64<true>(rb + k);
          while (bits) {
            const int32_t pc = (k << 6) + __builtin_ctzll(bits);
            bits &= bits - 1ull;
            const uint64_t* rc = rows + (int64_t)pc * NW;
            const int tc = ptype[pc];
            for (int u = 0; u < L; ++u) {
              const int32_t s0 = tstart[u], s1 = tstart[u + 1];
              if (s0 >= s1) continue;
              uint32_t nv = 0;
              for (int32_t w = s0 >> 6; w <= (s1 - 1) >> 6; ++w) {
                const int32_t b0 = max(s0 - (w << 6), 0), b1 = min(s1 - (w << 6), 64);
                const uint64_t msk = (b1 >= 64 ? ~0ull : ((1ull << b1) - 1ull)) & ~((1ull << b0) - 1ull);
                nv += (uint32_t)__popcll(k4_load64<true>(rb + w) & k4_load64<true>(rc + w) & msk);
              }
              if (nv) atomicAdd(&accw[pair_index(tc, u)], nv);
            }
          }
        }
        wave_sync();
        const int32_t e_ab = A.out_eid[oa + qpos[pb]];
        for (int p = ln; p < P; p += TG_WAVE) {
          const uint32_t v = accw[p];
          if (v) k4_credit(A, p, e_ab, v >> 1);
        }
        wave_sync();
      }
    }
    k4_sync<TSIZE>();
  }
  if (GLOB) gacc_flush(ga, gsm);
}

// Nodes by out-degree tier: 0 (|O| < 3: no clique has them lowest), 1
// (|O| <= 64), 2 (<= 256), 3 (> 2048), 4 (> 1024), 5 (> 512), 6 (> 256),
// 7 (> TG_K4_LDS_IDS: the pass does not run).  Tiers 3-6 form one launch
// whose list runs from the largest out-degrees down.
__device__ __forceinline__ int k4_tier(int32_t D) {
  if (D < 3) return 0;
  if (D <= 64) return 1;
  if (D <= 256) return 2;
  if (D > TG_K4_LDS_IDS) return 7;
  return D > 2048 ? 3 : (D > 1024 ? 4 : (D > 512 ? 5 : 6));
}

// Per-workgroup LDS histograms, one global atomic per (workgroup, tier).
__global__ void __launch_bounds__(256) k_k4_tier_count(int64_t n, const int32_t* __restrict__ out_off,
                                                       int32_t* __restrict__ cnt, int32_t* __restrict__ dmax) {
  __shared__ int32_t h[9];
  if (threadIdx.x < 9) h[threadIdx.x] = 0;
  __syncthreads();
  int32_t my = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t D = out_off[v + 1] - out_off[v];
    atomicAdd(&h[k4_tier(D)], 1);
    my = max(my, D);
  }
  atomicMax(&h[8], my);
  __syncthreads();
  if (threadIdx.x < 8 && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 8) atomicMax(dmax, h[8]);
}

__global__ void __launch_bounds__(256) k_k4_tier_scatter(int64_t n, const int32_t* __restrict__ out_off,
                                                         int32_t* __restrict__ cursor, int32_t* __restrict__ list) {
  __shared__ int32_t h[8];
  __shared__ int32_t base[8];
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < n; t0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < 8) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t v = t0 + threadIdx.x;
    int tier = 0, local = 0;
    if (v < n) {
      tier = k4_tier(out_off[v + 1] - out_off[v]);
      if (tier > 0 && tier < 7) local = atomicAdd(&h[tier], 1);
    }
    __syncthreads();
    if (threadIdx.x < 8) base[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0;
    __syncthreads();
    if (v < n && tier > 0 && tier < 7) list[base[tier] + local] = (int32_t)v;
    __syncthreads();
  }
}

// Largest |T_ij| = sum of tau over all edges.
__global__ void __launch_bounds__(256) k_max_tsum_all(int64_t m, const uint32_t* __restrict__ tau, int L,
                                                      uint32_t* __restrict__ out) {
  __shared__ uint32_t h;
  if (threadIdx.x == 0) h = 0;
  __syncthreads();
  uint32_t my = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    uint32_t s = 0;
    for (int t = 0; t < L; ++t) s += tau[e * L + t];
    my = max(my, s);
  }
  atomicMax(&h, my);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, h);
}

}  // namespace tg
