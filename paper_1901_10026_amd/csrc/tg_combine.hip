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
//
// Two kernels per batch of edges.  The gather kernel builds T_ij and the
// accumulators A_i, A_j, Q, Mu (one team of TSIZE lanes per edge: 16 or 64
// lanes of a wavefront, or a 256-lane workgroup; AccT is their width, 32
// bits when |T_ij| is small) and stores them per edge; the row kernel turns
// them into orbits, graphlets and global key sums.  Keeping the identities
// out of the gather kernel keeps its register count, and so its occupancy,
// set by the intersection and 4-clique loops alone.

template <int TSIZE>
__device__ __forceinline__ void tsync() {
  if (TSIZE <= TG_WAVE) wave_sync();
  else __syncthreads();
}

// lanes of this thread's team, as bits 0..TSIZE-1 (TSIZE <= 64)
template <int TSIZE>
__device__ __forceinline__ uint64_t team_bits(uint64_t mask) {
  if (TSIZE >= TG_WAVE) return mask;
  const int sh = (lane() / TSIZE) * TSIZE;
  return (mask >> sh) & ((1ull << TSIZE) - 1ull);
}

__device__ __forceinline__ uint64_t bits_below(int tl) { return tl == 0 ? 0ull : (~0ull >> (64 - tl)); }

// Exclusive prefix sum over the team; *total gets the team sum.  For
// TSIZE == 256, scratch holds 4 + 256 ints of LDS.
template <int TSIZE>
__device__ __forceinline__ int32_t team_excl_scan(int32_t v, int32_t* total, int32_t* scratch, int tid) {
  if (TSIZE <= TG_WAVE) {
    const int tl = tid;
    int32_t x = v;
    for (int off = 1; off < TSIZE; off <<= 1) {
      const int32_t y = __shfl_up(x, off, TSIZE);
      if (tl >= off) x += y;
    }
    *total = __shfl(x, TSIZE - 1, TSIZE);
    return x - v;
  } else {
    const int ln = lane(), wv = tid / TG_WAVE;
    int32_t x = v;
    for (int off = 1; off < TG_WAVE; off <<= 1) {
      const int32_t y = __shfl_up(x, off, TG_WAVE);
      if (ln >= off) x += y;
    }
    if (ln == TG_WAVE - 1) scratch[wv] = x;
    __syncthreads();
    int32_t before = 0, tot = 0;
    for (int q = 0; q < TSIZE / TG_WAVE; ++q) {
      const int32_t c = scratch[q];
      if (q < wv) before += c;
      tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
  }
}

// Hash of T_ij for workgroup teams: slot = (node id << 4) | type, -1 empty;
// 2^TG_THASH_LOG2 slots in LDS, or, for a T_ij too long for LDS, 2^hlog
// slots of global scratch (over_hash_log2 of the scratch capacity).
#define TG_THASH_LOG2 12
#ifndef TG_THASH16_LOG2
#define TG_THASH16_LOG2 0
#endif
__device__ __forceinline__ uint32_t thash_home(int32_t k, int hlog) {
  return ((uint32_t)k * 2654435761u) >> (32 - hlog);
}

__host__ __device__ inline int over_hash_log2(int64_t cap) {
  int k = 6;
  while ((1ll << k) < 2 * cap) ++k;
  return k;
}

// int32 units of the global overflow scratch of `grid` workgroups with
// capacity `cap`: ids, types (bytes, rounded up to ints), hash slots
inline int64_t over_scratch_ints(int64_t grid, int64_t cap) {
  return grid * cap + (grid * cap + 3) / 4 + grid * (1ll << over_hash_log2(cap));
}

// Copies of the 4-clique cell counters: hits of one cell from several lanes
// of a wavefront spread over this many LDS words.
template <int TSIZE>
struct MuCopies {
  static constexpr int value = TSIZE >= 64 ? 8 : 4;
};

template <int TSIZE, class AccT, bool PROBE>
__device__ __forceinline__ void gather_edge(const EdgeArgs& A, int32_t e, int32_t* Tid, uint8_t* Tty,
                                            AccT* __restrict__ acc, AccT* __restrict__ out, int32_t* scratch,
                                            int tid, int32_t* Th, int hlog, bool th_global) {
  const int L = A.L, LL = L * L, P = L * (L + 1) / 2;
  const int R = 2 * L + 6 * P;
  AccT* Aa = acc;
  AccT* Ab = acc + LL;
  AccT* Q = acc + 2 * LL;
  AccT* Mu = acc + 3 * LL;  // PROBE: MuCopies<TSIZE> copies, lane l adds to copy l % copies
  for (int x = tid; x < (PROBE ? 3 + MuCopies<TSIZE>::value : 3) * LL; x += TSIZE) acc[x] = 0;
  if (Th)
    for (int x = tid; x < (1 << hlog); x += TSIZE) Th[x] = -1;
  tsync<TSIZE>();
  const int32_t i = A.ei[e], j = A.ej[e];
  const int32_t di = A.deg[i], dj = A.deg[j];
  const bool a_is_i = di <= dj;
  const int32_t a = a_is_i ? i : j, b = a_is_i ? j : i;
  const int32_t la = a_is_i ? di : dj, lb = a_is_i ? dj : di;
  const int32_t ra = A.rp[a], rb = A.rp[b];
  const int wv = tid / TG_WAVE;

  // ---- T_ij with the sums of tau and D over its members
  // sa, sb: the CSR slots of k in the rows of a and b
  auto add_member = [&](int32_t k, int t, int64_t sa, int64_t sb) {
    for (int u = 0; u < L; ++u) {
      const uint32_t va = A.tau_s[sa * L + u];
      if (va) atomicAdd(&Aa[t * L + u], (AccT)va);
      const uint32_t vb = A.tau_s[sb * L + u];
      if (vb) atomicAdd(&Ab[t * L + u], (AccT)vb);
      const uint32_t vd = A.D[(int64_t)k * L + u];
      if (vd) atomicAdd(&Q[t * L + u], (AccT)vd);
    }
  };
  auto hash_member = [&](int32_t k, int t) {
    uint32_t h = thash_home(k, hlog);
    while (atomicCAS(&Th[h], -1, (k << 4) | t) != -1) h = (h + 1) & ((1u << hlog) - 1);
  };
  int32_t nT = 0;
  if (A.tl_off) {
    // kept by the tau pass, in id order: |T_ij| is the sum of tau(i, j)
    for (int u = 0; u < L; ++u) nT += (int32_t)A.tau[(int64_t)e * L + u];
    const int64_t base = A.tl_off[e];
    for (int32_t q = tid; q < nT; q += TSIZE) {
      const int32_t v = A.tl_k[base + q];
      const int32_t k = A.tl_packed ? (v >> 4) : v;
      const int t = A.tl_packed ? (v & 15) : A.ty[k];
      add_member(k, t, A.tl_e[2 * (base + q)], A.tl_e[2 * (base + q) + 1]);
      if (PROBE) {
        Tid[q] = k;
        Tty[q] = (uint8_t)t;
        if (Th) hash_member(k, t);
      }
    }
  } else {
  // without PROBE nothing keeps T: |T_ij| is the sum of tau(i, j), and the
  // members need no positions (no ballot, no barrier per chunk)
  if (!PROBE)
    for (int u = 0; u < L; ++u) nT += (int32_t)A.tau[(int64_t)e * L + u];
  // a hub's row is searched in its bitmap (two loads per id)
  const int32_t hb = A.hub_of ? A.hub_of[b] : -1;
  const uint64_t* hbits = hb >= 0 ? A.hub_bits + (int64_t)hb * A.hub_nw : nullptr;
  const int32_t* hrank = hb >= 0 ? A.hub_rank + (int64_t)hb * A.hub_nw : nullptr;
  for (int32_t b0 = 0; b0 < la; b0 += TSIZE) {
    const int32_t idx = b0 + tid;
    bool found = false;
    int32_t k = 0, p = 0;
    if (idx < la) {
      k = A.ci[ra + idx];
      if (hbits) {
        const uint64_t w = hbits[k >> 6];
        found = (w >> (k & 63)) & 1ull;
        if (found) p = hrank[k >> 6] + __popcll(w & ((1ull << (k & 63)) - 1ull));
      } else {
        p = lower_bound(A.ci + rb, lb, k);
        found = p < lb && A.ci[rb + p] == k;
      }
    }
    int t = 0;
    if (found) {
      t = A.ty[k];
      add_member(k, t, ra + idx, rb + p);
    }
    if (!PROBE) continue;
    const uint64_t wmask = ballot(found);
    int32_t before, total;
    if (TSIZE <= TG_WAVE) {
      const uint64_t tm = team_bits<TSIZE>(wmask);
      before = __popcll(tm & bits_below(tid));
      total = __popcll(tm);
    } else {
      if (lane() == 0) scratch[wv] = __popcll(wmask);
      __syncthreads();
      before = __popcll(wmask & bits_below(lane()));
      total = 0;
      for (int q = 0; q < TSIZE / TG_WAVE; ++q) {
        const int32_t c = scratch[q];
        if (q < wv) before += c;
        total += c;
      }
      __syncthreads();
    }
    if (PROBE && found) {
      Tid[nT + before] = k;
      Tty[nT + before] = (uint8_t)t;
      if (Th) hash_member(k, t);
    }
    nT += total;
  }
  }
  tsync<TSIZE>();

  // element visits: building T (three list words per member, or a search
  // of the longer row per element of the shorter one), then its tau/D sums
  uint64_t my_work = 0;
  if (A.work && tid == 0)
    my_work = (A.tl_off ? (uint64_t)nT * 3u : (uint64_t)la * (uint64_t)(1 + (lb > 0 ? 32 - __clz(lb) : 0))) +
              (uint64_t)nT * 3u * (uint64_t)L + (uint64_t)(P + L);

  // ---- typed edges inside T (4-cliques through (i, j)), each found from its
  // lower end's degree-ordered out-list; (member, out-slot) pairs are dealt
  // to lanes through a team prefix sum.  Without PROBE the clique pass has
  // counted them already.
  int32_t* s_excl = scratch + 8;  // TSIZE == 256 only
  for (int32_t q0 = 0; PROBE && q0 < nT; q0 += TSIZE) {
    const int32_t q = q0 + tid;
    int32_t ostart = 0, ocnt = 0, tk = 0;
    if (q < nT) {
      const int32_t k = Tid[q];
      ostart = A.out_off[k];
      ocnt = A.out_off[k + 1] - ostart;
      tk = Tty[q];
    }
    int32_t tot;
    const int32_t excl = team_excl_scan<TSIZE>(ocnt, &tot, scratch, tid);
    if (A.work && tid == 0) my_work += (uint64_t)tot + (uint64_t)min(TSIZE, nT - q0);
    if (TSIZE > TG_WAVE) {
      s_excl[tid] = excl;
      s_excl[TSIZE + tid] = ostart;
      s_excl[2 * TSIZE + tid] = tk;
      __syncthreads();
    }
    // U (member, out-slot) pairs per lane at a time; their owner searches,
    // out-list loads and first table reads are issued together so that the
    // lookups of the U pairs overlap
    constexpr int U = 4;
    for (int32_t c0 = 0; c0 < tot; c0 += TSIZE * U) {
      int32_t v[U], o[U], r[U];
      int rtk[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        v[k] = c0 + k * TSIZE + tid;
        o[k] = 0;
      }
      // owner of pair v: the largest member q with excl[q] <= v
#pragma unroll
      for (int step = TSIZE / 2; step > 0; step >>= 1) {
        int32_t ex[U];
#pragma unroll
        for (int k = 0; k < U; ++k) ex[k] = TSIZE <= TG_WAVE ? __shfl(excl, o[k] + step, TSIZE) : s_excl[o[k] + step];
#pragma unroll
        for (int k = 0; k < U; ++k)
          if (ex[k] <= v[k]) o[k] += step;
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        int32_t o_excl, o_start;
        if (TSIZE <= TG_WAVE) {
          o_excl = __shfl(excl, o[k], TSIZE);
          o_start = __shfl(ostart, o[k], TSIZE);
          rtk[k] = __shfl(tk, o[k], TSIZE);
        } else {
          o_excl = s_excl[o[k]];
          o_start = s_excl[TSIZE + o[k]];
          rtk[k] = s_excl[2 * TSIZE + o[k]];
        }
        r[k] = v[k] < tot ? A.out_col[o_start + (v[k] - o_excl)] : -1;
      }
      // membership of r in T and its type
      int cellv[U];
      if (Th) {
        const uint32_t hmask = (1u << hlog) - 1;
        // a table in global scratch was filled by device-scope atomics: read
        // it at device scope too, past this CU's cache
        auto th_read = [&](uint32_t hh) {
          return th_global ? __hip_atomic_load(&Th[hh], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : Th[hh];
        };
        // the home slot and the next one are read for all U ids at once and
        // decide almost every lookup without a branch; only a run of more
        // than two occupied slots goes on probing
        uint32_t h[U];
        int32_t sv[U], sw[U];
#pragma unroll
        for (int k = 0; k < U; ++k) h[k] = thash_home(r[k] >= 0 ? r[k] : 0, hlog);
#pragma unroll
        for (int k = 0; k < U; ++k) {
          sv[k] = r[k] >= 0 ? th_read(h[k]) : -1;
          sw[k] = r[k] >= 0 ? th_read((h[k] + 1) & hmask) : -1;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const bool hit0 = sv[k] != -1 && (sv[k] >> 4) == r[k];
          const bool hit1 = sv[k] != -1 && sw[k] != -1 && (sw[k] >> 4) == r[k];
          cellv[k] = hit0 ? rtk[k] * L + (sv[k] & 15) : (hit1 ? rtk[k] * L + (sw[k] & 15) : -1);
          if (!hit0 && !hit1 && sv[k] != -1 && sw[k] != -1) {
            uint32_t hh = (h[k] + 2) & hmask;
            int32_t x = th_read(hh);
            while (x != -1) {
              if ((x >> 4) == r[k]) {
                cellv[k] = rtk[k] * L + (x & 15);
                break;
              }
              hh = (hh + 1) & hmask;
              x = th_read(hh);
            }
          }
        }
      } else {
        // lower bound in the sorted ids, the same steps for all U pairs
        int32_t pos[U];
#pragma unroll
        for (int k = 0; k < U; ++k) pos[k] = 0;
        int top = 1;
        while (top * 2 <= nT) top *= 2;
        for (int step = top; step > 0; step >>= 1) {
          int32_t tv[U];
#pragma unroll
          for (int k = 0; k < U; ++k) tv[k] = pos[k] + step <= nT ? Tid[pos[k] + step - 1] : INT32_MAX;
#pragma unroll
          for (int k = 0; k < U; ++k)
            if (tv[k] < r[k]) pos[k] += step;
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
          cellv[k] = (r[k] >= 0 && pos[k] < nT && Tid[pos[k]] == r[k]) ? rtk[k] * L + Tty[pos[k]] : -1;
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        if (cellv[k] >= 0) atomicAdd(&Mu[(lane() % MuCopies<TSIZE>::value) * LL + cellv[k]], (AccT)1);
      }
    }
    if (TSIZE > TG_WAVE) __syncthreads();
  }
  if (A.work && tid == 0 && my_work) atomicAdd((unsigned long long*)&A.work[e], (unsigned long long)my_work);
  tsync<TSIZE>();
  if (PROBE) {
    for (int x = tid; x < LL; x += TSIZE) {
      AccT sum = Mu[x];
      for (int c = 1; c < MuCopies<TSIZE>::value; ++c) sum += Mu[c * LL + x];
      Mu[x] = sum;
    }
    tsync<TSIZE>();
  }
  if (out)
    for (int x = tid; x < (PROBE ? 4 : 3) * LL; x += TSIZE) out[x] = acc[x];
  tsync<TSIZE>();
}

// Orbits, graphlets (per-edge row) and global key sums of edge e from its
// gathered accumulators ea = [A_a | A_b | Q | Mu] (a = the endpoint with the
// shorter row).  One team of TSIZE lanes per edge.
template <int TSIZE, class AccT>
__device__ __forceinline__ void edge_rows(const EdgeArgs& A, int32_t e, const AccT* __restrict__ ea,
                                          uint64_t* gacc, int tid, uint64_t* stage = nullptr,
                                          int64_t* opos_out = nullptr) {
  const int L = A.L, LL = L * L, P = L * (L + 1) / 2;
  const int R = 2 * L + 6 * P;
  const int32_t i = A.ei[e], j = A.ej[e];
  const bool a_is_i = A.deg[i] <= A.deg[j];
  const AccT* Aa = ea;
  const AccT* Ab = ea + LL;
  const AccT* Q = ea + 2 * LL;
  const AccT* Mu = ea + 3 * LL;
  // ---- per type pair: every orbit, then every graphlet
  const int pi = A.ty[i], pj = A.ty[j];
  const AccT* Ai = a_is_i ? Aa : Ab;
  const AccT* Aj = a_is_i ? Ab : Aa;
  const uint32_t* tau_e = A.tau + (int64_t)e * L;
  const uint32_t* Di = A.D + (int64_t)i * L;
  const uint32_t* Dj = A.D + (int64_t)j * L;
  const uint64_t* Ui = A.Un + (int64_t)i * LL;
  const uint64_t* Uj = A.Un + (int64_t)j * LL;
  const uint64_t* Pi = A.Pn + (int64_t)i * LL;
  const uint64_t* Pj = A.Pn + (int64_t)j * LL;
  // output position of this edge (listed ids or range), -1 if none
  int64_t opos = -1;
  if (A.edge_counts || A.edge_orbits || A.sp_keys) {
    if (A.edge_ids) {
      int64_t lo = 0, hi = A.n_edge_ids;  // first id >= e
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (A.edge_ids[mid] < e) lo = mid + 1; else hi = mid;
      }
      if (lo < A.n_edge_ids && A.edge_ids[lo] == e) opos = lo;
    } else if (e >= A.edge_begin && e < A.edge_end) {
      opos = e - A.edge_begin;
    }
  }
  uint64_t* row = (A.edge_counts && opos >= 0) ? A.edge_counts + opos * R : nullptr;
  if (stage && opos >= 0) row = stage;  // sparse output: the row is staged, then emitted
  if (opos_out) *opos_out = opos;
  // orbit row: g1[t], g2[t], then g3..g12 in blocks of P
  uint64_t* orow = (A.edge_orbits && opos >= 0) ? A.edge_orbits + opos * (2 * L + 10 * P) : nullptr;
  auto gadd = [&](int64_t key, int64_t v) {
    if (v == 0) return;
    if (gacc) atomicAdd((unsigned long long*)&gacc[key], (unsigned long long)v);
    else if (A.global_sums) atomicAdd((unsigned long long*)&A.global_sums[key], (unsigned long long)v);
  };
  auto Tn = [&](int x) -> int64_t { return (int64_t)tau_e[x]; };
  auto Si = [&](int x) -> int64_t { return (int64_t)Di[x] - tau_e[x] - (pj == x ? 1 : 0); };
  auto Sj = [&](int x) -> int64_t { return (int64_t)Dj[x] - tau_e[x] - (pi == x ? 1 : 0); };
  for (int c = tid; c < L; c += TSIZE) {
    const int64_t wedge = Si(c) + Sj(c), tri = Tn(c);
    if (row) { row[c] = (uint64_t)wedge; row[L + c] = (uint64_t)tri; }
    if (orow) { orow[c] = (uint64_t)wedge; orow[L + c] = (uint64_t)tri; }
    gadd(key_of(L, 0, pi, pj, c, 0), wedge);
    gadd(key_of(L, 1, pi, pj, c, 0), tri);
  }
  for (int p = tid; p < P; p += TSIZE) {
    int u = 0;
    while ((u + 1) * (u + 2) / 2 <= p) ++u;
    const int t = p - u * (u + 1) / 2;
    auto sym = [&](auto f) -> int64_t { return t == u ? f(t, t) : f(t, u) + f(u, t); };
    // M(x, y): edges between T^x and T^y counted from both ends, i.e. the
    // 4-cliques through (i, j) with other types {x, y}, twice when x == y
    auto k4 = [&](int x, int y) -> int64_t {
      const int64_t q = (int64_t)e * P + pair_index(x, y);
      return A.K4w ? (int64_t)A.K4w[q] : (int64_t)A.K4n[q];
    };
    const bool have_k4 = A.K4w || A.K4n;
    auto M = [&](int x, int y) -> int64_t {
      if (have_k4) return (x == y ? 2 : 1) * k4(x, y);
      return (int64_t)Mu[x * L + y] + (int64_t)Mu[y * L + x];
    };
    auto ETSi = [&](int x, int y) -> int64_t { return (int64_t)Ai[x * L + y] - Tn(x) * (pj == y) - M(x, y); };
    auto ETSj = [&](int x, int y) -> int64_t { return (int64_t)Aj[x * L + y] - Tn(x) * (pi == y) - M(x, y); };
    auto ETI = [&](int x, int y) -> int64_t {
      return (int64_t)Q[x * L + y] - Tn(x) * ((pi == y) + (pj == y)) - M(x, y) - ETSi(x, y) - ETSj(x, y);
    };
    const int64_t g12 = have_k4 ? k4(t, u) : sym([&](int x, int y) -> int64_t { return (int64_t)Mu[x * L + y]; });
    const int64_t g10 = sym(ETSi) + sym(ETSj);
    const int64_t g8 = sym(ETI);
    const int64_t sSiSi = sym([&](int x, int y) -> int64_t { return (int64_t)Ui[x * L + y]; })
                        - sym([&](int x, int y) -> int64_t { return (pj == x) ? Tn(y) : 0; })
                        - sym([&](int x, int y) -> int64_t { return (int64_t)Ai[x * L + y]; }) - sym(ETSi);
    const int64_t sSjSj = sym([&](int x, int y) -> int64_t { return (int64_t)Uj[x * L + y]; })
                        - sym([&](int x, int y) -> int64_t { return (pi == x) ? Tn(y) : 0; })
                        - sym([&](int x, int y) -> int64_t { return (int64_t)Aj[x * L + y]; }) - sym(ETSj);
    const int64_t g7 = (sSiSi + sSjSj) / 2;
    const int64_t ci4 = A.c4_rows ? (int64_t)p * A.c4_rows + e : (int64_t)e * P + p;
    const int64_t c4 = A.c4_wide ? (int64_t)A.C4[ci4] : (int64_t)A.C4n[ci4];
    const int64_t g6 = c4 - g10 - 2 * g12;
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
    if (orow) {
      const int64_t g[10] = {g3, g4, g5, g6, g7, g8, g9, g10, g11, g12};
      for (int q = 0; q < 10; ++q) orow[2 * L + q * P + p] = (uint64_t)g[q];
    }
    const int64_t h[6] = {g3 + g4, g5, g6, g7 + g8 + g9, g10 + g11, g12};  // Eqs. 11-16
    for (int s = 0; s < 6; ++s) {
      if (row) row[2 * L + s * P + p] = (uint64_t)h[s];
      gadd(key_of(L, 2 + s, pi, pj, t, u), h[s]);
    }
  }
}

// Capacity of T_ij kept in LDS per team.
template <int TSIZE>
struct TeamCap {
  static constexpr int value = TSIZE == 16 ? 64 : (TSIZE == 64 ? 256 : TG_T_WG_CAP);
};

// log2 of the LDS hash slots of T_ij per team (0: no hash; the sorted ids are
// searched instead): four slots per id of capacity for wavefront teams, two
// for workgroup teams
template <int TSIZE>
struct THashLog2 {
  static constexpr int value = TSIZE == 16 ? TG_THASH16_LOG2 : (TSIZE == 64 ? 10 : TG_THASH_LOG2);
};

// Gather kernel: one team per edge, grid-stride over list[0, count); the
// accumulators of list[w] go to ea[w * 4L^2 ...] (or nowhere when ea is
// null: work measurement only).  LDS per team: [acc 4L^2 AccT][scan
// scratch][T hash (workgroup teams)][T ids][T types].  A T_ij larger than
// the team's capacity (workgroup teams only) is kept in this workgroup's
// slice of a global scratch.
template <int TSIZE, class AccT, bool PROBE>
__global__ void __launch_bounds__(256) k_combine(EdgeArgs A, int64_t count, const int32_t* __restrict__ list,
                                                 AccT* __restrict__ ea, int32_t* __restrict__ t_over,
                                                 int64_t t_over_cap) {
  extern __shared__ uint64_t smem_comb[];
  constexpr int TEAMS = 256 / TSIZE;
  // without PROBE, T_ij is streamed into the sums and not kept
  constexpr int TCAP = PROBE ? TeamCap<TSIZE>::value : 0;
  constexpr int SCR = TSIZE > TG_WAVE ? 8 + 3 * TSIZE : 8;
  const int LL = A.L * A.L;
  const int team = threadIdx.x / TSIZE, tid = threadIdx.x % TSIZE;
  // per-team region, in bytes, rounded to 8
  constexpr int HBYTES = (PROBE && THashLog2<TSIZE>::value) ? (4 << THashLog2<TSIZE>::value) : 0;
  const int acc_bytes = (PROBE ? 3 + MuCopies<TSIZE>::value : 3) * LL * (int)sizeof(AccT);
  const int region = ((acc_bytes + SCR * 4 + HBYTES + TCAP * 5) + 7) & ~7;
  char* base = (char*)smem_comb + (int64_t)team * region;
  AccT* acc = (AccT*)base;
  int32_t* scratch = (int32_t*)(base + acc_bytes);
  int32_t* Th = (HBYTES && A.thash_ok) ? scratch + SCR : nullptr;
  int32_t* Tid_l = scratch + SCR + HBYTES / 4;
  uint8_t* Tty_l = (uint8_t*)(Tid_l + TCAP);
  int32_t* Tid_g = t_over ? t_over + (int64_t)blockIdx.x * t_over_cap : nullptr;
  uint8_t* Tty_g = t_over ? (uint8_t*)(t_over + (int64_t)gridDim.x * t_over_cap) + (int64_t)blockIdx.x * t_over_cap
                          : nullptr;
  // a T_ij past the LDS capacity keeps its hash in global scratch too
  const int hlog_g = t_over ? over_hash_log2(t_over_cap) : 0;
  int32_t* Th_g = (t_over && A.thash_ok)
                      ? t_over + (int64_t)gridDim.x * t_over_cap + ((int64_t)gridDim.x * t_over_cap + 3) / 4 +
                            (int64_t)blockIdx.x * (1ll << hlog_g)
                      : nullptr;
  for (int64_t w = (int64_t)blockIdx.x * TEAMS + team; w < count; w += (int64_t)gridDim.x * TEAMS) {
    const int32_t e = list[w];
    bool big = false;
    uint32_t tsum = 0;
    if (PROBE && TSIZE > TG_WAVE) {
      for (int t = 0; t < A.L; ++t) tsum += A.tau[(int64_t)e * A.L + t];
      big = tsum > (uint32_t)TCAP;
    }
    // a global table sized for this T_ij (at most the block's 2^hlog_g slots)
    // keeps the probed region small
    gather_edge<TSIZE, AccT, PROBE>(A, e, big ? Tid_g : Tid_l, big ? Tty_g : Tty_l, acc,
                             ea ? ea + w * 4 * LL : nullptr, scratch, tid, big ? Th_g : Th,
                             big ? min(hlog_g, over_hash_log2(tsum)) : THashLog2<TSIZE>::value, big);
  }
}

// LDS bytes of k_combine<TSIZE, AccT, PROBE>
template <int TSIZE, class AccT, bool PROBE>
inline size_t combine_lds_bytes(int L) {
  constexpr int TCAP = PROBE ? TeamCap<TSIZE>::value : 0;
  constexpr int SCR = TSIZE > TG_WAVE ? 8 + 3 * TSIZE : 8;
  constexpr int HBYTES = (PROBE && THashLog2<TSIZE>::value) ? (4 << THashLog2<TSIZE>::value) : 0;
  const int acc_bytes = (PROBE ? 3 + MuCopies<TSIZE>::value : 3) * L * L * (int)sizeof(AccT);
  const int region = ((acc_bytes + SCR * 4 + HBYTES + TCAP * 5) + 7) & ~7;
  return (size_t)(256 / TSIZE) * region;
}

// Nonzero (global key, count) pairs of one row staged in LDS, in column
// order: columns are taken TS at a time, one per lane, and the nonzero ones
// are packed by a ballot; the edge's pairs go at a cursor reserved once per
// edge.
template <int TS>
__device__ __forceinline__ void sparse_emit(const EdgeArgs& A, int32_t e, int64_t opos, const uint64_t* stage,
                                            int R, int tid) {
  const int L = A.L, P = L * (L + 1) / 2;
  wave_sync();  // the staged row was written by the other lanes of the team
  int32_t nz = 0;
  for (int c0 = 0; c0 < R; c0 += TS) {
    const bool on = c0 + tid < R && stage[c0 + tid] != 0;
    nz += __popcll(team_bits<TS>(ballot(on)));
  }
  int64_t base = 0;
  if (tid == 0) base = (int64_t)atomicAdd(A.sp_cursor, (unsigned long long)nz);
  base = __shfl(base, (lane() / TS) * TS, TG_WAVE);
  if (tid == 0) {
    A.sp_start[opos] = base;
    A.sp_len[opos] = nz;
  }
  if (base + nz > A.sp_cap) return;  // counted, not written: the caller sees the total
  const int pi = A.ty[A.ei[e]], pj = A.ty[A.ej[e]];
  int64_t at = base;
  for (int c0 = 0; c0 < R; c0 += TS) {
    const int c = c0 + tid;
    const uint64_t v = c < R ? stage[c] : 0ull;
    const uint64_t mask = team_bits<TS>(ballot(v != 0));
    if (v) {
      int64_t key;
      if (c < 2 * L) {
        key = key_of(L, c / L, pi, pj, c % L, 0);
      } else {
        const int h = (c - 2 * L) / P, p = (c - 2 * L) % P;
        int u = 0;
        while ((u + 1) * (u + 2) / 2 <= p) ++u;
        key = key_of(L, 2 + h, pi, pj, p - u * (u + 1) / 2, u);
      }
      const int64_t q = at + __popcll(mask & bits_below(tid));
      A.sp_keys[q] = (uint32_t)key;
      A.sp_counts[q] = v;
    }
    at += __popcll(mask);
  }
  wave_sync();  // the stage is rewritten by the team's next edge
}

// Row kernel: one 16-lane team per edge of list[0, count), accumulators
// from ea (as written by the gather kernel over the same list); global key
// sums are gathered in LDS first when gacc_in_lds.
template <class AccT>
__global__ void __launch_bounds__(256) k_combine_rows(EdgeArgs A, int64_t count, const int32_t* __restrict__ list,
                                                      const AccT* __restrict__ ea, int nkeys) {
  extern __shared__ uint64_t smem_rows[];
  constexpr int TS = 16, TEAMS = 256 / TS;
  const int LL = A.L * A.L;
  uint64_t* gacc = A.gacc_in_lds ? smem_rows : nullptr;
  if (gacc)
    for (int x = threadIdx.x; x < nkeys; x += blockDim.x) gacc[x] = 0;
  __syncthreads();
  const int team = threadIdx.x / TS, tid = threadIdx.x % TS;
  const int P = A.L * (A.L + 1) / 2, R = 2 * A.L + 6 * P;
  // sparse output: each team's row staged in LDS after the key sums
  uint64_t* stage = A.sp_keys ? smem_rows + (A.gacc_in_lds ? nkeys : 0) + team * R : nullptr;
  for (int64_t w = (int64_t)blockIdx.x * TEAMS + team; w < count; w += (int64_t)gridDim.x * TEAMS) {
    const int32_t e = list[w];
    int64_t opos = -1;
    edge_rows<TS, AccT>(A, e, ea + w * 4 * LL, gacc, tid, stage, &opos);
    if (stage && opos >= 0) sparse_emit<TS>(A, e, opos, stage, R, tid);
  }
  __syncthreads();
  if (gacc)
    for (int x = threadIdx.x; x < nkeys; x += blockDim.x)
      if (gacc[x]) atomicAdd((unsigned long long*)&A.global_sums[x], (unsigned long long)gacc[x]);
}
