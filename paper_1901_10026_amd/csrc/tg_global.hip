// ------------------------------------------------------- global, once --
//
// Global typed-graphlet counts with every instance counted a fixed number of
// times instead of once per edge (the Global Typed Graphlet Counts section
// remarks that an ordering lets a global-only count avoid the per-edge
// repetitions).  The kernels below sum, per type multiset, NON-induced counts
// N of the eight shape patterns; the finalize kernel turns them into the
// induced counts that Eq. 17 gives from the per-edge rows.
//
// A node set whose induced subgraph is H holds a fixed number of copies of
// each pattern (edge subsets of H isomorphic to it), and every copy carries
// the set's type multiset, so per multiset
//   N_wedge   = I_wedge + 3 I_triangle
//   N_path    = I_path + 4 I_cycle + 2 I_tailed + 6 I_chordal + 12 I_clique
//   N_star    = I_star + I_tailed + 2 I_chordal + 4 I_clique
//   N_cycle   = I_cycle + I_chordal + 3 I_clique
//   N_tailed  = I_tailed + 4 I_chordal + 12 I_clique
//   N_chordal = I_chordal + 6 I_clique
//   N_clique  = I_clique
// Sources of the sums (the key vector holds them, shape by shape, until the
// finalize kernel):
//   wedges, stars: per centre c from its typed degrees D[c] (k_glob_nodes);
//   per edge (a, b) from tau_ab and D[a], D[b] (k_glob_edges): triangles
//   (each reached from its 3 edges), 4-paths (once, by the middle edge),
//   chordal cycles (once, by the chord), tailed triangles (twice: the
//   triangle edge at the tail's node that is not the other one);
//   4-cycles: twice, from the degree-ordered wedge pass (GLOB variants of
//   k_c4_hash, phase 3 of k_c4_group, k_c4_scan);
//   4-cliques: once, from their two lowest nodes a < b in degree order as the
//   typed edges inside T+_ab = {k ~ a, k ~ b, b before k} = out(a) ∩ out(b)
//   (k_glob_k4).

// Typed 4-cycles from the count rows of one heavy group of the wedge pass,
// after its counting phase: row (x, w) holds the typed middle counts c_t of
// x's wedges x-u-w, and the cycles with opposite corners x and w and middle
// types {s, t} number c_s c_t (s < t) or C(c_s, 2) -- each cycle once, since
// x is its highest node and w is fixed by x.  The sums are doubled to match
// the wedge-based sums of the other tiers.  Every nonzero row (and, for hash
// tables, its key) is cleared on the way, which replaces the clearing pass.
// Rows: dense groups, row q * n + w for group node q (count array of RW
// words per row); hashed groups, table row h of the node q with
// hoff[q] <= h < hoff[q + 1], far end hkeys[h] (-1: empty).
template <bool HALF, bool HASH>
__global__ void __launch_bounds__(256) k_c4_scan(int64_t nrows, uint32_t* __restrict__ cnt, int RW, int64_t n,
                                                 int Gg, const int32_t* __restrict__ gx,
                                                 const int64_t* __restrict__ hoff, int32_t* __restrict__ hkeys,
                                                 const uint8_t* __restrict__ ty, int L, GAcc ga) {
  extern __shared__ uint64_t gsm_scan[];
  gacc_init(ga, gsm_scan);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    int32_t w;
    int q;
    if (HASH) {
      w = hkeys[r];
      if (w < 0) continue;
      hkeys[r] = -1;
      int lo = 0, hi = Gg;  // largest q with hoff[q] <= r
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (hoff[mid] <= r) lo = mid; else hi = mid;
      }
      q = lo;
    } else {
      q = (int)(r / n);
      w = (int32_t)(r - (int64_t)q * n);
    }
    uint4* row = reinterpret_cast<uint4*>(cnt + r * RW);
    uint32_t c[16];
    bool any = false;
    for (int q4 = 0; q4 < RW / 4; ++q4) {
      const uint4 v4 = row[q4];
      any |= (v4.x | v4.y | v4.z | v4.w) != 0u;
      const uint32_t wd[4] = {v4.x, v4.y, v4.z, v4.w};
      for (int k = 0; k < 4; ++k) {
        if (HALF) {
          c[8 * q4 + 2 * k] = wd[k] & 0xffffu;
          c[8 * q4 + 2 * k + 1] = wd[k] >> 16;
        } else {
          c[4 * q4 + k] = wd[k];
        }
      }
    }
    if (!any) continue;
    for (int q4 = 0; q4 < RW / 4; ++q4) row[q4] = make_uint4(0u, 0u, 0u, 0u);
    const int phx = ty[gx[q]], phw = ty[w];
    for (int t = 0; t < L; ++t) {
      const uint64_t ct = c[t];
      if (!ct) continue;
      if (ct >= 2) gacc_add(ga, gsm_scan, key_of(L, 4, phx, phw, t, t), ct * (ct - 1));
      for (int s = 0; s < t; ++s)
        if (c[s]) gacc_add(ga, gsm_scan, key_of(L, 4, phx, phw, s, t), 2 * ct * c[s]);
    }
  }
  gacc_flush(ga, gsm_scan);
}

// multiset t1 <= t2 of colex rank q (q < L(L+1)/2)
__device__ __forceinline__ void unrank2(int q, int& t1, int& t2) {
  t2 = 0;
  while ((t2 + 1) * (t2 + 2) / 2 <= q) ++t2;
  t1 = q - t2 * (t2 + 1) / 2;
}

// multiset t1 <= t2 <= t3 of colex rank q (q < C(L+2, 3))
__device__ __forceinline__ void unrank3(int q, int& t1, int& t2, int& t3) {
  t3 = 0;
  while ((t3 + 1) * (t3 + 2) * (t3 + 3) / 6 <= q) ++t3;
  unrank2(q - t3 * (t3 + 1) * (t3 + 2) / 6, t1, t2);
}

// Non-induced wedges and 3-stars by centre, one 16-lane team per node.
__global__ void __launch_bounds__(256) k_glob_nodes(int64_t n, const int32_t* __restrict__ deg,
                                                    const uint32_t* __restrict__ D, const uint8_t* __restrict__ ty,
                                                    int L, GAcc ga) {
  extern __shared__ uint64_t gsm_nodes[];
  gacc_init(ga, gsm_nodes);
  constexpr int TS = 16;
  const int tl = threadIdx.x % TS;
  const int64_t teams = (int64_t)gridDim.x * (blockDim.x / TS);
  const int P = L * (L + 1) / 2, T3 = L * (L + 1) * (L + 2) / 6;
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / TS) + threadIdx.x / TS; v < n; v += teams) {
    const int32_t dv = deg[v];
    if (dv < 2) continue;
    const uint32_t* Dv = D + v * L;
    const int ph = ty[v];
    for (int q = tl; q < P; q += TS) {
      int t1, t2;
      unrank2(q, t1, t2);
      const uint64_t a = Dv[t1], b = Dv[t2];
      const uint64_t val = t1 == t2 ? (uint64_t)c2((int64_t)a) : a * b;
      if (val) gacc_add(ga, gsm_nodes, key_of(L, 0, ph, t1, t2, 0), val);
    }
    if (dv < 3) continue;
    for (int q = tl; q < T3; q += TS) {
      int t1, t2, t3;
      unrank3(q, t1, t2, t3);
      const uint64_t a = Dv[t1], b = Dv[t2], c = Dv[t3];
      uint64_t val;
      if (t1 == t3) val = (uint64_t)c3((int64_t)a);
      else if (t1 == t2) val = (uint64_t)c2((int64_t)a) * c;
      else if (t2 == t3) val = a * (uint64_t)c2((int64_t)b);
      else val = a * b * c;
      if (val) gacc_add(ga, gsm_nodes, key_of(L, 3, ph, t1, t2, t3), val);
    }
  }
  gacc_flush(ga, gsm_nodes);
}

// Per edge (a, b) with typed common-neighbour counts tau and typed degrees
// Da, Db (one 16-lane team per edge):
//   triangles  {phi_a, phi_b, t}: tau[t]                      (3 per triangle)
//   4-paths    {phi_a, phi_b, s, t}, s at a's side, t at b's:
//              (Da[s] - [phi_b = s]) (Db[t] - [phi_a = t]) - [s = t] tau[s]
//   chordal    {phi_a, phi_b, s, t}, s <= t: pairs of common neighbours
//   tailed     {phi_a, phi_b, t, s}: tau[t] (Da[s] + Db[s] - [phi_b = s]
//              - [phi_a = s] - 2 [s = t])   (2 per tailed triangle: the tail
//              node's triangle edges)
__global__ void __launch_bounds__(256) k_glob_edges(int64_t m, const int32_t* __restrict__ ei,
                                                    const int32_t* __restrict__ ej, const uint32_t* __restrict__ D,
                                                    const uint32_t* __restrict__ tau, const uint8_t* __restrict__ ty,
                                                    int L, GAcc ga) {
  extern __shared__ uint64_t gsm_edges[];
  gacc_init(ga, gsm_edges);
  constexpr int TS = 16;
  const int tl = threadIdx.x % TS;
  const int64_t teams = (int64_t)gridDim.x * (blockDim.x / TS);
  const int P = L * (L + 1) / 2, LL = L * L;
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / TS) + threadIdx.x / TS; e < m; e += teams) {
    const int32_t a = ei[e], b = ej[e];
    const int pa = ty[a], pb = ty[b];
    const uint32_t* Da = D + (int64_t)a * L;
    const uint32_t* Db = D + (int64_t)b * L;
    const uint32_t* te = tau + e * L;
    // any common neighbour at all (decides the triangle-based terms)
    uint32_t tsum = 0;
    for (int t = 0; t < L; ++t) tsum += te[t];
    for (int q = tl; q < LL; q += TS) {
      const int s = q / L, t = q % L;
      const uint64_t left = Da[s] - (pb == s ? 1u : 0u);
      const uint64_t right = Db[t] - (pa == t ? 1u : 0u);
      uint64_t val = left * right;
      if (s == t) val -= te[s];
      if (val) gacc_add(ga, gsm_edges, key_of(L, 2, pa, pb, s, t), val);
      if (tsum) {
        // here s is the tail's type and t the third triangle node's
        const uint64_t tt = te[t];
        if (tt) {
          const uint64_t tails = (uint64_t)Da[s] + Db[s] - (pb == s ? 1u : 0u) - (pa == s ? 1u : 0u) -
                                 (s == t ? 2u : 0u);
          if (tails) gacc_add(ga, gsm_edges, key_of(L, 5, pa, pb, t, s), tt * tails);
        }
      }
    }
    if (!tsum) continue;
    for (int q = tl; q < L; q += TS)
      if (te[q]) gacc_add(ga, gsm_edges, key_of(L, 1, pa, pb, q, 0), te[q]);
    for (int q = tl; q < P; q += TS) {
      int s, t;
      unrank2(q, s, t);
      const uint64_t x = te[s], y = te[t];
      const uint64_t val = s == t ? (uint64_t)c2((int64_t)x) : x * y;
      if (val) gacc_add(ga, gsm_edges, key_of(L, 6, pa, pb, s, t), val);
    }
  }
  gacc_flush(ga, gsm_edges);
}

// 4-clique edge classes: by the length of the T+ intersection loop,
// min(|out(a)|, |out(b)|), against lim = (16-lane team limit, wavefront
// limit); edges with fewer than two common neighbours hold no 4-clique and
// are left out.
__device__ __forceinline__ int k4_class(int32_t e, const int32_t* ei, const int32_t* ej, const int32_t* deg,
                                        const int32_t* out_off, const uint32_t* tau, int L, int2 lim,
                                        int32_t* len_out) {
  uint32_t tsum = 0;
  for (int t = 0; t < L; ++t) tsum += tau[(int64_t)e * L + t];
  if (tsum < 2) return -1;
  const int32_t i = ei[e], j = ej[e];
  const int32_t ni = out_off[i + 1] - out_off[i], nj = out_off[j + 1] - out_off[j];
  const int32_t loop = min(ni, nj);
  const int32_t len = min(loop, (int32_t)tsum);
  *len_out = len;
  if (len < 2) return -1;
  return loop <= lim.x ? 0 : (loop <= lim.y ? 1 : 2);
}

// counters: [0, 3) class sizes, [3] largest T+ bound of class 2
__global__ void __launch_bounds__(256) k_k4_class_count(int64_t m, const int32_t* __restrict__ ei,
                                                        const int32_t* __restrict__ ej,
                                                        const int32_t* __restrict__ deg,
                                                        const int32_t* __restrict__ out_off,
                                                        const uint32_t* __restrict__ tau, int L, int2 lim,
                                                        int32_t* __restrict__ cnt) {
  __shared__ int32_t local[4];
  if (threadIdx.x < 4) local[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t len = 0;
    const int c = k4_class((int32_t)e, ei, ej, deg, out_off, tau, L, lim, &len);
    if (c >= 0) atomicAdd(&local[c], 1);
    if (c == 2) atomicMax(&local[3], len);
  }
  __syncthreads();
  if (threadIdx.x < 3 && local[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], local[threadIdx.x]);
  if (threadIdx.x == 3 && local[3]) atomicMax(&cnt[3], local[3]);
}

// cur[c] holds the next free position of class c in list; one atomic per
// class and wavefront reserves the wavefront's positions
__global__ void __launch_bounds__(256) k_k4_class_scatter(int64_t m, const int32_t* __restrict__ ei,
                                                          const int32_t* __restrict__ ej,
                                                          const int32_t* __restrict__ deg,
                                                          const int32_t* __restrict__ out_off,
                                                          const uint32_t* __restrict__ tau, int L, int2 lim,
                                                          int32_t* __restrict__ cur, int32_t* __restrict__ list) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < m; e0 += stride) {
    const int64_t e = e0 + threadIdx.x;
    int32_t len = 0;
    const int c = e < m ? k4_class((int32_t)e, ei, ej, deg, out_off, tau, L, lim, &len) : -1;
    for (int k = 0; k < 3; ++k) {
      const uint64_t mask = ballot(c == k);
      if (!mask) continue;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      int32_t base = 0;
      if (lane() == leader) base = atomicAdd(&cur[k], __popcll(mask));
      base = __shfl(base, leader, TG_WAVE);
      if (c == k) list[base + lanes_below(mask)] = (int32_t)e;
    }
  }
}

template <int TSIZE>
struct K4Cap {
  static constexpr int value = TSIZE == 16 ? 64 : (TSIZE == 64 ? 1024 : 4096);
};

// LDS hash slots of T+ for workgroup teams (two per id of capacity; slot =
// id << 4 | type, -1 empty): their edges probe T+ hundreds of thousands of
// times, where a lookup of one or two reads beats a 12-step search
template <int TSIZE>
struct K4Hash {
  static constexpr int value = TSIZE > TG_WAVE ? 2 * K4Cap<TSIZE>::value : 0;
};

// per-team LDS bytes of k_glob_k4 after the key copies: scan scratch, the
// cell counters (mcopies copies of L x L), the T+ ids and types, the hash
template <int TSIZE>
__host__ __device__ inline int k4_team_bytes(int L, int mcopies) {
  return ((TSIZE > TG_WAVE ? 8 + 3 * TSIZE : 8) * 4 + mcopies * L * L * 4 + K4Cap<TSIZE>::value * 5 +
          K4Hash<TSIZE>::value * 4 + 7) & ~7;
}

template <int TSIZE>
inline size_t k4_lds_bytes(const GAcc& ga, int L, int mcopies) {
  return (size_t)ga.copies * ga.nk * sizeof(uint64_t) + (size_t)(256 / TSIZE) * k4_team_bytes<TSIZE>(L, mcopies);
}

// Typed 4-cliques, once each: one team of TSIZE lanes per edge (a, b) of
// list, a before b in degree order.  T+ = out(a) intersect out(b), built by
// searching the shorter list's ids in the longer one (both sorted), so it
// comes out sorted; each edge {c, d} inside T+ is then found once, from the
// out-list of its lower end, by binary search in T+, and counted in the
// edge's L x L cell (phi_c, phi_d) (mcopies lane-spread copies of 32-bit
// counters: an edge has fewer than 2^32 of them, as |T+| is at most the
// largest out-degree, below 2^16); the cells then go to the 4-clique keys.
// Each lane runs U searches at a time, step by step together, so that U
// loads are in flight.  A T+ that may exceed the team's LDS capacity
// (workgroup teams only: min(tcap, 4096) ids) lives in t_over, t_over_cap
// ids and types per workgroup (t_over_cap at least min(loop length,
// |T_ab|) over the list).
template <int TSIZE>
__global__ void __launch_bounds__(256) k_glob_k4(int64_t count, const int32_t* __restrict__ list,
                                                 const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
                                                 const int32_t* __restrict__ deg, const uint8_t* __restrict__ ty,
                                                 const int32_t* __restrict__ out_off,
                                                 const int32_t* __restrict__ out_col,
                                                 const uint32_t* __restrict__ tau, int L, int mcopies,
                                                 int tcap, int32_t* __restrict__ t_over, int64_t t_over_cap,
                                                 int thash_ok, GAcc ga) {
  extern __shared__ uint64_t gsm_k4[];
  gacc_init(ga, gsm_k4);
  constexpr int TEAMS = 256 / TSIZE;
  constexpr int TCAP = K4Cap<TSIZE>::value;
  constexpr int SCR = TSIZE > TG_WAVE ? 8 + 3 * TSIZE : 8;
  constexpr int U = 4;
  const int LL = L * L;
  const int team = threadIdx.x / TSIZE, tid = threadIdx.x % TSIZE, wv = tid / TG_WAVE;
  char* base = (char*)(gsm_k4 + (int64_t)ga.copies * ga.nk) + team * k4_team_bytes<TSIZE>(L, mcopies);
  int32_t* scratch = (int32_t*)base;
  uint32_t* cell = (uint32_t*)(scratch + SCR);
  int32_t* Tid_l = (int32_t*)(cell + mcopies * LL);
  uint8_t* Tty_l = (uint8_t*)(Tid_l + TCAP);
  constexpr int HS = K4Hash<TSIZE>::value;
  constexpr int HLOG = HS > 1 ? 31 - __builtin_clz((unsigned)(HS > 1 ? HS : 2)) : 1;
  int32_t* Th = HS ? (int32_t*)(Tty_l + TCAP) : nullptr;  // TCAP is a multiple of 4
  for (int64_t w = (int64_t)blockIdx.x * TEAMS + team; w < count; w += (int64_t)gridDim.x * TEAMS) {
    const int32_t e = list[w];
    const int32_t i = ei[e], j = ej[e];
    const int32_t di = deg[i], dj = deg[j];
    const bool i_first = precedes(di, i, dj, j);
    const int32_t a = i_first ? i : j, b = i_first ? j : i;
    // T+ = out(a) ∩ out(b): every member ranks above b, hence above a
    const int32_t oa = out_off[a], na = out_off[a + 1] - oa;
    const int32_t ob = out_off[b], nb = out_off[b + 1] - ob;
    const bool a_short = na <= nb;
    const int32_t os = a_short ? oa : ob, ns = a_short ? na : nb;  // scanned
    const int32_t ol = a_short ? ob : oa, nl = a_short ? nb : na;  // searched
    // |T+| is at most the loop length and at most |T_ab|
    bool big = false;
    if (TSIZE > TG_WAVE) {
      uint32_t tsum = 0;
      for (int t = 0; t < L; ++t) tsum += tau[(int64_t)e * L + t];
      big = min((int64_t)ns, (int64_t)tsum) > min(tcap, TCAP);
    }
    int32_t* Tid = big ? t_over + (int64_t)blockIdx.x * t_over_cap : Tid_l;
    uint8_t* Tty = big ? (uint8_t*)(t_over + (int64_t)gridDim.x * t_over_cap) + (int64_t)blockIdx.x * t_over_cap
                       : Tty_l;
    for (int x = tid; x < mcopies * LL; x += TSIZE) cell[x] = 0u;
    // an LDS T+ of a workgroup team also goes into the LDS hash
    const bool use_hash = HS && !big && thash_ok;
    if (use_hash)
      for (int x = tid; x < HS; x += TSIZE) Th[x] = -1;
    // ---- T+, in id order: U scanned ids per lane, searched together
    int32_t nT = 0;
    int top = 1;
    while (top * 2 <= nl) top *= 2;
    for (int32_t b0 = 0; b0 < ns; b0 += TSIZE * U) {
      int32_t kv[U], pos[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int32_t idx = b0 + k * TSIZE + tid;
        kv[k] = idx < ns ? out_col[os + idx] : -1;
        pos[k] = 0;
      }
      // lower bound of kv in the searched list, the same steps for all U
      for (int step = top; step > 0; step >>= 1) {
        int32_t tv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) tv[k] = pos[k] + step <= nl ? out_col[ol + pos[k] + step - 1] : INT32_MAX;
#pragma unroll
        for (int k = 0; k < U; ++k)
          if (tv[k] < kv[k]) pos[k] += step;
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const bool found = kv[k] >= 0 && pos[k] < nl && out_col[ol + pos[k]] == kv[k];
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
        if (found) {
          const int tk = ty[kv[k]];
          Tid[nT + before] = kv[k];
          Tty[nT + before] = (uint8_t)tk;
          if (use_hash) {
            uint32_t h = ((uint32_t)kv[k] * 2654435761u) >> (32 - HLOG);
            while (atomicCAS(&Th[h], -1, (kv[k] << 4) | tk) != -1) h = (h + 1) & (HS - 1);
          }
        }
        nT += total;
      }
    }
    tsync<TSIZE>();
    if (nT >= 2) {
      // (member, out-slot) pairs dealt to lanes through a team prefix sum
      int32_t* s_excl = scratch + 8;  // TSIZE == 256 only
      int ttop = 1;
      while (ttop * 2 <= nT) ttop *= 2;
      for (int32_t q0 = 0; q0 < nT; q0 += TSIZE) {
        const int32_t q = q0 + tid;
        int32_t ostart = 0, ocnt = 0, tk = 0;
        if (q < nT) {
          const int32_t k = Tid[q];
          ostart = out_off[k];
          ocnt = out_off[k + 1] - ostart;
          tk = Tty[q];
        }
        int32_t tot;
        const int32_t excl = team_excl_scan<TSIZE>(ocnt, &tot, scratch, tid);
        if (TSIZE > TG_WAVE) {
          s_excl[tid] = excl;
          s_excl[TSIZE + tid] = ostart;
          s_excl[2 * TSIZE + tid] = tk;
          __syncthreads();
        }
        for (int32_t c0 = 0; c0 < tot; c0 += TSIZE * U) {
          int32_t v[U], o[U], r[U], rtk[U], p[U];
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
            for (int k = 0; k < U; ++k)
              ex[k] = TSIZE <= TG_WAVE ? __shfl(excl, o[k] + step, TSIZE) : s_excl[o[k] + step];
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
            r[k] = v[k] < tot ? out_col[o_start + (v[k] - o_excl)] : -1;
            p[k] = 0;
          }
          if (use_hash) {
            // the home slot and the next one settle almost every lookup
            uint32_t h[U];
            int32_t sv[U], sw[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
              h[k] = ((uint32_t)(r[k] >= 0 ? r[k] : 0) * 2654435761u) >> (32 - HLOG);
              sv[k] = r[k] >= 0 ? Th[h[k]] : -1;
              sw[k] = r[k] >= 0 ? Th[(h[k] + 1) & (HS - 1)] : -1;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
              int cellv = -1;
              if (sv[k] != -1 && (sv[k] >> 4) == r[k]) {
                cellv = rtk[k] * L + (sv[k] & 15);
              } else if (sv[k] != -1 && sw[k] != -1) {
                if ((sw[k] >> 4) == r[k]) {
                  cellv = rtk[k] * L + (sw[k] & 15);
                } else {
                  uint32_t hh = (h[k] + 2) & (HS - 1);
                  int32_t x = Th[hh];
                  while (x != -1) {
                    if ((x >> 4) == r[k]) {
                      cellv = rtk[k] * L + (x & 15);
                      break;
                    }
                    hh = (hh + 1) & (HS - 1);
                    x = Th[hh];
                  }
                }
              }
              if (cellv >= 0) atomicAdd(&cell[(lane() % mcopies) * LL + cellv], 1u);
            }
          } else {
            // lower bound in the sorted T+, the same steps for all U pairs
            for (int step = ttop; step > 0; step >>= 1) {
              int32_t tv[U];
#pragma unroll
              for (int k = 0; k < U; ++k) tv[k] = p[k] + step <= nT ? Tid[p[k] + step - 1] : INT32_MAX;
#pragma unroll
              for (int k = 0; k < U; ++k)
                if (tv[k] < r[k]) p[k] += step;
            }
#pragma unroll
            for (int k = 0; k < U; ++k)
              if (r[k] >= 0 && p[k] < nT && Tid[p[k]] == r[k])
                atomicAdd(&cell[(lane() % mcopies) * LL + rtk[k] * L + Tty[p[k]]], 1u);
          }
        }
        if (TSIZE > TG_WAVE) __syncthreads();
      }
      tsync<TSIZE>();
      const int pa = ty[a], pb = ty[b];
      for (int x = tid; x < LL; x += TSIZE) {
        uint64_t sum = 0;
        for (int c = 0; c < mcopies; ++c) sum += cell[c * LL + x];
        if (sum) gacc_add(ga, gsm_k4, key_of(L, 7, pa, pb, x / L, x % L), sum);
      }
    }
    tsync<TSIZE>();
  }
  gacc_flush(ga, gsm_k4);
}

// Mean over nty count vectors of K keys (the type-permutation null model's
// average): exact 128-bit sums, then one division in double.
__global__ void k_mean_counts(int64_t nty, int64_t K, const uint64_t* __restrict__ counts,
                              double* __restrict__ mean) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  uint64_t lo = 0, hi = 0;
  for (int64_t b = 0; b < nty; ++b) {
    const uint64_t v = counts[b * K + k];
    lo += v;
    hi += lo < v ? 1u : 0u;
  }
  mean[k] = ((double)hi * 18446744073709551616.0 + (double)lo) / (double)nty;
}

// Induced counts from the non-induced sums, in place (inverting the
// relations above per type multiset); flag gets 1 when a sum is not a
// multiple of its repetition count or a result is negative.
__global__ void k_glob_finalize(uint64_t* __restrict__ g, int L, int32_t* __restrict__ flag) {
  const int64_t C3 = c3(L + 2), C4 = c4(L + 3);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (r < C3) {
    const uint64_t s_tri = g[C3 + r];
    bad |= s_tri % 3 != 0;
    const uint64_t tri = s_tri / 3;
    const uint64_t wedge = g[r] - 3 * tri;
    bad |= (int)(wedge >> 63);
    g[r] = wedge;
    g[C3 + r] = tri;
  }
  if (r < C4) {
    uint64_t* h = g + 2 * C3 + r;  // shape s (2..7) at h[(s - 2) * C4]
    const uint64_t n_path = h[0], n_star = h[C4], s_cyc = h[2 * C4], s_tail = h[3 * C4], n_chord = h[4 * C4];
    const uint64_t clique = h[5 * C4];
    bad |= (s_cyc & 1) != 0 || (s_tail & 1) != 0;
    const uint64_t chord = n_chord - 6 * clique;
    const uint64_t tail = s_tail / 2 - 4 * chord - 12 * clique;
    const uint64_t cyc = s_cyc / 2 - chord - 3 * clique;
    const uint64_t star = n_star - tail - 2 * chord - 4 * clique;
    const uint64_t path = n_path - 4 * cyc - 2 * tail - 6 * chord - 12 * clique;
    bad |= (int)((chord | tail | cyc | star | path) >> 63);
    h[0] = path;
    h[C4] = star;
    h[2 * C4] = cyc;
    h[3 * C4] = tail;
    h[4 * C4] = chord;
  }
  if (bad) atomicOr(flag, 1);
}
