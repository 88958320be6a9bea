// ----------------------------------------------------------- directed 4 --
//
// Directed typed 4-node graphlets (the Directed Typed Graphlets subsection:
// typed neighbour sets split into typed out- and in-neighbour sets, one id
// per directed typed motif), on the same input as the 3-node case: the
// symmetric support CSR plus one direction byte per slot.
//
// Keys: a 4-node digraph on ordered nodes 0..3 has one arc bit per ordered
// pair (x, y), x != y, in the order (0,1) (0,2) (0,3) (1,0) (1,2) (1,3) (2,0)
// (2,1) (2,3) (3,0) (3,1) (3,2), and its full code adds the four types, 4
// bits each from bit 12.  Its canonical code is the smallest full code over
// the 24 node orderings; the keys of L types number the canonical codes of
// the weakly connected digraphs with types below L in increasing order (199
// keys for L = 1).  The host builds a table from every local code (12 arc
// bits, types 2 bits each above them, so L <= 4) straight to its key.
//
// Per support edge (i, j), i < j (one wavefront): every other node k with a
// support edge to i or j has the direction codes a_k = c(i, k), b_k = c(j, k)
// (U, held in LDS with its codes).  A weakly connected 4-node
// set {i, j, k, l} has k in U and l either in U or a support neighbour of k
// only.  The wavefront
//   - walks the support rows of U's members: a neighbour l outside U (and not
//     i, j) gives the set with l reached from k alone; a neighbour l in U
//     with l > k gives an adjacent pair, whose key gains one while the key of
//     the same pair without the (k, l) arcs loses one;
//   - adds, for every unordered pair of (code, type) classes of U, the number
//     of pairs of nodes in those classes to the key of the pair without a
//     (k, l) arc (so that after the subtractions above only the non-adjacent
//     pairs remain counted there).
// The per-edge row (optional) and the global key sums take these signed
// contributions modulo 2^64; every final entry is a non-negative count.
// Global counts: the key sums divided by the key's support edges.

namespace dir4 {

constexpr int kLocalCodes = 1 << 20;  // 12 arc bits, 4 types of 2 bits
constexpr int kMaxL = 4;
constexpr int kUCap = 1024;           // |U| per edge kept in LDS

// ordered pair (x, y) -> arc bit
__host__ __device__ inline int arc_bit(int x, int y) { return 3 * x + (y < x ? y : y - 1); }

inline bool weakly_connected(int arcs) {
  int adj[4] = {0, 0, 0, 0};
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y)
      if (x != y && (arcs >> arc_bit(x, y) & 1)) {
        adj[x] |= 1 << y;
        adj[y] |= 1 << x;
      }
  int seen = 1, grew = 1;
  while (grew) {
    grew = 0;
    for (int x = 0; x < 4; ++x)
      if ((seen >> x & 1) && (adj[x] & ~seen)) {
        seen |= adj[x];
        grew = 1;
      }
  }
  return seen == 15;
}

inline int support_edges(int arcs) {
  int s = 0;
  for (int x = 0; x < 4; ++x)
    for (int y = x + 1; y < 4; ++y)
      if ((arcs >> arc_bit(x, y) & 1) || (arcs >> arc_bit(y, x) & 1)) ++s;
  return s;
}

// canonical full code (types 4 bits each) of arcs with node types t[4]
inline int64_t canonical(int arcs, const int* t) {
  int perm[4] = {0, 1, 2, 3};
  int64_t best = INT64_MAX;
  do {
    // old node perm[q] becomes new node q
    int inv[4];
    for (int q = 0; q < 4; ++q) inv[perm[q]] = q;
    int64_t a = 0;
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; ++y)
        if (x != y && (arcs >> arc_bit(x, y) & 1)) a |= 1ll << arc_bit(inv[x], inv[y]);
    for (int q = 0; q < 4; ++q) a |= (int64_t)t[perm[q]] << (12 + 4 * q);
    best = std::min(best, a);
  } while (std::next_permutation(perm, perm + 4));
  return best;
}

struct Tables {
  std::vector<int32_t> local2key;  // kLocalCodes entries, -1: not a key
  std::vector<int64_t> canon;      // canonical code of each key
  std::vector<uint8_t> divisor;    // support edges of each key
};

inline const Tables& tables(int L) {
  static std::mutex mu;
  static std::map<int, Tables> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(L);
  if (it != cache.end()) return it->second;
  Tables T;
  std::vector<int64_t> can(kLocalCodes, -1);
  for (int code = 0; code < kLocalCodes; ++code) {
    const int arcs = code & 0xFFF;
    int t[4];
    bool ok = weakly_connected(arcs);
    for (int q = 0; q < 4; ++q) {
      t[q] = (code >> (12 + 2 * q)) & 3;
      ok = ok && t[q] < L;
    }
    if (ok) can[code] = canonical(arcs, t);
  }
  std::vector<int64_t> sorted;
  for (int64_t c : can)
    if (c >= 0) sorted.push_back(c);
  std::sort(sorted.begin(), sorted.end());
  sorted.erase(std::unique(sorted.begin(), sorted.end()), sorted.end());
  T.canon = sorted;
  for (int64_t c : sorted) T.divisor.push_back((uint8_t)support_edges((int)(c & 0xFFF)));
  T.local2key.assign(kLocalCodes, -1);
  for (int code = 0; code < kLocalCodes; ++code)
    if (can[code] >= 0)
      T.local2key[code] = (int32_t)(std::lower_bound(sorted.begin(), sorted.end(), can[code]) - sorted.begin());
  return cache.emplace(L, std::move(T)).first->second;
}

}  // namespace dir4

// Local code of nodes (i, j, k, l) from the six direction codes (bit 0: the
// first node of the pair -> the second, bit 1: the reverse) and the types.
__device__ __forceinline__ int dir4_code(int cij, int ak, int bk, int al, int bl, int ckl, int ti, int tj, int tk,
                                         int tl) {
  using dir4::arc_bit;
  int a = 0;
  a |= (cij & 1) << arc_bit(0, 1) | (cij >> 1) << arc_bit(1, 0);
  a |= (ak & 1) << arc_bit(0, 2) | (ak >> 1) << arc_bit(2, 0);
  a |= (bk & 1) << arc_bit(1, 2) | (bk >> 1) << arc_bit(2, 1);
  a |= (al & 1) << arc_bit(0, 3) | (al >> 1) << arc_bit(3, 0);
  a |= (bl & 1) << arc_bit(1, 3) | (bl >> 1) << arc_bit(3, 1);
  a |= (ckl & 1) << arc_bit(2, 3) | (ckl >> 1) << arc_bit(3, 2);
  return a | ti << 12 | tj << 14 | tk << 16 | tl << 18;
}

// LDS bytes per wavefront of k_dir4: U's ids, codes and types, the class
// histogram (16 codes x 4 types) and |U|.
__host__ __device__ constexpr int dir4_wave_lds() { return dir4::kUCap * 6 + 64 * 4 + 16; }

// One wavefront per support edge e of [0, m): U in LDS (ids, codes a | b << 2,
// types), its class histogram, then the walks described above.  rows: m x K
// (or null); global sums through ga.
__global__ void __launch_bounds__(256) k_dir4(int64_t m, const int32_t* __restrict__ ei,
                                              const int32_t* __restrict__ ej, const int32_t* __restrict__ es_lo,
                                              const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                              const uint8_t* __restrict__ sdir, const uint8_t* __restrict__ ty,
                                              int L, const int32_t* __restrict__ l2k, uint64_t* __restrict__ rows,
                                              int64_t K, GAcc ga) {
  extern __shared__ uint64_t smem_dir4[];
  constexpr int WAVES = 4;
  const int wv = threadIdx.x / TG_WAVE, ln = lane();
  uint64_t* gsm = smem_dir4;
  char* base = reinterpret_cast<char*>(smem_dir4) + (size_t)ga.copies * ga.nk * sizeof(uint64_t) +
               (size_t)wv * dir4_wave_lds();
  int32_t* uid = reinterpret_cast<int32_t*>(base);                // [kUCap]
  uint8_t* ucode = reinterpret_cast<uint8_t*>(uid + dir4::kUCap);  // [kUCap] a | b << 2
  uint8_t* utype = ucode + dir4::kUCap;                            // [kUCap]
  uint32_t* hist = reinterpret_cast<uint32_t*>(utype + dir4::kUCap);  // [16][4]
  int32_t* nU_s = reinterpret_cast<int32_t*>(hist + 64);
  gacc_init(ga, gsm);
  auto add = [&](int64_t e, int code, uint64_t v) {
    const int32_t key = l2k[code];
    if (key < 0) return;  // not reached for inputs with types below L
    if (rows) atomicAdd((unsigned long long*)&rows[e * K + key], (unsigned long long)v);
    gacc_add(ga, gsm, key, v);
  };
  for (int64_t e = (int64_t)blockIdx.x * WAVES + wv; e < m; e += (int64_t)gridDim.x * WAVES) {
    const int32_t i = ei[e], j = ej[e];
    const int cij = sdir[es_lo[e]];
    const int ti = ty[i] & 3, tj = ty[j] & 3;
    const int32_t ri = rp[i], di = rp[i + 1] - ri, rj = rp[j], dj = rp[j + 1] - rj;
    for (int q = ln; q < 64; q += TG_WAVE) hist[q] = 0;
    if (ln == 0) *nU_s = 0;
    wave_sync();
    // U: i's row (codes from both rows), then j's row minus i's
    for (int32_t b0 = 0; b0 < di + dj; b0 += TG_WAVE) {
      const int32_t q = b0 + ln;
      bool keep = false;
      int32_t k = 0;
      int a = 0, b = 0;
      if (q < di) {
        k = ci[ri + q];
        if (k != j) {
          a = sdir[ri + q];
          const int32_t p = lower_bound(ci + rj, dj, k);
          b = (p < dj && ci[rj + p] == k) ? sdir[rj + p] : 0;
          keep = true;
        }
      } else if (q < di + dj) {
        k = ci[rj + (q - di)];
        if (k != i) {
          const int32_t p = lower_bound(ci + ri, di, k);
          if (!(p < di && ci[ri + p] == k)) {
            b = sdir[rj + (q - di)];
            keep = true;
          }
        }
      }
      const uint64_t mask = ballot(keep);
      const int32_t at = *nU_s;
      if (keep) {
        const int32_t s = at + lanes_below(mask);
        uid[s] = k;
        ucode[s] = (uint8_t)(a | b << 2);
        utype[s] = ty[k] & 3;
        atomicAdd(&hist[(a | b << 2) * 4 + (ty[k] & 3)], 1u);
      }
      wave_sync();
      if (ln == 0) *nU_s = at + __popcll(mask);
      wave_sync();
    }
    const int32_t nU = *nU_s;
    // (walks) every (k, slot) pair of U's rows, dealt 64 at a time
    for (int32_t q0 = 0; q0 < nU; q0 += TG_WAVE) {
      const int32_t q = q0 + ln;
      int32_t start = 0, cnt = 0;
      if (q < nU) {
        const int32_t k = uid[q];
        start = rp[k];
        cnt = rp[k + 1] - start;
      }
      int32_t tot = 0;
      int32_t x = cnt;
      for (int off = 1; off < TG_WAVE; off <<= 1) {
        const int32_t y = __shfl_up(x, off, TG_WAVE);
        if (ln >= off) x += y;
      }
      tot = __shfl(x, TG_WAVE - 1, TG_WAVE);
      const int32_t excl = x - cnt;
      for (int32_t v0 = 0; v0 < tot; v0 += TG_WAVE) {
        const int32_t v = v0 + ln;
        int o = 0;
        for (int step = 32; step > 0; step >>= 1) {
          const int32_t ex = __shfl(excl, o + step, TG_WAVE);
          if (ex <= v) o += step;
        }
        const int32_t o_excl = __shfl(excl, o, TG_WAVE), o_start = __shfl(start, o, TG_WAVE);
        if (v >= tot) continue;
        const int32_t qk = q0 + o;
        const int32_t k = uid[qk];
        const int32_t s = o_start + (v - o_excl);
        const int32_t l = ci[s];
        if (l == i || l == j) continue;
        const int ck = ucode[qk], tk = utype[qk];
        const int ckl = sdir[s];  // c(k, l)
        // l in U? (U is not sorted: search both rows of i and j)
        const int32_t pi = lower_bound(ci + ri, di, l), pj = lower_bound(ci + rj, dj, l);
        const int al = (pi < di && ci[ri + pi] == l) ? sdir[ri + pi] : 0;
        const int bl = (pj < dj && ci[rj + pj] == l) ? sdir[rj + pj] : 0;
        const int tl = ty[l] & 3;
        if (al == 0 && bl == 0) {
          add(e, dir4_code(cij, ck & 3, ck >> 2, 0, 0, ckl, ti, tj, tk, tl), 1ull);
        } else if (l > k) {
          add(e, dir4_code(cij, ck & 3, ck >> 2, al, bl, ckl, ti, tj, tk, tl), 1ull);
          add(e, dir4_code(cij, ck & 3, ck >> 2, al, bl, 0, ti, tj, tk, tl), ~0ull);  // minus one
        }
      }
    }
    // pairs of U by (code, type) class, counted without a (k, l) arc
    const int NC = 16 * 4;
    for (int x = ln; x < NC * NC; x += TG_WAVE) {
      const int c1 = x / NC, c2 = x % NC;
      if (c2 < c1) continue;
      const uint64_t n1 = hist[c1], n2 = hist[c2];
      if (!n1 || !n2) continue;
      const uint64_t pairs = c1 == c2 ? n1 * (n1 - 1) / 2 : n1 * n2;
      if (!pairs) continue;
      const int k1 = c1 >> 2, t1 = c1 & 3, k2 = c2 >> 2, t2 = c2 & 3;
      add(e, dir4_code(cij, k1 & 3, k1 >> 2, k2 & 3, k2 >> 2, 0, ti, tj, t1, t2), pairs);
    }
    wave_sync();
  }
  gacc_flush(ga, gsm);
}

// Largest |U| = d_i + d_j - 2 over the support edges.
__global__ void __launch_bounds__(256) k_dir4_max_u(int64_t m, const int32_t* __restrict__ ei,
                                                    const int32_t* __restrict__ ej, const int32_t* __restrict__ rp,
                                                    int32_t* __restrict__ out) {
  __shared__ int32_t h;
  if (threadIdx.x == 0) h = 0;
  __syncthreads();
  int32_t my = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    my = max(my, rp[ei[e] + 1] - rp[ei[e]] + rp[ej[e] + 1] - rp[ej[e]] - 2);
  atomicMax(&h, my);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, h);
}

tg_status directed4_impl(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const uint8_t* sdir,
                         const uint8_t* ty, int L, uint64_t* global_counts, uint64_t* edge_rows,
                         int32_t* edge_info, const tg_options* opt_in, hipStream_t st) {
  tg_options opt;
  tg_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (L < 1 || L > dir4::kMaxL) return fail(TG_ERR_UNSUPPORTED_L, "directed 4-node counting takes L in [1, 4]");
  if (n < 0 || nnz < 0 || n >= (1ll << 31) || nnz >= (1ll << 31))
    return fail(TG_ERR_INVALID_ARG, "n and nnz must be in [0, 2^31)");
  if (!rp || (!global_counts && !edge_rows) || (nnz > 0 && (!ci || !sdir)) || (n > 0 && !ty))
    return fail(TG_ERR_INVALID_ARG, "null input or output pointer");
  if (nnz % 2) return fail(TG_ERR_INVALID_GRAPH, "nnz is odd: some edge is stored in one direction only");
  const dir4::Tables& T = dir4::tables(L);
  const int64_t K = (int64_t)T.canon.size(), m = nnz / 2;
  keep_pool_cached();
  Scratch S(st);
  PhaseTimer timer(st, opt.phase_ms);
  if (global_counts) {
    k_fill_u64<<<grid_for(K, 256, 1024), 256, 0, st>>>(global_counts, K, 0);
    TG_LAUNCHED("k_fill_u64");
  }
  if (opt.validate && n > 0) {
    if (tg_status vs = validate_graph(S, st, n, nnz, rp, ci, ty, L)) return vs;
    int32_t* flags;
    TG_HIP(S.get(&flags, 1));
    TG_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t), st));
    k_validate_dir<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, rp, ci, sdir, flags);
    TG_LAUNCHED("k_validate_dir");
    int32_t h = 0;
    TG_HIP(hipMemcpyAsync(&h, flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (h) return fail(TG_ERR_INVALID_GRAPH, "direction bytes must be 1..3 and mirror each other on an edge's slots");
  }
  if (m == 0) return TG_OK;
  timer.mark(TG_PHASE_PREP);
  Work W;
  TG_HIP(S.get(&W.deg, n));
  TG_HIP(S.get(&W.D, n * L));
  TG_HIP(S.get(&W.n_upper, n));
  TG_HIP(S.get(&W.n_out, n));
  TG_HIP(S.get(&W.wedge_work, n));
  TG_HIP(S.get(&W.nbr_deg_sum, n));
  TG_HIP(S.get(&W.upper_off, n + 1));
  TG_HIP(S.get(&W.out_off, n + 1));
  TG_HIP(S.get(&W.ei, m));
  TG_HIP(S.get(&W.ej, m));
  TG_HIP(S.get(&W.s2e, nnz));
  TG_HIP(S.get(&W.es_lo, m));
  TG_HIP(S.get(&W.es_hi, m));
  TG_HIP(S.get(&W.out_col, m));
  k_degree<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, rp, W.deg);
  TG_LAUNCHED("k_degree");
  k_node_stats<<<grid_for(n, 4), 256, 0, st>>>(n, rp, ci, W.deg, ty, L, W.D, W.n_upper, W.n_out, W.wedge_work,
                                               W.nbr_deg_sum);
  TG_LAUNCHED("k_node_stats");
  if (tg_status s = scan(S, st, n, W.n_upper, W.upper_off)) return s;
  if (tg_status s = scan(S, st, n, W.n_out, W.out_off)) return s;
  k_fill_edges<<<grid_for(n, 4), 256, 0, st>>>(n, rp, ci, W.deg, W.n_upper, W.upper_off, W.out_off, W.ei, W.ej,
                                               W.s2e, W.es_lo, W.es_hi, W.out_col, nullptr);
  TG_LAUNCHED("k_fill_edges");
  // |U| of every edge must fit the wavefront's LDS
  int32_t* d_mu;
  TG_HIP(S.get(&d_mu, 1));
  TG_HIP(hipMemsetAsync(d_mu, 0, sizeof(int32_t), st));
  k_dir4_max_u<<<grid_for(m, 256, 2048), 256, 0, st>>>(m, W.ei, W.ej, rp, d_mu);
  TG_LAUNCHED("k_dir4_max_u");
  int32_t h_mu = 0;
  TG_HIP(hipMemcpyAsync(&h_mu, d_mu, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  if (h_mu > dir4::kUCap)
    return fail(TG_ERR_INVALID_ARG, "directed 4-node counting takes d_i + d_j - 2 <= " +
                                        std::to_string(dir4::kUCap) + " on every edge (found " +
                                        std::to_string(h_mu) + ")");
  int32_t* l2k;
  uint8_t* div;
  TG_HIP(S.get(&l2k, dir4::kLocalCodes));
  TG_HIP(S.get(&div, K));
  TG_HIP(hipMemcpyAsync(l2k, T.local2key.data(), dir4::kLocalCodes * sizeof(int32_t), hipMemcpyHostToDevice, st));
  TG_HIP(hipMemcpyAsync(div, T.divisor.data(), K, hipMemcpyHostToDevice, st));
  if (edge_rows) {
    k_fill_u64<<<grid_for(m * K, 256, 16384), 256, 0, st>>>(edge_rows, m * K, 0);
    TG_LAUNCHED("k_fill_u64");
  }
  timer.mark(TG_PHASE_TAU);
  timer.mark(TG_PHASE_TABLES);
  timer.mark(TG_PHASE_SCHEDULE);
  timer.mark(TG_PHASE_CYCLES);
  timer.mark(TG_PHASE_CLIQUES);
  // ---- per edge
  timer.mark(TG_PHASE_COMBINE);
  uint64_t* gsum = global_counts;
  if (!gsum) {
    TG_HIP(S.get(&gsum, K));
    k_fill_u64<<<grid_for(K, 256, 1024), 256, 0, st>>>(gsum, K, 0);
    TG_LAUNCHED("k_fill_u64");
  }
  const GAcc ga = make_gacc(gsum, 0, K, 32 << 10);
  const size_t lds = gacc_bytes(ga) + 4 * (size_t)dir4_wave_lds();
  k_dir4<<<grid_for(m, 4, 4096), 256, lds, st>>>(m, W.ei, W.ej, W.es_lo, rp, ci, sdir, ty, L, l2k, edge_rows, K, ga);
  TG_LAUNCHED("k_dir4");
  timer.mark(TG_PHASE_FINALIZE);
  int32_t* flag;
  TG_HIP(S.get(&flag, 1));
  TG_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  if (global_counts) {
    k_dir3_finalize<<<grid_for(K, 256), 256, 0, st>>>(global_counts, K, div, flag);
    TG_LAUNCHED("k_dir3_finalize");
  }
  if (edge_info) {
    k_dir_edge_info<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, W.ei, W.ej, W.es_lo, sdir, edge_info);
    TG_LAUNCHED("k_dir_edge_info");
  }
  timer.mark(TG_NUM_PHASES);
  if (opt.check) {
    int32_t hf = 0;
    TG_HIP(hipMemcpyAsync(&hf, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (hf) return fail(TG_ERR_INTERNAL, "a directed 4-node key sum is not a multiple of its support edge count");
  }
  timer.finish();
  return TG_OK;
}
