// ------------------------------------------------------------ directed --
//
// Directed typed 3-node graphlets (the Directed Typed Graphlets subsection:
// every typed neighbour set is split into typed out- and in-neighbour sets).
// The graph is its symmetric support CSR plus one direction byte per slot:
// bit 0 for the arc row -> column, bit 1 for column -> row; the direction
// code of a pair (u, v) is that byte at u's slot for v (1 out, 2 in, 3 both).
//
// For a support edge (i, j), i < j, and a third node k adjacent to i or j,
// the induced triad on (i, j, k) is fixed by c(i,j), c(i,k), c(j,k) and the
// three types.  The per-edge row has 15 L columns, ((4 c(i,k) + c(j,k)) - 1)
// L + phi_k over (c(i,k), c(j,k)) != (0, 0): the typed common neighbours T
// split by both codes, and S_i (S_j) split by c(i,k) (c(j,k)).  Only T needs
// an intersection; S_i and S_j follow from the per-node directed typed
// degrees Dd[v][c - 1][t] minus T's cells and the edge itself.
//
// Keys: a triad on ordered nodes (a, b, c) has the code of its six arc bits
// (a->b, b->a, a->c, c->a, b->c, c->b; bits 0-5) and types (bits 6-9,
// 10-13, 14-17); its canonical code is the smallest over the six orderings,
// and the keys of L types number the canonical codes of weakly connected
// triads with types below L in increasing order.  code2rank maps every code
// straight to its key (-1: not a connected triad with types below L), so no
// kernel canonicalises.  Global counts: the sum of the per-edge cells over
// the triad's support edges, divided by their number (2 or 3).

namespace dir3 {

constexpr int kCodes = 1 << 18;

__host__ __device__ inline int arc_bit(int x, int y) {
  // (0,1) (1,0) (0,2) (2,0) (1,2) (2,1)
  return x == 0 ? (y == 1 ? 0 : 2) : (x == 1 ? (y == 0 ? 1 : 4) : (y == 0 ? 3 : 5));
}

inline int support_edges(int adj) {
  return ((adj & 3) ? 1 : 0) + ((adj & 12) ? 1 : 0) + ((adj & 48) ? 1 : 0);
}

inline int canonical(int code) {
  const int adj = code & 63;
  const int t[3] = {(code >> 6) & 15, (code >> 10) & 15, (code >> 14) & 15};
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int best = INT32_MAX;
  for (const auto& p : perms) {
    // old node p[q] becomes new node q
    int inv[3];
    for (int q = 0; q < 3; ++q) inv[p[q]] = q;
    int a = 0;
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y)
        if (x != y && (adj >> arc_bit(x, y) & 1)) a |= 1 << arc_bit(inv[x], inv[y]);
    best = std::min(best, a | (t[p[0]] << 6) | (t[p[1]] << 10) | (t[p[2]] << 14));
  }
  return best;
}

struct Tables {
  std::vector<int32_t> code2rank;  // kCodes entries
  std::vector<int32_t> canon;      // canonical code of each key
  std::vector<uint8_t> divisor;    // support edges of each key
};

inline const Tables& tables(int L) {
  static std::mutex mu;
  static std::map<int, Tables> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(L);
  if (it != cache.end()) return it->second;
  Tables T;
  T.code2rank.assign(kCodes, -1);
  std::vector<int32_t> canon_of(kCodes, -1);
  std::vector<char> is_key(kCodes, 0);
  for (int code = 0; code < kCodes; ++code) {
    if (support_edges(code & 63) < 2) continue;
    if (((code >> 6) & 15) >= L || ((code >> 10) & 15) >= L || ((code >> 14) & 15) >= L) continue;
    canon_of[code] = canonical(code);
    is_key[canon_of[code]] = 1;
  }
  std::vector<int32_t> rank(kCodes, -1);
  for (int code = 0; code < kCodes; ++code)
    if (is_key[code]) {
      rank[code] = (int32_t)T.canon.size();
      T.canon.push_back(code);
      T.divisor.push_back((uint8_t)support_edges(code & 63));
    }
  for (int code = 0; code < kCodes; ++code)
    if (canon_of[code] >= 0) T.code2rank[code] = rank[canon_of[code]];
  return cache.emplace(L, std::move(T)).first->second;
}

}  // namespace dir3

// Direction bytes: every slot nonzero, and the two slots of an edge mirror
// each other (bits swapped); flags |= 1 on a violation.
__global__ void k_validate_dir(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const uint8_t* __restrict__ sdir, int32_t* __restrict__ flags) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    for (int32_t s = rp[u]; s < rp[u + 1]; ++s) {
      const int32_t v = ci[s];
      const int c = sdir[s];
      const int32_t p = rp[v] + lower_bound(ci + rp[v], rp[v + 1] - rp[v], (int32_t)u);
      const int mirror = (p < rp[v + 1] && ci[p] == (int32_t)u) ? sdir[p] : -1;
      if (c < 1 || c > 3 || mirror != (((c & 1) << 1) | (c >> 1))) atomicOr(flags, 1);
    }
  }
}

// Dd[v][c - 1][t]: neighbours k of v with direction code c(v, k) = c and type
// t; one wavefront per node, counted in LDS.
__global__ void __launch_bounds__(256) k_dir_degree(int64_t n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const uint8_t* __restrict__ sdir,
                                                    const uint8_t* __restrict__ ty, int L,
                                                    uint32_t* __restrict__ Dd) {
  __shared__ uint32_t cnt[4][48];
  const int wv = threadIdx.x / TG_WAVE, ln = lane();
  uint32_t* c = cnt[wv];
  for (int64_t v = (int64_t)blockIdx.x * 4 + wv; v < n; v += (int64_t)gridDim.x * 4) {
    for (int q = ln; q < 3 * L; q += TG_WAVE) c[q] = 0u;
    wave_sync();
    for (int32_t s = rp[v] + ln; s < rp[v + 1]; s += TG_WAVE) {
      const int d = sdir[s], t = ty[ci[s]];
      if (d >= 1 && d <= 3 && t < L) atomicAdd(&c[(d - 1) * L + t], 1u);
    }
    wave_sync();
    for (int q = ln; q < 3 * L; q += TG_WAVE) Dd[v * 3 * L + q] = c[q];
    wave_sync();
  }
}

// Per edge (one team of TSIZE lanes; edges whose shorter support row has a
// length in (dlo, dhi]): the typed common neighbours T split by both
// direction codes (team LDS cells), then the row and the key sums.
template <int TSIZE>
__global__ void __launch_bounds__(256) k_dir3(int64_t m, int32_t dlo, int32_t dhi, const int32_t* __restrict__ ei,
                                              const int32_t* __restrict__ ej, const int32_t* __restrict__ es_lo,
                                              const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                              const uint8_t* __restrict__ sdir, const uint8_t* __restrict__ ty,
                                              int L, const uint32_t* __restrict__ Dd,
                                              const int32_t* __restrict__ code2rank, uint64_t* __restrict__ rows,
                                              GAcc ga) {
  extern __shared__ uint64_t gsm_dir[];
  gacc_init(ga, gsm_dir);
  constexpr int TEAMS = 256 / TSIZE;
  const int team = threadIdx.x / TSIZE, tl = threadIdx.x % TSIZE;
  uint32_t* Tc = reinterpret_cast<uint32_t*>(gsm_dir + (int64_t)ga.copies * ga.nk) + team * 9 * L;
  const int W = 15 * L;
  for (int64_t e = (int64_t)blockIdx.x * TEAMS + team; e < m; e += (int64_t)gridDim.x * TEAMS) {
    const int32_t i = ei[e], j = ej[e];
    const int32_t di = rp[i + 1] - rp[i], dj = rp[j + 1] - rp[j];
    const bool a_is_i = di <= dj;
    const int32_t la = a_is_i ? di : dj, lb = a_is_i ? dj : di;
    if (la <= dlo || la > dhi) continue;
    for (int q = tl; q < 9 * L; q += TSIZE) Tc[q] = 0u;
    tsync<TSIZE>();
    const int32_t ra = rp[a_is_i ? i : j], rb = rp[a_is_i ? j : i];
    for (int32_t idx = tl; idx < la; idx += TSIZE) {
      const int32_t k = ci[ra + idx];
      const int32_t p = lower_bound(ci + rb, lb, k);
      if (p < lb && ci[rb + p] == k) {
        const int ca = sdir[ra + idx], cb = sdir[rb + p], tk = ty[k];
        const int cik = a_is_i ? ca : cb, cjk = a_is_i ? cb : ca;
        // codes outside 1..3 or types >= L (inputs that validation rejects)
        // are skipped rather than indexed
        if (cik >= 1 && cik <= 3 && cjk >= 1 && cjk <= 3 && tk < L)
          atomicAdd(&Tc[((cik - 1) * 3 + (cjk - 1)) * L + tk], 1u);
      }
    }
    tsync<TSIZE>();
    const int cij = sdir[es_lo[e]];
    const int cji = ((cij & 1) << 1) | (cij >> 1);
    const int pi = ty[i] & 15, pj = ty[j] & 15;
    const int base_code = (cij & 3) | (pi << 6) | (pj << 10);
    for (int col = tl; col < W; col += TSIZE) {
      const int cat = col / L + 1, t = col % L;
      const int cik = cat >> 2, cjk = cat & 3;
      uint64_t v;
      if (cik && cjk) {
        v = Tc[((cik - 1) * 3 + (cjk - 1)) * L + t];
      } else if (cik) {
        int64_t s = Dd[(int64_t)i * 3 * L + (cik - 1) * L + t];
        for (int c = 0; c < 3; ++c) s -= Tc[((cik - 1) * 3 + c) * L + t];
        if (cik == cij && t == pj) s -= 1;
        v = (uint64_t)s;
      } else {
        int64_t s = Dd[(int64_t)j * 3 * L + (cjk - 1) * L + t];
        for (int c = 0; c < 3; ++c) s -= Tc[(c * 3 + (cjk - 1)) * L + t];
        if (cjk == cji && t == pi) s -= 1;
        v = (uint64_t)s;
      }
      if (rows) rows[e * W + col] = v;
      if (v) {
        // arcs of (i, j, k): i<->j from cij, i<->k bits 2-3, j<->k bits 4-5
        const int code = base_code | (cik << 2) | (cjk << 4) | (t << 14);
        const int32_t r = code2rank[code];
        if (r >= 0) gacc_add(ga, gsm_dir, r, v);
      }
    }
    tsync<TSIZE>();
  }
  gacc_flush(ga, gsm_dir);
}

__global__ void k_dir_edge_info(int64_t m, const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
                                const int32_t* __restrict__ es_lo, const uint8_t* __restrict__ sdir,
                                int32_t* __restrict__ info) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    info[3 * e] = ei[e];
    info[3 * e + 1] = ej[e];
    info[3 * e + 2] = sdir[es_lo[e]];
  }
}

__global__ void k_dir3_finalize(uint64_t* __restrict__ g, int64_t K, const uint8_t* __restrict__ divisor,
                                int32_t* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint64_t d = divisor[k], s = g[k];
  if (s % d) atomicOr(flag, 1);
  g[k] = s / d;
}

tg_status directed3_impl(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const uint8_t* sdir,
                         const uint8_t* ty, int L, uint64_t* global_counts, uint64_t* edge_rows,
                         int32_t* edge_info, const tg_options* opt_in, hipStream_t st) {
  tg_options opt;
  tg_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (n < 0 || nnz < 0 || n >= (1ll << 31) || nnz >= (1ll << 31))
    return fail(TG_ERR_INVALID_ARG, "n and nnz must be in [0, 2^31)");
  if (!rp || (!global_counts && !edge_rows) || (nnz > 0 && (!ci || !sdir)) || (n > 0 && !ty))
    return fail(TG_ERR_INVALID_ARG, "null input or output pointer");
  if (nnz % 2) return fail(TG_ERR_INVALID_GRAPH, "nnz is odd: some edge is stored in one direction only");
  const dir3::Tables& T = dir3::tables(L);
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
  // canonical edges (degree, offsets, slot maps) as for tg_count
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
  uint32_t* Dd;
  int32_t* c2r;
  uint8_t* div;
  TG_HIP(S.get(&Dd, n * 3 * L));
  TG_HIP(S.get(&c2r, dir3::kCodes));
  TG_HIP(S.get(&div, K));
  TG_HIP(hipMemcpyAsync(c2r, T.code2rank.data(), dir3::kCodes * sizeof(int32_t), hipMemcpyHostToDevice, st));
  TG_HIP(hipMemcpyAsync(div, T.divisor.data(), K, hipMemcpyHostToDevice, st));
  // phases: prep (canonical edges), tables (directed typed degrees),
  // combine (per-edge kernels), finalize; the others stay empty
  timer.mark(TG_PHASE_TAU);
  timer.mark(TG_PHASE_TABLES);
  k_dir_degree<<<grid_for(n, 4, 8192), 256, 0, st>>>(n, rp, ci, sdir, ty, L, Dd);
  TG_LAUNCHED("k_dir_degree");
  timer.mark(TG_PHASE_SCHEDULE);
  timer.mark(TG_PHASE_CYCLES);
  timer.mark(TG_PHASE_CLIQUES);
  // ---- per edge
  timer.mark(TG_PHASE_COMBINE);
  uint64_t* gsum = global_counts;
  if (!gsum) TG_HIP(S.get(&gsum, K));
  const GAcc ga = make_gacc(gsum, 0, K, 40 << 10);
  const size_t lds16 = gacc_bytes(ga) + 16 * 9 * L * sizeof(uint32_t);
  const size_t lds64 = gacc_bytes(ga) + 4 * 9 * L * sizeof(uint32_t);
  k_dir3<16><<<grid_for(m, 16, 2048), 256, lds16, st>>>(m, -1, 48, W.ei, W.ej, W.es_lo, rp, ci, sdir, ty, L, Dd, c2r,
                                                        edge_rows, ga);
  TG_LAUNCHED("k_dir3<16>");
  k_dir3<64><<<grid_for(m, 4, 2048), 256, lds64, st>>>(m, 48, INT32_MAX, W.ei, W.ej, W.es_lo, rp, ci, sdir, ty, L,
                                                       Dd, c2r, edge_rows, ga);
  TG_LAUNCHED("k_dir3<64>");
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
    if (hf) return fail(TG_ERR_INTERNAL, "a directed triad sum is not a multiple of its support edge count");
  }
  timer.finish();
  return TG_OK;
}
