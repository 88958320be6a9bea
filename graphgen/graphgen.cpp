// Seeded synthetic graph and node-type generators.
//
// This module only produces inputs: undirected simple graphs in CSR form
// (both directions stored, rows sorted, no self loops, no duplicates) and
// per-node uint8 types.  It holds none of the graphlet-counting arithmetic and
// is shared by the oracle tests and by the GPU benchmarks.
//
// Random numbers: SplitMix64 (Steele, Lea, Flood 2014).  Every generator
// derives an independent stream per node (or per graph) from (seed, index), so
// the output does not depend on the number of threads.
//
// Graph models:
//  * Chung-Lu G(w): pair {u,v} present with probability min(1, w_u w_v / S),
//    S = sum of weights, sampled exactly in O(n + m) with the skipping method
//    of Miller and Hagberg (2011) over weights sorted in decreasing order;
//    node ids are then shuffled so that id carries no degree information.
//  * Bipartite and k-partite Chung-Lu: the same model restricted to pairs in
//    different parts.
//  * Erdos-Renyi G(n, p) with geometric skipping (Batagelj, Brandes 2005).
// Weight sequences follow a power law in rank: w_r = c (r + r0)^(-1/(gamma-1)),
// with w_0 = wmax and r0 solved so that the mean weight equals the target.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Rng {
  uint64_t s;
  Rng(uint64_t seed, uint64_t stream) {
    uint64_t a = seed * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull;
    uint64_t b = stream;
    s = splitmix64(a) ^ splitmix64(b);
    splitmix64(s);
  }
  uint64_t next() { return splitmix64(s); }
  // uniform in [0, 1)
  double u01() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  // uniform in (0, 1]
  double u01_open0() { return (double)((next() >> 11) + 1) * (1.0 / 9007199254740992.0); }
  uint64_t below(uint64_t k) { return (uint64_t)(u01() * (double)k); }
};

// Sum over r in [0, n) of (r + r0)^(-a): the first terms exactly, the tail by
// the midpoint-rule integral (smooth, monotone integrand).
double power_sum(int64_t n, double r0, double a) {
  const int64_t K = std::min<int64_t>(n, 4096);
  double s = 0.0;
  for (int64_t r = 0; r < K; ++r) s += std::pow((double)r + r0, -a);
  if (n > K) {
    double x0 = (double)K - 0.5 + r0, x1 = (double)n - 0.5 + r0;
    if (std::fabs(a - 1.0) < 1e-12) s += std::log(x1 / x0);
    else s += (std::pow(x1, 1.0 - a) - std::pow(x0, 1.0 - a)) / (1.0 - a);
  }
  return s;
}

// Power-law weights in decreasing order with w[0] = wmax and mean = target.
std::vector<double> power_law_weights(int64_t n, double gamma, double wmax, double mean) {
  const double a = 1.0 / (gamma - 1.0);
  auto mean_of = [&](double r0) { return wmax * std::pow(r0, a) * power_sum(n, r0, a) / (double)n; };
  // mean weight grows with r0 (flatter sequence); bisection in log space
  double lo = 1e-9, hi = 1e15;
  for (int it = 0; it < 120; ++it) {
    double mid = std::sqrt(lo * hi);
    if (mean_of(mid) < mean) lo = mid; else hi = mid;
  }
  const double r0 = std::sqrt(lo * hi);
  const double c = wmax * std::pow(r0, a);
  std::vector<double> w(n);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) w[r] = c * std::pow((double)r + r0, -a);
  return w;
}

struct EdgeBuf {
  std::vector<std::vector<std::pair<int64_t, int64_t>>> per_thread;
  EdgeBuf() : per_thread(omp_get_max_threads()) {}
  void add(int64_t u, int64_t v) { per_thread[omp_get_thread_num()].emplace_back(u, v); }
};

// Miller-Hagberg walk of u against the sorted candidate list cand[v0..v1),
// with weights wv; emits pairs (u, cand[v]).
template <class Emit>
void mh_walk(double wu, const double* wv, int64_t v0, int64_t v1, double S, Rng& rng, Emit emit) {
  int64_t v = v0;
  if (v >= v1) return;
  double p = std::min(1.0, wu * wv[v] / S);
  while (v < v1 && p > 0.0) {
    if (p != 1.0) {
      double r = rng.u01_open0();
      double skip = std::floor(std::log(r) / std::log1p(-p));
      if (skip >= (double)(v1 - v)) return;
      v += (int64_t)skip;
    }
    if (v < v1) {
      double q = std::min(1.0, wu * wv[v] / S);
      double r = rng.u01();
      if (r < q / p) emit(v);
      p = q;
      ++v;
    }
  }
}

void shuffle_ids(std::vector<int32_t>& perm, uint64_t seed) {
  Rng rng(seed, 0xA5A5A5A5ull);
  for (int64_t i = (int64_t)perm.size() - 1; i > 0; --i) {
    int64_t k = (int64_t)rng.below((uint64_t)i + 1);
    std::swap(perm[i], perm[k]);
  }
}

}  // namespace

struct gg_graph {
  int64_t n = 0;
  std::vector<int32_t> row_ptr;  // n + 1
  std::vector<int32_t> col_idx;  // 2m
  std::vector<uint8_t> part;     // part id per node (k-partite models), else empty
};

namespace {

gg_graph* build_csr(int64_t n, EdgeBuf& eb, const std::vector<int32_t>* relabel) {
  gg_graph* g = new gg_graph();
  g->n = n;
  std::vector<int64_t> deg(n + 1, 0);
  for (auto& v : eb.per_thread)
    for (auto& e : v) {
      int64_t a = relabel ? (*relabel)[e.first] : e.first;
      int64_t b = relabel ? (*relabel)[e.second] : e.second;
      deg[a]++; deg[b]++;
    }
  g->row_ptr.assign(n + 1, 0);
  int64_t acc = 0;
  for (int64_t i = 0; i < n; ++i) { g->row_ptr[i] = (int32_t)acc; acc += deg[i]; }
  g->row_ptr[n] = (int32_t)acc;
  g->col_idx.assign(acc, 0);
  std::vector<int64_t> fillp(g->row_ptr.begin(), g->row_ptr.end() - 1);
  for (auto& v : eb.per_thread) {
    for (auto& e : v) {
      int64_t a = relabel ? (*relabel)[e.first] : e.first;
      int64_t b = relabel ? (*relabel)[e.second] : e.second;
      g->col_idx[fillp[a]++] = (int32_t)b;
      g->col_idx[fillp[b]++] = (int32_t)a;
    }
    std::vector<std::pair<int64_t, int64_t>>().swap(v);
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i)
    std::sort(g->col_idx.begin() + g->row_ptr[i], g->col_idx.begin() + g->row_ptr[i + 1]);
  return g;
}

}  // namespace

extern "C" {

// Chung-Lu graph with n nodes, power-law weights (exponent gamma, max wmax,
// mean mean_deg).  Expected edge count n*mean_deg/2 minus the loss from
// probabilities capped at 1.
gg_graph* gg_chung_lu(int64_t n, double gamma, double wmax, double mean_deg, uint64_t seed) {
  if (n < 2 || n >= (1ll << 31)) return nullptr;
  std::vector<double> w = power_law_weights(n, gamma, wmax, mean_deg);
  double S = 0.0;
  for (double x : w) S += x;
  EdgeBuf eb;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t u = 0; u < n - 1; ++u) {
    Rng rng(seed, (uint64_t)u);
    mh_walk(w[u], w.data(), u + 1, n, S, rng, [&](int64_t v) { eb.add(u, v); });
  }
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  shuffle_ids(perm, seed);
  return build_csr(n, eb, &perm);
}

// k-partite Chung-Lu: part p has sizes[p] nodes, power-law weights with
// exponent gammas[p], cap wmaxs[p], mean means[p].  Only pairs in different
// parts can be edges; p(u,v) = min(1, w_u w_v / S) with S chosen so that the
// expected edge count (before capping) is m.  Nodes of part p get part id p.
gg_graph* gg_kpartite_cl(int nparts, const int64_t* sizes, const double* gammas,
                         const double* wmaxs, const double* means, int64_t m, uint64_t seed) {
  if (nparts < 2 || nparts > 255 || m <= 0) return nullptr;
  int64_t n = 0;
  std::vector<int64_t> off(nparts + 1, 0);
  for (int p = 0; p < nparts; ++p) { off[p + 1] = off[p] + sizes[p]; }
  n = off[nparts];
  if (n >= (1ll << 31)) return nullptr;
  std::vector<double> w(n);
  std::vector<double> W(nparts, 0.0);
  for (int p = 0; p < nparts; ++p) {
    std::vector<double> wp = power_law_weights(sizes[p], gammas[p], wmaxs[p], means[p]);
    for (int64_t r = 0; r < sizes[p]; ++r) { w[off[p] + r] = wp[r]; W[p] += wp[r]; }
  }
  double cross = 0.0;
  for (int p = 0; p < nparts; ++p)
    for (int q = p + 1; q < nparts; ++q) cross += W[p] * W[q];
  const double S = cross / (double)m;
  EdgeBuf eb;
  for (int p = 0; p < nparts; ++p) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < sizes[p]; ++r) {
      int64_t u = off[p] + r;
      for (int q = p + 1; q < nparts; ++q) {
        Rng rng(seed ^ (0x1000003ull * (uint64_t)(q + 1)), (uint64_t)u);
        mh_walk(w[u], w.data() + off[q], 0, sizes[q], S, rng,
                [&](int64_t v) { eb.add(u, off[q] + v); });
      }
    }
  }
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  shuffle_ids(perm, seed);
  gg_graph* g = build_csr(n, eb, &perm);
  g->part.assign(n, 0);
  for (int p = 0; p < nparts; ++p)
    for (int64_t r = off[p]; r < off[p + 1]; ++r) g->part[perm[r]] = (uint8_t)p;
  return g;
}

// Erdos-Renyi G(n, p).
gg_graph* gg_gnp(int64_t n, double p, uint64_t seed) {
  if (n < 1 || n >= (1ll << 31) || p < 0.0 || p > 1.0) return nullptr;
  EdgeBuf eb;
  if (p > 0.0) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < n - 1; ++u) {
      Rng rng(seed, (uint64_t)u);
      int64_t v = u + 1;
      while (v < n) {
        if (p < 1.0) {
          double skip = std::floor(std::log(rng.u01_open0()) / std::log1p(-p));
          if (skip >= (double)(n - v)) break;
          v += (int64_t)skip;
        }
        eb.add(u, v);
        ++v;
      }
    }
  }
  return build_csr(n, eb, nullptr);
}

int64_t gg_num_nodes(const gg_graph* g) { return g ? g->n : 0; }
int64_t gg_num_slots(const gg_graph* g) { return g ? (int64_t)g->col_idx.size() : 0; }
const int32_t* gg_row_ptr(const gg_graph* g) { return g->row_ptr.data(); }
const int32_t* gg_col_idx(const gg_graph* g) { return g->col_idx.data(); }
int gg_has_parts(const gg_graph* g) { return g && !g->part.empty(); }
const uint8_t* gg_parts(const gg_graph* g) { return g->part.data(); }
void gg_free(gg_graph* g) { delete g; }

// Types drawn iid uniform in [0, L).
void gg_types_uniform(int64_t n, int L, uint64_t seed, uint8_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Rng rng(seed ^ 0x7F4A7C159E3779B9ull, (uint64_t)i);
    out[i] = (uint8_t)rng.below((uint64_t)L);
  }
}

namespace {
std::vector<double> zipf_cdf(int L, double s) {
  std::vector<double> c(L);
  double acc = 0.0;
  for (int t = 0; t < L; ++t) { acc += std::pow((double)(t + 1), -s); c[t] = acc; }
  for (int t = 0; t < L; ++t) c[t] /= acc;
  c[L - 1] = 1.0;
  return c;
}
uint8_t zipf_draw(const std::vector<double>& cdf, double u) {
  int t = 0;
  while (t + 1 < (int)cdf.size() && u >= cdf[t]) ++t;
  return (uint8_t)t;
}
}  // namespace

// Types drawn iid with P(t) proportional to (t+1)^(-s).
void gg_types_zipf(int64_t n, int L, double s, uint64_t seed, uint8_t* out) {
  std::vector<double> cdf = zipf_cdf(L, s);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Rng rng(seed ^ 0x2545F4914F6CDD1Dull, (uint64_t)i);
    out[i] = zipf_draw(cdf, rng.u01());
  }
}

// Homophilous Zipf types: nodes are visited in a seeded random order; with
// probability p_follow a node takes the most frequent type among its already
// typed neighbours (ties to the smallest type; no typed neighbour: a Zipf
// draw), otherwise a Zipf(s) draw.
void gg_types_homophily(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int L, double s,
                        double p_follow, uint64_t seed, uint8_t* out) {
  std::vector<double> cdf = zipf_cdf(L, s);
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  shuffle_ids(order, seed ^ 0x94D049BB133111EBull);
  const uint8_t NONE = 0xFF;
  std::fill(out, out + n, NONE);
  Rng rng(seed, 0x5EEDull);
  std::vector<int64_t> cnt(L);
  for (int64_t idx = 0; idx < n; ++idx) {
    int32_t v = order[idx];
    double u1 = rng.u01();
    double u2 = rng.u01();
    uint8_t t = NONE;
    if (u1 < p_follow) {
      std::fill(cnt.begin(), cnt.end(), 0);
      int64_t seen = 0;
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        uint8_t tn = out[col_idx[e]];
        if (tn != NONE) { cnt[tn]++; ++seen; }
      }
      if (seen > 0) {
        int best = 0;
        for (int q = 1; q < L; ++q) if (cnt[q] > cnt[best]) best = q;
        t = (uint8_t)best;
      }
    }
    if (t == NONE) t = zipf_draw(cdf, u2);
    out[v] = t;
  }
}

// ---------------------------------------------------------------------------
// Batches of small G(n, rho) graphs.  Graph g uses its own stream (seed, g):
// n = round(exp(U(ln nmin, ln nmax))), rho ~ U(rmin, rmax), L ~ U{lmin..lmax},
// types uniform in [0, L).  Output is concatenated with local node ids.
struct gg_batch {
  int64_t G = 0;
  std::vector<int64_t> node_off, slot_off;
  std::vector<int32_t> row_ptr;  // node_off[G] + G entries (n_g + 1 per graph)
  std::vector<int32_t> col_idx;  // slot_off[G]
  std::vector<uint8_t> types;    // node_off[G]
  std::vector<uint8_t> L;        // G
};

gg_batch* gg_batch_gnp(int64_t G, double nmin, double nmax, double rmin, double rmax, int lmin, int lmax,
                       uint64_t seed) {
  if (G < 0 || nmin < 1 || nmax < nmin || nmax > 65535 || lmin < 1 || lmax < lmin || lmax > 255) return nullptr;
  gg_batch* b = new gg_batch();
  b->G = G;
  std::vector<int64_t> ns(G), ms(G);
  std::vector<double> rhos(G);
  std::vector<uint8_t> Ls(G);
  std::vector<std::vector<int32_t>> rp(G), ci(G);
  std::vector<std::vector<uint8_t>> ty(G);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < G; ++g) {
    Rng rng(seed, (uint64_t)g);
    double ln0 = std::log(nmin), ln1 = std::log(nmax);
    int64_t n = (int64_t)std::llround(std::exp(ln0 + (ln1 - ln0) * rng.u01()));
    if (n < 1) n = 1;
    double rho = rmin + (rmax - rmin) * rng.u01();
    int L = lmin + (int)rng.below((uint64_t)(lmax - lmin + 1));
    ns[g] = n; rhos[g] = rho; Ls[g] = (uint8_t)L;
    // adjacency by pair skipping, local to this graph
    std::vector<std::vector<int32_t>> adj(n);
    Rng er(seed ^ 0xE7037ED1A0B428DBull, (uint64_t)g);
    for (int64_t u = 0; u + 1 < n; ++u) {
      int64_t v = u + 1;
      while (v < n) {
        double skip = std::floor(std::log(er.u01_open0()) / std::log1p(-rho));
        if (skip >= (double)(n - v)) break;
        v += (int64_t)skip;
        adj[u].push_back((int32_t)v);
        adj[v].push_back((int32_t)u);
        ++v;
      }
    }
    rp[g].resize(n + 1);
    int64_t acc = 0;
    for (int64_t u = 0; u < n; ++u) {
      rp[g][u] = (int32_t)acc;
      std::sort(adj[u].begin(), adj[u].end());
      acc += (int64_t)adj[u].size();
    }
    rp[g][n] = (int32_t)acc;
    ci[g].reserve(acc);
    for (int64_t u = 0; u < n; ++u) ci[g].insert(ci[g].end(), adj[u].begin(), adj[u].end());
    ty[g].resize(n);
    Rng tr(seed ^ 0x7F4A7C159E3779B9ull, (uint64_t)g);
    for (int64_t u = 0; u < n; ++u) ty[g][u] = (uint8_t)tr.below((uint64_t)L);
    ms[g] = acc;
  }
  b->node_off.assign(G + 1, 0);
  b->slot_off.assign(G + 1, 0);
  for (int64_t g = 0; g < G; ++g) {
    b->node_off[g + 1] = b->node_off[g] + ns[g];
    b->slot_off[g + 1] = b->slot_off[g] + ms[g];
  }
  b->row_ptr.resize(b->node_off[G] + G);
  b->col_idx.resize(b->slot_off[G]);
  b->types.resize(b->node_off[G]);
  b->L = Ls;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t g = 0; g < G; ++g) {
    std::copy(rp[g].begin(), rp[g].end(), b->row_ptr.begin() + b->node_off[g] + g);
    std::copy(ci[g].begin(), ci[g].end(), b->col_idx.begin() + b->slot_off[g]);
    std::copy(ty[g].begin(), ty[g].end(), b->types.begin() + b->node_off[g]);
  }
  return b;
}

int64_t gg_batch_num_graphs(const gg_batch* b) { return b->G; }
const int64_t* gg_batch_node_off(const gg_batch* b) { return b->node_off.data(); }
const int64_t* gg_batch_slot_off(const gg_batch* b) { return b->slot_off.data(); }
const int32_t* gg_batch_row_ptr(const gg_batch* b) { return b->row_ptr.data(); }
const int32_t* gg_batch_col_idx(const gg_batch* b) { return b->col_idx.data(); }
const uint8_t* gg_batch_types(const gg_batch* b) { return b->types.data(); }
const uint8_t* gg_batch_L(const gg_batch* b) { return b->L.data(); }
void gg_batch_free(gg_batch* b) { delete b; }

}  // extern "C"
