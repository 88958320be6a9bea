// C ABI of libtg.so: argument checks, scratch management, launch sequence.
// The kernels live in tg_kernels.hip, compiled into this translation unit.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tg.h"
#include "tg_kernels.hip"
#include "tg_batch.hip"
#include "tg_mlp.hip"
#include "tg_sparse.hip"
#include "tg_global.hip"

namespace {

thread_local std::string g_last_error;

tg_status fail(tg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

int64_t binom(int64_t n, int64_t k) {
  if (k < 0 || n < k) return 0;
  int64_t r = 1;
  for (int64_t q = 1; q <= k; ++q) r = r * (n - k + q) / q;
  return r;
}

int64_t per_shape(int L, int K) { return binom(L + K - 1, K); }

int64_t nkeys(int L) { return 2 * per_shape(L, 3) + 6 * per_shape(L, 4); }

// Per-edge log2 cost predicted by a learned model (defined with the model).
tg_status tg_internal_predict_costs(const tg_cost_model* model, int64_t n, const int32_t* rp, const int32_t* ci,
                                    const uint8_t* ty, int L, const tg::Work& W, int64_t m, float* out,
                                    hipStream_t st);

#define TG_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t err_ = (call);                                                                 \
    if (err_ != hipSuccess)                                                                   \
      return fail(TG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(err_));           \
  } while (0)

#define TG_LAUNCHED(name)                                                                     \
  do {                                                                                        \
    hipError_t err_ = hipGetLastError();                                                      \
    if (err_ != hipSuccess)                                                                   \
      return fail(TG_ERR_HIP, std::string("launch of ") + name + ": " + hipGetErrorString(err_)); \
  } while (0)

// Stream-ordered scratch: every allocation is released on the same stream when
// the owner goes out of scope.  The default pool keeps freed memory cached.
// A per-device workspace reused by successive calls: allocation through the
// stream-ordered pool costs tens of microseconds per buffer, which a call
// with forty buffers pays twice, with the device idle in between once the
// caller waits for a result.  One call at a time holds the workspace (others
// allocate from the pool as before); its buffers are carved out of it in
// order, and requests beyond its size go to the pool and make the next
// holder grow it to the last call's total.  A holder on another stream
// first waits for the previous holder's work.
struct Workspace {
  std::atomic<bool> busy{false};
  char* base = nullptr;
  size_t cap = 0;
  size_t want = 0;  // total of the last holder's requests
  hipEvent_t done = nullptr;
  hipStream_t last = nullptr;
  bool used = false;
};

inline Workspace* device_workspace() {
  static Workspace ws[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  return &ws[dev];
}

struct Scratch {
  hipStream_t stream;
  std::vector<void*> ptrs;  // pool allocations
  Workspace* ws = nullptr;  // held workspace, or null
  size_t off = 0, total = 0, peak = 0;
  explicit Scratch(hipStream_t s) : stream(s) {
    Workspace* w = device_workspace();
    bool expect = false;
    if (!w || !w->busy.compare_exchange_strong(expect, true)) return;
    ws = w;
    if (ws->used && ws->last != stream && ws->done) (void)hipStreamWaitEvent(stream, ws->done, 0);
    if (ws->want > ws->cap) {
      // grow to the last call's total (a tenth more), freed in stream order
      if (ws->base) (void)hipFreeAsync(ws->base, stream);
      ws->base = nullptr;
      ws->cap = 0;
      const size_t cap = ws->want + ws->want / 10;
      void* p = nullptr;
      if (hipMallocAsync(&p, cap, stream) != hipSuccess) {
        // A workspace that does not fit is no error: the call then takes its
        // memory piece by piece.  Clear the error (the launch checks read
        // it), give the pool's cached memory back and try once more.
        p = nullptr;
        (void)hipGetLastError();
        int dev = 0;
        hipMemPool_t pool;
        if (hipStreamSynchronize(stream) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && hipMemPoolTrimTo(pool, 0) == hipSuccess &&
            hipMallocAsync(&p, cap, stream) != hipSuccess) {
          p = nullptr;
        }
        (void)hipGetLastError();
      }
      if (p) {
        ws->base = (char*)p;
        ws->cap = cap;
      }
    }
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFreeAsync(p, stream);
    if (!ws) return;
    if (!ws->done) (void)hipEventCreateWithFlags(&ws->done, hipEventDisableTiming);
    if (ws->done) (void)hipEventRecord(ws->done, stream);
    ws->last = stream;
    ws->used = true;
    ws->want = std::max(peak, total);
    ws->busy.store(false);
  }
  // Everything obtained after a mark is given back by release(mark), in
  // stream order: later allocations reuse it once the work enqueued before
  // the release is done with it.
  struct Mark {
    size_t off, total, nptrs;
  };
  Mark mark() const { return Mark{off, total, ptrs.size()}; }
  void release(const Mark& mk) {
    for (size_t i = mk.nptrs; i < ptrs.size(); ++i) (void)hipFreeAsync(ptrs[i], stream);
    ptrs.resize(mk.nptrs);
    peak = std::max(peak, total);
    off = mk.off;
    total = mk.total;
  }
  // bytes left in the held workspace
  size_t room() const { return (ws && ws->base && ws->cap > off) ? ws->cap - off : 0; }
  template <class T>
  hipError_t get(T** out, int64_t count) {
    *out = nullptr;
    if (count <= 0) count = 1;
    const size_t bytes = ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
    if (ws) {
      total += bytes;
      if (ws->base && off + bytes <= ws->cap) {
        *out = (T*)(ws->base + off);
        off += bytes;
        return hipSuccess;
      }
    }
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes, stream);
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    *out = (T*)p;
    return hipSuccess;
  }
};
// Frees the current device's workspace once its last holder's work is done
// and trims the default pool.  Fails while a call holds the workspace.
tg_status release_scratch() {
  Workspace* w = device_workspace();
  if (!w) return fail(TG_ERR_HIP, "no current device");
  bool expect = false;
  if (!w->busy.compare_exchange_strong(expect, true))
    return fail(TG_ERR_INVALID_ARG, "a call on another thread holds the scratch workspace");
  hipError_t e = hipSuccess;
  if (w->done) e = hipEventSynchronize(w->done);
  if (e == hipSuccess && w->base) e = hipFree(w->base);
  if (e == hipSuccess) {
    w->base = nullptr;
    w->cap = 0;
    w->want = 0;
    int dev = 0;
    hipMemPool_t pool;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipDeviceGetDefaultMemPool(&pool, dev);
    if (e == hipSuccess) e = hipMemPoolTrimTo(pool, 0);
  }
  w->busy.store(false);
  if (e != hipSuccess) return fail(TG_ERR_HIP, std::string("releasing scratch: ") + hipGetErrorString(e));
  return TG_OK;
}

void keep_pool_cached() {
  static bool done[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

// HIP events around each phase, on the caller's stream.
struct PhaseTimer {
  hipStream_t st;
  float* out;
  hipEvent_t ev[TG_NUM_PHASES + 1];
  int created = 0;
  int marked = 0;
  PhaseTimer(hipStream_t s, float* o) : st(s), out(o) {
    if (!out) return;
    for (int q = 0; q < TG_NUM_PHASES; ++q) out[q] = 0.0f;
    for (int q = 0; q <= TG_NUM_PHASES; ++q) {
      if (hipEventCreate(&ev[q]) != hipSuccess) return;
      ++created;
    }
  }
  ~PhaseTimer() {
    for (int q = 0; q < created; ++q) (void)hipEventDestroy(ev[q]);
  }
  // start of phase q (q == TG_NUM_PHASES: end of the last phase)
  void mark(int q) {
    if (created == TG_NUM_PHASES + 1 && q == marked) {
      if (hipEventRecord(ev[q], st) == hipSuccess) ++marked;
    }
  }
  void finish() {
    if (marked != TG_NUM_PHASES + 1) return;
    if (hipEventSynchronize(ev[TG_NUM_PHASES]) != hipSuccess) return;
    for (int q = 0; q < TG_NUM_PHASES; ++q) (void)hipEventElapsedTime(&out[q], ev[q], ev[q + 1]);
  }
};

inline unsigned grid_for(int64_t items, int64_t per_block, int64_t cap = (1ll << 30)) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

int64_t dense_budget_bytes() {
  const char* s = std::getenv("TG_DENSE_BUDGET_MB");
  int64_t mb = s ? std::atoll(s) : 4096;
  if (mb < 64) mb = 64;
  return mb << 20;
}

// Exclusive scan of in[0, n) into out[0, n], out[n] = total.
template <class T>
tg_status scan(Scratch& S, hipStream_t st, int64_t n, const T* in, T* out) {
  const int64_t nb = (n + 1023) / 1024;
  T* sums;
  TG_HIP(S.get(&sums, nb + 1));
  if (nb > 0) {
    k_scan_blocks<T><<<(unsigned)nb, 256, 0, st>>>(n, in, out, sums);
    TG_LAUNCHED("k_scan_blocks");
  }
  k_scan_sums<T><<<1, 256, 0, st>>>(nb, sums, sums + nb);
  TG_LAUNCHED("k_scan_sums");
  k_scan_add<T><<<grid_for(n + 1, 256, 8192), 256, 0, st>>>(n, out, sums, sums + nb);
  TG_LAUNCHED("k_scan_add");
  return TG_OK;
}

// Gather and row kernels over list[0, count) of one edge class, in batches
// whose accumulators fit ea (ea_budget bytes).
template <int TSIZE, class AccT, bool PROBE>
tg_status combine_class(hipStream_t st, const EdgeArgs& A, int64_t count, const int32_t* list, unsigned grid,
                        int32_t* t_over, int64_t t_cap, int64_t K, void* ea, int64_t ea_budget,
                        unsigned rows_grid) {
  const int64_t per = 4ll * A.L * A.L * (int64_t)sizeof(AccT);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(count, ea_budget / per));
  const size_t lds = combine_lds_bytes<TSIZE, AccT, PROBE>(A.L);
  const int R = 2 * A.L + 3 * A.L * (A.L + 1);
  const size_t rlds = (A.gacc_in_lds ? (size_t)K * sizeof(uint64_t) : 0) +
                      (A.sp_keys ? (size_t)16 * R * sizeof(uint64_t) : 0);
  for (int64_t c0 = 0; c0 < count; c0 += chunk) {
    const int64_t c = std::min(chunk, count - c0);
    const unsigned g = std::min(grid, grid_for(c, 256 / TSIZE));
    k_combine<TSIZE, AccT, PROBE><<<g, 256, lds, st>>>(A, c, list + c0, reinterpret_cast<AccT*>(ea), t_over, t_cap);
    TG_LAUNCHED("k_combine");
    k_combine_rows<AccT><<<grid_for(c, 16, rows_grid), 256, rlds, st>>>(A, c, list + c0,
                                                                         reinterpret_cast<const AccT*>(ea), (int)K);
    TG_LAUNCHED("k_combine_rows");
  }
  return TG_OK;
}

tg_status validate_graph(Scratch& S, hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                         const uint8_t* ty, int L) {
  int32_t* flags;
  TG_HIP(S.get(&flags, 1));
  TG_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t), st));
  int32_t h = 0;
  k_validate_rows<<<grid_for(n + 1, 256, 8192), 256, 0, st>>>(n, nnz, rp, ty, L, flags);
  TG_LAUNCHED("k_validate_rows");
  TG_HIP(hipMemcpyAsync(&h, flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  if (h & TG_VFLAG_ROWPTR) return fail(TG_ERR_INVALID_GRAPH, "row_ptr is not a valid offset array for nnz slots");
  if (h & TG_VFLAG_TYPE) return fail(TG_ERR_TYPE_RANGE, "a node type is >= L");
  k_validate_slots<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, rp, ci, flags);
  TG_LAUNCHED("k_validate_slots");
  TG_HIP(hipMemcpyAsync(&h, flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  if (h & TG_VFLAG_RANGE) return fail(TG_ERR_INVALID_GRAPH, "a column index is outside [0, n)");
  if (h & TG_VFLAG_SELFLOOP) return fail(TG_ERR_INVALID_GRAPH, "self loop");
  if (h & TG_VFLAG_ORDER) return fail(TG_ERR_INVALID_GRAPH, "a row is not strictly increasing (unsorted or duplicate)");
  k_validate_symmetry<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, rp, ci, flags);
  TG_LAUNCHED("k_validate_symmetry");
  TG_HIP(hipMemcpyAsync(&h, flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  if (h & TG_VFLAG_ASYMMETRIC) return fail(TG_ERR_INVALID_GRAPH, "edge stored in one direction only");
  return TG_OK;
}

// Scratch allocation, preprocessing, typed triangles and node tables: the
// part of the pipeline shared by counting and by cost-model training.
// Without `tables` (global counts counted once) the node tables P, U and the
// per-edge 4-cycle counters are neither allocated nor filled.  When the
// common-neighbour lists of all edges fit in `list_budget` bytes the tau
// pass also keeps them.
tg_status prepare_graph(Scratch& S, hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                        const uint8_t* ty, int L, Work& W, PhaseTimer* timer, bool tables = true,
                        int64_t list_budget = 0, bool out_eids = false, int32_t hub_min_degree = 4096) {
  const int64_t m = nnz / 2, P = (int64_t)L * (L + 1) / 2, LL = (int64_t)L * L;
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
  W.out_eid = nullptr;
  if (out_eids) TG_HIP(S.get(&W.out_eid, m));
  TG_HIP(S.get(&W.tau, m * L));
  W.Pn = W.Un = W.C4 = nullptr;
  W.tau_s = nullptr;
  if (tables) {
    TG_HIP(S.get(&W.tau_s, nnz * L));
    TG_HIP(S.get(&W.Pn, n * LL));
    TG_HIP(S.get(&W.Un, n * LL));
    TG_HIP(S.get(&W.C4, m * P));
  }
  TG_HIP(S.get(&W.elist, m));
  TG_HIP(S.get(&W.nlist, n));
  TG_HIP(S.get(&W.counters, 512));

  // ---- prep
  if (timer) timer->mark(TG_PHASE_PREP);
  k_degree<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, rp, W.deg);
  TG_LAUNCHED("k_degree");
  k_node_stats<<<grid_for(n, 4), 256, 0, st>>>(n, rp, ci, W.deg, ty, L, W.D, W.n_upper, W.n_out, W.wedge_work,
                                               W.nbr_deg_sum);
  TG_LAUNCHED("k_node_stats");
  if (tg_status s = scan(S, st, n, W.n_upper, W.upper_off)) return s;
  if (tg_status s = scan(S, st, n, W.n_out, W.out_off)) return s;
  k_fill_edges<<<grid_for(n, 4), 256, 0, st>>>(n, rp, ci, W.deg, W.n_upper, W.upper_off, W.out_off, W.ei, W.ej,
                                               W.s2e, W.es_lo, W.es_hi, W.out_col, W.out_eid);
  TG_LAUNCHED("k_fill_edges");

  // ---- typed triangles per edge, node tables
  if (timer) timer->mark(TG_PHASE_TAU);
  // common-neighbour lists of the edges, so that the per-edge gather does not
  // intersect the rows again (only when the bound on their size fits the
  // budget)
  W.tl_off = nullptr;
  W.tl_k = W.tl_e = nullptr;
  if (m > 0 && 12 * m <= list_budget) {  // every list holds at least one id
    uint64_t* d_total;
    TG_HIP(S.get(&d_total, 1));
    k_fill_u64<<<1, 64, 0, st>>>(d_total, 1, 0);
    TG_LAUNCHED("k_fill_u64");
    k_tl_total<<<grid_for(m, 256, 2048), 256, 0, st>>>(m, W.ei, W.ej, W.deg, d_total);
    TG_LAUNCHED("k_tl_total");
    uint64_t total = 0;
    TG_HIP(hipMemcpyAsync(&total, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (total * 12 <= (uint64_t)list_budget) {
      int64_t* bound;
      TG_HIP(S.get(&bound, m));
      TG_HIP(S.get(&W.tl_off, m + 1));
      k_tl_bound<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, W.ei, W.ej, W.deg, bound);
      TG_LAUNCHED("k_tl_bound");
      if (tg_status s = scan(S, st, m, (const int64_t*)bound, W.tl_off)) return s;
      TG_HIP(S.get(&W.tl_k, (int64_t)total));
      TG_HIP(S.get(&W.tl_e, 2 * (int64_t)total));
    }
  }
  W.tl_packed = n < (1ll << 27) ? 1 : 0;
  // Edges whose longer row is a hub's (degree above hub_min) are searched
  // in a bitmap of the hub's row instead (k_tau_hub); the threshold rises
  // until the bitmaps and their ranks (12 B per 64 node ids per hub) fit in
  // 4 GiB.
  int32_t hub_min = INT32_MAX;
  int64_t nh = 0, hub_slots = 0;
  W.hub_of = nullptr;
  W.hub_bits = nullptr;
  W.hub_rank = nullptr;
  W.hub_nw = 0;
  const int64_t nw = (n + 63) / 64;
  int32_t* hubs = nullptr;
  int64_t* hoff = nullptr;
  uint64_t* hbits = nullptr;
  int32_t* hrank = nullptr;
  if (hub_min_degree > 0 && m > 0) {
    int32_t* d_cnt;
    TG_HIP(S.get(&d_cnt, 1));
    for (int32_t h = hub_min_degree; h > 0 && h < (1 << 30); h *= 2) {
      k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(d_cnt), 1, 0u);
      k_hubs_above<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, W.deg, h, 1, d_cnt, nullptr, nullptr);
      TG_LAUNCHED("k_hubs_above");
      int32_t c = 0;
      TG_HIP(hipMemcpyAsync(&c, d_cnt, sizeof(c), hipMemcpyDeviceToHost, st));
      TG_HIP(hipStreamSynchronize(st));
      if ((int64_t)c * nw * 12 <= (4ll << 30)) {
        hub_min = h;
        nh = c;
        break;
      }
    }
    if (nh > 0) {
      int64_t* hdeg;
      TG_HIP(S.get(&hubs, nh));
      TG_HIP(S.get(&hdeg, nh));
      TG_HIP(S.get(&hoff, nh + 1));
      k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(d_cnt), 1, 0u);
      k_hubs_above<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, W.deg, hub_min, 0, d_cnt, hubs, hdeg);
      TG_LAUNCHED("k_hubs_above");
      if (tg_status s = scan(S, st, nh, (const int64_t*)hdeg, hoff)) return s;
      TG_HIP(hipMemcpyAsync(&hub_slots, hoff + nh, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      TG_HIP(S.get(&hbits, nh * nw));
      TG_HIP(S.get(&hrank, nh * nw));
      k_fill_u64<<<grid_for(nh * nw, 256, 16384), 256, 0, st>>>(hbits, nh * nw, 0);
      TG_LAUNCHED("k_fill_u64");
      TG_HIP(hipStreamSynchronize(st));
      k_hub_bits<<<grid_for(hub_slots, 256, 16384), 256, 0, st>>>(hub_slots, nh, hubs, hoff, rp, ci, nw, hbits);
      TG_LAUNCHED("k_hub_bits");
      k_hub_rank<<<(unsigned)nh, 256, 0, st>>>(nw, hbits, hrank);
      TG_LAUNCHED("k_hub_rank");
      // kept for the gather's row intersections
      TG_HIP(S.get(&W.hub_of, n));
      k_fill_u32<<<grid_for(n, 256, 16384), 256, 0, st>>>(reinterpret_cast<uint32_t*>(W.hub_of), n, 0xffffffffu);
      k_hub_index<<<grid_for(nh, 256, 1024), 256, 0, st>>>(nh, hubs, W.hub_of);
      TG_LAUNCHED("k_hub_index");
      W.hub_bits = hbits;
      W.hub_rank = hrank;
      W.hub_nw = nw;
    } else {
      hub_min = INT32_MAX;
    }
  }
  k_tau<16><<<grid_for(m, 16, 8192), 256, 0, st>>>(m, -1, 48, W.ei, W.ej, rp, ci, W.deg, ty, L, W.tau, W.es_lo,
                                                   W.es_hi, W.tau_s, W.tl_off, W.tl_k, W.tl_e, W.tl_packed, hub_min);
  TG_LAUNCHED("k_tau<16>");
  k_tau<64><<<grid_for(m, 4, 8192), 256, 0, st>>>(m, 48, INT32_MAX, W.ei, W.ej, rp, ci, W.deg, ty, L, W.tau, W.es_lo,
                                                  W.es_hi, W.tau_s, W.tl_off, W.tl_k, W.tl_e, W.tl_packed, hub_min);
  TG_LAUNCHED("k_tau<64>");
  if (nh > 0) {
    k_tau_hub<<<grid_for(hub_slots, 4, 16384), 256, 0, st>>>(hub_slots, nh, hubs, hoff, nw, hbits, hrank, rp, ci,
                                                             W.deg, W.s2e, ty, L, W.tau, W.es_lo, W.es_hi, W.tau_s,
                                                             W.tl_off, W.tl_k, W.tl_e, W.tl_packed);
    TG_LAUNCHED("k_tau_hub");
  }
  if (timer) timer->mark(TG_PHASE_TABLES);
  if (tables) {
    k_node_tables<<<grid_for(n, 4), 256, (size_t)(4 * 2 * LL * sizeof(uint64_t)), st>>>(n, rp, ci, ty, L, W.D,
                                                                                       W.tau_s, W.Pn, W.Un);
    TG_LAUNCHED("k_node_tables");
  }

  return TG_OK;
}

// List budget of the default tuning: work labels measure the gather as
// tg_count runs it by default.
inline int64_t default_list_budget() {
  tg_tuning t;
  tg_tuning_default(&t);
  return (int64_t)std::max(0, t.tlist_budget_mib) << 20;
}

// Host-side choice of LDS copies for the key sums [k0, k0 + nk) of one kernel
// within `budget` bytes (no copies: straight global atomics).
GAcc make_gacc(uint64_t* g, int64_t k0, int64_t nk, int64_t budget) {
  const int64_t c = budget / std::max<int64_t>(1, nk * (int64_t)sizeof(uint64_t));
  return GAcc{g, k0, nk, (int)std::min<int64_t>(8, std::max<int64_t>(0, c))};
}

size_t gacc_bytes(const GAcc& a) { return (size_t)a.copies * a.nk * sizeof(uint64_t); }

// The gather and row kernels over the three edge classes (16-lane teams,
// wavefronts, workgroups).  PROBE: the gather finds each edge's 4-cliques
// from out-lists (else the clique pass has counted them).
template <bool PROBE>
tg_status combine_classes(Scratch& S, hipStream_t st, const EdgeArgs& A, const Work& W, const int64_t* class_begin,
                          const int64_t* class_count, int64_t K, void* ea, int64_t ea_budget, const tg_tuning& tune,
                          int cus, int64_t max_t_heavy) {
  const int L = A.L;
  // workgroups that fit the device at once for a launch of `kernel` with
  // `lds` bytes (the default caps)
  auto resident = [&](const void* kernel, size_t lds) -> int64_t {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds) != hipSuccess) per_cu = 1;
    return (int64_t)std::max(1, cus) * std::max(1, per_cu);
  };
  const unsigned rows_grid = tune.combine_grid > 0 ? (unsigned)tune.combine_grid : 8192u;
  if (class_count[0] > 0) {
    const int64_t cap = tune.combine_grid > 0 ? tune.combine_grid
                                              : resident((const void*)k_combine<16, uint32_t, PROBE>,
                                                         combine_lds_bytes<16, uint32_t, PROBE>(L));
    if (tg_status s2 = combine_class<16, uint32_t, PROBE>(st, A, class_count[0], W.elist + class_begin[0],
                                                   grid_for(class_count[0], 16, cap), nullptr, 0, K, ea, ea_budget,
                                                   rows_grid))
      return s2;
  }
  if (class_count[1] > 0) {
    const int64_t cap = tune.combine_grid > 0 ? tune.combine_grid
                                              : resident((const void*)k_combine<64, uint32_t, PROBE>,
                                                         combine_lds_bytes<64, uint32_t, PROBE>(L));
    if (tg_status s2 = combine_class<64, uint32_t, PROBE>(st, A, class_count[1], W.elist + class_begin[1],
                                                   grid_for(class_count[1], 4, cap), nullptr, 0, K, ea, ea_budget,
                                                   rows_grid))
      return s2;
  }
  if (class_count[2] > 0) {
    // default: one workgroup per resident slot (CUs x workgroups per CU at
    // this launch's LDS), so that no second partial wave of workgroups runs
    const int64_t cap = tune.wg_grid > 0 ? tune.wg_grid
                                         : resident((const void*)k_combine<256, uint64_t, PROBE>,
                                                    combine_lds_bytes<256, uint64_t, PROBE>(L));
    const unsigned grid = grid_for(class_count[2], 1, cap);
    int32_t* t_over = nullptr;
    int64_t t_cap = 0;
    if (PROBE && max_t_heavy > TG_T_WG_CAP) {
      t_cap = max_t_heavy;
      TG_HIP(S.get(&t_over, over_scratch_ints(grid, t_cap)));
    }
    if (tg_status s2 = combine_class<256, uint64_t, PROBE>(st, A, class_count[2], W.elist + class_begin[2], grid, t_over,
                                                    t_cap, K, ea, ea_budget, rows_grid))
      return s2;
  }

  return TG_OK;
}

// Node plan of the clique pass (tg_clique.hip): tier sizes, the largest
// out-degree, and the nodes listed by tier (tiers 3-6 in decreasing
// out-degree order).  ok = false when a node has more out-neighbours than
// the pass supports (nothing listed then).
struct K4Plan {
  bool ok = false;
  int64_t count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t start[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int32_t dmax = 0;
  int32_t* list = nullptr;
};

tg_status k4_plan(Scratch& S, hipStream_t st, int64_t n, const int32_t* out_off, K4Plan& plan) {
  int32_t* c;
  TG_HIP(S.get(&c, 32));
  k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(c), 32, 0u);
  TG_LAUNCHED("k_fill_u32");
  k_k4_tier_count<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, out_off, c, c + 8);
  TG_LAUNCHED("k_k4_tier_count");
  int32_t h[9];
  TG_HIP(hipMemcpyAsync(h, c, sizeof(h), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  plan.dmax = h[8];
  if (h[7] > 0) return TG_OK;  // out-degree above TG_K4_LDS_IDS
  int64_t acc = 0;
  int32_t cur[8];
  for (int t = 0; t < 8; ++t) {
    plan.count[t] = t == 0 ? 0 : h[t];
    plan.start[t] = acc;
    cur[t] = (int32_t)acc;
    acc += plan.count[t];
  }
  TG_HIP(S.get(&plan.list, std::max<int64_t>(1, acc)));
  TG_HIP(hipMemcpyAsync(c + 16, cur, sizeof(cur), hipMemcpyHostToDevice, st));
  k_k4_tier_scatter<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, out_off, c + 16, plan.list);
  TG_LAUNCHED("k_k4_tier_scatter");
  plan.ok = true;
  return TG_OK;
}

// Launches the clique pass over the planned nodes.  Each tier takes a
// wavefront team per node with LDS rows when they fit in lds_kib KiB per
// workgroup (at most 64), else a workgroup team with LDS rows, else a
// workgroup team with rows in global scratch.
template <bool GLOB>
tg_status k4_launch(Scratch& S, hipStream_t st, const K4Args& K, const K4Plan& plan, int cus, int grid_big,
                    int lds_kib, GAcc ga) {
  const int L = K.L;
  const size_t gb = GLOB ? gacc_bytes(ga) : 0;
  const size_t cap = (size_t)std::max(0, std::min(lds_kib, 64)) << 10;
  auto run = [&](int64_t cnt, const int32_t* list, int dcap) -> tg_status {
    if (cnt <= 0) return TG_OK;
    const size_t l64 = 4 * (size_t)k4_team_lds<64, false>(dcap, L);
    const size_t l256 = (size_t)k4_team_lds<256, false>(dcap, L);
    if (dcap <= 64 && l64 + gb <= cap) {
      k_k4_low<64, false, GLOB><<<grid_for(cnt, 4, 8192), 256, l64 + gb, st>>>(K, cnt, list, dcap, nullptr, 0, ga);
      TG_LAUNCHED("k_k4_low<64>");
    } else if (l256 + gb <= cap) {
      k_k4_low<256, false, GLOB><<<grid_for(cnt, 1, 4096), 256, l256 + gb, st>>>(K, cnt, list, dcap, nullptr, 0, ga);
      TG_LAUNCHED("k_k4_low<256>");
    } else {
      const int64_t grid = std::min<int64_t>(cnt, grid_big > 0 ? grid_big : 2 * (int64_t)cus);
      const int64_t stride = k4_gscr_bytes(dcap, L);
      char* g;
      TG_HIP(S.get(&g, grid * stride));
      k_k4_low<256, true, GLOB><<<(unsigned)grid, 256, (size_t)k4_team_lds<256, true>(dcap, L) + gb, st>>>(
          K, cnt, list, dcap, g, stride, ga);
      TG_LAUNCHED("k_k4_low<256, global rows>");
    }
    return TG_OK;
  };
  if (tg_status s = run(plan.count[1], plan.list + plan.start[1], 64)) return s;
  if (tg_status s = run(plan.count[2], plan.list + plan.start[2], 256)) return s;
  const int64_t big = plan.count[3] + plan.count[4] + plan.count[5] + plan.count[6];
  if (tg_status s = run(big, plan.list + plan.start[3], std::max(257, plan.dmax))) return s;
  return TG_OK;
}

// once: global counts only, every instance counted a fixed number of times
// (tg_count_global); otherwise per-edge counting with Eq. 17 (tg_count).
// With once, ty may hold nty type vectors of n entries each and
// global_counts then receives nty vectors of K(L) counts; the work that does
// not depend on types (degree order, out-lists, 4-cycle groups, 4-clique
// edge classes) is done once.
// Sparse per-edge output of tg_count_sparse: nonzero (key, count) pairs of
// the requested edges, edge q's at [start[q], start[q] + len[q]).
struct SparseOut {
  uint32_t* keys = nullptr;
  uint64_t* counts = nullptr;
  int64_t* start = nullptr;
  int32_t* len = nullptr;
  int64_t cap = 0;
  int64_t* total = nullptr;  // host
};

tg_status count_impl(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const uint8_t* ty, int L,
                     uint64_t* global_counts, uint64_t* edge_counts, int32_t* edge_endpoints,
                     const tg_options* opt_in, hipStream_t st, bool once = false, int64_t nty = 1,
                     const SparseOut* sparse = nullptr) {
  tg_options opt;
  tg_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (nty < 1 || (nty > 1 && !once)) return fail(TG_ERR_INVALID_ARG, "bad number of type vectors");
  if (once) {
    if (!global_counts) return fail(TG_ERR_INVALID_ARG, "null global_counts");
    edge_counts = nullptr;
    edge_endpoints = nullptr;
    opt.edge_orbits = nullptr;
    opt.edge_ids = nullptr;
    opt.num_edge_ids = 0;
    opt.edge_begin = 0;
    opt.edge_end = -1;
    opt.schedule = TG_SCHED_DEGREE;
  }
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (n < 0 || nnz < 0 || n >= (1ll << 31) || nnz >= (1ll << 31))
    return fail(TG_ERR_INVALID_ARG, "n and nnz must be in [0, 2^31)");
  if (n * (int64_t)L >= (1ll << 31)) return fail(TG_ERR_INVALID_ARG, "n * L must be below 2^31");
  if (!rp || (!global_counts && !edge_counts && !opt.edge_orbits && !sparse) || (nnz > 0 && !ci) || (n > 0 && !ty))
    return fail(TG_ERR_INVALID_ARG, "null input or output pointer");
  if (sparse && L > 8) return fail(TG_ERR_UNSUPPORTED_L, "sparse per-edge output takes L <= 8");
  if (sparse && (!sparse->start || !sparse->len || !sparse->total || sparse->cap < 0 ||
                 (sparse->cap > 0 && (!sparse->keys || !sparse->counts))))
    return fail(TG_ERR_INVALID_ARG, "null sparse output pointer or negative capacity");
  if (sparse) *sparse->total = 0;
  if (nnz % 2) return fail(TG_ERR_INVALID_GRAPH, "nnz is odd: some edge is stored in one direction only");
  if (opt.schedule < TG_SCHED_NONE || opt.schedule > TG_SCHED_LEARNED)
    return fail(TG_ERR_INVALID_ARG, "unknown schedule");
  if (opt.schedule == TG_SCHED_LEARNED && !opt.model)
    return fail(TG_ERR_INVALID_ARG, "TG_SCHED_LEARNED needs a cost model");
  const int64_t m = nnz / 2;
  const int64_t eb = opt.edge_begin, ee = opt.edge_end < 0 ? m : opt.edge_end;
  if (eb < 0 || eb > ee || ee > m) return fail(TG_ERR_INVALID_ARG, "edge range outside [0, m]");
  const int64_t K = nkeys(L), P = (int64_t)L * (L + 1) / 2, LL = (int64_t)L * L;
  if (opt.edge_ids && opt.num_edge_ids < 0) return fail(TG_ERR_INVALID_ARG, "negative num_edge_ids");
  const int64_t* ids = (opt.edge_ids && opt.num_edge_ids > 0) ? opt.edge_ids : nullptr;
  const int64_t nids = ids ? opt.num_edge_ids : 0;
  keep_pool_cached();
  Scratch S(st);
  if (ids) {
    int32_t* bad;
    TG_HIP(S.get(&bad, 1));
    TG_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
    k_check_ids<<<grid_for(nids, 256, 4096), 256, 0, st>>>(ids, nids, m, bad);
    TG_LAUNCHED("k_check_ids");
    int32_t hb = 0;
    TG_HIP(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (hb) return fail(TG_ERR_INVALID_ARG, "edge_ids must be strictly increasing canonical edge ids in [0, m)");
  }
  PhaseTimer timer(st, opt.phase_ms);

  if (global_counts) {
    k_fill_u64<<<grid_for(K * nty, 256, 1024), 256, 0, st>>>(global_counts, K * nty, 0);
    TG_LAUNCHED("k_fill_u64");
  }
  // without global counts only the edges whose rows are asked for go through
  // the per-edge combine (the 4-cycle pass still covers the whole graph)
  const int64_t* sel = global_counts ? nullptr : ids;
  const int64_t sel_e0 = (global_counts || ids) ? 0 : eb;
  const int64_t sel_count = global_counts ? m : (ids ? nids : ee - eb);
  if (opt.validate && n > 0) {
    for (int64_t b = 0; b < nty; ++b) {
      tg_status vs = validate_graph(S, st, n, nnz, rp, ci, ty + b * n, L);
      if (vs != TG_OK) return vs;
    }
  } else if (opt.validate) {
    int32_t h0 = -1;
    TG_HIP(hipMemcpyAsync(&h0, rp, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (h0 != 0 || nnz != 0) return fail(TG_ERR_INVALID_GRAPH, "empty graph must have row_ptr[0] == 0 and nnz == 0");
  }
  if (m == 0) return TG_OK;

  tg_tuning tune;
  tg_tuning_default(&tune);
  if (opt.tuning) tune = *opt.tuning;
  Work W;
  const int64_t list_budget = once ? 0 : (int64_t)std::max(0, tune.tlist_budget_mib) << 20;
  // 4-cliques of every edge in one pass over the graph (when the per-edge
  // step covers enough of the edges for a whole-graph pass to pay)
  const bool want_k4_pass = !once && tune.clique_pass != 0 && sel_count * 8 >= m;
  if (tg_status s = prepare_graph(S, st, n, nnz, rp, ci, ty, L, W, &timer, !once, list_budget, want_k4_pass,
                                  std::max(0, tune.tau_hub_min_degree)))
    return s;

  // ---- schedule: edge classes and cost buckets, node tiers
  timer.mark(TG_PHASE_SCHEDULE);
  const int mode = opt.schedule == TG_SCHED_NONE ? 0 : (opt.schedule == TG_SCHED_DEGREE ? 1 : 2);
  BinParams bp{mode,
               std::max(1, tune.light_max_degree),
               std::max(1, tune.heavy_min_degree),
               std::min(64, std::max(0, tune.mid_log2_cost)),
               std::min(64, std::max(0, tune.heavy_log2_cost)),
               L <= 8 ? 1 : 0};
  const float* pred = nullptr;
  if (mode == 2) {
    float* p;
    TG_HIP(S.get(&p, m));
    tg_status s = tg_internal_predict_costs(opt.model, n, rp, ci, ty, L, W, m, p, st);
    if (s != TG_OK) return s;
    pred = p;
  }
  // counters: [0,192) edge bins (class * 64 + bucket), [256,260) node tiers,
  // [264] max |T| of workgroup-class edges, [272] divisibility flag
  int32_t* cnt = W.counters;
  TG_HIP(hipMemsetAsync(cnt, 0, 512 * sizeof(int32_t), st));
  if (!once) {
    k_edge_bin_count<<<grid_for(sel_count, 256, 8192), 256, 0, st>>>(sel_count, sel, sel_e0, W.ei, W.ej, W.deg,
                                                                     W.tau, L, bp, pred, cnt,
                                                                     (uint32_t*)(cnt + 264));
    TG_LAUNCHED("k_edge_bin_count");
  }
  k_node_tier_count<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, W.wedge_work, cnt + 256);
  TG_LAUNCHED("k_node_tier_count");
  k_max_degree<<<grid_for(n, 256, 1024), 256, 0, st>>>(n, W.deg, cnt + 268);
  TG_LAUNCHED("k_max_degree");
  int32_t h_cnt[512];
  TG_HIP(hipMemcpyAsync(h_cnt, cnt, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  int32_t cur[512];
  memset(cur, 0, sizeof(cur));
  int64_t acc = 0, class_begin[3], class_count[3];
  for (int c = 0; c < 3; ++c) {
    class_begin[c] = acc;
    for (int b = 0; b < 64; ++b) { cur[c * 64 + b] = (int32_t)acc; acc += h_cnt[c * 64 + b]; }
    class_count[c] = acc - class_begin[c];
  }
  int64_t nacc = 0;
  for (int t = 0; t < 4; ++t) { cur[256 + t] = (int32_t)nacc; nacc += h_cnt[256 + t]; }
  const int64_t max_t_heavy = (uint32_t)h_cnt[264];
  const int64_t max_deg = h_cnt[268];
  // 32-bit 4-cycle counters when (d_i - 1)(d_j - 1) < 2^32 on every edge
  const bool c4_wide = (max_deg - 1) * (max_deg - 1) >= (1ll << 32);
  // the heavy pass sums the credits of one window's x-side edges in 32-bit
  // LDS counters (a window holds at most one chunk of wedges, each credit at
  // most the maximum degree)
  TG_HIP(hipMemcpyAsync(cnt, cur, 264 * sizeof(int32_t), hipMemcpyHostToDevice, st));
  if (!once) {
    k_edge_bin_scatter<<<grid_for(sel_count, 256, 8192), 256, 0, st>>>(sel_count, sel, sel_e0, W.ei, W.ej, W.deg,
                                                                       W.tau, L, bp, pred, cnt, W.elist);
    TG_LAUNCHED("k_edge_bin_scatter");
  }
  k_node_tier_scatter<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, W.wedge_work, cnt + 256, W.nlist);
  TG_LAUNCHED("k_node_tier_scatter");

  // ---- non-induced typed 4-cycles per edge
  timer.mark(TG_PHASE_CYCLES);
  const int64_t n_t1 = h_cnt[257], n_t2 = h_cnt[258], n_t3 = h_cnt[259];
  uint32_t* C4n = reinterpret_cast<uint32_t*>(W.C4);
  // Credits go to one row per CSR slot when those rows fit the budget
  // (consecutive wedges then credit consecutive rows), folded into per-edge
  // rows afterwards; else straight to per-edge rows.
  const int64_t c4_width = c4_wide ? 8 : 4;
  const bool slot_rows = !once && nnz * P * c4_width <= ((int64_t)std::max(0, tune.c4_slot_budget_mb) << 20);
  // what the 4-cycle pass allocates from here on is given back after its fold
  const Scratch::Mark c4_mark = S.mark();
  // Split counters (C4Split): when 64-bit slot rows do not fit the budget,
  // 32-bit slot rows if the device has room for them, the edges that may
  // pass 2^c4_split_log2 cycles counted in their 64-bit per-edge counters.
  bool split = false;
  if (!once && c4_wide && !slot_rows && tune.c4_split_log2 > 0) {
    size_t free_b = 0, total_b = 0;
    TG_HIP(hipMemGetInfo(&free_b, &total_b));
    // memory the default pool holds but has not handed out counts as free
    int pdev = 0;
    hipMemPool_t pool;
    uint64_t reserved = 0, used = 0;
    if (hipGetDevice(&pdev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, pdev) == hipSuccess &&
        hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &reserved) == hipSuccess &&
        hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemCurrent, &used) == hipSuccess && reserved > used)
      free_b += (size_t)(reserved - used);
    const size_t need = (size_t)nnz * (size_t)P * sizeof(uint32_t);
    split = need + (8ull << 30) <= free_b + S.room();
  }
  const bool srows = slot_rows || split;  // counters per CSR slot
  const bool c4s_wide = c4_wide && !split;  // width of the counters the walks credit
  const int32_t* s2x = srows ? nullptr : W.s2e;
  const int64_t crows = srows ? nnz : m;  // counters are C4[p * crows + row]
  uint64_t* C4w_t = W.C4;
  uint32_t* C4n_t = C4n;
  C4Split c4x{};
  if (slot_rows) {
    uint64_t* c4s;
    TG_HIP(S.get(&c4s, (nnz * P * c4_width + 7) / 8));
    k_fill_u64<<<grid_for((nnz * P * c4_width + 7) / 8, 256, 8192), 256, 0, st>>>(c4s, (nnz * P * c4_width + 7) / 8,
                                                                                 0);
    C4w_t = c4s;
    C4n_t = reinterpret_cast<uint32_t*>(c4s);
  } else if (split) {
    TG_HIP(S.get(&C4n_t, nnz * P));
    k_fill_u32<<<grid_for(nnz * P, 256, 16384), 256, 0, st>>>(C4n_t, nnz * P, 0);
    k_fill_u64<<<grid_for(m * P, 256, 8192), 256, 0, st>>>(W.C4, m * P, 0);
    c4x.C4e = W.C4;
    c4x.s2e = W.s2e;
    c4x.lim = 1ull << std::min(32, tune.c4_split_log2);
    c4x.P = (int)P;
  } else if (!once) {
    k_fill_u64<<<grid_for(m * P, 256, 8192), 256, 0, st>>>(W.C4, m * P, 0);
  }
  TG_LAUNCHED("k_fill_u64");
  // degree and type of every slot's column node, so that the wedge walks read
  // them in row order (one type vector only; degrees below 2^28)
  uint32_t* cdt = nullptr;
  if (nty == 1 && max_deg < (1ll << 28)) {
    TG_HIP(S.get(&cdt, nnz));
    k_slot_dt<<<grid_for(nnz, 256, 16384), 256, 0, st>>>(nnz, ci, W.deg, ty, cdt);
    TG_LAUNCHED("k_slot_dt");
  }
  // once: the 4-cycle keys, summed twice per cycle
  const int64_t C3k = per_shape(L, 3), C4k = per_shape(L, 4);
  // key copies of type vector b's 4-cycle sums within `budget` bytes
  auto gacc_cyc = [&](int64_t b, int64_t budget) {
    return make_gacc(global_counts + b * K, 2 * C3k + 2 * C4k, C4k, budget);
  };
  for (int64_t b = 0; once && b < nty; ++b) {
    const GAcc ga_cyc = gacc_cyc(b, 8 << 10);
    if (n_t1 > 0) {
      k_c4_hash<1, 8, uint32_t, true><<<grid_for(n_t1, 4, 4096), 256, gacc_bytes(ga_cyc), st>>>(
          n_t1, W.nlist + cur[257], rp, ci, W.deg, ty + b * n, L, nullptr, nullptr, 0, ga_cyc, cdt, C4Split{});
      TG_LAUNCHED("k_c4_hash<1, glob>");
    }
    if (n_t2 > 0) {
      k_c4_hash<4, 12, uint32_t, true><<<grid_for(n_t2, 1, 2048), 256, gacc_bytes(ga_cyc), st>>>(
          n_t2, W.nlist + cur[258], rp, ci, W.deg, ty + b * n, L, nullptr, nullptr, 0, ga_cyc, cdt, C4Split{});
      TG_LAUNCHED("k_c4_hash<4, glob>");
    }
  }
  if (!once && n_t1 > 0) {
    if (c4s_wide)
      k_c4_hash<1, 8, uint64_t><<<grid_for(n_t1, 4, 4096), 256, 0, st>>>(n_t1, W.nlist + cur[257], rp, ci, W.deg, ty,
                                                                         L, s2x, C4w_t, crows, GAcc{}, cdt, c4x);
    else
      k_c4_hash<1, 8, uint32_t><<<grid_for(n_t1, 4, 4096), 256, 0, st>>>(n_t1, W.nlist + cur[257], rp, ci, W.deg, ty,
                                                                         L, s2x, C4n_t, crows, GAcc{}, cdt, c4x);
    TG_LAUNCHED("k_c4_hash<1>");
  }
  if (!once && n_t2 > 0) {
    if (c4s_wide)
      k_c4_hash<4, 12, uint64_t><<<grid_for(n_t2, 1, 2048), 256, 0, st>>>(n_t2, W.nlist + cur[258], rp, ci, W.deg,
                                                                          ty, L, s2x, C4w_t, crows, GAcc{}, cdt, c4x);
    else
      k_c4_hash<4, 12, uint32_t><<<grid_for(n_t2, 1, 2048), 256, 0, st>>>(n_t2, W.nlist + cur[258], rp, ci, W.deg,
                                                                          ty, L, s2x, C4n_t, crows, GAcc{}, cdt, c4x);
    TG_LAUNCHED("k_c4_hash<4>");
  }
  if (n_t3 > 0) {
    // heaviest nodes first, in groups sharing one launch per phase
    std::vector<int32_t> hx(n_t3);
    std::vector<uint64_t> hw(n_t3);
    std::vector<int32_t> hd(n_t3);
    TG_HIP(hipMemcpyAsync(hx.data(), W.nlist + cur[259], n_t3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    // gather W and degree of the listed nodes on the host side of the copy
    {
      int32_t* d_idx;
      uint64_t* d_w;
      int32_t* d_d;
      TG_HIP(S.get(&d_idx, n_t3));
      TG_HIP(S.get(&d_w, n_t3));
      TG_HIP(S.get(&d_d, n_t3));
      k_gather_node_info<<<grid_for(n_t3, 256, 8192), 256, 0, st>>>(n_t3, W.nlist + cur[259], W.wedge_work, W.deg,
                                                                    d_w, d_d);
      TG_LAUNCHED("k_gather_node_info");
      TG_HIP(hipMemcpyAsync(hw.data(), d_w, n_t3 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
      TG_HIP(hipMemcpyAsync(hd.data(), d_d, n_t3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      TG_HIP(hipStreamSynchronize(st));
    }
    std::vector<int64_t> order(n_t3);
    for (int64_t q = 0; q < n_t3; ++q) order[q] = q;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return hw[a] != hw[b] ? hw[a] > hw[b] : hx[a] < hx[b];
    });
    // dense rows: 16-bit counts (two per word) when no count can exceed
    // 65535 (a count is at most d_x), else 32-bit
    const bool half = max_deg < 65536;
    const int CS = L <= 8 ? 8 : 16;
    const int RW = half ? CS / 2 : CS;
    const int64_t stride = n * RW;
    // Nodes whose far ends are few compared with n (a table of 2^k >= 2
    // min(W, n) rows is at least c4_hash_ratio times smaller than a dense
    // array) use hash tables; the rest (the heaviest, a prefix of the
    // order) use dense arrays.
    auto hash_log2 = [&](uint64_t wq) {
      const int64_t want = 2 * std::min<int64_t>((int64_t)wq, n);
      int lg = 6;
      while ((1ll << lg) < want) ++lg;
      return lg;
    };
    // the bucketed counts of dense groups (below) shift the balance towards
    // hash tables for the lighter nodes: their own ratio applies then
    const bool parts_ok = !once && tune.c4_parts != 0 && cdt && L <= 8 && nty == 1;
    const int hash_ratio = std::max(0, parts_ok ? tune.c4_part_hash_ratio : tune.c4_hash_ratio);
    int64_t qd = n_t3;  // nodes [0, qd) dense, [qd, n_t3) hashed
    if (hash_ratio > 0) {
      qd = 0;
      while (qd < n_t3 && ((1ll << hash_log2(hw[order[qd]])) * (1 + RW)) * hash_ratio > stride) ++qd;
    }
    int64_t Gmax = dense_budget_bytes() / (stride * (int64_t)sizeof(uint32_t));
    Gmax = std::max<int64_t>(1, std::min<int64_t>(Gmax, std::min<int64_t>(256, n_t3)));
    // groups of consecutive nodes (heaviest first): a group closes once its
    // wedges fill the chip (c4_group_kwedges thousand) or its count rows
    // would touch more than c4_footprint_mb, so that they can stay in the
    // last-level cache; at most Gmax nodes per dense group
    const int64_t foot = (int64_t)std::max(1, tune.c4_footprint_mb) << 20;
    const int64_t wtarget = (int64_t)std::max(1, tune.c4_group_kwedges) * 1000;
    // dense groups split their far ends into one slice per XCD (c4_slices);
    // a group's count rows are then capped at 2 MiB per slice so that each
    // XCD's L2 can hold its part
    int64_t dense_slots = 0;
    for (int64_t q = 0; q < qd; ++q) dense_slots += hd[order[q]];
    const int nsl = (tune.c4_slices > 1 && dense_slots > 0 && dense_slots * tune.c4_slices * 16 <= (4ll << 30))
                        ? tune.c4_slices : 1;
    // (with the bucketed counts, slices only split the credit walk, whose
    // workgroups run node after node, so the groups keep their full size)
    const int64_t foot_dense = (nsl > 1 && !parts_ok) ? (int64_t)nsl << 21 : foot;
    const int CH = std::max(64, tune.c4_chunk);
    std::vector<int64_t> gstart, gcount;
    std::vector<int64_t> hoff(n_t3, 0);
    std::vector<uint8_t> hlog(n_t3, 0);
    std::vector<int64_t> grows;  // hash rows of each group (0 for dense groups)
    int64_t G = 0, max_hrows = 0;
    {
      int64_t q = 0;
      while (q < n_t3) {
        const bool hashed = q >= qd;
        const int64_t qend = hashed ? n_t3 : qd;
        int64_t c = 0, bytes = 0, wsum = 0, rows = 0;
        while (q + c < qend && (hashed ? c < (1 << 20) : c < Gmax)) {
          const uint64_t wq = hw[order[q + c]];
          int64_t touched;
          if (hashed) {
            const int lg = hash_log2(wq);
            touched = (1ll << lg) * (1 + RW) * (int64_t)sizeof(uint32_t);
            if (c > 0 && (bytes + touched > foot || wsum >= wtarget)) break;
            hoff[q + c] = rows;
            hlog[q + c] = (uint8_t)lg;
            rows += 1ll << lg;
          } else {
            touched = std::min<int64_t>((int64_t)wq, n) * RW * (int64_t)sizeof(uint32_t);
            if (c > 0 && (bytes + touched > foot_dense || wsum >= wtarget)) break;
          }
          bytes += touched;
          wsum += (int64_t)wq;
          ++c;
        }
        gstart.push_back(q);
        gcount.push_back(c);
        grows.push_back(rows);
        if (hashed) max_hrows = std::max(max_hrows, rows);
        else G = std::max(G, c);
        q += c;
      }
    }
    const int64_t ngroups = (int64_t)gstart.size();
    // heavy nodes in processing order, prefix of their degrees (slots),
    // and prefix of their wedge counts (W(x), summed over the node's slots)
    std::vector<int32_t> gx(n_t3);
    std::vector<int64_t> hs(n_t3 + 1, 0), hwp(n_t3 + 1, 0);
    for (int64_t q = 0; q < n_t3; ++q) {
      gx[q] = hx[order[q]];
      hs[q + 1] = hs[q] + hd[order[q]];
      hwp[q + 1] = hwp[q] + (int64_t)hw[order[q]];
    }
    const int64_t nslots = hs[n_t3];
    int32_t* d_gx;
    int64_t *d_hs, *d_sc, *d_wp, *d_hoff = nullptr;
    uint8_t* d_hlog = nullptr;
    int32_t* hkeys = nullptr;
    uint32_t* dense = nullptr;
    uint32_t* hcnt = nullptr;
    TG_HIP(S.get(&d_gx, n_t3));
    TG_HIP(S.get(&d_hs, n_t3 + 1));
    TG_HIP(S.get(&d_sc, nslots));
    TG_HIP(S.get(&d_wp, nslots + 1));
    TG_HIP(hipMemcpyAsync(d_gx, gx.data(), n_t3 * sizeof(int32_t), hipMemcpyHostToDevice, st));
    TG_HIP(hipMemcpyAsync(d_hs, hs.data(), (n_t3 + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    // Dense groups may take their middle counts from records bucketed by
    // far-end id range and summed in LDS (k_c4_bwalk, k_c4_bcount) instead of
    // from global atomics; every row that the credit walk reads is then
    // written, so the array needs no clearing.
    bool use_parts = false;
    int64_t partR = 0, partK = 0;
    size_t bw_lds = 0, bc_lds = 0;
    const int part_rw = (L + 1) / 2;
    int CHW = std::max(256, std::min(32768, tune.c4_part_chunk));
    std::vector<int64_t> gwalk(ngroups + 1, 0);  // walk items of each group (a prefix)
    std::vector<char> gpart(ngroups, 0);          // dense groups counted by the bucketed pass
    std::vector<int64_t> gnit(ngroups + 1, 0);   // each group's per-node item starts in d_nit
    int32_t* d_nit = nullptr;
    uint32_t* d_region = nullptr;
    int32_t* d_runs = nullptr;
    if (parts_ok && qd > 0) {
      int dev = 0, max_lds = 0;
      TG_HIP(hipGetDevice(&dev));
      TG_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      const size_t cap = std::min<size_t>((size_t)std::max(0, max_lds),
                                          (size_t)std::max(0, tune.c4_part_lds_kib) << 10);
      const size_t fixed = c4_bcount_lds(0, 0, 256);
      // R rows of part_rw words, R a multiple of 4 so that the table is whole uint4s
      partR = cap > fixed ? (int64_t)((cap - fixed) / ((size_t)part_rw * 4)) / 4 * 4 : 0;
      partK = partR > 0 ? (n + partR - 1) / partR : 0;
      // every (node, range) workgroup reads its range's start in each walk
      // item of the node: items of at least 2K wedges keep those reads below
      // the records' own bytes, and graphs with more ranges than that allows
      // keep the grouped count (20M nodes, K = 8461 at 40 KiB: the bucketed
      // pass with 4096-wedge items took 73.3 s against 70.6 s)
      while (CHW < 16384 && CHW < 2 * partK) CHW *= 2;
      bw_lds = c4_bwalk_lds(CHW, (int)std::min<int64_t>(partK, 1 << 20));
      bc_lds = c4_bcount_lds((int)partR, part_rw, 256);
      if (partR >= 64 && 2 * partK <= CHW && bw_lds <= (size_t)max_lds) {
        // per dense group whose counts fit 16 bits (every node's degree below
        // 65536: a count is at most d_x): each node's first walk item
        // (group-local), then the total
        std::vector<int32_t> nit;
        int64_t max_items = 0, total = 0;
        for (int64_t g = 0; g < ngroups; ++g) {
          gwalk[g] = total;
          gnit[g] = (int64_t)nit.size();
          if (gstart[g] >= qd) continue;
          int32_t gmax = 0;
          for (int64_t c = 0; c < gcount[g]; ++c) gmax = std::max(gmax, hd[order[gstart[g] + c]]);
          if (gmax >= 65536) continue;
          gpart[g] = 1;
          int64_t items = 0;
          for (int64_t c = 0; c < gcount[g]; ++c) {
            nit.push_back((int32_t)items);
            items += ((int64_t)hw[order[gstart[g] + c]] + CHW - 1) / CHW;
          }
          nit.push_back((int32_t)items);
          total += items;
          max_items = std::max(max_items, items);
        }
        gwalk[ngroups] = total;
        gnit[ngroups] = (int64_t)nit.size();
        if (max_items > 0 && max_items < (1ll << 31)) {
          TG_HIP(S.get(&d_nit, (int64_t)nit.size()));
          TG_HIP(S.get(&d_region, max_items * CHW));
          TG_HIP(S.get(&d_runs, max_items * (partK + 1)));
          TG_HIP(hipMemcpyAsync(d_nit, nit.data(), nit.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
          // the copy reads the host vector until it is done
          TG_HIP(hipStreamSynchronize(st));
          use_parts = true;
        }
      }
    }
    // dense rows left by a bucketed group are not zero: a grouped count
    // after one clears its rows first
    bool dense_dirty = false;
    if (G > 0) {
      TG_HIP(S.get(&dense, G * stride));
      if (!use_parts) {
        k_fill_u32<<<grid_for(G * stride, 256, 16384), 256, 0, st>>>(dense, G * stride, 0);
        TG_LAUNCHED("k_fill_u32");
      } else {
        dense_dirty = true;
      }
    }
    if (max_hrows > 0) {
      TG_HIP(S.get(&d_hoff, n_t3));
      TG_HIP(S.get(&d_hlog, n_t3));
      TG_HIP(S.get(&hkeys, max_hrows));
      TG_HIP(S.get(&hcnt, max_hrows * RW));
      TG_HIP(hipMemcpyAsync(d_hoff, hoff.data(), n_t3 * sizeof(int64_t), hipMemcpyHostToDevice, st));
      TG_HIP(hipMemcpyAsync(d_hlog, hlog.data(), n_t3 * sizeof(uint8_t), hipMemcpyHostToDevice, st));
      k_fill_u32<<<grid_for(max_hrows, 256, 16384), 256, 0, st>>>(reinterpret_cast<uint32_t*>(hkeys), max_hrows,
                                                                  0xffffffffu);
      k_fill_u32<<<grid_for(max_hrows * RW, 256, 16384), 256, 0, st>>>(hcnt, max_hrows * RW, 0);
      TG_LAUNCHED("k_fill_u32");
    }
    k_c4_slot_wedges<<<grid_for(nslots, 256, 16384), 256, 0, st>>>(nslots, n_t3, d_gx, d_hs, rp, ci, W.deg, d_sc);
    TG_LAUNCHED("k_c4_slot_wedges");
    if (tg_status s2 = scan(S, st, nslots, (const int64_t*)d_sc, d_wp)) return s2;
    // per-slice prefixes over the dense nodes' slots (slots [0, dense_slots))
    int32_t* bnd = nullptr;
    int64_t* d_wps = nullptr;
    const int64_t wstride = dense_slots + 1;
    if (nsl > 1) {
      int64_t* d_scs;
      TG_HIP(S.get(&bnd, n * (nsl + 1)));
      TG_HIP(S.get(&d_scs, dense_slots * nsl));
      TG_HIP(S.get(&d_wps, wstride * nsl));
      k_slice_bounds<<<grid_for(n * (nsl + 1), 256, 16384), 256, 0, st>>>(n, nsl, rp, ci, bnd);
      TG_LAUNCHED("k_slice_bounds");
      k_c4_slot_wedges_sliced<<<grid_for(dense_slots, 256, 16384), 256, 0, st>>>(dense_slots, qd, nsl, d_gx, d_hs,
                                                                                  rp, ci, W.deg, bnd, d_scs);
      TG_LAUNCHED("k_c4_slot_wedges_sliced");
      for (int k = 0; k < nsl; ++k)
        if (tg_status s2 = scan(S, st, dense_slots, (const int64_t*)(d_scs + k * dense_slots), d_wps + k * wstride))
          return s2;
    }
    const size_t xu_lds = (size_t)4 * TG_WAVE * P * sizeof(uint32_t);
    for (int64_t g = 0; g < ngroups; ++g) {
      const int Gg = (int)gcount[g];
      const int64_t q0 = gstart[g];
      const bool hashed = q0 >= qd;
      const int64_t Wn = hwp[q0 + Gg] - hwp[q0];
      if (Wn == 0) continue;
      int64_t ch = CH;
      while ((Wn + ch - 1) / ch > (1ll << 24)) ch *= 2;
      const int gsl_n = hashed ? 1 : nsl;
      // sliced: blocks per slice for a quarter more than an even split of
      // the group's wedges; the kernel strides over any further chunks
      const unsigned grid = gsl_n == 1 ? grid_for((Wn + ch - 1) / ch, 4)
                                       : (unsigned)(gsl_n * ((Wn * 5 / 4 / gsl_n + 4 * ch - 1) / (4 * ch) + 1));
      // the group's nodes, slot prefix (global base), wedge prefix and
      // (hashed groups) table offsets and sizes
      const int32_t* gxg = d_gx + q0;
      const int64_t* gsl = d_hs + q0;
      const int64_t* wpg = gsl_n == 1 ? d_wp + hs[q0] : d_wps + hs[q0];
      const int64_t* hog = hashed ? d_hoff + q0 : nullptr;
      const uint8_t* hlg = hashed ? d_hlog + q0 : nullptr;
      uint32_t* cnt_base = hashed ? hcnt : dense;
      const int64_t rows = grows[g];
      // dense groups are cleared by a fill when that is cheaper than a second
      // walk over their wedges (a streamed byte costs about 1/128 of a walked
      // wedge: 64, 128, 256 and 512 were measured); hashed groups always by a
      // fill of their rows
      const bool fill_clear = hashed || Gg * stride * (int64_t)sizeof(uint32_t) < Wn * 128;
      // bucketed groups keep 16-bit counts (4-word rows) whatever the
      // maximum degree
      const bool gp = !hashed && use_parts && gpart[g];
      const bool ghalf = half || gp;
      const int RWg = ghalf ? CS / 2 : CS;
      if (!hashed && !gp && dense_dirty) {
        k_fill_u32<<<grid_for(Gg * stride, 256, 16384), 256, 0, st>>>(dense, Gg * stride, 0);
        TG_LAUNCHED("k_fill_u32");
      }
      if (!hashed) dense_dirty = gp;
      const int stage_xu = (L <= 8 && ch * max_deg < (1ll << 32)) ? 1 : 0;
      // phase 3 (once): at most a few resident waves of workgroups, so that
      // few LDS key copies are flushed
      const unsigned grid3 = std::min<unsigned>(grid, 4096u);
#define TG_C4_GROUP(PH, T, HF, HS, C4P, STG)                                                                       \
  k_c4_group<PH, T, HF, HS><<<PH == 3 ? grid3 : grid, 256,                                                         \
                              PH == 3 ? gacc_bytes(ga_cyc_g) : ((PH == 1 && STG) ? xu_lds : 0), st>>>(             \
      Gg, gxg, gsl, wpg, wstride, gsl_n, bnd, (int)ch, cnt_base, stride, RWg, hog, hlg, hkeys, rp, ci, W.deg, tyb,  \
      L, s2x, C4P, crows, STG, ga_cyc_g, cdt, c4x)
#define TG_C4_PHASES(T, HF, HS, C4P, STG)                                                                          \
  do {                                                                                                             \
    if (!HS && gp) {                                                                                               \
      if (gwalk[g + 1] > gwalk[g]) {                                                                               \
        k_c4_bwalk<TG_C4P_NW><<<(unsigned)(gwalk[g + 1] - gwalk[g]), TG_C4P_NW * TG_WAVE, bw_lds, st>>>(           \
            d_nit + gnit[g], Gg, CHW, (int)partR, (int)partK, gxg, gsl, d_wp + hs[q0], rp, ci, cdt, d_region,     \
            d_runs);                                                                                               \
        k_c4_bcount<256><<<(unsigned)(Gg * partK), 256, bc_lds, st>>>((int)partK, (int)partR, part_rw, n,          \
                                                                      d_nit + gnit[g], d_region, CHW, d_runs,      \
                                                                      dense, stride);                              \
      }                                                                                                            \
    } else {                                                                                                       \
      TG_C4_GROUP(0, T, HF, HS, C4P, STG);                                                                         \
    }                                                                                                              \
    if (once && (HS || fill_clear)) {                                                                              \
      const int64_t nrows = HS ? rows : Gg * n;                                                                    \
      k_c4_scan<HF, HS><<<grid_for(nrows, 256, 2048), 256, gacc_bytes(ga_cyc_g), st>>>(                            \
          nrows, cnt_base, RWg, n, Gg, gxg, hog, hkeys, tyb, L, ga_cyc_g);                                         \
      break;                                                                                                       \
    }                                                                                                              \
    if (once) TG_C4_GROUP(3, T, HF, HS, C4P, STG);                                                                 \
    else TG_C4_GROUP(1, T, HF, HS, C4P, STG);                                                                      \
    if (HS) {                                                                                                      \
      k_fill_u32<<<grid_for(rows, 256, 16384), 256, 0, st>>>(reinterpret_cast<uint32_t*>(hkeys), rows,             \
                                                             0xffffffffu);                                         \
      k_fill_u32<<<grid_for(rows * RW, 256, 16384), 256, 0, st>>>(hcnt, rows * RW, 0);                             \
    } else if (gp) {                                                                                               \
      /* the next dense group's counts overwrite every row it reads */                                                      \
    } else if (fill_clear) {                                                                                       \
      k_fill_u32<<<grid_for(Gg * stride, 256, 16384), 256, 0, st>>>(dense, Gg * stride, 0);                        \
    } else {                                                                                                       \
      TG_C4_GROUP(2, T, HF, HS, C4P, STG);                                                                         \
    }                                                                                                              \
  } while (0)
#define TG_C4_ALL(HS)                                                  \
  do {                                                                 \
    if (c4s_wide) {                                                    \
      if (ghalf) TG_C4_PHASES(uint64_t, true, HS, C4w_t, stage_xu);    \
      else TG_C4_PHASES(uint64_t, false, HS, C4w_t, stage_xu);         \
    } else {                                                           \
      if (ghalf) TG_C4_PHASES(uint32_t, true, HS, C4n_t, stage_xu);    \
      else TG_C4_PHASES(uint32_t, false, HS, C4n_t, stage_xu);         \
    }                                                                  \
  } while (0)
      // every type vector in turn reuses the group's count rows
      for (int64_t b = 0; b < nty; ++b) {
        const uint8_t* tyb = ty + b * n;
        const GAcc ga_cyc_g = once ? gacc_cyc(b, 16 << 10) : GAcc{};
        if (hashed) TG_C4_ALL(true);
        else TG_C4_ALL(false);
      }
#undef TG_C4_ALL
#undef TG_C4_PHASES
#undef TG_C4_GROUP
      TG_LAUNCHED("k_c4_group");
    }
  }

  if (slot_rows) {
    if (c4_wide)
      k_c4_fold<uint64_t><<<grid_for(m * P, 256, 16384), 256, 0, st>>>(m, (int)P, nnz, W.es_lo, W.es_hi, C4w_t,
                                                                       W.C4);
    else
      k_c4_fold<uint32_t><<<grid_for(m * P, 256, 16384), 256, 0, st>>>(m, (int)P, nnz, W.es_lo, W.es_hi, C4n_t, C4n);
    TG_LAUNCHED("k_c4_fold");
  } else if (split) {
    k_c4_fold_add<<<grid_for(m * P, 256, 16384), 256, 0, st>>>(m, (int)P, nnz, W.es_lo, W.es_hi, C4n_t, W.C4);
    TG_LAUNCHED("k_c4_fold_add");
  }
  S.release(c4_mark);

  int dev = 0, cus = 0;
  TG_HIP(hipGetDevice(&dev));
  TG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

  // ---- typed 4-cliques of every edge, each clique once from its lowest node
  timer.mark(TG_PHASE_CLIQUES);
  uint32_t* K4n = nullptr;
  uint64_t* K4w = nullptr;
  bool k4_glob_done = false;
  if (once && tune.clique_pass != 0) {
    // global counts: every clique adds one to its key, per type vector
    K4Plan plan;
    if (tg_status s2 = k4_plan(S, st, n, W.out_off, plan)) return s2;
    for (int64_t b = 0; plan.ok && b < nty; ++b) {
      const K4Args K{W.deg, ty + b * n, L, W.out_off, W.out_col, nullptr, m, nullptr, nullptr};
      const GAcc ga_k4 = make_gacc(global_counts + b * nkeys(L), 2 * C3k + 5 * C4k, C4k, 16 << 10);
      if (tg_status s2 = k4_launch<true>(S, st, K, plan, cus, tune.clique_pass_grid, tune.clique_pass_lds_kib,
                                         ga_k4))
        return s2;
    }
    k4_glob_done = plan.ok;
  }
  if (W.out_eid) {
    K4Plan plan;
    if (tg_status s2 = k4_plan(S, st, n, W.out_off, plan)) return s2;
    if (plan.ok) {
      // a count on edge e is at most C(|T_e|, 2)
      uint32_t* d_mt;
      TG_HIP(S.get(&d_mt, 1));
      k_fill_u32<<<1, 64, 0, st>>>(d_mt, 1, 0u);
      k_max_tsum_all<<<grid_for(m, 256, 4096), 256, 0, st>>>(m, W.tau, L, d_mt);
      TG_LAUNCHED("k_max_tsum_all");
      uint32_t mt = 0;
      TG_HIP(hipMemcpyAsync(&mt, d_mt, sizeof(mt), hipMemcpyDeviceToHost, st));
      TG_HIP(hipStreamSynchronize(st));
      const bool k4_wide = (uint64_t)mt * (mt > 0 ? mt - 1 : 0) / 2 >= (1ull << 32);
      K4Args K{W.deg, ty, L, W.out_off, W.out_col, W.out_eid, m, nullptr, nullptr};
      if (k4_wide) {
        TG_HIP(S.get(&K4w, m * P));
        k_fill_u64<<<grid_for(m * P, 256, 16384), 256, 0, st>>>(K4w, m * P, 0);
        K.K4w = K4w;
      } else {
        TG_HIP(S.get(&K4n, m * P));
        k_fill_u32<<<grid_for(m * P, 256, 16384), 256, 0, st>>>(K4n, m * P, 0u);
        K.K4n = K4n;
      }
      TG_LAUNCHED("k_fill");
      if (tg_status s2 = k4_launch<false>(S, st, K, plan, cus, tune.clique_pass_grid, tune.clique_pass_lds_kib,
                                          GAcc{}))
        return s2;
    }
  }

  if (once) {
    // ---- the other shapes, each instance a fixed number of times
    timer.mark(TG_PHASE_COMBINE);
    // 4-cliques: edges in three classes by intersection length (|T_ij| does
    // not depend on the types, so neither do the classes)
    // (none when the clique pass has added every 4-clique already)
    int32_t* kc = cnt + 280;
    int32_t hk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int32_t kcur[4] = {0, 0, 0, 0};
    const int team_max = std::min(64, std::max(0, tune.clique_team_max));
    const int tcap = std::min(K4Cap<256>::value, std::max(0, tune.clique_lds_ids));
    if (!k4_glob_done) {
      TG_HIP(hipMemsetAsync(kc, 0, 8 * sizeof(int32_t), st));
      const int2 lim = make_int2(team_max, std::min(1024, std::max(team_max, tune.clique_wave_max)));
      k_k4_class_count<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, W.ei, W.ej, W.deg, W.out_off, W.tau, L, lim, kc);
      TG_LAUNCHED("k_k4_class_count");
      TG_HIP(hipMemcpyAsync(hk, kc, sizeof(hk), hipMemcpyDeviceToHost, st));
      TG_HIP(hipStreamSynchronize(st));
      kcur[1] = hk[0];
      kcur[2] = hk[0] + hk[1];
      TG_HIP(hipMemcpyAsync(kc + 4, kcur, 3 * sizeof(int32_t), hipMemcpyHostToDevice, st));
      k_k4_class_scatter<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, W.ei, W.ej, W.deg, W.out_off, W.tau, L, lim,
                                                                 kc + 4, W.elist);
      TG_LAUNCHED("k_k4_class_scatter");
    }
    // lane-spread copies of each edge's L x L clique cells: about 2 KiB per team
    const int mcop = (int)std::max<int64_t>(1, std::min<int64_t>(8, 512 / (LL)));
    const unsigned grid_wg = grid_for(hk[2], 1, 2048);
    int32_t* t_over = nullptr;
    int64_t t_cap = 0;
    if (hk[2] > 0 && hk[3] > tcap) {
      t_cap = hk[3];
      TG_HIP(S.get(&t_over, ((int64_t)grid_wg * t_cap * 5 + 3) / 4));
    }
    int32_t* flag = cnt + 272;
    TG_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
    for (int64_t b = 0; b < nty; ++b) {
      const uint8_t* tyb = ty + b * n;
      uint64_t* gb = global_counts + b * K;
      if (b > 0) {
        // typed degrees and typed common-neighbour counts of this type vector
        k_node_stats<<<grid_for(n, 4), 256, 0, st>>>(n, rp, ci, W.deg, tyb, L, W.D, W.n_upper, W.n_out,
                                                     W.wedge_work, W.nbr_deg_sum);
        TG_LAUNCHED("k_node_stats");
        k_tau<16><<<grid_for(m, 16, 8192), 256, 0, st>>>(m, -1, 48, W.ei, W.ej, rp, ci, W.deg, tyb, L, W.tau,
                                                         nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                                                         INT32_MAX);
        k_tau<64><<<grid_for(m, 4, 8192), 256, 0, st>>>(m, 48, INT32_MAX, W.ei, W.ej, rp, ci, W.deg, tyb, L, W.tau,
                                                        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                                                        INT32_MAX);
        TG_LAUNCHED("k_tau");
      }
      const GAcc ga_all = make_gacc(gb, 0, K, 32 << 10);
      k_glob_nodes<<<grid_for(n, 16, 2048), 256, gacc_bytes(ga_all), st>>>(n, W.deg, W.D, tyb, L, ga_all);
      TG_LAUNCHED("k_glob_nodes");
      k_glob_edges<<<grid_for(m, 16, 2048), 256, gacc_bytes(ga_all), st>>>(m, W.ei, W.ej, W.D, W.tau, tyb, L,
                                                                            ga_all);
      TG_LAUNCHED("k_glob_edges");
      const GAcc ga_k4 = make_gacc(gb, 2 * C3k + 5 * C4k, C4k, 16 << 10);
      if (hk[0] > 0) {
        k_glob_k4<16><<<grid_for(hk[0], 16, 4096), 256, k4_lds_bytes<16>(ga_k4, L, mcop), st>>>(
            hk[0], W.elist, W.ei, W.ej, W.deg, tyb, W.out_off, W.out_col, W.tau, L, mcop, 0, nullptr, 0, 0, ga_k4);
        TG_LAUNCHED("k_glob_k4<16>");
      }
      if (hk[1] > 0) {
        k_glob_k4<64><<<grid_for(hk[1], 4, 4096), 256, k4_lds_bytes<64>(ga_k4, L, mcop), st>>>(
            hk[1], W.elist + kcur[1], W.ei, W.ej, W.deg, tyb, W.out_off, W.out_col, W.tau, L, mcop, 0, nullptr, 0,
            0, ga_k4);
        TG_LAUNCHED("k_glob_k4<64>");
      }
      if (hk[2] > 0) {
        k_glob_k4<256><<<grid_wg, 256, k4_lds_bytes<256>(ga_k4, L, mcop), st>>>(
            hk[2], W.elist + kcur[2], W.ei, W.ej, W.deg, tyb, W.out_off, W.out_col, W.tau, L, mcop, tcap, t_over,
            t_cap, n < (1ll << 27) ? 1 : 0, ga_k4);
        TG_LAUNCHED("k_glob_k4<256>");
      }
      k_glob_finalize<<<grid_for(std::max(C3k, C4k), 256), 256, 0, st>>>(gb, L, flag);
      TG_LAUNCHED("k_glob_finalize");
    }
    timer.mark(TG_PHASE_FINALIZE);
    timer.mark(TG_NUM_PHASES);
    if (opt.check) {
      int32_t hf = 0;
      TG_HIP(hipMemcpyAsync(&hf, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      TG_HIP(hipStreamSynchronize(st));
      if (hf) return fail(TG_ERR_INTERNAL, "a non-induced key sum is inconsistent (odd, not a multiple of 3, or "
                                           "larger than its pattern total)");
    }
    timer.finish();
    return TG_OK;
  }

  // ---- per-edge combine
  timer.mark(TG_PHASE_COMBINE);
  EdgeArgs A;
  A.rp = rp; A.ci = ci; A.ty = ty; A.deg = W.deg; A.D = W.D; A.ei = W.ei; A.ej = W.ej; A.s2e = W.s2e;
  A.out_off = W.out_off; A.out_col = W.out_col; A.tau = W.tau; A.Pn = W.Pn; A.Un = W.Un; A.C4 = W.C4; A.L = L;
  A.tau_s = W.tau_s; A.tl_off = W.tl_off; A.tl_k = W.tl_k; A.tl_e = W.tl_e; A.tl_packed = W.tl_packed;
  A.hub_of = W.hub_of; A.hub_bits = W.hub_bits; A.hub_rank = W.hub_rank; A.hub_nw = W.hub_nw;
  A.C4n = C4n;
  A.c4_wide = c4_wide ? 1 : 0;
  A.c4_rows = srows ? 0 : m;
  A.edge_counts = edge_counts; A.edge_begin = eb; A.edge_end = ee; A.global_sums = global_counts;
  A.edge_ids = ids; A.n_edge_ids = nids;
  A.edge_orbits = opt.edge_orbits;
  A.gacc_in_lds = (global_counts && K <= TG_GACC_MAX_KEYS) ? 1 : 0;
  A.work = nullptr;
  A.thash_ok = n < (1ll << 27) ? 1 : 0;
  A.K4n = K4n;
  A.K4w = K4w;
  A.m = m;
  A.sp_keys = nullptr;
  A.sp_counts = nullptr;
  A.sp_start = nullptr;
  A.sp_len = nullptr;
  A.sp_cursor = nullptr;
  A.sp_cap = 0;
  if (sparse) {
    TG_HIP(S.get(&A.sp_cursor, 1));
    k_fill_u64<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t*>(A.sp_cursor), 1, 0);
    TG_LAUNCHED("k_fill_u64");
    // the keys pointer also switches the row kernel to sparse output; with
    // no capacity it points at a dummy word that is never written
    A.sp_keys = sparse->keys ? sparse->keys : reinterpret_cast<uint32_t*>(A.sp_cursor);
    A.sp_counts = sparse->counts;
    A.sp_start = sparse->start;
    A.sp_len = sparse->len;
    A.sp_cap = sparse->cap;
  }
  const bool probe = !K4n && !K4w;
  // gathered accumulators of one batch of edges (reused by every class and
  // batch: all launches are ordered on st)
  const int64_t ea_budget = 4ll << 30;
  void* ea = nullptr;
  {
    int64_t need = 0;
    for (int c = 0; c < 3; ++c)
      need = std::max<int64_t>(need, class_count[c] * 4 * LL * (c == 2 ? 8 : 4));
    need = std::min(need, ea_budget);
    if (need > 0) TG_HIP(S.get(reinterpret_cast<uint64_t**>(&ea), (need + 7) / 8));
  }
  {
    tg_status s2 = probe ? combine_classes<true>(S, st, A, W, class_begin, class_count, K, ea, ea_budget, tune, cus,
                                                 max_t_heavy)
                         : combine_classes<false>(S, st, A, W, class_begin, class_count, K, ea, ea_budget, tune, cus,
                                                  max_t_heavy);
    if (s2 != TG_OK) return s2;
  }

  // ---- Eq. 17 and outputs
  timer.mark(TG_PHASE_FINALIZE);
  int32_t* flag = cnt + 272;
  TG_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  if (global_counts) {
    k_finalize<<<grid_for(K, 256, 64), 256, 0, st>>>(global_counts, L, flag);
    TG_LAUNCHED("k_finalize");
  }
  if (edge_endpoints && ids) {
    k_copy_endpoints_ids<<<grid_for(nids, 256, 8192), 256, 0, st>>>(ids, nids, W.ei, W.ej, edge_endpoints);
    TG_LAUNCHED("k_copy_endpoints_ids");
  } else if (edge_endpoints && ee > eb) {
    k_copy_endpoints<<<grid_for(ee - eb, 256, 8192), 256, 0, st>>>(eb, ee, W.ei, W.ej, edge_endpoints);
    TG_LAUNCHED("k_copy_endpoints");
  }
  timer.mark(TG_NUM_PHASES);
  if (opt.check) {
    int32_t hf = 0;
    TG_HIP(hipMemcpyAsync(&hf, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (hf) return fail(TG_ERR_INTERNAL, "a global sum is not a multiple of its shape's edge count");
  }
  timer.finish();
  if (sparse) {
    uint64_t tot = 0;
    TG_HIP(hipMemcpyAsync(&tot, A.sp_cursor, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    *sparse->total = (int64_t)tot;
    if ((int64_t)tot > sparse->cap)
      return fail(TG_ERR_INVALID_ARG, "sparse capacity " + std::to_string(sparse->cap) + " is below the " +
                                          std::to_string(tot) + " nonzero pairs (reported in *total)");
  }
  return TG_OK;
}


// ------------------------------------------------------------------ batch --

struct BatchLaunch {
  int variant;
  int64_t offset, count;
};

// Cached HIP graph of the per-bucket launches: replayed while the call's
// pointers and bucket plan repeat.
struct BatchGraphCache {
  bool valid = false;
  int device = -1;
  std::vector<uint64_t> sig;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    valid = false;
  }
};

BatchGraphCache& batch_cache() {
  static thread_local BatchGraphCache c;
  return c;
}

tg_status enqueue_batch_variant(int variant, const BatchArgs& A, int64_t count, const int32_t* list, int32_t* queue,
                                hipStream_t st) {
  const unsigned grid4 = grid_for(count, 4, 4096), grid1 = grid_for(count, 1, 2048);
  switch (variant) {
    case 0: k_batch<1, 1, false><<<grid4, 256, 0, st>>>(A, count, list, queue); break;
    case 1: k_batch<2, 1, false><<<grid4, 256, 0, st>>>(A, count, list, queue); break;
    case 2: k_batch<2, 4, true><<<grid1, 256, 0, st>>>(A, count, list, queue); break;
    case 3: k_batch<4, 1, false><<<grid4, 256, 0, st>>>(A, count, list, queue); break;
    case 4: k_batch<4, 4, true><<<grid1, 256, 0, st>>>(A, count, list, queue); break;
    case 5: k_batch<8, 4, true><<<grid1, 256, 0, st>>>(A, count, list, queue); break;
    default: return fail(TG_ERR_INVALID_ARG, "unknown batch kernel variant");
  }
  TG_LAUNCHED("k_batch");
  return TG_OK;
}

// largest size class W (words per bit row) a variant handles
int variant_wmax(int v) {
  static const int w[6] = {1, 2, 2, 4, 4, 8};
  return (v >= 0 && v < 6) ? w[v] : 0;
}

tg_status batch_check(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* rp,
                      const int32_t* ci, const uint8_t* ty, const uint8_t* Lg, const int64_t* key_off, uint64_t* out,
                      const tg_tuning& tune) {
  if (G < 0 || G >= (1ll << 31)) return fail(TG_ERR_INVALID_ARG, "G must be in [0, 2^31)");
  if (G == 0) return TG_OK;
  if (!node_off || !slot_off || !rp || !ci || !ty || !Lg || !key_off || !out)
    return fail(TG_ERR_INVALID_ARG, "null input or output pointer");
  for (int w = 0; w <= 8; ++w)
    if (variant_wmax(tune.batch_variant[w]) < std::max(1, w))
      return fail(TG_ERR_INVALID_ARG, "tuning assigns a size class to a kernel variant that is too small");
  return TG_OK;
}

// The batch pipeline on caller-provided scratch: ctr[128] ([0,72) sub-bucket
// counts, [80] bad flag, [96,112) queues, [120] divisibility flag) and
// list[G].  use_graph: replay the per-bucket launches from a cached HIP graph
// (else launch them directly).
tg_status batch_run(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* rp,
                    const int32_t* ci, const uint8_t* ty, const uint8_t* Lg, const int64_t* key_off, uint64_t* out,
                    const tg_options& opt, const tg_tuning& tune, int32_t* ctr, int32_t* list, bool use_graph,
                    hipStream_t st) {
  k_zero_i32<<<1, 128, 0, st>>>(ctr, 128);
  TG_LAUNCHED("k_zero_i32");
  k_batch_classify<<<grid_for(G, 256, 4096), 256, 0, st>>>(G, node_off, Lg, key_off, ctr + 80);
  TG_LAUNCHED("k_batch_classify");
  k_batch_subcount<<<grid_for(G, 256, 4096), 256, 0, st>>>(G, node_off, ctr);
  TG_LAUNCHED("k_batch_subcount");
  int32_t h[128];
  TG_HIP(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  if (h[80] & 1) return fail(TG_ERR_INVALID_ARG, "a graph has more than 512 nodes or a negative size");
  if (h[80] & 2) return fail(TG_ERR_UNSUPPORTED_L, "a graph's L is outside [1, 8]");
  if (h[80] & 4) return fail(TG_ERR_INVALID_ARG, "key_off does not match tg_num_keys(L_g)");
  if (opt.validate) {
    k_batch_validate<<<grid_for(G, 4, 4096), 256, 0, st>>>(G, node_off, slot_off, rp, ci, ty, Lg, ctr + 80);
    TG_LAUNCHED("k_batch_validate");
    TG_HIP(hipMemcpyAsync(&h[80], ctr + 80, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (h[80] & 16)
      return fail(TG_ERR_INVALID_GRAPH, "a graph's CSR is invalid (row pointers, column range, self loop, unsorted "
                                        "or duplicate row, or an edge stored in one direction only)");
    if (h[80] & 8) return fail(TG_ERR_TYPE_RANGE, "a node type is >= its graph's L");
  }
  // list order: size class W from 8 down to 0, largest first inside a class
  int32_t cur[128];
  memset(cur, 0, sizeof(cur));
  int64_t acc = 0;
  int64_t cls_begin[9], cls_count[9];
  for (int w = 8; w >= 0; --w) {
    cls_begin[w] = acc;
    for (int sb = 0; sb < 8; ++sb) { cur[w * 8 + sb] = (int32_t)acc; acc += h[w * 8 + sb]; }
    cls_count[w] = acc - cls_begin[w];
  }
  TG_HIP(hipMemcpyAsync(ctr, cur, 72 * sizeof(int32_t), hipMemcpyHostToDevice, st));
  k_batch_scatter<<<grid_for(G, 256, 4096), 256, 0, st>>>(G, node_off, ctr, list);
  TG_LAUNCHED("k_batch_scatter");
  // launches: consecutive classes with the same variant share one queue
  std::vector<BatchLaunch> plan;
  for (int w = 8; w >= 0; --w) {
    if (cls_count[w] == 0) continue;
    const int v = tune.batch_variant[w];
    if (!plan.empty() && plan.back().variant == v && plan.back().offset + plan.back().count == cls_begin[w])
      plan.back().count += cls_count[w];
    else
      plan.push_back({v, cls_begin[w], cls_count[w]});
  }
  if (plan.size() > 16) return fail(TG_ERR_INTERNAL, "too many batch launches");
  BatchArgs A{node_off, slot_off, rp, ci, ty, Lg, key_off, out, ctr + 120};
  if (!use_graph) {
    k_zero_i32<<<1, 64, 0, st>>>(ctr + 96, 32);
    TG_LAUNCHED("k_zero_i32");
    for (size_t q = 0; q < plan.size(); ++q)
      if (tg_status s2 = enqueue_batch_variant(plan[q].variant, A, plan[q].count, list + plan[q].offset,
                                               ctr + 96 + (int)q, st))
        return s2;
  } else {
  // HIP graph: zero the queues and flag, then one persistent launch per bucket
  int dev = 0;
  TG_HIP(hipGetDevice(&dev));
  std::vector<uint64_t> sig = {(uint64_t)dev, (uint64_t)G, (uint64_t)node_off, (uint64_t)slot_off, (uint64_t)rp,
                               (uint64_t)ci, (uint64_t)ty, (uint64_t)Lg, (uint64_t)key_off, (uint64_t)out,
                               (uint64_t)ctr, (uint64_t)list};
  for (auto& l : plan) {
    sig.push_back((uint64_t)l.variant);
    sig.push_back((uint64_t)l.offset);
    sig.push_back((uint64_t)l.count);
  }
  BatchGraphCache& C = batch_cache();
  if (!C.valid || C.sig != sig) {
    C.reset();
    if (!C.cap_stream || C.device != dev) {
      C.device = dev;
      TG_HIP(hipStreamCreateWithFlags(&C.cap_stream, hipStreamNonBlocking));
    }
    TG_HIP(hipStreamBeginCapture(C.cap_stream, hipStreamCaptureModeThreadLocal));
    k_zero_i32<<<1, 64, 0, C.cap_stream>>>(ctr + 96, 32);
    tg_status s2 = TG_OK;
    for (size_t q = 0; q < plan.size() && s2 == TG_OK; ++q)
      s2 = enqueue_batch_variant(plan[q].variant, A, plan[q].count, list + plan[q].offset, ctr + 96 + (int)q,
                                 C.cap_stream);
    hipGraph_t gph = nullptr;
    hipError_t e2 = hipStreamEndCapture(C.cap_stream, &gph);
    if (s2 != TG_OK) { if (gph) (void)hipGraphDestroy(gph); return s2; }
    if (e2 != hipSuccess) return fail(TG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    C.graph = gph;
    TG_HIP(hipGraphInstantiate(&C.exec, C.graph, nullptr, nullptr, 0));
    C.sig = sig;
    C.valid = true;
  }
  TG_HIP(hipGraphLaunch(C.exec, st));
  }
  if (opt.check) {
    int32_t hf = 0;
    TG_HIP(hipMemcpyAsync(&hf, ctr + 120, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (hf) return fail(TG_ERR_INTERNAL, "a global sum is not a multiple of its shape's edge count");
  }
  return TG_OK;
}

tg_status batch_impl(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* rp,
                     const int32_t* ci, const uint8_t* ty, const uint8_t* Lg, const int64_t* key_off, uint64_t* out,
                     const tg_options* opt_in, hipStream_t st) {
  tg_options opt;
  tg_options_default(&opt);
  if (opt_in) opt = *opt_in;
  tg_tuning tune;
  tg_tuning_default(&tune);
  if (opt.tuning) tune = *opt.tuning;
  if (tg_status s = batch_check(G, node_off, slot_off, rp, ci, ty, Lg, key_off, out, tune)) return s;
  if (G == 0) return TG_OK;
  keep_pool_cached();
  Scratch S(st);  // its buffers are released stream-ordered after the launches
  int32_t* ctr;
  int32_t* list;
  TG_HIP(S.get(&ctr, 128));
  TG_HIP(S.get(&list, G));
  return batch_run(G, node_off, slot_off, rp, ci, ty, Lg, key_off, out, opt, tune, ctr, list, true, st);
}

// ------------------------------------------------- batch, no allocation --
//
// Scratch of tg_count_batch_noalloc: a fixed device array (its 128 counters
// and a list of up to TG_NOALLOC_MAX_GRAPHS graph ids), one copy per device,
// held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
#define TG_NOALLOC_MAX_GRAPHS (1 << 21)
static __device__ __align__(256) int32_t noalloc_scratch[128 + TG_NOALLOC_MAX_GRAPHS];

std::mutex g_noalloc_mu;
int32_t* g_noalloc_ptr[64] = {};

// Device address of the current device's copy of noalloc_scratch, looked up
// on the first call on that device.
tg_status noalloc_scratch_ptr(int32_t** out) {
  int dev = 0;
  TG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(TG_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p)
      return fail(TG_ERR_HIP, std::string("hipGetSymbolAddress(noalloc_scratch): ") + hipGetErrorString(e));
    g_noalloc_ptr[dev] = reinterpret_cast<int32_t*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return TG_OK;
}

tg_status batch_noalloc_impl(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* rp,
                             const int32_t* ci, const uint8_t* ty, const uint8_t* Lg, const int64_t* key_off,
                             uint64_t* out, const tg_options* opt_in, hipStream_t st) {
  tg_options opt;
  tg_options_default(&opt);
  if (opt_in) opt = *opt_in;
  tg_tuning tune;
  tg_tuning_default(&tune);
  if (opt.tuning) tune = *opt.tuning;
  if (G > TG_NOALLOC_MAX_GRAPHS)
    return fail(TG_ERR_INVALID_ARG, "tg_count_batch_noalloc takes at most " +
                                        std::to_string(TG_NOALLOC_MAX_GRAPHS) + " graphs");
  if (tg_status s = batch_check(G, node_off, slot_off, rp, ci, ty, Lg, key_off, out, tune)) return s;
  if (G == 0) return TG_OK;
  int32_t* scr = nullptr;
  if (tg_status s = noalloc_scratch_ptr(&scr)) return s;
  return batch_run(G, node_off, slot_off, rp, ci, ty, Lg, key_off, out, opt, tune, scr, scr + 128, false, st);
}

tg_status tg_internal_predict_costs(const tg_cost_model* model, int64_t n, const int32_t* rp, const int32_t* ci,
                                    const uint8_t* ty, int L, const tg::Work& W, int64_t m, float* out,
                                    hipStream_t st);

}  // namespace

// ------------------------------------------------------------- cost model --

struct tg_cost_model {
  int device = -1;
  float* W = nullptr;       // fp32 master parameters
  float* M = nullptr;       // Adam first moment
  float* V = nullptr;       // Adam second moment
  uint16_t* Wbf = nullptr;  // bf16 copy used by the kernels
  float* stats = nullptr;   // feature mean[16], deviation[16]
  int64_t steps = 0;        // Adam steps taken
};

namespace {

void model_init_host(std::vector<float>& w, std::vector<float>& stats, uint64_t seed) {
  // seeded uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases
  w.assign(TG_MLP_NPARAM, 0.0f);
  uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  for (int p = 0; p < TG_MLP_OFF_B1; ++p) w[p] = (float)((2 * next() - 1) / std::sqrt((double)TG_MLP_IN));
  for (int p = TG_MLP_OFF_W2; p < TG_MLP_OFF_B2; ++p) w[p] = (float)((2 * next() - 1) / std::sqrt((double)TG_MLP_H));
  for (int p = TG_MLP_OFF_W3; p < TG_MLP_OFF_B3; ++p) w[p] = (float)((2 * next() - 1) / std::sqrt((double)TG_MLP_H));
  stats.assign(2 * TG_MLP_IN, 0.0f);
  for (int c = 0; c < TG_MLP_IN; ++c) stats[TG_MLP_IN + c] = 1.0f;
}

tg_status model_upload(tg_cost_model* md, const float* w, const float* stats, hipStream_t st) {
  TG_HIP(hipMemcpyAsync(md->W, w, TG_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
  TG_HIP(hipMemcpyAsync(md->stats, stats, 2 * TG_MLP_IN * sizeof(float), hipMemcpyHostToDevice, st));
  TG_HIP(hipMemsetAsync(md->M, 0, TG_MLP_NPARAM * sizeof(float), st));
  TG_HIP(hipMemsetAsync(md->V, 0, TG_MLP_NPARAM * sizeof(float), st));
  k_mlp_to_bf16<<<grid_for(TG_MLP_NPARAM, 256, 64), 256, 0, st>>>(md->W, md->Wbf);
  TG_LAUNCHED("k_mlp_to_bf16");
  TG_HIP(hipStreamSynchronize(st));
  md->steps = 0;
  return TG_OK;
}

tg_status check_model_device(const tg_cost_model* md) {
  int dev = 0;
  TG_HIP(hipGetDevice(&dev));
  if (dev != md->device) return fail(TG_ERR_INVALID_ARG, "cost model lives on another device");
  return TG_OK;
}

tg_status check_graph_args(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const uint8_t* ty, int L) {
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (n < 0 || nnz < 0 || n >= (1ll << 31) || nnz >= (1ll << 31) || n * (int64_t)L >= (1ll << 31))
    return fail(TG_ERR_INVALID_ARG, "graph size out of range");
  if (!rp || (nnz > 0 && !ci) || (n > 0 && !ty)) return fail(TG_ERR_INVALID_ARG, "null graph pointer");
  if (nnz % 2) return fail(TG_ERR_INVALID_GRAPH, "nnz is odd");
  return TG_OK;
}

// Instrumented element-visit counts of the per-edge counting kernel for the
// listed edges (work indexed by edge id).
tg_status measure_work(Scratch& S, hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                       const uint8_t* ty, int L, const Work& W, const int32_t* list, int64_t count,
                       uint64_t* work_by_edge) {
  const int64_t m = nnz / 2, P = (int64_t)L * (L + 1) / 2, LL = (int64_t)L * L, K = nkeys(L);
  uint64_t* gsink;
  uint32_t* tmax;
  TG_HIP(S.get(&gsink, K));
  TG_HIP(S.get(&tmax, 1));
  k_fill_u64<<<grid_for(m, 256, 8192), 256, 0, st>>>(work_by_edge, m, 0);
  TG_LAUNCHED("k_fill_u64");
  k_fill_u64<<<1, 64, 0, st>>>(gsink, K, 0);
  TG_LAUNCHED("k_fill_u64");
  k_fill_u32<<<1, 64, 0, st>>>(tmax, 1, 0);
  TG_LAUNCHED("k_fill_u32");
  k_max_tsum<<<grid_for(count, 256, 4096), 256, 0, st>>>(count, list, W.tau, L, tmax);
  TG_LAUNCHED("k_max_tsum");
  uint32_t h_tmax = 0;
  TG_HIP(hipMemcpyAsync(&h_tmax, tmax, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  EdgeArgs A;
  A.rp = rp; A.ci = ci; A.ty = ty; A.deg = W.deg; A.D = W.D; A.ei = W.ei; A.ej = W.ej; A.s2e = W.s2e;
  A.out_off = W.out_off; A.out_col = W.out_col; A.tau = W.tau; A.Pn = W.Pn; A.Un = W.Un; A.C4 = W.C4; A.L = L;
  A.tau_s = W.tau_s; A.tl_off = W.tl_off; A.tl_k = W.tl_k; A.tl_e = W.tl_e; A.tl_packed = W.tl_packed;
  A.hub_of = W.hub_of; A.hub_bits = W.hub_bits; A.hub_rank = W.hub_rank; A.hub_nw = W.hub_nw;
  A.C4n = reinterpret_cast<const uint32_t*>(W.C4);
  A.c4_wide = 1;
  A.c4_rows = 0;
  A.edge_counts = nullptr; A.edge_begin = 0; A.edge_end = 0; A.global_sums = gsink;
  A.edge_ids = nullptr; A.n_edge_ids = 0;
  A.edge_orbits = nullptr;
  A.gacc_in_lds = 0;
  A.work = work_by_edge;
  A.thash_ok = n < (1ll << 27) ? 1 : 0;
  A.K4n = nullptr;
  A.K4w = nullptr;
  A.m = m;
  A.sp_keys = nullptr;
  A.sp_counts = nullptr;
  A.sp_start = nullptr;
  A.sp_len = nullptr;
  A.sp_cursor = nullptr;
  A.sp_cap = 0;
  const unsigned grid = grid_for(count, 1, 1024);
  int32_t* t_over = nullptr;
  int64_t t_cap = 0;
  if (h_tmax > TG_T_WG_CAP) {
    t_cap = h_tmax;
    TG_HIP(S.get(&t_over, over_scratch_ints(grid, t_cap)));
  }
  // the gather as tg_count runs it by default: without the 4-clique probes
  // when the clique pass covers the graph
  tg_tuning dflt;
  tg_tuning_default(&dflt);
  bool probe = dflt.clique_pass == 0;
  if (!probe) {
    int32_t* c;
    TG_HIP(S.get(&c, 16));
    k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(c), 16, 0u);
    k_k4_tier_count<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, W.out_off, c, c + 8);
    TG_LAUNCHED("k_k4_tier_count");
    int32_t h[8];
    TG_HIP(hipMemcpyAsync(h, c, sizeof(h), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    probe = h[7] > 0;
  }
  if (probe) {
    k_combine<256, uint64_t, true><<<grid, 256, combine_lds_bytes<256, uint64_t, true>(L), st>>>(
        A, count, list, nullptr, t_over, t_cap);
  } else {
    k_combine<256, uint64_t, false><<<grid, 256, combine_lds_bytes<256, uint64_t, false>(L), st>>>(
        A, count, list, nullptr, nullptr, 0);
  }
  TG_LAUNCHED("k_combine<256>");
  return TG_OK;
}

// Seeded uniform sample of canonical edges, in increasing edge order.
tg_status sample_edges(Scratch& S, hipStream_t st, int64_t m, double frac, uint64_t seed, int32_t** list_out,
                       int64_t* count_out) {
  int32_t* flag;
  int32_t* pos;
  int32_t* list;
  TG_HIP(S.get(&flag, m));
  TG_HIP(S.get(&pos, m + 1));
  TG_HIP(S.get(&list, m));
  const uint64_t thr = frac >= 1.0 ? ~0ull : (uint64_t)(frac * 18446744073709551616.0);
  k_sample_flags<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, seed, thr, flag);
  TG_LAUNCHED("k_sample_flags");
  if (tg_status s = scan(S, st, m, flag, pos)) return s;
  k_compact<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, flag, pos, list);
  TG_LAUNCHED("k_compact");
  int32_t total = 0;
  TG_HIP(hipMemcpyAsync(&total, pos + m, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TG_HIP(hipStreamSynchronize(st));
  *list_out = list;
  *count_out = total;
  return TG_OK;
}

tg_status train_impl(tg_cost_model* md, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                     const uint8_t* ty, int L, double frac, uint64_t seed, int epochs, float* loss_hist,
                     hipStream_t st) {
  if (!md) return fail(TG_ERR_INVALID_ARG, "null model");
  if (tg_status s = check_model_device(md)) return s;
  if (tg_status s = check_graph_args(n, nnz, rp, ci, ty, L)) return s;
  if (!(frac > 0.0 && frac <= 1.0) || epochs < 0) return fail(TG_ERR_INVALID_ARG, "bad sample fraction or epochs");
  const int64_t m = nnz / 2;
  if (m == 0) return fail(TG_ERR_INVALID_ARG, "graph has no edges to learn from");
  keep_pool_cached();
  Scratch S(st);
  Work W;
  if (tg_status s = prepare_graph(S, st, n, nnz, rp, ci, ty, L, W, nullptr, true, default_list_budget())) return s;
  int32_t* list;
  int64_t ns = 0;
  if (tg_status s = sample_edges(S, st, m, frac, seed, &list, &ns)) return s;
  if (ns < TG_MLP_ROWS) return fail(TG_ERR_INVALID_ARG, "edge sample too small to train on");
  uint64_t* work;
  float *X, *Yall, *Y;
  TG_HIP(S.get(&work, m));
  TG_HIP(S.get(&X, ns * TG_MLP_IN));
  TG_HIP(S.get(&Yall, m));
  TG_HIP(S.get(&Y, ns));
  if (tg_status s = measure_work(S, st, n, nnz, rp, ci, ty, L, W, list, ns, work)) return s;
  k_work_to_target<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, work, Yall);
  TG_LAUNCHED("k_work_to_target");
  k_gather_f32<<<grid_for(ns, 256, 8192), 256, 0, st>>>(ns, list, Yall, Y);
  TG_LAUNCHED("k_gather_f32");
  k_mlp_features<<<grid_for(ns, 256, 8192), 256, 0, st>>>(ns, list, W.ei, W.ej, W.deg, W.D, W.tau, ty, L,
                                                          X);
  TG_LAUNCHED("k_mlp_features");
  k_mlp_feature_stats<<<1, 256, 0, st>>>(ns, X, md->stats);
  TG_LAUNCHED("k_mlp_feature_stats");
  // mini-batch Adam over seeded shuffles of the sample
  const int64_t B = 1024;
  const int max_blocks = (int)(B / TG_MLP_ROWS);
  float *partial, *ploss, *grad, *loss;
  int32_t* perm_d;
  TG_HIP(S.get(&partial, (int64_t)max_blocks * TG_MLP_NPARAM));
  TG_HIP(S.get(&ploss, max_blocks));
  TG_HIP(S.get(&grad, TG_MLP_NPARAM));
  TG_HIP(S.get(&loss, 1));
  TG_HIP(S.get(&perm_d, ns));
  std::vector<int32_t> perm(ns);
  std::vector<float> step_loss;
  uint64_t rs = seed ^ 0xD6E8FEB86659FD93ull;
  auto next = [&]() {
    uint64_t z = (rs += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const float lr = 2e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t q = 0; q < ns; ++q) perm[q] = (int32_t)q;
    for (int64_t q = ns - 1; q > 0; --q) std::swap(perm[q], perm[next() % (uint64_t)(q + 1)]);
    TG_HIP(hipMemcpyAsync(perm_d, perm.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const int64_t nsteps = (ns + B - 1) / B;
    step_loss.assign(nsteps, 0.0f);
    for (int64_t stp = 0; stp < nsteps; ++stp) {
      const int64_t r0 = stp * B, rows = std::min(B, ns - r0);
      const int nb = (int)((rows + TG_MLP_ROWS - 1) / TG_MLP_ROWS);
      k_mlp_backward<<<nb, 256, 0, st>>>(rows, rows, perm_d + r0, md->Wbf, md->stats, X, Y, partial, ploss);
      TG_LAUNCHED("k_mlp_backward");
      k_mlp_reduce<<<grid_for(TG_MLP_NPARAM, 256, 64), 256, 0, st>>>(nb, partial, ploss, grad, loss);
      TG_LAUNCHED("k_mlp_reduce");
      md->steps += 1;
      const float c1 = 1.0f - std::pow(b1, (float)md->steps), c2 = 1.0f - std::pow(b2, (float)md->steps);
      k_mlp_adam<<<grid_for(TG_MLP_NPARAM, 256, 64), 256, 0, st>>>(md->W, md->M, md->V, grad, md->Wbf, lr, b1, b2,
                                                                   eps, c1, c2);
      TG_LAUNCHED("k_mlp_adam");
      if (loss_hist) TG_HIP(hipMemcpyAsync(&step_loss[stp], loss, sizeof(float), hipMemcpyDeviceToHost, st));
    }
    if (loss_hist) {
      TG_HIP(hipStreamSynchronize(st));
      double accl = 0.0;
      for (int64_t q = 0; q < nsteps; ++q) accl += step_loss[q];
      loss_hist[ep] = (float)(accl / (double)nsteps);
    }
  }
  TG_HIP(hipStreamSynchronize(st));
  return TG_OK;
}

}  // namespace

namespace {

tg_status tg_internal_predict_costs(const tg_cost_model* model, int64_t, const int32_t*, const int32_t*,
                                    const uint8_t* ty, int L, const tg::Work& W, int64_t m, float* out,
                                    hipStream_t st) {
  if (tg_status s = check_model_device(model)) return s;
  k_mlp_predict<<<grid_for(m, 256, 8192), 256, 0, st>>>(m, model->Wbf, model->stats, nullptr, W.ei, W.ej, W.deg,
                                                         W.D, W.tau, ty, L, out);
  TG_LAUNCHED("k_mlp_predict");
  return TG_OK;
}

}  // namespace

// ------------------------------------------------------------------ ABI --

#include "tg_directed.hip"
#include "tg_directed4.hip"

extern "C" {

void tg_options_default(tg_options* opt) {
  if (!opt) return;
  opt->schedule = TG_SCHED_DEGREE;
  opt->model = nullptr;
  opt->tuning = nullptr;
  opt->validate = 0;
  opt->check = 1;
  opt->edge_begin = 0;
  opt->edge_end = -1;
  opt->phase_ms = nullptr;
  opt->edge_ids = nullptr;
  opt->num_edge_ids = 0;
  opt->edge_orbits = nullptr;
}

void tg_tuning_default(tg_tuning* t) {
  if (!t) return;
  t->light_max_degree = 1024;
  t->heavy_min_degree = 4096;
  t->mid_log2_cost = 16;
  t->heavy_log2_cost = 64;
  t->combine_grid = 16384;
  t->wg_grid = 1024;
  t->c4_footprint_mb = 1024;
  t->c4_group_kwedges = 65536;
  t->c4_chunk = 1024;
  t->c4_hash_ratio = 16;
  t->c4_slot_budget_mb = 16384;
  t->c4_slices = 1;
  const int v[9] = {0, 0, 1, 4, 4, 5, 5, 5, 5};
  for (int w = 0; w <= 8; ++w) t->batch_variant[w] = v[w];
  t->clique_team_max = 64;
  t->clique_wave_max = 1024;
  t->clique_lds_ids = 4096;
  t->tlist_budget_mib = 16384;
  t->clique_pass = 1;
  t->clique_pass_grid = 0;
  t->clique_pass_lds_kib = 64;
  t->c4_parts = 1;
  t->c4_part_lds_kib = 40;
  t->c4_part_chunk = 4096;
  t->c4_part_hash_ratio = 16;
  t->tau_hub_min_degree = 4096;
  t->c4_split_log2 = 32;
}

tg_status tg_count_batch(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* row_ptr_local,
                         const int32_t* col_idx_local, const uint8_t* node_types, const uint8_t* L_per_graph,
                         const int64_t* key_off, uint64_t* global_counts, const tg_options* opt,
                         hipStream_t stream) {
  try {
    return batch_impl(G, node_off, slot_off, row_ptr_local, col_idx_local, node_types, L_per_graph, key_off,
                      global_counts, opt, stream);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

tg_status tg_count_batch_noalloc(int64_t G, const int64_t* node_off, const int64_t* slot_off,
                                 const int32_t* row_ptr_local, const int32_t* col_idx_local, const uint8_t* node_types,
                                 const uint8_t* L_per_graph, const int64_t* key_off, uint64_t* global_counts,
                                 const tg_options* opt, hipStream_t stream) {
  try {
    return batch_noalloc_impl(G, node_off, slot_off, row_ptr_local, col_idx_local, node_types, L_per_graph, key_off,
                              global_counts, opt, stream);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

size_t tg_num_keys(int L) { return (L < 1 || L > 16) ? 0 : (size_t)nkeys(L); }

size_t tg_edge_row_width(int L) { return (L < 1 || L > 16) ? 0 : (size_t)(2 * L + 3 * L * (L + 1)); }

tg_status tg_rows_sparse(int64_t E, int L, const uint64_t* rows, const int32_t* endpoints,
                         const uint8_t* node_types, int64_t* offsets, uint32_t* keys, uint64_t* counts,
                         int64_t capacity, int64_t* total, hipStream_t stream) {
  try {
    if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
    if (E < 0 || !offsets || (E > 0 && (!rows || !endpoints || !node_types)))
      return fail(TG_ERR_INVALID_ARG, "null input or offsets pointer");
    const int R = (int)tg_edge_row_width(L);
    hipStream_t st = stream;
    if (!keys) {
      // pass 1: nonzero counts and their exclusive prefix
      if (!total) return fail(TG_ERR_INVALID_ARG, "pass 1 needs a total pointer");
      keep_pool_cached();
      Scratch S(st);
      int64_t* cnt;
      TG_HIP(S.get(&cnt, std::max<int64_t>(E, 1)));
      if (E > 0) {
        k_sparse_count<<<grid_for(E, 4, 16384), 256, 0, st>>>(E, R, rows, cnt);
        TG_LAUNCHED("k_sparse_count");
      }
      if (tg_status s2 = scan(S, st, E, (const int64_t*)cnt, offsets)) return s2;
      TG_HIP(hipMemcpyAsync(total, offsets + E, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      TG_HIP(hipStreamSynchronize(st));
      return TG_OK;
    }
    // pass 2: the pairs, at the offsets of pass 1
    if (!counts) return fail(TG_ERR_INVALID_ARG, "null counts pointer");
    int64_t need = 0;
    TG_HIP(hipMemcpyAsync(&need, offsets + E, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TG_HIP(hipStreamSynchronize(st));
    if (need > capacity) return fail(TG_ERR_INVALID_ARG, "keys/counts capacity below the number of nonzeros");
    if (E > 0) {
      k_sparse_fill<<<grid_for(E, 4, 16384), 256, 0, st>>>(E, L, rows, endpoints, node_types, offsets, keys, counts);
      TG_LAUNCHED("k_sparse_fill");
    }
    if (total) *total = need;
    return TG_OK;
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, ex.what());
  }
}

size_t tg_edge_orbit_width(int L) { return (L < 1 || L > 16) ? 0 : (size_t)(2 * L + 5 * L * (L + 1)); }

tg_status tg_key_encode(int L, int shape, const uint8_t types[4], size_t* key) {
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (shape < 0 || shape >= TG_NUM_SHAPES || !types || !key) return fail(TG_ERR_INVALID_ARG, "bad shape or pointer");
  const int k = shape < 2 ? 3 : 4;
  int v[4];
  for (int a = 0; a < k; ++a) {
    if (types[a] >= L) return fail(TG_ERR_TYPE_RANGE, "type >= L");
    v[a] = types[a];
  }
  std::sort(v, v + k);
  int64_t r = 0;
  for (int a = 0; a < k; ++a) r += binom(v[a] + a, a + 1);
  const int64_t off = shape <= 2 ? shape * per_shape(L, 3) : 2 * per_shape(L, 3) + (shape - 2) * per_shape(L, 4);
  *key = (size_t)(off + r);
  return TG_OK;
}

tg_status tg_key_decode(int L, size_t key, int* shape, uint8_t types[4]) {
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (!shape || !types || key >= (size_t)nkeys(L)) return fail(TG_ERR_INVALID_ARG, "bad key or pointer");
  const int64_t c3 = per_shape(L, 3), c4 = per_shape(L, 4);
  int64_t k = (int64_t)key;
  int h, K;
  if (k < 2 * c3) { h = (int)(k / c3); k -= h * c3; K = 3; }
  else { h = 2 + (int)((k - 2 * c3) / c4); k -= 2 * c3 + (h - 2) * c4; K = 4; }
  // colex unranking: the largest element first
  int v[4] = {0, 0, 0, 0};
  for (int a = K - 1; a >= 0; --a) {
    int x = a;  // element x = type + a, find the largest with binom(x, a+1) <= k
    while (binom(x + 1, a + 1) <= k) ++x;
    k -= binom(x, a + 1);
    v[a] = x - a;
  }
  *shape = h;
  for (int a = 0; a < 4; ++a) types[a] = a < K ? (uint8_t)v[a] : (uint8_t)0xFF;
  return TG_OK;
}

tg_status tg_edge_row_key(int L, uint8_t phi_i, uint8_t phi_j, size_t col, size_t* key) {
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (phi_i >= L || phi_j >= L) return fail(TG_ERR_TYPE_RANGE, "type >= L");
  const int64_t P = (int64_t)L * (L + 1) / 2;
  if (!key || col >= (size_t)(2 * L + 6 * P)) return fail(TG_ERR_INVALID_ARG, "bad column or pointer");
  uint8_t ty[4] = {phi_i, phi_j, 0, 0};
  int shape;
  if ((int64_t)col < 2 * L) {
    shape = (int)col / L;
    ty[2] = (uint8_t)(col % L);
  } else {
    const int64_t c = (int64_t)col - 2 * L;
    shape = 2 + (int)(c / P);
    const int64_t p = c % P;
    int u = 0;
    while ((int64_t)(u + 1) * (u + 2) / 2 <= p) ++u;
    ty[2] = (uint8_t)(p - (int64_t)u * (u + 1) / 2);
    ty[3] = (uint8_t)u;
  }
  return tg_key_encode(L, shape, ty, key);
}

tg_status tg_count(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                   const uint8_t* node_types, int L, uint64_t* global_counts, uint64_t* edge_counts,
                   int32_t* edge_endpoints, const tg_options* opt, hipStream_t stream) {
  try {
    return count_impl(n, nnz, row_ptr, col_idx, node_types, L, global_counts, edge_counts, edge_endpoints, opt,
                      stream);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

tg_status tg_count_sparse(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                          const uint8_t* node_types, int L, uint64_t* global_counts, int64_t capacity,
                          uint32_t* keys, uint64_t* counts, int64_t* edge_start, int32_t* edge_len,
                          int64_t* total, const tg_options* opt, hipStream_t stream) {
  try {
    SparseOut sp;
    sp.keys = keys;
    sp.counts = counts;
    sp.start = edge_start;
    sp.len = edge_len;
    sp.cap = capacity;
    sp.total = total;
    tg_options o;
    tg_options_default(&o);
    if (opt) o = *opt;
    o.edge_orbits = nullptr;
    return count_impl(n, nnz, row_ptr, col_idx, node_types, L, global_counts, nullptr, nullptr, &o, stream, false,
                      1, &sp);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

tg_status tg_count_global(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                          const uint8_t* node_types, int L, uint64_t* global_counts, const tg_options* opt,
                          hipStream_t stream) {
  try {
    return count_impl(n, nnz, row_ptr, col_idx, node_types, L, global_counts, nullptr, nullptr, opt, stream, true);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

tg_status tg_count_global_types(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                                int64_t num_type_vectors, const uint8_t* node_types, int L,
                                uint64_t* global_counts, double* mean_counts, const tg_options* opt,
                                hipStream_t stream) {
  try {
    if (num_type_vectors < 1) return fail(TG_ERR_INVALID_ARG, "num_type_vectors must be at least 1");
    if (!global_counts) return fail(TG_ERR_INVALID_ARG, "null global_counts");
    tg_status s = count_impl(n, nnz, row_ptr, col_idx, node_types, L, global_counts, nullptr, nullptr, opt, stream,
                             true, num_type_vectors);
    if (s != TG_OK || !mean_counts) return s;
    const int64_t K = nkeys(L);
    k_mean_counts<<<grid_for(K, 256), 256, 0, stream>>>(num_type_vectors, K, global_counts, mean_counts);
    TG_LAUNCHED("k_mean_counts");
    return TG_OK;
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

tg_status tg_count_directed3(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                             const uint8_t* slot_dir, const uint8_t* node_types, int L, uint64_t* global_counts,
                             uint64_t* edge_rows, int32_t* edge_info, const tg_options* opt, hipStream_t stream) {
  try {
    return directed3_impl(n, nnz, row_ptr, col_idx, slot_dir, node_types, L, global_counts, edge_rows, edge_info,
                          opt, stream);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

tg_status tg_count_directed4(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                             const uint8_t* slot_dir, const uint8_t* node_types, int L, uint64_t* global_counts,
                             uint64_t* edge_rows, int32_t* edge_info, const tg_options* opt, hipStream_t stream) {
  try {
    return directed4_impl(n, nnz, row_ptr, col_idx, slot_dir, node_types, L, global_counts, edge_rows, edge_info,
                          opt, stream);
  } catch (const std::exception& ex) {
    return fail(TG_ERR_INTERNAL, std::string("exception: ") + ex.what());
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "unknown exception");
  }
}

size_t tg_directed4_num_keys(int L) {
  if (L < 1 || L > dir4::kMaxL) return 0;
  try {
    return dir4::tables(L).canon.size();
  } catch (...) {
    return 0;
  }
}

tg_status tg_directed4_key_decode(int L, size_t key, uint16_t* arcs, uint8_t types[4]) {
  if (L < 1 || L > dir4::kMaxL) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 4]");
  if (!arcs || !types) return fail(TG_ERR_INVALID_ARG, "null pointer");
  const dir4::Tables& T = dir4::tables(L);
  if (key >= T.canon.size()) return fail(TG_ERR_INVALID_ARG, "key out of range");
  const int64_t c = T.canon[key];
  *arcs = (uint16_t)(c & 0xFFF);
  for (int q = 0; q < 4; ++q) types[q] = (uint8_t)((c >> (12 + 4 * q)) & 15);
  return TG_OK;
}

size_t tg_directed3_num_keys(int L) {
  if (L < 1 || L > 16) return 0;
  try {
    return dir3::tables(L).canon.size();
  } catch (...) {
    return 0;
  }
}

tg_status tg_directed3_key_decode(int L, size_t key, uint8_t* arcs, uint8_t types[3]) {
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (!arcs || !types) return fail(TG_ERR_INVALID_ARG, "null output pointer");
  try {
    const dir3::Tables& T = dir3::tables(L);
    if (key >= T.canon.size()) return fail(TG_ERR_INVALID_ARG, "key out of range");
    const int c = T.canon[key];
    *arcs = (uint8_t)(c & 63);
    types[0] = (uint8_t)((c >> 6) & 15);
    types[1] = (uint8_t)((c >> 10) & 15);
    types[2] = (uint8_t)((c >> 14) & 15);
    return TG_OK;
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "table construction failed");
  }
}

tg_status tg_directed3_key_encode(int L, uint8_t arcs, const uint8_t types[3], size_t* key) {
  if (L < 1 || L > 16) return fail(TG_ERR_UNSUPPORTED_L, "L must be in [1, 16]");
  if (!types || !key) return fail(TG_ERR_INVALID_ARG, "null pointer");
  if (arcs > 63) return fail(TG_ERR_INVALID_ARG, "arcs must be six bits");
  for (int q = 0; q < 3; ++q)
    if (types[q] >= L) return fail(TG_ERR_TYPE_RANGE, "type >= L");
  try {
    const int32_t r = dir3::tables(L).code2rank[arcs | (types[0] << 6) | (types[1] << 10) | (types[2] << 14)];
    if (r < 0) return fail(TG_ERR_INVALID_ARG, "the triad is not weakly connected");
    *key = (size_t)r;
    return TG_OK;
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "table construction failed");
  }
}

size_t tg_cost_model_num_params(void) { return (size_t)TG_MLP_NPARAM; }

tg_status tg_cost_model_create(tg_cost_model** out, uint64_t seed) {
  if (!out) return fail(TG_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  tg_cost_model* md = new (std::nothrow) tg_cost_model();
  if (!md) return fail(TG_ERR_OUT_OF_MEMORY, "host allocation failed");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { delete md; return fail(TG_ERR_HIP, "hipGetDevice failed"); }
  md->device = dev;
  bool ok = hipMalloc(&md->W, TG_MLP_NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&md->M, TG_MLP_NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&md->V, TG_MLP_NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&md->Wbf, TG_MLP_NPARAM * sizeof(uint16_t)) == hipSuccess &&
            hipMalloc(&md->stats, 2 * TG_MLP_IN * sizeof(float)) == hipSuccess;
  if (!ok) { tg_cost_model_destroy(md); return fail(TG_ERR_OUT_OF_MEMORY, "device allocation failed"); }
  std::vector<float> w, st;
  model_init_host(w, st, seed);
  tg_status s = model_upload(md, w.data(), st.data(), nullptr);
  if (s != TG_OK) { tg_cost_model_destroy(md); return s; }
  *out = md;
  return TG_OK;
}

tg_status tg_cost_model_destroy(tg_cost_model* md) {
  if (!md) return TG_OK;
  if (md->W) (void)hipFree(md->W);
  if (md->M) (void)hipFree(md->M);
  if (md->V) (void)hipFree(md->V);
  if (md->Wbf) (void)hipFree(md->Wbf);
  if (md->stats) (void)hipFree(md->stats);
  delete md;
  return TG_OK;
}

tg_status tg_cost_model_get_params(const tg_cost_model* md, float* params) {
  if (!md || !params) return fail(TG_ERR_INVALID_ARG, "null pointer");
  TG_HIP(hipMemcpy(params, md->W, TG_MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  TG_HIP(hipMemcpy(params + TG_MLP_NPARAM, md->stats, 2 * TG_MLP_IN * sizeof(float), hipMemcpyDeviceToHost));
  return TG_OK;
}

tg_status tg_cost_model_set_params(tg_cost_model* md, const float* params) {
  if (!md || !params) return fail(TG_ERR_INVALID_ARG, "null pointer");
  return model_upload(md, params, params + TG_MLP_NPARAM, nullptr);
}

tg_status tg_cost_model_save(const tg_cost_model* md, const char* path) {
  if (!md || !path) return fail(TG_ERR_INVALID_ARG, "null pointer");
  std::vector<float> p(TG_MLP_NPARAM + 2 * TG_MLP_IN);
  if (tg_status s = tg_cost_model_get_params(md, p.data())) return s;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(TG_ERR_INVALID_ARG, std::string("cannot open ") + path);
  const char magic[8] = {'T', 'G', 'M', 'L', 'P', '1', '6', '\0'};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  return ok ? TG_OK : fail(TG_ERR_INVALID_ARG, "short write");
}

tg_status tg_cost_model_load(tg_cost_model* md, const char* path) {
  if (!md || !path) return fail(TG_ERR_INVALID_ARG, "null pointer");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(TG_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  std::vector<float> p(TG_MLP_NPARAM + 2 * TG_MLP_IN);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "TGMLP16", 8) == 0 &&
            std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  if (!ok) return fail(TG_ERR_INVALID_ARG, "not a cost model file");
  return tg_cost_model_set_params(md, p.data());
}

tg_status tg_cost_model_train(tg_cost_model* md, int64_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, const uint8_t* node_types, int L, double sample_frac,
                              uint64_t seed, int epochs, float* loss_history, hipStream_t stream) {
  try {
    return train_impl(md, n, nnz, row_ptr, col_idx, node_types, L, sample_frac, seed, epochs, loss_history, stream);
  } catch (...) {
    return fail(TG_ERR_INTERNAL, "exception during training");
  }
}

tg_status tg_cost_model_predict(const tg_cost_model* md, int64_t n, int64_t nnz, const int32_t* row_ptr,
                                const int32_t* col_idx, const uint8_t* node_types, int L, float* cost,
                                hipStream_t stream) {
  if (!md || !cost) return fail(TG_ERR_INVALID_ARG, "null pointer");
  if (tg_status s = check_graph_args(n, nnz, row_ptr, col_idx, node_types, L)) return s;
  if (nnz == 0) return TG_OK;
  keep_pool_cached();
  Scratch S(stream);
  Work W;
  if (tg_status s = prepare_graph(S, stream, n, nnz, row_ptr, col_idx, node_types, L, W, nullptr)) return s;
  return tg_internal_predict_costs(md, n, row_ptr, col_idx, node_types, L, W, nnz / 2, cost, stream);
}

tg_status tg_edge_work(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                       const uint8_t* node_types, int L, const int32_t* edges, int64_t count, uint64_t* work,
                       hipStream_t stream) {
  if (tg_status s = check_graph_args(n, nnz, row_ptr, col_idx, node_types, L)) return s;
  if (!work || count < 0 || (count > 0 && !edges)) return fail(TG_ERR_INVALID_ARG, "bad edge list or output");
  if (nnz == 0 || count == 0) return TG_OK;
  keep_pool_cached();
  Scratch S(stream);
  Work W;
  if (tg_status s = prepare_graph(S, stream, n, nnz, row_ptr, col_idx, node_types, L, W, nullptr, true,
                                  default_list_budget()))
    return s;
  return measure_work(S, stream, n, nnz, row_ptr, col_idx, node_types, L, W, edges, count, work);
}

tg_status tg_cost_model_gradient(const tg_cost_model* md, const float* X, const float* Y, int64_t rows,
                                 float* grad, float* loss, hipStream_t stream) {
  if (!md || !X || !Y || !grad || rows <= 0) return fail(TG_ERR_INVALID_ARG, "bad arguments");
  if (tg_status s = check_model_device(md)) return s;
  Scratch S(stream);
  const int nb = (int)((rows + TG_MLP_ROWS - 1) / TG_MLP_ROWS);
  float *partial, *ploss;
  TG_HIP(S.get(&partial, (int64_t)nb * TG_MLP_NPARAM));
  TG_HIP(S.get(&ploss, nb));
  k_mlp_backward<<<nb, 256, 0, stream>>>(rows, rows, nullptr, md->Wbf, md->stats, X, Y, partial, ploss);
  TG_LAUNCHED("k_mlp_backward");
  k_mlp_reduce<<<grid_for(TG_MLP_NPARAM, 256, 64), 256, 0, stream>>>(nb, partial, ploss, grad, loss);
  TG_LAUNCHED("k_mlp_reduce");
  return TG_OK;
}

tg_status tg_autotune(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      const uint8_t* node_types, int L, uint64_t* global_counts, uint64_t* edge_counts,
                      const tg_options* base, tg_tuning* tuning, float* best_ms, hipStream_t stream) {
  if (!tuning) return fail(TG_ERR_INVALID_ARG, "null tuning output");
  tg_options opt;
  tg_options_default(&opt);
  if (base) opt = *base;
  opt.edge_begin = 0;
  opt.edge_end = -1;
  tg_tuning cur;
  tg_tuning_default(&cur);
  if (base && base->tuning) cur = *base->tuning;
  float ph[TG_NUM_PHASES];
  opt.phase_ms = ph;
  // a trial is the faster of two calls (the phase times vary by about 1%)
  auto trial = [&](const tg_tuning& t, float* ms) -> tg_status {
    opt.tuning = &t;
    *ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      tg_status s = tg_count(n, nnz, row_ptr, col_idx, node_types, L, global_counts, edge_counts, nullptr, &opt,
                             stream);
      if (s) return s;
      const float v = ph[TG_PHASE_CYCLES] + ph[TG_PHASE_COMBINE];
      *ms = rep == 0 ? v : std::min(*ms, v);
    }
    return TG_OK;
  };
  float best = 0.0f;
  if (tg_status s = trial(cur, &best)) return s;   // warm-up of the pool and caches
  if (tg_status s = trial(cur, &best)) return s;
  const bool learned = opt.schedule == TG_SCHED_LEARNED;
  // coordinate descent over one parameter at a time (counts never change)
  std::vector<std::pair<int32_t*, std::vector<int32_t>>> axes;
  tg_tuning t = cur;
  axes.push_back({&t.light_max_degree, {16, 64, 256, 1024}});
  axes.push_back({&t.heavy_min_degree, {1024, 4096, 16384}});
  if (opt.schedule != TG_SCHED_NONE) {
    if (learned) {
      axes.push_back({&t.mid_log2_cost, {64, 8, 10, 12, 14, 16}});
      axes.push_back({&t.heavy_log2_cost, {64, 14, 16, 18, 20, 22}});
    } else {
      axes.push_back({&t.mid_log2_cost, {64, 12, 14, 16, 18}});
      axes.push_back({&t.heavy_log2_cost, {64, 18, 20, 22, 24}});
    }
  }
  axes.push_back({&t.combine_grid, {4096, 8192, 16384}});
  axes.push_back({&t.wg_grid, {0, 1024, 2048, 4096}});
  axes.push_back({&t.c4_footprint_mb, {64, 192, 1024}});
  axes.push_back({&t.c4_group_kwedges, {4096, 16384, 32768, 65536}});
  axes.push_back({&t.c4_chunk, {256, 1024, 4096}});
  axes.push_back({&t.c4_hash_ratio, {0, 4, 16}});
  axes.push_back({&t.c4_slices, {1, 8}});
  axes.push_back({&t.c4_part_hash_ratio, {2, 4, 8, 16}});
  axes.push_back({&t.c4_part_lds_kib, {32, 40, 64}});
  axes.push_back({&t.c4_part_chunk, {2048, 4096, 8192}});
  axes.push_back({&t.tau_hub_min_degree, {0, 256, 1024, 4096}});
  for (auto& ax : axes) {
    int32_t best_v = *ax.first;
    for (int32_t v : ax.second) {
      if (v == best_v) continue;
      *ax.first = v;
      float ms = 0.0f;
      if (tg_status s = trial(t, &ms)) return s;
      if (ms < best) { best = ms; best_v = v; }
    }
    *ax.first = best_v;
  }
  *tuning = t;
  if (best_ms) *best_ms = best;
  return TG_OK;
}

tg_status tg_autotune_batch(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* row_ptr_local,
                            const int32_t* col_idx_local, const uint8_t* node_types, const uint8_t* L_per_graph,
                            const int64_t* key_off, uint64_t* global_counts, tg_tuning* tuning, float* best_ms,
                            hipStream_t stream) {
  if (!tuning) return fail(TG_ERR_INVALID_ARG, "null tuning output");
  tg_tuning t = *tuning;
  tg_options opt;
  tg_options_default(&opt);
  opt.check = 1;
  hipEvent_t e0, e1;
  TG_HIP(hipEventCreate(&e0));
  TG_HIP(hipEventCreate(&e1));
  auto trial = [&](const tg_tuning& tt, float* ms) -> tg_status {
    opt.tuning = &tt;
    tg_status s = TG_OK;
    float best_of = 1e30f;
    for (int rep = 0; rep < 2 && s == TG_OK; ++rep) {
      if (hipEventRecord(e0, stream) != hipSuccess) return fail(TG_ERR_HIP, "hipEventRecord");
      s = tg_count_batch(G, node_off, slot_off, row_ptr_local, col_idx_local, node_types, L_per_graph, key_off,
                         global_counts, &opt, stream);
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(TG_ERR_HIP, "hipEvent timing");
      float x = 0.0f;
      (void)hipEventElapsedTime(&x, e0, e1);
      best_of = std::min(best_of, x);
    }
    *ms = best_of;
    return s;
  };
  float best = 0.0f;
  tg_status st = trial(t, &best);
  // variants able to hold each size class W (words per bit row)
  const int wmax[6] = {1, 2, 2, 4, 4, 8};
  for (int w = 8; w >= 1 && st == TG_OK; --w) {
    int best_v = t.batch_variant[w];
    for (int v = 0; v < 6 && st == TG_OK; ++v) {
      if (wmax[v] < w || v == best_v) continue;
      t.batch_variant[w] = v;
      float ms = 0.0f;
      st = trial(t, &ms);
      if (st == TG_OK && ms < best) { best = ms; best_v = v; }
    }
    t.batch_variant[w] = best_v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TG_OK) return st;
  t.batch_variant[0] = t.batch_variant[1];
  *tuning = t;
  if (best_ms) *best_ms = best;
  return TG_OK;
}

tg_status tg_release_scratch(void) { return release_scratch(); }

const char* tg_status_string(tg_status s) {
  switch (s) {
    case TG_OK: return "TG_OK";
    case TG_ERR_INVALID_ARG: return "TG_ERR_INVALID_ARG";
    case TG_ERR_INVALID_GRAPH: return "TG_ERR_INVALID_GRAPH";
    case TG_ERR_TYPE_RANGE: return "TG_ERR_TYPE_RANGE";
    case TG_ERR_UNSUPPORTED_L: return "TG_ERR_UNSUPPORTED_L";
    case TG_ERR_OUT_OF_MEMORY: return "TG_ERR_OUT_OF_MEMORY";
    case TG_ERR_INTERNAL: return "TG_ERR_INTERNAL";
    case TG_ERR_HIP: return "TG_ERR_HIP";
  }
  return "unknown status";
}

const char* tg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
