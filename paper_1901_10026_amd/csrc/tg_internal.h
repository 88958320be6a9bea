// Internal declarations shared by the kernel and API translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tg_device.h"

// validation flags (device-side, OR-ed together)
#define TG_VFLAG_ROWPTR 1
#define TG_VFLAG_TYPE 2
#define TG_VFLAG_RANGE 4
#define TG_VFLAG_SELFLOOP 8
#define TG_VFLAG_ORDER 16
#define TG_VFLAG_ASYMMETRIC 32

// light/heavy limits
#define TG_C4_LIGHT_W 128     // wedge work handled by one wavefront with an LDS hash
#define TG_C4_LIGHT_CAP 256
#define TG_C4_MED_W 2048      // wedge work handled by one workgroup with an LDS hash
#define TG_C4_MED_CAP 4096
#define TG_T_WAVE_CAP 128     // |T_ij| handled by one wavefront
#define TG_T_WG_CAP 2048      // |T_ij| kept in LDS by a workgroup (larger: global scratch)
#define TG_GACC_MAX_KEYS 5120 // global keys accumulated in LDS per workgroup
#define TG_C4P_NW 8           // wavefronts of a k_c4_part workgroup

namespace tg {

struct Graph {
  int64_t n, nnz, m;
  int L;
  const int32_t* rp;
  const int32_t* ci;
  const uint8_t* ty;
};

// Device scratch of one tg_count call.
struct Work {
  int32_t* deg;          // n
  uint32_t* D;           // n*L typed degree
  int32_t* n_upper;      // n
  int32_t* n_out;        // n
  uint64_t* wedge_work;  // n   W(v)
  uint64_t* nbr_deg_sum; // n   s(v)
  int32_t* upper_off;    // n+1
  int32_t* out_off;      // n+1
  int32_t* scan_tmp;     // blocks + 1
  int32_t* ei;           // m
  int32_t* ej;           // m
  int32_t* s2e;          // nnz
  int32_t* es_lo;        // m     slot of each edge in its lower end's row
  int32_t* es_hi;        // m     slot of each edge in its upper end's row
  int32_t* out_col;      // m
  int32_t* out_eid;      // m     canonical edge id of each out-list slot (clique pass only), or null
  uint32_t* tau;         // m*L
  uint32_t* tau_s;       // nnz*L: tau of each edge again at both of its CSR slots (per-edge counting only)
  int64_t* tl_off;       // m+1, or null: start of each edge's common-neighbour list kept by the tau pass
  int tl_packed;         // list ids hold their node's type in the low 4 bits (n < 2^27)
  int32_t* hub_of;       // n, or null: index of each hub node (row bitmaps below), -1 for the others
  uint64_t* hub_bits;    // hubs x hub_nw: bit k of a hub's bitmap = node k in its row
  int32_t* hub_rank;     // hubs x hub_nw: set bits before each word (the row position)
  int64_t hub_nw;        // words per hub bitmap, ceil(n / 64)
  int32_t* tl_k;         // list entries: member ids (id << 4 | type when tl_packed) ...
  int32_t* tl_e;         // ... and the CSR slots of k in the rows of a and b, two per member
  uint64_t* Pn;          // n*L*L
  uint64_t* Un;          // n*L*L
  uint64_t* C4;          // m*P (32-bit counters when they suffice: see c4_wide)
  int32_t* elist;        // m     edge ids grouped by class and bucket
  int32_t* nlist;        // n     node ids grouped by tier
  int32_t* counters;     // small
  uint64_t* ecost;       // m     per-edge cost used for binning
};

struct EdgeArgs {
  const int32_t* rp;
  const int32_t* ci;
  const uint8_t* ty;
  const int32_t* deg;
  const uint32_t* D;
  const int32_t* ei;
  const int32_t* ej;
  const int32_t* s2e;
  const int32_t* out_off;
  const int32_t* out_col;
  const uint32_t* tau;
  const uint32_t* tau_s;  // tau by CSR slot
  const int64_t* tl_off;  // common-neighbour lists of the edges (from the tau pass), or null
  int tl_packed;          // list ids are id << 4 | type
  const int32_t* hub_of;  // row bitmaps of the hubs (see Work), or null
  const uint64_t* hub_bits;
  const int32_t* hub_rank;
  int64_t hub_nw;
  const int32_t* tl_k;
  const int32_t* tl_e;
  const uint64_t* Pn;
  const uint64_t* Un;
  const uint64_t* C4;     // 64-bit 4-cycle counters (c4_wide), or
  const uint32_t* C4n;    // 32-bit ones
  int c4_wide;
  int64_t c4_rows;        // 0: P counters per edge; else type-pair major, C4[p * c4_rows + e]
  int L;
  uint64_t* edge_counts;  // rows for [edge_begin, edge_end) or for edge_ids, or null
  int64_t edge_begin, edge_end;
  const int64_t* edge_ids;  // sorted sample of edges whose rows are written, or null
  uint64_t* edge_orbits;    // orbit rows g1..g12 (2L + 10P per edge) for the same edges, or null
  int64_t n_edge_ids;
  uint64_t* global_sums;  // K(L)
  int gacc_in_lds;
  uint64_t* work;         // null, or per-edge element-visit counts (added atomically, by edge id)
  int thash_ok;           // node ids fit the packed (id << 4 | type) hash slots
  // per-edge typed 4-clique counts from the clique pass, edge major
  // (K4[e * P + p]), 32- or 64-bit; both null: the gather probes out-lists
  const uint32_t* K4n;
  const uint64_t* K4w;
  int64_t m;
  // sparse per-edge output (instead of dense rows, L <= 8): each team of
  // the row kernel stages its edge's row in LDS and appends the nonzero
  // (key, count) pairs at an atomic cursor; sp_start[q] and sp_len[q] give
  // edge q's pairs; pairs past sp_cap are not written (the cursor still
  // counts them).  sp_keys null: dense rows as usual.
  uint32_t* sp_keys;
  uint64_t* sp_counts;
  int64_t* sp_start;
  int32_t* sp_len;
  unsigned long long* sp_cursor;
  int64_t sp_cap;
};

// Global key sums of one kernel: keys [k0, k0 + nk) are summed in `copies`
// LDS copies (lane l adds to copy l % copies) and flushed once per
// workgroup; other keys, or all keys when copies == 0, go straight to g.
struct GAcc {
  uint64_t* g;  // global key vector
  int64_t k0, nk;
  int copies;
};

__device__ __forceinline__ void gacc_init(const GAcc& a, uint64_t* s) {
  for (int64_t x = threadIdx.x; x < (int64_t)a.copies * a.nk; x += blockDim.x) s[x] = 0;
  __syncthreads();
}

__device__ __forceinline__ void gacc_add(const GAcc& a, uint64_t* s, int64_t key, uint64_t v) {
  const int64_t r = key - a.k0;
  if (a.copies && r >= 0 && r < a.nk)
    atomicAdd((unsigned long long*)&s[(int64_t)(lane() % a.copies) * a.nk + r], (unsigned long long)v);
  else
    atomicAdd((unsigned long long*)&a.g[key], (unsigned long long)v);
}

__device__ __forceinline__ void gacc_flush(const GAcc& a, uint64_t* s) {
  if (!a.copies) return;
  __syncthreads();
  for (int64_t x = threadIdx.x; x < a.nk; x += blockDim.x) {
    uint64_t v = 0;
    for (int c = 0; c < a.copies; ++c) v += s[(int64_t)c * a.nk + x];
    if (v) atomicAdd((unsigned long long*)&a.g[a.k0 + x], (unsigned long long)v);
  }
}

}  // namespace tg
