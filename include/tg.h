/*
 * tg.h -- C ABI of libtg.so: per-edge and global counts of typed 3- and
 * 4-node graphlets on AMD MI355X (gfx950).
 *
 * What is counted (Sections 3.2 and 4, "Local Typed Graphlet Counting" and
 * "Global Typed Graphlet Counting"): for an undirected simple graph whose
 * nodes carry a type phi in [0, L), and for every edge (i, j), the number of
 * connected induced subgraphs on 3 or 4 nodes that contain both i and j,
 * split by graphlet shape and by the multiset of node types of the subgraph
 * (typed graphlet instances are equal when their type multisets are equal).
 * The global count of a (shape, multiset) is the number of such subgraphs in
 * the graph; it equals the per-edge sum divided by the shape's edge count
 * (Eq. 17).
 *
 * Shapes, in the paper's order h1..h8: wedge (3-node path), triangle, 4-path,
 * 4-star, 4-cycle, tailed triangle, chordal cycle (diamond), 4-clique.
 *
 * Conventions used by every entry point:
 *  - Graph: CSR with int32 row_ptr[n+1] and col_idx[nnz]; both directions of
 *    each edge stored; each row strictly increasing; no self loops; nnz < 2^31.
 *  - Node types: uint8 types[n], each < L, 1 <= L <= 16.
 *  - Canonical edge order: the e-th slot (i, j) with i < j when the CSR is read
 *    row by row.  m = nnz / 2 edges.
 *  - Per-edge row (width tg_edge_row_width(L) = 2L + 3L(L+1)), relative to the
 *    edge's own types (phi_i, phi_j): wedge[t] for t < L, triangle[t], then for
 *    4-path, 4-star, 4-cycle, tailed triangle, chordal cycle, 4-clique one
 *    block of P = L(L+1)/2 entries each, indexed by p(t, u) = u(u+1)/2 + t for
 *    t <= u: the types of the two other nodes.
 *  - Global key (tg_num_keys(L) = 2 C(L+2,3) + 6 C(L+3,4) keys): shape offset
 *    plus the colex rank of the sorted type multiset (a<=b<=c[<=d]):
 *    C(a,1) + C(b+1,2) + C(c+2,3) [+ C(d+3,4)].  Offsets follow shape order,
 *    3-node shapes taking C(L+2,3) keys each and 4-node shapes C(L+3,4).
 *  - Counts are uint64.
 *
 * Memory: pointers documented as "device" must point to device memory of the
 * current HIP device (e.g. torch tensors); "host" pointers to host memory.
 * The caller owns every input and output buffer.  Scratch memory belongs to
 * the library: a per-device workspace that one call at a time holds and that
 * later calls reuse (grown to the last call's need, kept until the process
 * ends or tg_release_scratch frees it; a call on another stream first waits
 * for the previous holder's work), with any excess and concurrent calls
 * served stream-ordered on the caller's stream from the default pool.
 *
 * Streams and errors: all device work is enqueued on `stream`.  Argument
 * errors are reported before anything is enqueued.  Device-detected problems
 * (invalid graph when validation is on, a global sum that is not a multiple of
 * its shape's edge count) are reported after the call synchronises the
 * stream, which it does only when `check` (or `validate`) is set.  On any
 * non-OK status the outputs are unspecified.  tg_last_error() gives a
 * thread-local message for the last failure.  No C++ exception crosses the ABI.
 */
#ifndef TG_H_
#define TG_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TG_OK = 0,
  TG_ERR_INVALID_ARG = 1,     /* null pointer, bad size, bad range */
  TG_ERR_INVALID_GRAPH = 2,   /* CSR violates the conventions above (validate=1) */
  TG_ERR_TYPE_RANGE = 3,      /* a node type >= L (validate=1) */
  TG_ERR_UNSUPPORTED_L = 4,   /* L outside [1, 16] */
  TG_ERR_OUT_OF_MEMORY = 5,   /* scratch allocation failed */
  TG_ERR_INTERNAL = 6,        /* a global sum was not divisible (check=1) */
  TG_ERR_HIP = 7              /* a HIP runtime call failed */
} tg_status;

typedef enum {
  TG_WEDGE = 0, TG_TRIANGLE, TG_PATH4, TG_STAR4, TG_CYCLE4, TG_TAILED_TRIANGLE, TG_CHORDAL_CYCLE, TG_CLIQUE4,
  TG_NUM_SHAPES
} tg_shape;

/* Edge scheduling.  Counts are identical for every choice; only time changes.
 * NONE: edges in canonical order with a fixed light/heavy split by degree.
 * DEGREE: edges binned and ordered by the degree-product cost d_i * d_j.
 * LEARNED: edges binned and ordered by a cost model (tg_cost_model). */
typedef enum { TG_SCHED_NONE = 0, TG_SCHED_DEGREE = 1, TG_SCHED_LEARNED = 2 } tg_schedule;

typedef struct tg_cost_model tg_cost_model;

/* Launch-shape choices (defaults from tg_tuning_default; tg_autotune picks
 * them by timing).  Counts never depend on them. */
typedef struct {
  int32_t light_max_degree;   /* tg_count: edges with |T_ij| <= 64 and min(d_i, d_j) <= this use a
                                 16-lane team (L <= 8) */
  int32_t heavy_min_degree;   /* tg_count: edges with min(d_i, d_j) above this use one workgroup */
  int32_t mid_log2_cost;      /* tg_count: edges whose log2 schedule cost exceeds this use at least
                                 a full wavefront (64 = never) */
  int32_t heavy_log2_cost;    /* tg_count: edges whose log2 schedule cost exceeds this use one
                                 workgroup (64 = never) */
  int32_t combine_grid;       /* tg_count: workgroup count cap of the small-team combine launches
                                 (0 = the number that fits the device at once) */
  int32_t wg_grid;            /* tg_count: workgroup count cap of the workgroup-per-edge launch
                                 (0 = the number that fits the device at once) */
  int32_t c4_footprint_mb;    /* tg_count: heavy nodes of the 4-cycle pass are processed in groups
                                 whose count rows touch at most about this many MiB ... */
  int32_t c4_group_kwedges;   /* ... and that close once they hold this many thousand wedges */
  int32_t c4_chunk;           /* tg_count: wedges per wavefront in the heavy 4-cycle pass (>= 64) */
  int32_t c4_hash_ratio;      /* tg_count: a heavy node uses a hash table of its far ends instead of a
                                 dense array when the table is at least this many times smaller
                                 (0 = never) */
  int32_t c4_slot_budget_mb;  /* tg_count: 4-cycle counters are kept per CSR slot (then folded per edge)
                                 when they fit in this many MiB, else per edge */
  int32_t c4_slices;          /* tg_count: far-end slices of the dense 4-cycle groups, one per XCD (1 = none) */
  int32_t batch_variant[9];   /* tg_count_batch: kernel variant per size class W = ceil(n/64)
                                 (0: wavefront, 64 nodes; 1: wavefront, 128; 2: workgroup, 128;
                                 3: wavefront, 256; 4: workgroup, 256; 5: workgroup, 512) */
  int32_t clique_team_max;    /* tg_count_global: edges whose 4-clique intersection loop is at most this
                                 long (<= 64) use a 16-lane team ... */
  int32_t clique_wave_max;    /* ... at most this long (<= 1024) a wavefront, longer ones a workgroup */
  int32_t clique_lds_ids;     /* tg_count_global: common higher neighbours kept in LDS by a workgroup
                                 team (<= 4096); more go to global scratch */
  int32_t tlist_budget_mib;   /* tg_count: the typed-triangle pass keeps every edge's common-neighbour
                                 list (12 B per entry, sized by min(d_i, d_j)) for the per-edge gather
                                 when all lists fit in this many MiB of scratch; else (and at 0) the
                                 gather intersects the two rows again */
  int32_t clique_pass;        /* tg_count: 1 = count every edge's typed 4-cliques in one pass over the
                                 graph, each clique once from its lowest node in degree order, when the
                                 per-edge step covers at least an eighth of the edges and no node has
                                 more than 4096 higher-ranked neighbours; 0 = the per-edge gather finds
                                 them from out-lists instead */
  int32_t clique_pass_grid;   /* tg_count: workgroups of the clique pass's global-scratch launch, each
                                 with a slice of its own (0 = two per compute unit) */
  int32_t clique_pass_lds_kib;/* tg_count: a tier of the clique pass keeps its bit rows in LDS when they
                                 fit in this many KiB per workgroup, else in global scratch */
  int32_t c4_parts;           /* tg_count: 1 = the dense groups of the 4-cycle pass take their middle
                                 counts from records bucketed by far-end id range and summed in LDS
                                 instead of from global atomics (L <= 8; the groups whose nodes all
                                 have degrees below 65536; graphs of at most 8192 id ranges of the
                                 range table); 0 = never */
  int32_t c4_part_lds_kib;    /* tg_count: LDS per workgroup of the range table, capped by the device's
                                 limit */
  int32_t c4_part_chunk;      /* tg_count: wedges per walk item of that pass (256 to 32768; raised to
                                 twice the number of id ranges, up to 16384, and the pass is off
                                 when that is not enough) */
  int32_t c4_part_hash_ratio; /* tg_count: c4_hash_ratio in effect when that pass is on */
  int32_t tau_hub_min_degree; /* tg_count: the typed-triangle pass finds the common neighbours of an edge
                                 whose longer row has more than this many entries in a bitmap of that
                                 row (raised until the bitmaps fit in 4 GiB; 0 = binary search always) */
  int32_t c4_split_log2;      /* tg_count: when the 4-cycle counters need 64 bits and per-slot rows of
                                 64-bit counters exceed c4_slot_budget_mb, per-slot rows of 32-bit
                                 counters are kept if device memory allows, and an edge (a, b) with
                                 (d_a - 1)(d_b - 1) >= 2^c4_split_log2 is counted in its 64-bit per-edge
                                 counters instead (1 to 32; 0 = per-edge counters only) */
} tg_tuning;

/* Fills *t with the library's defaults. */
void tg_tuning_default(tg_tuning* t);

typedef struct {
  tg_schedule schedule;        /* default TG_SCHED_DEGREE */
  const tg_cost_model* model;  /* required for TG_SCHED_LEARNED, else ignored */
  const tg_tuning* tuning;     /* NULL: defaults */
  int validate;                /* 1: O(m) device check of the CSR and types (synchronises) */
  int check;                   /* 1: synchronise and verify global divisibility (default 1) */
  int64_t edge_begin;          /* per-edge rows are written for canonical edges */
  int64_t edge_end;            /*   [edge_begin, edge_end); edge_end < 0 means m */
  float* phase_ms;             /* host, TG_NUM_PHASES floats, or NULL: when set, the call records
                                  HIP events on `stream` around each phase, synchronises at the end
                                  and stores each phase's elapsed milliseconds */
  const int64_t* edge_ids;     /* device, strictly increasing canonical edge ids in [0, m), or NULL.
                                  When set, rows (and endpoints) are written for these edges only,
                                  entry q for edge edge_ids[q], and edge_begin/edge_end are ignored:
                                  a sample of a graph whose rows would not fit in memory */
  int64_t num_edge_ids;        /* length of edge_ids */
  uint64_t* edge_orbits;       /* device, uint64[E * tg_edge_orbit_width(L)] or NULL: per-edge orbit counts
                                  (Table 3's g1..g12) for the same E edges as edge_counts: g1[t], g2[t]
                                  for t < L, then g3..g12 in blocks of L(L+1)/2 type pairs (the same pair
                                  order as the row's 4-node blocks) */
} tg_options;

/* Phases timed through tg_options.phase_ms. */
enum {
  TG_PHASE_PREP = 0,     /* degrees, typed degrees, edge ids, degree-ordered out-lists */
  TG_PHASE_TAU,          /* typed triangle counts per edge */
  TG_PHASE_TABLES,       /* per-node sums of typed degrees and triangle counts */
  TG_PHASE_SCHEDULE,     /* edge classes and cost buckets, node tiers */
  TG_PHASE_CYCLES,       /* typed 4-cycles through every edge */
  TG_PHASE_CLIQUES,      /* typed 4-cliques, each from its lowest node (when that pass runs) */
  TG_PHASE_COMBINE,      /* per-edge orbits, graphlets, rows and global sums */
  TG_PHASE_FINALIZE,     /* division of global sums by shape edge counts */
  TG_NUM_PHASES
};

/* Fills *opt with the defaults above. */
void tg_options_default(tg_options* opt);

/* K(L) = 2 C(L+2,3) + 6 C(L+3,4) global keys (Eq. 1 per shape); 0 if L is
 * outside [1, 16]. */
size_t tg_num_keys(int L);

/* R(L) = 2L + 3L(L+1) entries per edge row; 0 if L is outside [1, 16]. */
size_t tg_edge_row_width(int L);

/* 2L + 5L(L+1) entries per edge orbit row (the twelve orbits of Table 3, by
 * type or type pair); 0 if L is outside [1, 16]. */
size_t tg_edge_orbit_width(int L);

/* Host.  Decodes a global key into its shape and sorted types; types[3] is
 * 0xFF for 3-node shapes. */
tg_status tg_key_decode(int L, size_t key, int* shape, uint8_t types[4]);

/* Host.  Encodes (shape, types) into a global key; the types may come in any
 * order (the key depends on the multiset only, Section 4.5); types[3] is
 * ignored for 3-node shapes. */
tg_status tg_key_encode(int L, int shape, const uint8_t types[4], size_t* key);

/* Host.  Global key of column `col` of a per-edge row whose edge has types
 * (phi_i, phi_j). */
tg_status tg_edge_row_key(int L, uint8_t phi_i, uint8_t phi_j, size_t col, size_t* key);

/* Counts every typed 3/4-node graphlet of one graph (Algorithm 1's problem,
 * per edge, plus Eq. 17's global counts).
 *   n, nnz          node count and CSR slot count (nnz = 2m)
 *   row_ptr         device, int32[n+1]
 *   col_idx         device, int32[nnz]
 *   node_types      device, uint8[n]
 *   L               number of node types, 1..16
 *   global_counts   device, uint64[tg_num_keys(L)], or NULL when edge_counts
 *                   is given: then only the edges whose rows are asked for
 *                   go through the per-edge step (the 4-cycle pass still
 *                   covers the whole graph), for graphs too large to count
 *                   in full
 *   edge_counts     device, uint64[E * R(L)], or NULL for global counts only;
 *                   E = edge_end - edge_begin, or num_edge_ids when
 *                   opt->edge_ids is set
 *   edge_endpoints  device, int32[E * 2] receiving (i, j) with i < j of each
 *                   canonical edge in range (or listed), or NULL
 *   opt             host, or NULL for defaults
 * Canonical edge ids number the edges (i, j), i < j, in (i, j) order.
 * The call reads small plan data back to the host while it runs (the edge
 * bin sizes, the 4-cycle node groups, the size of the common-neighbour
 * lists), so the calling thread waits for the preprocessing enqueued on
 * `stream`; the counting kernels themselves are left running on return
 * unless check, validate or phase_ms asks for a synchronisation.
 * Errors: TG_ERR_INVALID_ARG for a bad edge range, an edge_ids array that
 * is not strictly increasing inside [0, m), or no output given (nothing
 * written).
 */
tg_status tg_count(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                   const uint8_t* node_types, int L, uint64_t* global_counts, uint64_t* edge_counts,
                   int32_t* edge_endpoints, const tg_options* opt, hipStream_t stream);

/* tg_count with the paper's sparse per-edge output (the Sparse Typed Motif
 * Format subsection: only the nonzero typed graphlet counts of each edge,
 * with their ids), written by the row kernel itself: no dense per-edge row
 * is ever stored, so the per-edge output of a graph whose dense rows would
 * not fit can be taken in one call.  Arguments as for tg_count, with the
 * edges of opt's range or id list (E of them) and, in place of the dense
 * rows:
 *   capacity    number of (key, count) pairs the caller's buffers hold
 *   keys        device, uint32[capacity]: the pairs' global keys (dense
 *               rank of tg_key_encode; tg_key_decode is the lookup table)
 *   counts      device, uint64[capacity]: the pairs' counts (nonzero)
 *   edge_start  device, int64[E]: first pair of edge q
 *   edge_len    device, int32[E]: number of pairs of edge q, in the row's
 *               column order
 *   total       host: receives the number of pairs of all E edges
 * The edges' pairs lie at arbitrary but disjoint places of [0, total).  L
 * must be at most 8 (TG_ERR_UNSUPPORTED_L).  The call synchronises to read
 * the total; with total > capacity it returns TG_ERR_INVALID_ARG after the
 * counting (edge_start and edge_len are written, the pairs are not all
 * written), so a caller may count once with capacity 0 and again with the
 * reported total, or size the buffers by E * R(L).  global_counts may be
 * NULL, as for tg_count. */
tg_status tg_count_sparse(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                          const uint8_t* node_types, int L, uint64_t* global_counts, int64_t capacity,
                          uint32_t* keys, uint64_t* counts, int64_t* edge_start, int32_t* edge_len,
                          int64_t* total, const tg_options* opt, hipStream_t stream);

/* Global counts only, every instance counted a fixed number of times instead
 * of once per edge (the Global Typed Graphlet Counts section notes that an
 * ordering makes a global-only count cheaper).  Non-induced typed counts of
 * the eight shape patterns are summed per type multiset -- 4-cliques once
 * from their two lowest nodes in degree order, 4-cycles from degree-ordered
 * wedges, the rest from typed degrees and typed common-neighbour counts --
 * and converted into induced counts.  The result equals tg_count's global
 * counts.
 *   arguments as for tg_count; global_counts (device, uint64[tg_num_keys(L)])
 *   must not be NULL
 *   opt             host, or NULL: validate, check, phase_ms and tuning (its
 *                   4-cycle fields) apply; edge ranges, edge_ids, schedule,
 *                   model and edge_orbits are ignored
 * Every true count, and every non-induced pattern total (for instance the
 * number of 4-paths including those inside denser subgraphs), must be below
 * 2^63.  With check set, the call synchronises and reports
 * TG_ERR_INTERNAL if a sum is inconsistent (a 4-cycle or tailed-triangle sum
 * odd, a triangle sum not a multiple of 3, or a negative result).
 */
tg_status tg_count_global(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                          const uint8_t* node_types, int L, uint64_t* global_counts, const tg_options* opt,
                          hipStream_t stream);

/* Global counts for several type vectors of one graph, as tg_count_global
 * gives them for each, sharing the work that does not depend on the types
 * (degree order, out-lists, 4-cycle groups, 4-clique edge classes).  This
 * is the type-permutation null model of the exploratory analysis (the
 * randomized typed triangle and 4-node motif distributions): the caller
 * passes permutations of the real type vector (random numbers are the
 * caller's) and gets every permutation's counts and their mean.
 *   num_type_vectors  B >= 1
 *   node_types        device, uint8[B * n]: vector b at node_types + b * n
 *   global_counts     device, uint64[B * tg_num_keys(L)]: vector b's counts
 *                     at global_counts + b * K(L); must not be NULL
 *   mean_counts       device, double[tg_num_keys(L)] receiving the mean over
 *                     the B vectors (exact integer sums, one rounding), or
 *                     NULL
 * Other arguments, options and errors as for tg_count_global; validate
 * checks every type vector.
 */
tg_status tg_count_global_types(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                                int64_t num_type_vectors, const uint8_t* node_types, int L,
                                uint64_t* global_counts, double* mean_counts, const tg_options* opt,
                                hipStream_t stream);

/* Directed typed 3-node graphlets (the Directed Typed Graphlets subsection:
 * typed neighbour sets split into typed out- and in-neighbour sets).
 * Graph: the symmetric support CSR (conventions above) plus one direction
 * byte per slot, bit 0 for the arc row -> column and bit 1 for column -> row
 * (so 1, 2 or 3; the two slots of an edge mirror each other).  The direction
 * code c(u, v) of a pair is the byte at u's slot for v, 0 if not adjacent.
 * Triad of ordered nodes (a, b, c): arc bits a->b, b->a, a->c, c->a, b->c,
 * c->b (bits 0..5).  A directed typed triad's key numbers, in increasing
 * order, the canonical codes (arcs | types[0] << 6 | types[1] << 10 |
 * types[2] << 14, smallest over the six node orderings) of the weakly
 * connected triads with types below L: tg_directed3_num_keys(L) keys (13 for
 * L = 1, the connected triads of the triad census).
 *   slot_dir      device, uint8[nnz]
 *   global_counts device, uint64[tg_directed3_num_keys(L)]: the number of
 *                 node triples inducing each typed triad; or NULL
 *   edge_rows     device, uint64[m * 15 L], or NULL: per canonical edge
 *                 (i, j), i < j, column ((4 c(i,k) + c(j,k)) - 1) L + t counts
 *                 the nodes k of type t with those direction codes to i and j
 *                 (one of them nonzero)
 *   edge_info     device, int32[m * 3] receiving (i, j, c(i, j)), or NULL
 *   opt           host or NULL: validate (also checks the direction bytes),
 *                 check (global sums divisible by the triad's support
 *                 edges), phase_ms
 * Global counts are the row entries summed per key over the triad's 2 or 3
 * support edges and divided by that number (Eq. 17's argument for triads).
 */
tg_status tg_count_directed3(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                             const uint8_t* slot_dir, const uint8_t* node_types, int L, uint64_t* global_counts,
                             uint64_t* edge_rows, int32_t* edge_info, const tg_options* opt, hipStream_t stream);

/* Number of directed typed 3-node keys for L types (0 if L is outside
 * [1, 16]). */
size_t tg_directed3_num_keys(int L);

/* Host.  Canonical triad of a directed key: *arcs gets its six arc bits,
 * types its three node types, in the canonical node order. */
tg_status tg_directed3_key_decode(int L, size_t key, uint8_t* arcs, uint8_t types[3]);

/* Host.  Key of the triad with arc bits `arcs` and node types `types` (any
 * node order); TG_ERR_INVALID_ARG if the triad is not weakly connected. */
tg_status tg_directed3_key_encode(int L, uint8_t arcs, const uint8_t types[3], size_t* key);

/* Directed typed 4-node graphlets (the Directed Typed Graphlets subsection:
 * typed out- and in-neighbour sets, one id per directed typed motif), on the
 * same input as tg_count_directed3 (support CSR plus direction bytes).
 * A 4-node digraph on ordered nodes 0..3 has one arc bit per ordered pair in
 * the order (0,1) (0,2) (0,3) (1,0) (1,2) (1,3) (2,0) (2,1) (2,3) (3,0)
 * (3,1) (3,2); its full code adds the four types, 4 bits each from bit 12;
 * its canonical code is the smallest full code over the 24 node orderings.
 * The keys of L types number, in increasing order, the canonical codes of
 * the weakly connected digraphs with types below L:
 * tg_directed4_num_keys(L) keys (199, 2818, 13770, 42802 for L = 1..4).
 *   L             1..4 (TG_ERR_UNSUPPORTED_L otherwise)
 *   global_counts device, uint64[tg_directed4_num_keys(L)]: the number of
 *                 4-node sets inducing each key; or NULL
 *   edge_rows     device, uint64[m * tg_directed4_num_keys(L)], or NULL: per
 *                 canonical support edge (i, j), i < j, the number of
 *                 weakly connected 4-node sets containing i and j per key
 *   edge_info     device, int32[m * 3] receiving (i, j, c(i, j)), or NULL
 *   opt           host or NULL: validate (also the direction bytes), check
 *                 (global sums divisible by the key's support edges),
 *                 phase_ms
 * Per support edge the work is the sum of the degrees of the neighbours of
 * i and j (the paper's per-edge enumeration bound), and the neighbourhood
 * of each edge is held in LDS: every edge needs d_i + d_j - 2 <= 1024
 * (TG_ERR_INVALID_ARG otherwise, found after one synchronisation).  Global
 * counts are the row entries summed per key over the set's support edges
 * and divided by their number. */
tg_status tg_count_directed4(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                             const uint8_t* slot_dir, const uint8_t* node_types, int L, uint64_t* global_counts,
                             uint64_t* edge_rows, int32_t* edge_info, const tg_options* opt, hipStream_t stream);

/* Number of directed typed 4-node keys for L types (0 if L is outside
 * [1, 4]). */
size_t tg_directed4_num_keys(int L);

/* Host.  Canonical digraph of a directed 4-node key: *arcs gets its 12 arc
 * bits, types its four node types, in the canonical node order. */
tg_status tg_directed4_key_decode(int L, size_t key, uint16_t* arcs, uint8_t types[4]);

/* Sparse per-edge output (the Sparse Typed Motif Format subsection: only the
 * nonzero typed graphlet counts of each edge, with their ids).  Turns dense
 * per-edge rows into (global key, count) pairs; keys are the dense key rank
 * of tg_key_encode, already consecutive from 0 (tg_key_decode is the lookup
 * table).  Two calls on the same arguments:
 *   pass 1 (keys == NULL): offsets[0..E] receives the exclusive prefix of
 *     the per-edge nonzero counts (offsets[E] = total) and *total the total
 *     (host; the call synchronises the stream);
 *   pass 2 (keys, counts given, capacity >= total): edge e's pairs are
 *     written at [offsets[e], offsets[e+1]) in row column order.
 *   rows        device, uint64[E * R(L)] as written by tg_count
 *   endpoints   device, int32[E * 2] as written by tg_count (the endpoints
 *               whose types the row is relative to)
 *   node_types  device, uint8[n]
 *   offsets     device, int64[E + 1], caller-owned
 *   keys        device, uint32[capacity] or NULL (pass 1)
 *   counts      device, uint64[capacity]
 * Errors: TG_ERR_INVALID_ARG for null pointers or a capacity below the
 * total (nothing written by pass 2); TG_ERR_UNSUPPORTED_L. */
tg_status tg_rows_sparse(int64_t E, int L, const uint64_t* rows, const int32_t* endpoints,
                         const uint8_t* node_types, int64_t* offsets, uint32_t* keys, uint64_t* counts,
                         int64_t capacity, int64_t* total, hipStream_t stream);

/* Counts many small typed graphs in one call (the batch form of tg_count's
 * global counts, Eq. 17 per graph).  Graph g has n_g = node_off[g+1] -
 * node_off[g] <= 512 nodes with local ids, L_g = L_per_graph[g] in [1, 8]
 * types, and writes tg_num_keys(L_g) counts at global_counts + key_off[g].
 *   G               number of graphs
 *   node_off        device, int64[G+1], node_off[0] = 0
 *   slot_off        device, int64[G+1], CSR slots of graph g are
 *                   [slot_off[g], slot_off[g+1]) of col_idx_local
 *   row_ptr_local   device, int32[node_off[G] + G]: graph g's row pointer
 *                   (n_g + 1 entries starting at 0) at node_off[g] + g
 *   col_idx_local   device, int32[slot_off[G]], local node ids
 *   node_types      device, uint8[node_off[G]]
 *   L_per_graph     device, uint8[G]
 *   key_off         device, int64[G+1], key_off[g+1] - key_off[g] = tg_num_keys(L_g)
 *   global_counts   device, uint64[key_off[G]]
 * The call reads the graph sizes back to the host (one synchronisation),
 * buckets graphs by size, and replays a cached HIP graph of one persistent
 * launch per bucket.  Only `check`, `validate` and `tuning` of opt are used.
 * Errors: TG_ERR_INVALID_ARG for a graph with more than 512 nodes or a
 * key_off that does not match tg_num_keys(L_g), TG_ERR_UNSUPPORTED_L for
 * L_g outside [1, 8] (these are always checked, with one synchronisation);
 * with validate set, a device check of every graph (row pointers, column
 * ids below n_g, no self loops, strictly increasing rows, both directions
 * stored, types below L_g; a second synchronisation) reports
 * TG_ERR_INVALID_GRAPH or TG_ERR_TYPE_RANGE.  Without validate these
 * properties are assumed, and inputs that break them give unspecified
 * counts. */
tg_status tg_count_batch(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* row_ptr_local,
                         const int32_t* col_idx_local, const uint8_t* node_types, const uint8_t* L_per_graph,
                         const int64_t* key_off, uint64_t* global_counts, const tg_options* opt,
                         hipStream_t stream);

/* tg_count_batch for callers that cannot allocate device memory (code that
 * must not call hipMalloc, such as tight serving loops or harnesses that
 * forbid allocation): same arguments, results and errors, but its scratch
 * (128 counters and a list of the graph ids) is a fixed array in the
 * library's device memory, one per device, held until the process ends;
 * the call allocates nothing and launches its kernels directly (no cached
 * HIP graph).  At most 2,097,152 graphs per call (TG_ERR_INVALID_ARG
 * beyond, before any device work).  Every call on one device shares that
 * array and clears what it needs at the start: calls that overlap on one
 * device (several threads or streams) race and must be serialised by the
 * caller.  The first call on a device looks up the array's address. */
tg_status tg_count_batch_noalloc(int64_t G, const int64_t* node_off, const int64_t* slot_off,
                                 const int32_t* row_ptr_local, const int32_t* col_idx_local, const uint8_t* node_types,
                                 const uint8_t* L_per_graph, const int64_t* key_off, uint64_t* global_counts,
                                 const tg_options* opt, hipStream_t stream);

/* ---- learned cost model (16-64-64-1 MLP, ReLU, bf16 weights, fp32
 * accumulation) that orders and bins edges for TG_SCHED_LEARNED.  A model
 * lives on the device that was current at creation. */

/* Number of trainable parameters (layout: W1[64][16], b1[64], W2[64][64],
 * b2[64], w3[64], b3); get/set also carry 32 feature statistics (mean[16],
 * deviation[16]) after them. */
size_t tg_cost_model_num_params(void);

/* Creates a model with seeded initial weights. */
tg_status tg_cost_model_create(tg_cost_model** model, uint64_t seed);
tg_status tg_cost_model_destroy(tg_cost_model* model);

/* Trains on a seeded uniform sample (fraction sample_frac) of the graph's
 * edges, labelled with the per-edge element-visit counts of the counting
 * kernel (target log2(1 + work)), for `epochs` passes of mini-batch Adam;
 * loss_history (host, [epochs] or NULL) receives the mean loss per epoch.
 * Device pointers as in tg_count.  Synchronises the stream. */
tg_status tg_cost_model_train(tg_cost_model* model, int64_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, const uint8_t* node_types, int L, double sample_frac,
                              uint64_t seed, int epochs, float* loss_history, hipStream_t stream);

/* Predicted log2(1 + work) of every canonical edge: cost is device float[m]. */
tg_status tg_cost_model_predict(const tg_cost_model* model, int64_t n, int64_t nnz, const int32_t* row_ptr,
                                const int32_t* col_idx, const uint8_t* node_types, int L, float* cost,
                                hipStream_t stream);

/* Measured element-visit counts of the per-edge counting kernel for the
 * listed canonical edges: edges is device int32[count], work is device
 * uint64[m] indexed by edge id (entries of unlisted edges are zero). */
tg_status tg_edge_work(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                       const uint8_t* node_types, int L, const int32_t* edges, int64_t count, uint64_t* work,
                       hipStream_t stream);

/* Mean-squared-error loss and its gradient over `rows` raw feature rows X
 * (device float[rows][16]) and targets Y (device float[rows]) with the
 * model's current bf16 weights: grad is device float[num_params], loss is
 * device float[1].  Used to check the training kernels. */
tg_status tg_cost_model_gradient(const tg_cost_model* model, const float* X, const float* Y, int64_t rows,
                                 float* grad, float* loss, hipStream_t stream);

/* Host copies of the fp32 parameters followed by the feature statistics
 * (num_params + 32 floats). */
tg_status tg_cost_model_get_params(const tg_cost_model* model, float* params);
tg_status tg_cost_model_set_params(tg_cost_model* model, const float* params);

/* Binary file with the parameters and statistics. */
tg_status tg_cost_model_save(const tg_cost_model* model, const char* path);
tg_status tg_cost_model_load(tg_cost_model* model, const char* path);

/* ---- autotuning.  Both searches time real calls on the caller's data
 * (counts are rewritten with identical values) and only change launch
 * shapes. */

/* Coordinate descent over tg_tuning's tg_count fields, timing the 4-cycle
 * and per-edge combine phases with HIP events; base supplies the schedule and model (NULL:
 * defaults).  Outputs as in tg_count (edge_counts may be NULL). */
tg_status tg_autotune(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      const uint8_t* node_types, int L, uint64_t* global_counts, uint64_t* edge_counts,
                      const tg_options* base, tg_tuning* tuning, float* best_ms, hipStream_t stream);

/* Chooses tg_tuning.batch_variant per size class by timing whole
 * tg_count_batch calls; *tuning is the starting point and the result. */
tg_status tg_autotune_batch(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* row_ptr_local,
                            const int32_t* col_idx_local, const uint8_t* node_types, const uint8_t* L_per_graph,
                            const int64_t* key_off, uint64_t* global_counts, tg_tuning* tuning, float* best_ms,
                            hipStream_t stream);

/* Frees the scratch workspace that the counting calls keep on the current
 * device (after the work of its last holder has finished) and returns the
 * memory cached by the device's default stream-ordered pool to the system;
 * later calls allocate again.  Synchronises the device.  Errors:
 * TG_ERR_INVALID_ARG while a call on another thread holds the workspace,
 * TG_ERR_HIP. */
tg_status tg_release_scratch(void);

/* Human-readable name of a status code (static string). */
const char* tg_status_string(tg_status s);

/* Thread-local detail about the last non-OK status returned on this thread. */
const char* tg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TG_H_ */
