/*
 * Oracle for per-edge typed 3/4-node graphlet counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * Two independent counters live here, both plain, slow and single-purpose:
 *
 *  1. or_brute: the definition.  Every 3- and 4-node subset of V is taken,
 *     its induced subgraph is built, connectivity is checked and the shape is
 *     classified; each edge inside the subgraph is credited with
 *     (shape, multiset of node types) -- the typed graphlet of Definition
 *     "Typed Graphlet" / "Typed Graphlet Instance" (Section 3.2) and the local
 *     counting problem of Section 4 (Definition "Local Typed Graphlet
 *     Counting").  Orbit roles (g1..g12 of Table 3) are credited as well.
 *
 *  2. or_count_edges / or_count_all: the same definition, written per edge
 *     (the local counting problem of Section 4): the other two nodes of
 *     every connected induced 4-node subgraph through edge (i, j) are
 *     classified by their adjacency to i and j (the sets T_ij, S_i, S_j of
 *     Section 4.1 and the rest), each configuration's shape is found from
 *     its explicit 4-node adjacency, and non-adjacent pairs inside the
 *     neighbourhood are counted as all pairs minus the adjacent ones.  Its
 *     cost per edge is the sum of the degrees of the neighbours of i and j,
 *     the bound of Theorem 2.  Global counts follow from Eq. 17.  The
 *     paper's Eqs. 7-10 (g4, g5, g9, g11 from g6, g7, g10, g12 and the set
 *     sizes) are not used here; tests check them against these counts.
 *
 * Readings of points the paper leaves open (each is also listed with the
 * design notes of the repository):
 *  - T_ij is the intersection of the neighbourhoods (Sections 4.1 and 4.3).
 *  - S_i excludes j (left-hand form of the S_i definition, Section 4.1).
 *  - Every S-based orbit covers both the S_i and the S_j side.
 *  - The graph is undirected and simple; only node types are used.
 *  - Keys are (graphlet shape h1..h8, sorted multiset of node types); the
 *    paper's decimal hash (Eqs. 18-19) is replaced by a dense rank, which is
 *    equally invertible (Section 4.5 requires only invertibility).
 *  - Counters are 64-bit.
 *
 * Layouts (shared with the library only as a documented format):
 *  - Canonical edge order: e-th slot (i, j) with i < j of the CSR, row-major.
 *  - Per-edge graphlet row, relative to (phi_i, phi_j): wedge[t] (t < L),
 *    triangle[t], then for h3..h8 a block of P = L(L+1)/2 entries indexed by
 *    p(t, u) = u(u+1)/2 + t with t <= u (types of the two other nodes).
 *    Width R(L) = 2L + 6P.
 *  - Per-edge orbit row: g1[t], g2[t], then g3..g12 blocks of P entries.
 *    Width 2L + 10P.
 *  - Global key = shape offset + rank of the sorted type multiset; 3-node
 *    rank of a<=b<=c is C(a,1)+C(b+1,2)+C(c+2,3), 4-node adds C(d+3,4).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_NOT_DIVISIBLE -2
#define OR_ERR_NOMEM -3

/* ---------------------------------------------------------------- keys -- */

static int64_t binom(int64_t n, int64_t k) {
  if (k < 0 || n < k) return 0;
  int64_t r = 1;
  for (int64_t q = 1; q <= k; ++q) r = r * (n - k + q) / q;
  return r;
}

/* Number of typed graphlets of one shape with K nodes and L types: the
 * multiset coefficient C(L+K-1, K) (Eq. 1, Table 2). */
int64_t or_typed_per_shape(int L, int K) { return binom(L + K - 1, K); }

int64_t or_num_keys(int L) { return 2 * or_typed_per_shape(L, 3) + 6 * or_typed_per_shape(L, 4); }
int64_t or_row_width(int L) { return 2 * (int64_t)L + 3 * (int64_t)L * (L + 1); }
int64_t or_orbit_row_width(int L) { return 2 * (int64_t)L + 5 * (int64_t)L * (L + 1); }

static void sort_small(int* v, int k) {
  for (int a = 1; a < k; ++a) {
    int x = v[a], b = a - 1;
    while (b >= 0 && v[b] > x) { v[b + 1] = v[b]; --b; }
    v[b + 1] = x;
  }
}

/* rank of a multiset of k types (k = 3 or 4) in colex order */
int64_t or_rank(int k, const int* types) {
  int v[4];
  for (int a = 0; a < k; ++a) v[a] = types[a];
  sort_small(v, k);
  int64_t r = 0;
  for (int a = 0; a < k; ++a) r += binom(v[a] + a, a + 1);
  return r;
}

/* shape index h = 0..7 for h1..h8 (wedge, triangle, 4-path, 4-star, 4-cycle,
 * tailed triangle, chordal cycle, 4-clique) */
int64_t or_shape_offset(int L, int h) {
  int64_t c3 = or_typed_per_shape(L, 3), c4 = or_typed_per_shape(L, 4);
  if (h <= 2) return h * c3;
  return 2 * c3 + (h - 2) * c4;
}

int64_t or_key(int L, int h, const int* types) {
  return or_shape_offset(L, h) + or_rank(h < 2 ? 3 : 4, types);
}

/* number of edges of each shape h1..h8 (divisor of Eq. 17) */
static const int kShapeEdges[8] = {2, 3, 3, 3, 4, 4, 5, 6};

static inline uint64_t choose2(uint64_t x) { return x ? x * (x - 1) / 2 : 0; }

static inline int64_t pair_index(int t, int u) {
  if (t > u) { int s = t; t = u; u = s; }
  return (int64_t)u * (u + 1) / 2 + t;
}

/* ------------------------------------------------------- the definition -- */

/* Shape of a connected 4-node graph with ne edges and node degrees deg[4]
 * (h = 2..7: 4-path, 4-star, 4-cycle, tailed triangle, chordal cycle,
 * 4-clique; Section 3.1's 4-node graphlets). */
static int shape4(int ne, const int* deg) {
  int maxd = 0;
  for (int x = 0; x < 4; ++x) if (deg[x] > maxd) maxd = deg[x];
  if (ne == 3) return (maxd == 3) ? 3 : 2;       /* star : path */
  if (ne == 4) return (maxd == 3) ? 5 : 4;       /* tailed triangle : cycle */
  if (ne == 5) return 6;                         /* chordal cycle */
  return 7;                                      /* clique */
}

/* Orbit g3..g12 of Table 3 of an edge whose ends have degrees dx, dy inside a
 * 4-node graphlet of shape h. */
static int orbit4(int h, int dx, int dy) {
  const int lo = dx < dy ? dx : dy, hi = dx < dy ? dy : dx;
  switch (h) {
    case 2: return (lo == 2 && hi == 2) ? 4 : 3;        /* 4-path: centre : end */
    case 3: return 5;                                   /* 4-star */
    case 4: return 6;                                   /* 4-cycle */
    case 5: return (lo == 1) ? 7 : (hi == 3 ? 9 : 8);   /* tailed triangle: tail, tri-edge at the centre, far */
    case 6: return (lo == 3) ? 11 : 10;                 /* chordal cycle: chord : rim */
    default: return 12;                                 /* 4-clique */
  }
}

/* Brute force over all 3- and 4-subsets.  adjacency is read from a CSR with
 * both directions stored.  rows: [m][R(L)] graphlet rows in canonical edge
 * order (may be NULL); orbit_rows: [m][2L+10P] (may be NULL); global: [K(L)]
 * (may be NULL) receives the number of subgraphs per key.  Requires n <= 64. */
int or_brute(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* types, int L,
             uint64_t* rows, uint64_t* orbit_rows, uint64_t* global) {
  if (n < 0 || n > 64 || L < 1) return OR_ERR_ARG;
  uint64_t adj[64];
  int64_t eid[64][64];
  memset(adj, 0, sizeof(adj));
  for (int a = 0; a < 64; ++a)
    for (int b = 0; b < 64; ++b) eid[a][b] = -1;
  int64_t m = 0;
  for (int64_t a = 0; a < n; ++a)
    for (int32_t s = row_ptr[a]; s < row_ptr[a + 1]; ++s) {
      int64_t b = col_idx[s];
      adj[a] |= 1ull << b;
      if (a < b) { eid[a][b] = eid[b][a] = m++; }
    }
  const int64_t R = or_row_width(L), RO = or_orbit_row_width(L), P = (int64_t)L * (L + 1) / 2;
  if (rows) memset(rows, 0, sizeof(uint64_t) * m * R);
  if (orbit_rows) memset(orbit_rows, 0, sizeof(uint64_t) * m * RO);
  if (global) memset(global, 0, sizeof(uint64_t) * or_num_keys(L));

  /* 3-node subsets */
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b)
      for (int c = b + 1; c < n; ++c) {
        int v[3] = {a, b, c};
        int ne = 0;
        for (int x = 0; x < 3; ++x)
          for (int y = x + 1; y < 3; ++y) ne += (adj[v[x]] >> v[y]) & 1;
        if (ne < 2) continue; /* 2 edges on 3 nodes is always connected */
        int h = (ne == 2) ? 0 : 1;
        int ty[3] = {types[a], types[b], types[c]};
        if (global) global[or_key(L, h, ty)]++;
        for (int x = 0; x < 3; ++x)
          for (int y = x + 1; y < 3; ++y) {
            if (!((adj[v[x]] >> v[y]) & 1)) continue;
            int z = 3 - x - y;
            int64_t e = eid[v[x]][v[y]];
            if (rows) rows[e * R + (int64_t)h * L + types[v[z]]]++;
            if (orbit_rows) orbit_rows[e * RO + (int64_t)h * L + types[v[z]]]++;
          }
      }
  /* 4-node subsets */
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b)
      for (int c = b + 1; c < n; ++c)
        for (int d = c + 1; d < n; ++d) {
          int v[4] = {a, b, c, d};
          int deg[4] = {0, 0, 0, 0};
          int ne = 0;
          for (int x = 0; x < 4; ++x)
            for (int y = x + 1; y < 4; ++y)
              if ((adj[v[x]] >> v[y]) & 1) { ++ne; deg[x]++; deg[y]++; }
          if (ne < 3) continue;
          /* connectivity: grow from v[0] inside the subset */
          int seen = 1, grew = 1;
          while (grew) {
            grew = 0;
            for (int x = 0; x < 4; ++x)
              if ((seen >> x) & 1)
                for (int y = 0; y < 4; ++y)
                  if (!((seen >> y) & 1) && ((adj[v[x]] >> v[y]) & 1)) { seen |= 1 << y; grew = 1; }
          }
          if (seen != 15) continue;
          const int h = shape4(ne, deg);
          int ty[4] = {types[a], types[b], types[c], types[d]};
          if (global) global[or_key(L, h, ty)]++;
          for (int x = 0; x < 4; ++x)
            for (int y = x + 1; y < 4; ++y) {
              if (!((adj[v[x]] >> v[y]) & 1)) continue;
              int o[2], q = 0;
              for (int z = 0; z < 4; ++z) if (z != x && z != y) o[q++] = z;
              int64_t e = eid[v[x]][v[y]];
              int64_t p = pair_index(types[v[o[0]]], types[v[o[1]]]);
              if (rows) rows[e * R + 2 * L + (int64_t)(h - 2) * P + p]++;
              if (orbit_rows) orbit_rows[e * RO + 2 * L + (int64_t)(orbit4(h, deg[x], deg[y]) - 3) * P + p]++;
            }
        }
  return OR_OK;
}

/* ------------------------------------------------ per edge, by definition */

/* Per-edge counts straight from the local counting problem of Section 4:
 * for edge (i, j), every other node k adjacent to i or j has a class
 *   cls(k) = [k ~ i] + 2 [k ~ j]  (1: only i, the set S_i; 2: only j, S_j;
 *                                  3: both, T_ij),
 * and a connected induced 4-node subgraph {i, j, k, l} has either
 *   (a) k in that neighbourhood U and l outside U, adjacent to k only
 *       (reached through k), or
 *   (b) both k and l in U.
 * Each configuration is written out as a 4-node adjacency (nodes 0, 1 = i, j;
 * 2, 3 = k, l) and classified with the same shape and orbit functions as the
 * brute force.  Configurations of (a) and the adjacent pairs of (b) are
 * enumerated one by one; the non-adjacent pairs of (b) are counted per
 * (class, type) combination as all pairs minus the adjacent ones.  3-node
 * subgraphs {i, j, k}: a triangle when cls(k) = 3, else a wedge (3-path). */

typedef struct {
  int L;
  uint8_t* cls;   /* n entries: class of each node for the current edge, 0 elsewhere */
  int32_t* U;     /* members of U */
  uint64_t* cnt;  /* [4][L]: |class c of type t| */
  uint64_t* adjc; /* [4][L][4][L]: adjacent ordered pairs inside U by (class, type) */
} or_work;

static int work_init(or_work* w, int64_t n, int64_t maxdeg, int L) {
  memset(w, 0, sizeof(*w));
  w->L = L;
  w->cls = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  w->U = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * maxdeg + 1));
  w->cnt = (uint64_t*)malloc(sizeof(uint64_t) * 4 * L);
  w->adjc = (uint64_t*)malloc(sizeof(uint64_t) * 16 * L * L);
  if (!w->cls || !w->U || !w->cnt || !w->adjc) return OR_ERR_NOMEM;
  return OR_OK;
}

static void work_free(or_work* w) {
  free(w->cls); free(w->U); free(w->cnt); free(w->adjc);
}

/* Shape and orbit of edge (0, 1) in the 4-node graph {i, j, k, l} whose
 * other edges are: k-i iff (ck & 1), k-j iff (ck & 2), l-i iff (cl & 1),
 * l-j iff (cl & 2), k-l iff kl.  Returns -1 if it is not connected. */
static int classify_config(int ck, int cl, int kl, int* orbit) {
  int adj[4][4];
  memset(adj, 0, sizeof(adj));
  adj[0][1] = adj[1][0] = 1;
  adj[2][0] = adj[0][2] = ck & 1;
  adj[2][1] = adj[1][2] = (ck >> 1) & 1;
  adj[3][0] = adj[0][3] = cl & 1;
  adj[3][1] = adj[1][3] = (cl >> 1) & 1;
  adj[2][3] = adj[3][2] = kl;
  int deg[4] = {0, 0, 0, 0}, ne = 0;
  for (int x = 0; x < 4; ++x)
    for (int y = x + 1; y < 4; ++y)
      if (adj[x][y]) { ++ne; deg[x]++; deg[y]++; }
  int seen = 1, grew = 1;
  while (grew) {
    grew = 0;
    for (int x = 0; x < 4; ++x)
      if ((seen >> x) & 1)
        for (int y = 0; y < 4; ++y)
          if (!((seen >> y) & 1) && adj[x][y]) { seen |= 1 << y; grew = 1; }
  }
  if (seen != 15) return -1;
  const int h = shape4(ne, deg);
  *orbit = orbit4(h, deg[0], deg[1]);
  return h;
}

/* classify_config for every (ck, cl, kl): the shapes and orbits of the 32
 * configurations, computed once by that function. */
typedef struct { int h, orbit; } or_config;
static or_config g_config[4][4][2];
static int g_config_ready = 0;

static void config_table_init(void) {
  if (g_config_ready) return;
  for (int ck = 0; ck < 4; ++ck)
    for (int cl = 0; cl < 4; ++cl)
      for (int kl = 0; kl < 2; ++kl) {
        int orb = 0;
        const int h = classify_config(ck, cl, kl, &orb);
        g_config[ck][cl][kl].h = h;
        g_config[ck][cl][kl].orbit = orb;
      }
  g_config_ready = 1;
}

/* Counts one edge (i, j) into a graphlet row (width R) and, optionally, an
 * orbit row (width 2L + 10P). */
static void count_edge(or_work* w, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* phi,
                       int32_t i, int32_t j, uint64_t* row, uint64_t* orow) {
  const int L = w->L;
  const int64_t P = (int64_t)L * (L + 1) / 2, R = 2 * L + 6 * P, RO = 2 * L + 10 * P;
  uint8_t* cls = w->cls;
  memset(row, 0, sizeof(uint64_t) * R);
  if (orow) memset(orow, 0, sizeof(uint64_t) * RO);
  memset(w->cnt, 0, sizeof(uint64_t) * 4 * L);
  memset(w->adjc, 0, sizeof(uint64_t) * 16 * L * L);
#define CNT(c, t) w->cnt[(c) * L + (t)]
#define ADJC(c1, t1, c2, t2) w->adjc[(((int64_t)(c1) * L + (t1)) * 4 + (c2)) * L + (t2)]
  /* classes of the neighbours of i and j (i and j themselves excluded) */
  int64_t nU = 0;
  for (int32_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s)
    if (col_idx[s] != j) cls[col_idx[s]] |= 1;
  for (int32_t s = row_ptr[j]; s < row_ptr[j + 1]; ++s)
    if (col_idx[s] != i) cls[col_idx[s]] |= 2;
  for (int32_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s)
    if (col_idx[s] != j) w->U[nU++] = col_idx[s];
  for (int32_t s = row_ptr[j]; s < row_ptr[j + 1]; ++s)
    if (col_idx[s] != i && cls[col_idx[s]] == 2) w->U[nU++] = col_idx[s];
  /* 3-node subgraphs */
  for (int64_t a = 0; a < nU; ++a) {
    const int32_t k = w->U[a];
    const int c = cls[k];
    CNT(c, phi[k])++;
    const int h = c == 3 ? 1 : 0;
    row[(int64_t)h * L + phi[k]]++;
    if (orow) orow[(int64_t)h * L + phi[k]]++;
  }
  /* (a) l outside U and not i or j, adjacent to k in U; (b) adjacent pairs
   * inside U, each once (from its smaller id) */
  for (int64_t a = 0; a < nU; ++a) {
    const int32_t k = w->U[a];
    const int ck = cls[k];
    for (int32_t s = row_ptr[k]; s < row_ptr[k + 1]; ++s) {
      const int32_t l = col_idx[s];
      if (l == i || l == j) continue;
      const int cl = cls[l];
      if (cl != 0) {
        ADJC(ck, phi[k], cl, phi[l])++;  /* every adjacent pair twice, once per order */
        if (l < k) continue;
      }
      const or_config c = g_config[ck][cl][1];
      const int64_t p = pair_index(phi[k], phi[l]);
      row[2 * L + (int64_t)(c.h - 2) * P + p]++;
      if (orow) orow[2 * L + (int64_t)(c.orbit - 3) * P + p]++;
    }
  }
  /* (b) non-adjacent pairs of U, per unordered (class, type) combination */
  for (int c1 = 1; c1 <= 3; ++c1)
    for (int t1 = 0; t1 < L; ++t1)
      for (int c2 = c1; c2 <= 3; ++c2)
        for (int t2 = (c2 == c1 ? t1 : 0); t2 < L; ++t2) {
          const int same = c1 == c2 && t1 == t2;
          const uint64_t all = same ? choose2(CNT(c1, t1)) : CNT(c1, t1) * CNT(c2, t2);
          const uint64_t adjacent = same ? ADJC(c1, t1, c2, t2) / 2 : ADJC(c1, t1, c2, t2);
          const uint64_t v = all - adjacent;
          if (!v) continue;
          const or_config c = g_config[c1][c2][0];
          const int64_t p = pair_index(t1, t2);
          row[2 * L + (int64_t)(c.h - 2) * P + p] += v;
          if (orow) orow[2 * L + (int64_t)(c.orbit - 3) * P + p] += v;
        }
#undef CNT
#undef ADJC
  /* reset the classes */
  for (int64_t a = 0; a < nU; ++a) cls[w->U[a]] = 0;
}

static int64_t max_degree(int64_t n, const int32_t* row_ptr) {
  int64_t d = 0;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] - row_ptr[v] > d) d = row_ptr[v + 1] - row_ptr[v];
  return d;
}

/* Per-edge rows for an explicit list of edges (ei[q], ej[q]), each an edge of
 * the graph.  rows: [ne][R(L)]; orbit_rows: [ne][2L+10P] or NULL.
 * nthreads > 1 splits the list into contiguous chunks, one mark table each. */
int or_count_edges(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* types, int L,
                   int64_t ne, const int32_t* ei, const int32_t* ej, uint64_t* rows, uint64_t* orbit_rows,
                   int nthreads) {
  if (n < 0 || L < 1 || ne < 0) return OR_ERR_ARG;
  const int64_t R = or_row_width(L), RO = or_orbit_row_width(L);
  const int64_t dmax = max_degree(n, row_ptr);
  int status = OR_OK;
  if (nthreads < 1) nthreads = 1;
  config_table_init();
#pragma omp parallel num_threads(nthreads) reduction(min : status)
  {
    or_work w;
    int st = work_init(&w, n, dmax, L);
    if (st != OR_OK) status = st;
    else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t q = 0; q < ne; ++q)
        count_edge(&w, row_ptr, col_idx, types, ei[q], ej[q], rows + q * R, orbit_rows ? orbit_rows + q * RO : NULL);
    }
    work_free(&w);
  }
  return status;
}

/* Global key of column c of a per-edge row for an edge with types (a, b). */
static int64_t row_key(int L, int a, int b, int64_t c) {
  const int64_t P = (int64_t)L * (L + 1) / 2;
  if (c < 2 * L) {
    int ty[3] = {a, b, (int)(c % L)};
    return or_key(L, (int)(c / L), ty);
  }
  int64_t h = (c - 2 * L) / P, p = (c - 2 * L) % P;
  int u = 0;
  while ((int64_t)(u + 1) * (u + 2) / 2 <= p) ++u;
  int t = (int)(p - (int64_t)u * (u + 1) / 2);
  int ty[4] = {a, b, t, u};
  return or_key(L, (int)h + 2, ty);
}

int64_t or_row_key(int L, int phi_i, int phi_j, int64_t col) { return row_key(L, phi_i, phi_j, col); }

/* All edges in canonical order.  rows: [m][R(L)] or NULL; global: [K(L)].
 * Global count = (sum over edges) / (edges of the shape), Eq. 17; returns
 * OR_ERR_NOT_DIVISIBLE if any sum is not a multiple of its divisor. */
int or_count_all(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* types, int L,
                 uint64_t* rows, uint64_t* global, int nthreads) {
  if (n < 0 || L < 1) return OR_ERR_ARG;
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int32_t s = row_ptr[v]; s < row_ptr[v + 1]; ++s) m += col_idx[s] > v;
  int32_t* ei = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
  int32_t* ej = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
  const int64_t R = or_row_width(L), K = or_num_keys(L);
  uint64_t* r = rows ? rows : (uint64_t*)malloc(sizeof(uint64_t) * (size_t)((m + 1) * R));
  if (!ei || !ej || !r) { free(ei); free(ej); if (!rows) free(r); return OR_ERR_NOMEM; }
  int64_t q = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int32_t s = row_ptr[v]; s < row_ptr[v + 1]; ++s)
      if (col_idx[s] > v) { ei[q] = (int32_t)v; ej[q] = col_idx[s]; ++q; }
  int st = or_count_edges(n, row_ptr, col_idx, types, L, m, ei, ej, r, NULL, nthreads);
  if (st == OR_OK && global) {
    memset(global, 0, sizeof(uint64_t) * K);
    for (int64_t e = 0; e < m; ++e)
      for (int64_t c = 0; c < R; ++c)
        if (r[e * R + c]) global[row_key(L, types[ei[e]], types[ej[e]], c)] += r[e * R + c];
    for (int h = 0; h < 8; ++h) {
      int64_t k0 = or_shape_offset(L, h), k1 = h < 7 ? or_shape_offset(L, h + 1) : K;
      for (int64_t k = k0; k < k1; ++k) {
        if (global[k] % kShapeEdges[h]) st = OR_ERR_NOT_DIVISIBLE;
        global[k] /= kShapeEdges[h];
      }
    }
  }
  free(ei); free(ej);
  if (!rows) free(r);
  return st;
}

/* Global counts of many independent graphs (the batch workload): graph g has
 * nodes [node_off[g], node_off[g+1]), its row pointer (n_g + 1 entries from
 * 0) at row_ptr + node_off[g] + g, local column ids at col_idx + slot_off[g],
 * L_g = Ls[g] types, and its K(L_g) counts go to global + key_off[g].  Each
 * graph is counted by or_count_all; graphs are spread over nthreads. */
int or_count_batch(int64_t G, const int64_t* node_off, const int64_t* slot_off, const int32_t* row_ptr,
                   const int32_t* col_idx, const uint8_t* types, const uint8_t* Ls, const int64_t* key_off,
                   uint64_t* global, int nthreads) {
  if (G < 0) return OR_ERR_ARG;
  int status = OR_OK;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(min : status)
  for (int64_t g = 0; g < G; ++g) {
    const int64_t n0 = node_off[g];
    const int st = or_count_all(node_off[g + 1] - n0, row_ptr + n0 + g, col_idx + slot_off[g], types + n0, Ls[g],
                                NULL, global + key_off[g], 1);
    if (st != OR_OK) status = st;
  }
  return status;
}
