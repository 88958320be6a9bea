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
 *  2. or_count_edges / or_count_all: the paper's method, step by step:
 *     Algorithm 1 (mark table Psi, typed sets T_ij^t, S_i^t, S_j^t),
 *     Algorithm 2 (path-based orbits g3, g6, g7), Algorithm 3 (triangle-based
 *     orbits g8, g10, g12), Eqs. 7-10 (g4, g5, g9, g11 derived per type pair),
 *     Eqs. 11-16 (orbits to graphlets) and Eq. 17 (global counts).
 *
 * Readings of points the paper leaves open (each is also listed with the
 * design notes of the repository):
 *  - T_ij is the intersection of the neighbourhoods (Sections 4.1 and 4.3).
 *  - S_i excludes j (left-hand form of the S_i definition, Section 4.1), so
 *    Algorithm 1's S_i loop skips j.
 *  - "w_r <= w_k" is the strict order w_r < w_k on node ids (no self loops).
 *  - i and j are skipped wherever they would be classified (Psi never marks
 *    them, so they would otherwise look like members of I).
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
          int maxd = 0;
          for (int x = 0; x < 4; ++x) if (deg[x] > maxd) maxd = deg[x];
          int h;
          if (ne == 3) h = (maxd == 3) ? 3 : 2;       /* star : path */
          else if (ne == 4) h = (maxd == 3) ? 5 : 4;  /* tailed triangle : cycle */
          else if (ne == 5) h = 6;                    /* chordal cycle */
          else h = 7;                                 /* clique */
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
              if (orbit_rows) {
                /* orbit of the edge inside its graphlet (Table 3) */
                int dx = deg[x], dy = deg[y], g;
                int lo = dx < dy ? dx : dy, hi = dx < dy ? dy : dx;
                switch (h) {
                  case 2: g = (lo == 2 && hi == 2) ? 4 : 3; break; /* centre : end */
                  case 3: g = 5; break;
                  case 4: g = 6; break;
                  case 5: g = (lo == 1) ? 7 : (hi == 3 ? 9 : 8); break; /* tail, tri-edge, tri-centre */
                  case 6: g = (lo == 3) ? 11 : 10; break; /* chord : rim */
                  default: g = 12; break;
                }
                orbit_rows[e * RO + 2 * L + (int64_t)(g - 3) * P + p]++;
              }
            }
        }
  return OR_OK;
}

/* ------------------------------------------------------ the paper's method */

/* Mark values of the table Psi (Table 1): 0 = unmarked (I, or i / j),
 * LAMBDA1 = only in Gamma_i, LAMBDA2 = only in Gamma_j, LAMBDA3 = both. */
enum { LAMBDA1 = 1, LAMBDA2 = 2, LAMBDA3 = 3 };

/* orbit slot of the explicit counters X[g][t][t'] */
enum { X_G3 = 0, X_G6, X_G7, X_G8, X_G10, X_G12, X_N };

typedef struct {
  int L;
  uint8_t* psi;   /* n marks */
  int32_t* Tset;  /* members of T_ij */
  int32_t* Siset; /* members of S_i */
  int32_t* Sjset; /* members of S_j */
  uint64_t *T, *Si, *Sj; /* |T^t|, |S_i^t|, |S_j^t| */
  uint64_t* X;    /* [X_N][L][L] ordered (type of w_k, type of w_r) */
} or_work;

static int work_init(or_work* w, int64_t n, int64_t maxdeg, int L) {
  memset(w, 0, sizeof(*w));
  w->L = L;
  w->psi = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  w->Tset = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
  w->Siset = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
  w->Sjset = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
  w->T = (uint64_t*)malloc(sizeof(uint64_t) * 3 * L);
  w->X = (uint64_t*)malloc(sizeof(uint64_t) * X_N * L * L);
  if (!w->psi || !w->Tset || !w->Siset || !w->Sjset || !w->T || !w->X) return OR_ERR_NOMEM;
  w->Si = w->T + L;
  w->Sj = w->T + 2 * L;
  return OR_OK;
}

static void work_free(or_work* w) {
  free(w->psi); free(w->Tset); free(w->Siset); free(w->Sjset); free(w->T); free(w->X);
}

#define XAT(w, g, t, u) ((w)->X[((int64_t)(g) * (w)->L + (t)) * (w)->L + (u)])

/* Symmetrised explicit count for the unordered type pair {t, u}. */
static uint64_t sym(const or_work* w, int g, int t, int u) {
  return t == u ? XAT(w, g, t, t) : XAT(w, g, t, u) + XAT(w, g, u, t);
}

/* Counts one edge (i, j) into a graphlet row (width R) and, optionally, an
 * orbit row (width 2L + 10P). */
static void count_edge(or_work* w, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* phi,
                       int32_t i, int32_t j, uint64_t* row, uint64_t* orow) {
  const int L = w->L;
  const int64_t P = (int64_t)L * (L + 1) / 2;
  uint8_t* psi = w->psi;
  int64_t nT = 0, nSi = 0, nSj = 0;
  memset(w->T, 0, sizeof(uint64_t) * 3 * L);
  memset(w->X, 0, sizeof(uint64_t) * X_N * L * L);

  /* Algorithm 1: mark Gamma_i (except j) with lambda1 */
  for (int32_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s)
    if (col_idx[s] != j) psi[col_idx[s]] = LAMBDA1;
  /* scan Gamma_j: triangle nodes (lambda3) and 3-path nodes centred at j (lambda2) */
  for (int32_t s = row_ptr[j]; s < row_ptr[j + 1]; ++s) {
    int32_t k = col_idx[s];
    if (k == i) continue;
    if (psi[k] == LAMBDA1) { psi[k] = LAMBDA3; w->Tset[nT++] = k; w->T[phi[k]]++; }
    else { psi[k] = LAMBDA2; w->Sjset[nSj++] = k; w->Sj[phi[k]]++; }
  }
  /* 3-path nodes centred at i: Gamma_i minus T_ij minus {j} */
  for (int32_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s) {
    int32_t k = col_idx[s];
    if (k == j || psi[k] != LAMBDA1) continue;
    w->Siset[nSi++] = k; w->Si[phi[k]]++;
  }

  /* Algorithm 2: path-based orbits from S_i, then S_j */
  for (int64_t a = 0; a < nSi; ++a) {
    int32_t wk = w->Siset[a];
    for (int32_t s = row_ptr[wk]; s < row_ptr[wk + 1]; ++s) {
      int32_t wr = col_idx[s];
      if (wr == i || wr == j) continue;
      if (psi[wr] == 0) XAT(w, X_G3, phi[wk], phi[wr])++;                       /* 4-path end edge */
      else if (psi[wr] == LAMBDA1 && wr < wk) XAT(w, X_G7, phi[wk], phi[wr])++; /* tailed-tri tail */
    }
  }
  for (int64_t a = 0; a < nSj; ++a) {
    int32_t wk = w->Sjset[a];
    for (int32_t s = row_ptr[wk]; s < row_ptr[wk + 1]; ++s) {
      int32_t wr = col_idx[s];
      if (wr == i || wr == j) continue;
      if (psi[wr] == 0) XAT(w, X_G3, phi[wk], phi[wr])++;
      else if (psi[wr] == LAMBDA2 && wr < wk) XAT(w, X_G7, phi[wk], phi[wr])++;
      else if (psi[wr] == LAMBDA1) XAT(w, X_G6, phi[wk], phi[wr])++;          /* 4-cycle */
    }
  }
  /* Algorithm 3: triangle-based orbits from T_ij */
  for (int64_t a = 0; a < nT; ++a) {
    int32_t wk = w->Tset[a];
    for (int32_t s = row_ptr[wk]; s < row_ptr[wk + 1]; ++s) {
      int32_t wr = col_idx[s];
      if (wr == i || wr == j) continue;
      if (psi[wr] == LAMBDA3) { if (wr < wk) XAT(w, X_G12, phi[wk], phi[wr])++; } /* 4-clique */
      else if (psi[wr] == LAMBDA1 || psi[wr] == LAMBDA2) XAT(w, X_G10, phi[wk], phi[wr])++; /* chordal rim */
      else XAT(w, X_G8, phi[wk], phi[wr])++;                                   /* tailed-tri centre */
    }
  }

  /* 3-node graphlets: typed 3-stars |S_i^t| + |S_j^t| and triangles |T^t| */
  const int64_t R = 2 * L + 6 * P;
  memset(row, 0, sizeof(uint64_t) * R);
  if (orow) memset(orow, 0, sizeof(uint64_t) * (2 * L + 10 * P));
  for (int t = 0; t < L; ++t) {
    row[t] = w->Si[t] + w->Sj[t];
    row[L + t] = w->T[t];
    if (orow) { orow[t] = row[t]; orow[L + t] = row[L + t]; }
  }
  /* type-pair loop: Eqs. 7-10 for t <= u, then Eqs. 11-16 */
  for (int u = 0; u < L; ++u)
    for (int t = 0; t <= u; ++t) {
      const uint64_t g3 = sym(w, X_G3, t, u), g6 = sym(w, X_G6, t, u), g7 = sym(w, X_G7, t, u);
      const uint64_t g8 = sym(w, X_G8, t, u), g10 = sym(w, X_G10, t, u), g12 = sym(w, X_G12, t, u);
      const uint64_t Si_t = w->Si[t], Si_u = w->Si[u], Sj_t = w->Sj[t], Sj_u = w->Sj[u];
      const uint64_t T_t = w->T[t], T_u = w->T[u];
      uint64_t g4, g5, g9, g11;
      if (t == u) {
        g4 = Si_t * Sj_t - g6;                                            /* Eq. 7 */
        g5 = choose2(Si_t) + choose2(Sj_t) - g7;                         /* Eq. 8 */
        g9 = T_t * (Si_t + Sj_t) - g10;                                   /* Eq. 9 */
        g11 = choose2(T_t) - g12;                                         /* Eq. 10 */
      } else {
        g4 = Si_t * Sj_u + Si_u * Sj_t - g6;
        g5 = Si_t * Si_u + Sj_t * Sj_u - g7;
        g9 = T_t * (Si_u + Sj_u) + T_u * (Si_t + Sj_t) - g10;
        g11 = T_t * T_u - g12;
      }
      const int64_t p = (int64_t)u * (u + 1) / 2 + t;
      uint64_t* H = row + 2 * L;
      H[0 * P + p] = g3 + g4;        /* Eq. 11: 4-path */
      H[1 * P + p] = g5;             /* Eq. 12: 4-star */
      H[2 * P + p] = g6;             /* Eq. 13: 4-cycle */
      H[3 * P + p] = g7 + g8 + g9;   /* Eq. 14: tailed triangle */
      H[4 * P + p] = g10 + g11;      /* Eq. 15: chordal cycle */
      H[5 * P + p] = g12;            /* Eq. 16: 4-clique */
      if (orow) {
        uint64_t* O = orow + 2 * L;
        const uint64_t g[10] = {g3, g4, g5, g6, g7, g8, g9, g10, g11, g12};
        for (int q = 0; q < 10; ++q) O[q * P + p] = g[q];
      }
    }

  /* reset Psi on Gamma_i and Gamma_j */
  for (int32_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s) psi[col_idx[s]] = 0;
  for (int32_t s = row_ptr[j]; s < row_ptr[j + 1]; ++s) psi[col_idx[s]] = 0;
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
