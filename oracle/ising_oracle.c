/*
 * ising_oracle.c -- plain, slow, obviously correct CPU reference for the
 * annealed Ising max-cut method of Cook, Zhao, Sato, Hiromoto and Tan,
 * "GPU Ising Computing for Combinatorial Optimization Problems in VLSI
 * Physical Design" (arXiv:1807.10750).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant
 * generator with the GPU library.  All arithmetic is integer and exact.
 *
 * What it computes, in the paper's terms:
 *   - local field and local spin update: Sec. II-A, Eq. (1)-(2);
 *   - global energy: Sec. II-A Eq. (3), Sec. III Eq. (5);
 *   - cut value: Sec. III Eq. (4);
 *   - annealing with a per-spin random flip of probability F_p, reduced each
 *     sweep: Sec. II-B and Sec. IV-B (Algorithm 2 and the flip mechanism
 *     described just before it).
 *
 * Readings taken where the paper is silent or ambiguous (each is listed in
 * the design notes of the repository):
 *   R1  Sign of the max-cut mapping.  Minimising -sum J s s with J = w
 *       aligns neighbours, i.e. minimises the cut; Eq. (4) is maximised by
 *       J = -w.  So the field is h_v = sum_u w_vu s_u and the update sets
 *       s_v = -sign(h_v).
 *   R2  Tie S = 0 (Eq. 2 allows either value): keep the current spin.
 *   R3  Initial spins: Philox-random +-1 (counter domain 1) or caller-given.
 *   R4  Update, then flip the updated value, immediately (Algorithm 2).
 *   R5  F_p schedule: integer thresholds T_t; flip iff a 32-bit uniform
 *       x < T_t.  p -> T = min(2^32-1, floor(p * 2^32)), linear in t.
 *   R6  Exactly M sweeps; the last linear threshold is T_end.
 *   R7  RNG: Philox4x32-10 with key = seed.  The flip draw of vertex v,
 *       sweep t, replica r is word (t mod 4) of the block at counter
 *       {v, t div 4, r, 0}, so one block serves four consecutive sweeps; the
 *       initial-spin draw of replica r is word (r mod 4) of the block at
 *       {v, 0, r div 4, 1}.  The paper only asks for one independent
 *       uniform per spin and sweep.
 *   R8  The RNG is keyed by the caller's vertex id.
 *   R9  Each unordered edge counted once in W, E and the cut.
 *   R10 Self-loops and duplicate edges are rejected; int8 weights; the
 *       field fits in int32 (checked).
 *   R14 External field (Eq. 1 and Eq. 3, which the max-cut mapping sets to
 *       zero in Sec. III): with J = -w the quantity whose sign sets the spin
 *       is S_v = h_v - sum_u w_vu s_u; s_v = +1 if S_v > 0, -1 if S_v < 0,
 *       unchanged if S_v = 0 (R2); the energy is
 *       H = sum_{u<v} w_uv s_u s_v - sum_v h_v s_v.  The cut ignores h.
 *       h is int32 and every row must keep sum |w| + |h_v| <= 2^30 - 1, which
 *       leaves headroom for exact integer arithmetic on 2 h.
 *   R15 Per-vertex flip temperature (not in the paper; it only lets a learned
 *       warm start choose how much each vertex is shaken): vertex v flips
 *       in sweep t iff its draw x < min(2^32 - 1, floor(T_t * m_v / 8))
 *       for an integer multiplier m_v in [0, 15]; m = 8 everywhere is the
 *       plain anneal, m = 0 never flips that vertex.  scale == NULL is m = 8.
 *   R12 The deterministic ("coloured") schedule: vertices are visited in
 *       (colour, id) order of a greedy colouring, sequentially.  Because no
 *       two vertices of one colour are adjacent, any order inside a colour
 *       class gives the same result; this is the checkerboard update the
 *       paper cites as prior art (Sec. IV-B), generalised to any graph.
 *   Jacobi variant: every vertex reads the spins as they stood at the start
 *       of the sweep; used only to bracket the asynchronous mode, in which a
 *       neighbour's value may be from the current or the previous sweep
 *       (Sec. IV-B).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_GRAPH 2
#define OR_ERR_SELF_LOOP 3
#define OR_ERR_DUPLICATE 4
#define OR_ERR_ASYMMETRIC 5
#define OR_ERR_OVERFLOW 6
#define OR_ERR_NOMEM 7
#define OR_ERR_INTERNAL 9

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  One round maps (c0,c1,c2,c3) with key (k0,k1)  */
/* to (hi(B*c2)^c1^k0, lo(B*c2), hi(A*c0)^c3^k1, lo(A*c0)) with the two      */
/* multipliers A, B below; the key is bumped by the two Weyl constants       */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_A = 0xD2511F53u;
static const uint32_t PHILOX_B = 0xCD9E8D57u;
static const uint32_t WEYL_0 = 0x9E3779B9u;
static const uint32_t WEYL_1 = 0xBB67AE85u;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t pa = (uint64_t)PHILOX_A * (uint64_t)c0;
    uint64_t pb = (uint64_t)PHILOX_B * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)pb;
    uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)pa;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += WEYL_0;
    k1 += WEYL_1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Word w of Philox4x32-10 at counter {a, b, c, d}, key {lo(seed), hi(seed)}. */
static uint32_t philox_word(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t w, uint64_t seed) {
  uint32_t ctr[4] = {a, b, c, d};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return out[w];
}

/* Flip draw of vertex v in sweep t for replica r (reading R7). */
static uint32_t flip_draw(uint32_t v, uint32_t t, uint32_t r, uint64_t seed) {
  return philox_word(v, t / 4u, r, 0u, t % 4u, seed);
}

/* Initial-spin draw of vertex v for replica r (reading R7). */
static uint32_t init_draw(uint32_t v, uint32_t r, uint64_t seed) {
  return philox_word(v, 0u, r / 4u, 1u, r % 4u, seed);
}

/* ------------------------------------------------------------------------ */
/* Flip-probability thresholds (reading R5).                                 */
/* ------------------------------------------------------------------------ */
static uint32_t prob_to_threshold(double p) {
  /* p * 2^32 is exact in binary64 (a power-of-two scale); the cast truncates. */
  double x = p * 4294967296.0;
  if (x >= 4294967295.0) return 4294967295u;
  return (uint32_t)x;
}

/* kind 0 = linear p_start -> p_end over M sweeps; fills T[0..M). */
int oracle_thresholds(int kind, double p_start, double p_end, int64_t M, uint32_t *T) {
  if (kind != 0 || M < 1 || T == NULL) return OR_ERR_ARG;
  if (!(p_start >= 0.0 && p_start <= 1.0 && p_end >= 0.0 && p_end <= 1.0)) return OR_ERR_ARG;
  uint32_t ts = prob_to_threshold(p_start);
  uint32_t te = prob_to_threshold(p_end);
  for (int64_t t = 0; t < M; ++t) {
    if (M == 1) { T[t] = ts; continue; }
    if (ts >= te) {
      unsigned __int128 step = (unsigned __int128)(ts - te) * (unsigned __int128)t / (unsigned __int128)(M - 1);
      T[t] = ts - (uint32_t)step;
    } else {
      unsigned __int128 step = (unsigned __int128)(te - ts) * (unsigned __int128)t / (unsigned __int128)(M - 1);
      T[t] = ts + (uint32_t)step;
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Graph validation (reading R10) and the total weight W (reading R9).      */
/* Checks run in this order, each over rows in id order: structure,         */
/* self-loop, duplicate, symmetry, field overflow.  The first failure wins; */
/* *bad_row / *bad_k name it.                                               */
/* ------------------------------------------------------------------------ */
static const int64_t *g_sym_row;
static const int32_t *g_sym_col;
static int cmp_entry_row_col(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  if (g_sym_row[x] != g_sym_row[y]) return g_sym_row[x] < g_sym_row[y] ? -1 : 1;
  if (g_sym_col[x] != g_sym_col[y]) return g_sym_col[x] < g_sym_col[y] ? -1 : 1;
  return 0;
}

int oracle_validate(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                    const int8_t *w, int64_t *W_out, int64_t *bad_row, int64_t *bad_k) {
  *bad_row = -1; *bad_k = -1;
  if (n < 0 || nnz < 0 || n > 2147483647LL - 64 || row_ptr == NULL) return OR_ERR_ARG;
  if (nnz > 0 && (col == NULL || w == NULL)) return OR_ERR_ARG;
  /* structure */
  if (row_ptr[0] != 0) { *bad_row = 0; return OR_ERR_GRAPH; }
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) { *bad_row = v; return OR_ERR_GRAPH; }
  if (row_ptr[n] != nnz) { *bad_row = n; return OR_ERR_GRAPH; }
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
      if (col[k] < 0 || (int64_t)col[k] >= n) { *bad_row = v; *bad_k = k; return OR_ERR_GRAPH; }
  /* self-loops */
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
      if ((int64_t)col[k] == v) { *bad_row = v; *bad_k = k; return OR_ERR_SELF_LOOP; }
  /* duplicates: last_row[u] == v marks u already seen in row v */
  int64_t *last_row = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!last_row) return OR_ERR_NOMEM;
  for (int64_t u = 0; u < n; ++u) last_row[u] = -1;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      if (last_row[col[k]] == v) { free(last_row); *bad_row = v; *bad_k = k; return OR_ERR_DUPLICATE; }
      last_row[col[k]] = v;
    }
  free(last_row);
  /* symmetry: entry (v -> u, w) needs an entry (u -> v, w).  Entries are
   * sorted by (row, col) once; each reverse entry is found by binary search. */
  {
    int64_t *rowof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!rowof || !idx) { free(rowof); free(idx); return OR_ERR_NOMEM; }
    for (int64_t v = 0; v < n; ++v)
      for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) { rowof[k] = v; idx[k] = k; }
    g_sym_row = rowof; g_sym_col = col;
    qsort(idx, (size_t)nnz, sizeof(int64_t), cmp_entry_row_col);
    for (int64_t k = 0; k < nnz; ++k) {
      int64_t v = rowof[k], u = col[k];
      int64_t lo = 0, hi = nnz, found = -1;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int64_t q = idx[mid];
        if (rowof[q] < u || (rowof[q] == u && (int64_t)col[q] < v)) lo = mid + 1;
        else hi = mid;
      }
      if (lo < nnz && rowof[idx[lo]] == u && (int64_t)col[idx[lo]] == v) found = idx[lo];
      if (found < 0 || w[found] != w[k]) {
        free(rowof); free(idx);
        *bad_row = v; *bad_k = k;
        return OR_ERR_ASYMMETRIC;
      }
    }
    free(rowof); free(idx);
  }
  /* the local field sum_u w_vu s_u must fit in int32 */
  for (int64_t v = 0; v < n; ++v) {
    int64_t s = 0;
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) s += (w[k] < 0) ? -(int64_t)w[k] : (int64_t)w[k];
    if (s > 2147483647LL) { *bad_row = v; return OR_ERR_OVERFLOW; }
  }
  int64_t W = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
      if (v < (int64_t)col[k]) W += w[k];
  *W_out = W;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Greedy colouring that defines the deterministic schedule (reading R12).  */
/* largest_first = 0: visit ids 0..n-1.  largest_first = 1: visit in        */
/* (degree descending, id ascending) order.  Each visited vertex takes the  */
/* smallest colour not used by an already-coloured neighbour.               */
/* ------------------------------------------------------------------------ */
static const int64_t *g_sort_deg;
static int cmp_deg_desc_id_asc(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  if (g_sort_deg[x] != g_sort_deg[y]) return g_sort_deg[x] > g_sort_deg[y] ? -1 : 1;
  return (x > y) - (x < y);
}

int oracle_color(int64_t n, const int64_t *row_ptr, const int32_t *col, int largest_first,
                 int32_t *color, int32_t *n_colors) {
  int32_t *visit = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *used_by = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!visit || !deg || !used_by) { free(visit); free(deg); free(used_by); return OR_ERR_NOMEM; }
  for (int64_t v = 0; v < n; ++v) { visit[v] = (int32_t)v; deg[v] = row_ptr[v + 1] - row_ptr[v]; color[v] = -1; }
  if (largest_first) { g_sort_deg = deg; qsort(visit, (size_t)n, sizeof(int32_t), cmp_deg_desc_id_asc); }
  for (int64_t c = 0; c <= n; ++c) used_by[c] = -1;
  int32_t nc = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t v = visit[i];
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      int32_t cu = color[col[k]];
      if (cu >= 0) used_by[cu] = v;
    }
    int32_t c = 0;
    while (used_by[c] == v) ++c;
    color[v] = c;
    if (c + 1 > nc) nc = c + 1;
  }
  *n_colors = nc;
  free(visit); free(deg); free(used_by);
  return OR_OK;
}

/* Vertices sorted by (colour, id): the sequential visiting order. */
void oracle_order(int64_t n, const int32_t *color, int32_t n_colors, int32_t *order) {
  int64_t pos = 0;
  for (int32_t c = 0; c < n_colors; ++c)
    for (int64_t v = 0; v < n; ++v)
      if (color[v] == c) order[pos++] = (int32_t)v;
}

/* ------------------------------------------------------------------------ */
/* Initial spins (reading R3): s = +1 if bit 31 of the domain-1 draw is set. */
/* spins is [R][n].                                                         */
/* ------------------------------------------------------------------------ */
void oracle_init_spins(int64_t n, int32_t R, uint64_t seed, int8_t *spins) {
  for (int32_t r = 0; r < R; ++r)
    for (int64_t v = 0; v < n; ++v) {
      uint32_t x = init_draw((uint32_t)v, (uint32_t)r, seed);
      spins[(int64_t)r * n + v] = (x >> 31) ? 1 : -1;
    }
}

/* Flip threshold of vertex v in a sweep with threshold T (R15). */
static uint32_t vertex_threshold(uint32_t T, const uint8_t *scale, int64_t v) {
  if (scale == NULL) return T;
  uint64_t x = ((uint64_t)T * (uint64_t)scale[v]) >> 3;
  return x > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)x;
}

/* Local field h_v = sum_u w_vu s_u (Eq. 2 with J = -w, reading R1). */
static int32_t local_field(int64_t v, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                           const int8_t *s) {
  int32_t h = 0;
  for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) h += (int32_t)w[k] * (int32_t)s[col[k]];
  return h;
}

/* Local spin update, Eq. (2): minimise H_v(s) = h_v * s over s in {-1,+1}
 * (R1), keeping the spin on a tie (R2). */
static int8_t local_update(int32_t h, int8_t s) {
  if (h > 0) return -1;
  if (h < 0) return 1;
  return s;
}

/* With an external field (R14): Eq. (1)-(2) give H_v(s) = -S_v s with
 * S_v = sum_u J_vu s_u + h_v = -(sum_u w_vu s_u) + h_v; the spin takes the
 * sign of S_v and keeps its value when S_v = 0.  field == NULL is h = 0. */
static int8_t field_update(int64_t v, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                           const int32_t *field, const int8_t *s_read, int8_t s_v) {
  if (field == NULL) return local_update(local_field(v, row_ptr, col, w, s_read), s_v);
  int64_t S = (int64_t)field[v];
  for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) S -= (int64_t)w[k] * (int64_t)s_read[col[k]];
  if (S > 0) return 1;
  if (S < 0) return -1;
  return s_v;
}

/* ------------------------------------------------------------------------ */
/* Deterministic anneal: Algorithm 2 with the parallel "for all" replaced   */
/* by a sequential visit in the given order (the (colour, id) order makes   */
/* this equal to any colour-phased parallel execution).  For each sweep t   */
/* in [t_begin, t_end): update each vertex from its local field, then flip  */
/* it when its flip draw is below T[t] (R4, R5, R7).  T holds the whole     */
/* schedule (indexed by absolute sweep).                                    */
/* ------------------------------------------------------------------------ */
int oracle_anneal(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                  const int32_t *field, const uint8_t *scale, const int32_t *order, int32_t R, int8_t *spins,
                  const uint32_t *T, uint64_t seed, int64_t t_begin, int64_t t_end) {
  if (t_begin < 0 || t_end < t_begin) return OR_ERR_ARG;
  for (int32_t r = 0; r < R; ++r) {
    int8_t *s = spins + (int64_t)r * n;
    for (int64_t t = t_begin; t < t_end; ++t) {
      for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i];
        s[v] = field_update(v, row_ptr, col, w, field, s, s[v]);
        if (flip_draw((uint32_t)v, (uint32_t)t, (uint32_t)r, seed) < vertex_threshold(T[t], scale, v))
          s[v] = (int8_t)-s[v];
      }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* The same deterministic anneal with each colour class swept by all host   */
/* threads at once (OpenMP).  No two vertices of a class are adjacent, so a */
/* vertex's field reads only spins of other classes, all final for this     */
/* phase: the result equals oracle_anneal in (colour, id) order bit for     */
/* bit, whatever the thread count.  Used to time the oracle on every core.  */
/* ------------------------------------------------------------------------ */
int oracle_anneal_colour_parallel(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                                  const int32_t *field, const uint8_t *scale, const int32_t *order,
                                  const int32_t *color,
                                  int32_t n_colors, int32_t R, int8_t *spins, const uint32_t *T, uint64_t seed,
                                  int64_t t_begin, int64_t t_end) {
  if (t_begin < 0 || t_end < t_begin || n_colors < 0) return OR_ERR_ARG;
  /* class c is order[first[c] .. first[c+1]) */
  int64_t *first = (int64_t *)calloc((size_t)n_colors + 2, sizeof(int64_t));
  if (!first) return OR_ERR_NOMEM;
  for (int64_t v = 0; v < n; ++v) first[color[v] + 1] += 1;
  for (int32_t c = 0; c < n_colors; ++c) first[c + 1] += first[c];
  for (int32_t r = 0; r < R; ++r) {
    int8_t *s = spins + (int64_t)r * n;
    for (int64_t t = t_begin; t < t_end; ++t) {
      for (int32_t c = 0; c < n_colors; ++c) {
#pragma omp parallel for schedule(static)
        for (int64_t i = first[c]; i < first[c + 1]; ++i) {
          int64_t v = order[i];
          int8_t x = field_update(v, row_ptr, col, w, field, s, s[v]);
          if (flip_draw((uint32_t)v, (uint32_t)t, (uint32_t)r, seed) < vertex_threshold(T[t], scale, v))
            x = (int8_t)-x;
          s[v] = x;
        }
      }
    }
  }
  free(first);
  return OR_OK;
}

/* Host threads the colour-parallel anneal uses. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Jacobi bracket: all vertices of sweep t read the spins of sweep t-1. */
int oracle_anneal_jacobi(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                         const int32_t *field, int32_t R, int8_t *spins, const uint32_t *T, uint64_t seed,
                         int64_t t_begin, int64_t t_end) {
  if (t_begin < 0 || t_end < t_begin) return OR_ERR_ARG;
  int8_t *prev = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
  if (!prev) return OR_ERR_NOMEM;
  for (int32_t r = 0; r < R; ++r) {
    int8_t *s = spins + (int64_t)r * n;
    for (int64_t t = t_begin; t < t_end; ++t) {
      memcpy(prev, s, (size_t)n);
      for (int64_t v = 0; v < n; ++v) {
        int8_t x = field_update(v, row_ptr, col, w, field, prev, prev[v]);
        if (flip_draw((uint32_t)v, (uint32_t)t, (uint32_t)r, seed) < T[t]) x = (int8_t)-x;
        s[v] = x;
      }
    }
  }
  free(prev);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Cut and energy per replica, each unordered edge once (R9).               */
/*   cut = sum_{u<v, s_u != s_v} w_uv          (Eq. 4 evaluated directly)   */
/*   E   = sum_{u<v} w_uv s_u s_v              (Eq. 5 with J = -w, R1)      */
/* and the identity 2 cut = W - E, which follows from Eq. (4), is checked.  */
/* With a field (R14) the energy adds -sum_v h_v s_v (Eq. 3); the cut and   */
/* the identity use the edge part alone.                                    */
/* ------------------------------------------------------------------------ */
int oracle_cut(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
               const int32_t *field, int32_t R, const int8_t *spins, int64_t *cut, int64_t *energy) {
  for (int32_t r = 0; r < R; ++r) {
    const int8_t *s = spins + (int64_t)r * n;
    int64_t W = 0, E = 0, C = 0, F = 0;
    if (field)
      for (int64_t v = 0; v < n; ++v) F -= (int64_t)field[v] * s[v];
    for (int64_t u = 0; u < n; ++u)
      for (int64_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
        int64_t v = col[k];
        if (u >= v) continue;
        W += w[k];
        E += (int64_t)w[k] * s[u] * s[v];
        if (s[u] != s[v]) C += w[k];
      }
    if (2 * C != W - E) return OR_ERR_INTERNAL;
    cut[r] = C;
    if (energy) energy[r] = E + F;
  }
  return OR_OK;
}

/* Field contract (R10, R14): every row keeps sum |w| + |h_v| <= 2^30 - 1,
 * so S_v and twice it fit int32.  Returns OR_ERR_OVERFLOW and the first
 * offending vertex in *bad otherwise. */
int oracle_validate_field(int64_t n, const int64_t *row_ptr, const int8_t *w, const int32_t *field,
                          int64_t *bad) {
  for (int64_t v = 0; v < n; ++v) {
    int64_t a = field[v] < 0 ? -(int64_t)field[v] : (int64_t)field[v];
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) a += w[k] < 0 ? -(int64_t)w[k] : (int64_t)w[k];
    if (a > (INT32_MAX >> 1)) {
      if (bad) *bad = v;
      return OR_ERR_OVERFLOW;
    }
  }
  return OR_OK;
}

/* Local field of every vertex for one replica (used by tests of the update
 * rule: a single flip of v changes the cut by s_v * h_v). */
void oracle_fields(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                   const int8_t *s, int32_t *h) {
  for (int64_t v = 0; v < n; ++v) h[v] = local_field(v, row_ptr, col, w, s);
}
