/* Exercises the oracle (validation, colourings, order, initial spins, the
 * sequential, colour-parallel and Jacobi anneals with and without a field
 * and flip multipliers, cut and energy) on a seeded random graph, for a
 * build with AddressSanitizer and UBSan.  Exits nonzero on a broken
 * invariant; the sanitizers abort on a memory or UB error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_thresholds(int kind, double p_start, double p_end, int64_t M, uint32_t *T);
int oracle_validate(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                    int64_t *W_out, int64_t *bad_row, int64_t *bad_k);
int oracle_color(int64_t n, const int64_t *row_ptr, const int32_t *col, int largest_first, int32_t *color,
                 int32_t *n_colors);
void oracle_order(int64_t n, const int32_t *color, int32_t n_colors, int32_t *order);
void oracle_init_spins(int64_t n, int32_t R, uint64_t seed, int8_t *spins);
int oracle_anneal(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w, const int32_t *field,
                  const uint8_t *scale, const int32_t *order, int32_t R, int8_t *spins, const uint32_t *T,
                  uint64_t seed, int64_t t_begin, int64_t t_end);
int oracle_anneal_colour_parallel(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                                  const int32_t *field, const uint8_t *scale, const int32_t *order,
                                  const int32_t *color, int32_t n_colors, int32_t R, int8_t *spins,
                                  const uint32_t *T, uint64_t seed, int64_t t_begin, int64_t t_end);
int oracle_anneal_jacobi(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                         const int32_t *field, int32_t R, int8_t *spins, const uint32_t *T, uint64_t seed,
                         int64_t t_begin, int64_t t_end);
int oracle_cut(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w, const int32_t *field,
               int32_t R, const int8_t *spins, int64_t *cut, int64_t *energy);

static uint64_t rng_state = 88172645463325252ull;
static uint32_t next_u32(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (uint32_t)(rng_state >> 11);
}

int main(void) {
  enum { N = 400, M = 900, R = 3, S = 40 };
  static int32_t adj[N][N];
  static int8_t wt[N][N];
  for (int k = 0; k < M; ++k) {
    int u = (int)(next_u32() % N), v = (int)(next_u32() % N);
    if (u == v || adj[u][v]) continue;
    adj[u][v] = adj[v][u] = 1;
    wt[u][v] = wt[v][u] = (int8_t)((next_u32() & 1) ? 1 : -1);
  }
  int64_t *rp = calloc(N + 1, sizeof(int64_t));
  int32_t *col = malloc(sizeof(int32_t) * 2 * M);
  int8_t *w = malloc(2 * M);
  int64_t nnz = 0;
  for (int u = 0; u < N; ++u) {
    for (int v = 0; v < N; ++v)
      if (adj[u][v]) { col[nnz] = v; w[nnz] = wt[u][v]; ++nnz; }
    rp[u + 1] = nnz;
  }
  int64_t W = 0, br = 0, bk = 0;
  int fails = 0;
  if (oracle_validate(N, nnz, rp, col, w, &W, &br, &bk) != 0) { fprintf(stderr, "validate\n"); ++fails; }
  int32_t *color = malloc(sizeof(int32_t) * N), *order = malloc(sizeof(int32_t) * N), nc = 0;
  uint32_t *T = malloc(sizeof(uint32_t) * S);
  oracle_thresholds(0, 0.2, 0.0, S, T);
  int32_t *field = malloc(sizeof(int32_t) * N);
  uint8_t *scale = malloc(N);
  for (int v = 0; v < N; ++v) { field[v] = (int32_t)(next_u32() % 7) - 3; scale[v] = (uint8_t)(next_u32() % 16); }
  int8_t *a = malloc(R * N), *b = malloc(R * N), *c = malloc(R * N);
  int64_t cut[R], energy[R];
  for (int lf = 0; lf < 2; ++lf) {
    oracle_color(N, rp, col, lf, color, &nc);
    oracle_order(N, color, nc, order);
    for (int variant = 0; variant < 3; ++variant) {
      const int32_t *f = variant == 1 ? field : NULL;
      const uint8_t *m = variant == 2 ? scale : NULL;
      oracle_init_spins(N, R, 5, a);
      memcpy(b, a, R * N);
      memcpy(c, a, R * N);
      oracle_anneal(N, rp, col, w, f, m, order, R, a, T, 9, 0, S);
      oracle_anneal_colour_parallel(N, rp, col, w, f, m, order, color, nc, R, b, T, 9, 0, S);
      if (memcmp(a, b, R * N) != 0) { fprintf(stderr, "colour-parallel differs\n"); ++fails; }
      oracle_anneal_jacobi(N, rp, col, w, f, R, c, T, 9, 0, S);
      if (oracle_cut(N, rp, col, w, f, R, a, cut, energy) != 0) { fprintf(stderr, "cut identity\n"); ++fails; }
      if (oracle_cut(N, rp, col, w, f, R, c, cut, energy) != 0) { fprintf(stderr, "cut identity (jacobi)\n"); ++fails; }
    }
  }
  free(rp); free(col); free(w); free(color); free(order); free(T); free(field); free(scale);
  free(a); free(b); free(c);
  if (fails) return 1;
  printf("oracle driver ok\n");
  return 0;
}
