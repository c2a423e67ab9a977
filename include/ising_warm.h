/*
 * ising_warm.h -- kernels of the learned warm start (not part of the
 * paper's method).
 *
 * A small message-passing network proposes initial spins; the anneal of
 * ising.h then starts from them (isingSetSpins) with a shorter schedule.
 * Plain random-start annealing stays the reference: the network only
 * changes where the exact, oracle-checked anneal begins.
 */
#ifndef ISING_WARM_H
#define ISING_WARM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Weighted neighbour sum of node features:
 *   y[v][c] = sum_{k = row_ptr[v]}^{row_ptr[v+1]-1} w[k] * x[col[k]][c],
 * for v < n and c < f.  The graph is the symmetric CSR of ising.h (int64
 * row_ptr [n+1], int32 col [nnz], int8 w [nnz]); x and y are float32
 * [n][f], row-major, and must not overlap.  Every pointer is device memory
 * owned by the caller.  Because the graph is symmetric this product is its
 * own transpose, so it also serves the backward pass.  Stream-ordered on
 * stream (hipStream_t, NULL = default), no synchronisation.  Returns 0, 1
 * for an invalid argument, 8 for a launch error (isingWarmLastError). */
int isingWarmAggregate(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w, const float *x,
                       float *y, int32_t f, void *stream);

const char *isingWarmLastError(void);

/* One 64-wide message-passing layer on the matrix cores, the neighbour sum
 * fused in (the network is not part of the paper; its spins only choose
 * where the exact anneal starts):
 *   m[v]   = (1 / max(deg v, 1)) * sum_{k in row v} w[k] * h[col[k]]
 *            (fp32 sum, rounded to bfloat16),
 *   out[v] = max(0, h[v] W_self + m[v] W_nb + b)
 *            (bfloat16 operands, fp32 accumulation, rounded to bfloat16).
 * Graph: the CSR of ising.h.  h, out, m_out: bfloat16 bit patterns, [n][64]
 * row-major; W_self, W_nb: bfloat16 [64][64] row-major (input feature,
 * output feature); b: fp32 [64].  m_out (may be NULL) receives m for the
 * backward pass.  out must not alias h.  All pointers are caller-owned
 * device memory.  Stream-ordered, no synchronisation.  Returns 0, 1 for an
 * invalid argument, 8 for a launch error (isingWarmLayerLastError). */
int isingWarmLayerForward(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                          const uint16_t *h, const uint16_t *W_self, const uint16_t *W_nb, const float *b,
                          uint16_t *out, uint16_t *m_out, void *stream);

/* Gradients of that layer from g = dL/d out (fp32 [n][64]) and the forward's
 * h, m and out:  dz = g * [out > 0] (rounded to bfloat16),
 *   dh      = dz W_self^T + A (D^-1 dz W_nb^T)   (fp32 [n][64], written;
 *             A is the weighted adjacency, D the degrees),
 *   dW_self += h^T dz,  dW_nb += m^T dz  (fp32 [64][64], accumulated),
 *   db      += sum over v of dz           (fp32 [64], accumulated),
 * all products on the matrix cores with fp32 accumulation.  work: fp32
 * [n][64] caller-owned scratch.  Returns as isingWarmLayerForward. */
int isingWarmLayerBackward(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                           const uint16_t *h, const uint16_t *m, const uint16_t *out, const uint16_t *W_self,
                           const uint16_t *W_nb, const float *g, float *dh, float *dW_self, float *dW_nb,
                           float *db, float *work, void *stream);

const char *isingWarmLayerLastError(void);

#ifdef __cplusplus
}
#endif

#endif
