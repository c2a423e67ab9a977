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

#ifdef __cplusplus
}
#endif

#endif
