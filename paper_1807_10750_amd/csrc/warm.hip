// warm.hip -- neighbour aggregation of the learned warm-start model.
//
// Y[v][:] = sum over the CSR row of v of w_vk * X[col_k][:], float32
// features.  One wavefront per row and 64 lanes per 64 features, so every
// neighbour costs one coalesced 256-byte read per 64 features.  The graph is
// symmetric, so the same product is its own transpose (the backward pass).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_warm.h"

namespace {

constexpr int kWave = 64;
constexpr int kRowsPerBlock = 4;

__global__ __launch_bounds__(kWave * kRowsPerBlock) void k_aggregate(int64_t n, const int64_t *row_ptr,
                                                                     const int32_t *col, const int8_t *w,
                                                                     const float *x, float *y, int32_t f) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * kRowsPerBlock;
  for (int64_t v = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave; v < n; v += stride) {
    const int64_t b = row_ptr[v], e = row_ptr[v + 1];
    for (int32_t c0 = 0; c0 < f; c0 += kWave) {
      const int32_t c = c0 + lane;
      float acc = 0.f;
      if (c < f) {
        for (int64_t k = b; k < e; ++k) acc += (float)w[k] * x[(int64_t)col[k] * f + c];
        y[v * f + c] = acc;
      }
    }
  }
}

thread_local char g_err[256];

}  // namespace

extern "C" {

const char *isingWarmLastError(void) { return g_err; }

int isingWarmAggregate(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w, const float *x,
                       float *y, int32_t f, void *stream) {
  g_err[0] = 0;
  if (n < 0 || f <= 0 || (n > 0 && (row_ptr == nullptr || x == nullptr || y == nullptr))) {
    snprintf(g_err, sizeof g_err, "invalid argument");
    return 1;
  }
  if (n == 0) return 0;
  const int64_t blocks = (n + kRowsPerBlock - 1) / kRowsPerBlock;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(k_aggregate, dim3(grid), dim3(kWave * kRowsPerBlock), 0, reinterpret_cast<hipStream_t>(stream),
                     n, row_ptr, col, w, x, y, f);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(g_err, sizeof g_err, "aggregate launch: %s", hipGetErrorString(e));
    return 8;
  }
  return 0;
}

}  // extern "C"
