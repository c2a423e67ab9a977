// mpnn.hip -- the 64-wide layers of the learned warm start on MFMA.
//
// One layer of the message-passing network maps node features h (n x 64)
// to relu(h W_self + m W_nb + b), where m is the degree-normalised weighted
// neighbour sum m_v = (1 / max(deg v, 1)) sum_k w_k h_{col k}.  Features and
// weights are bfloat16; products accumulate in fp32 on the matrix cores
// (v_mfma_f32_16x16x16_bf16).  A workgroup of four wavefronts owns a tile of
// 64 vertices: it gathers the tile's neighbour sums into LDS, then each
// wavefront computes 16 rows x 64 columns of the layer as four 16 x 16
// accumulators over K = 128 (64 self features, then 64 aggregated ones).
//
// The backward kernel takes g = dL/d out (fp32) and the layer's saved
// inputs: dz = g * [out > 0] (out > 0 exactly where z > 0), the input
// gradient's self part dz W_self^T, the neighbour part's pre-sum
// dz W_nb^T / deg (summed over neighbours by a second kernel: the graph is
// symmetric, so that sum is the transpose of the forward one), and the
// weight gradients h^T dz, m^T dz, sum dz, all on the matrix cores from
// transposed LDS tiles and added into fp32 accumulators.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "ising_warm.h"

namespace {

constexpr int kWave = 64;
constexpr int kF = 64;          // features
constexpr int kTile = 64;       // vertices per workgroup
constexpr int kThreads = 256;   // four wavefronts
constexpr int kPad = 4;         // bf16 padding per LDS row (keeps 8-byte reads aligned, spreads banks)
constexpr int kLd = kF + kPad;  // LDS row length in bf16

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t x) { return __uint_as_float((uint32_t)x << 16); }
// round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Four consecutive bf16 of an LDS row as one MFMA operand.
__device__ __forceinline__ bf16x4 ld4(const uint16_t *p) {
  const uint2 v = *reinterpret_cast<const uint2 *>(p);
  bf16x4 r;
  r[0] = (short)(v.x & 0xFFFFu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFFu);
  r[3] = (short)(v.y >> 16);
  return r;
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Forward.  MFMA 16x16x16 operand layout (lane l, j = 0..3):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + j;  B[k][c]: k = 4 (l / 16) + j,
//   c = l % 16;  D[r][c]: r = 4 (l / 16) + j, c = l % 16.
// A comes from row-major feature tiles (four consecutive k), B from the
// transposed weights WT[c][k] (four consecutive k).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_layer_fwd(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                                        const int8_t *w, const uint16_t *h, const uint16_t *Ws,
                                                        const uint16_t *Wn, const float *b, uint16_t *out,
                                                        uint16_t *m_out) {
  __shared__ __align__(16) uint16_t Xs[kTile * kLd];  // self features of the tile
  __shared__ __align__(16) uint16_t Xm[kTile * kLd];  // aggregated features
  __shared__ __align__(16) uint16_t WsT[kF * kLd];    // WsT[c][k] = W_self[k][c]
  __shared__ __align__(16) uint16_t WnT[kF * kLd];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t v0 = (int64_t)blockIdx.x * kTile;
  for (int i = threadIdx.x; i < kF * kF; i += kThreads) {
    const int k = i / kF, c = i % kF;
    WsT[c * kLd + k] = Ws[i];
    WnT[c * kLd + k] = Wn[i];
  }
  for (int i = threadIdx.x; i < kTile * kF; i += kThreads) {
    const int r = i / kF, c = i % kF;
    Xs[r * kLd + c] = v0 + r < n ? h[(v0 + r) * kF + c] : (uint16_t)0;
  }
  // neighbour sums: wavefront wv takes rows wv, wv + 4, ...; lane = feature
  for (int r = wv; r < kTile; r += kThreads / kWave) {
    const int64_t v = v0 + r;
    float acc = 0.f;
    int64_t deg = 0;
    if (v < n) {
      const int64_t e0 = row_ptr[v], e1 = row_ptr[v + 1];
      deg = e1 - e0;
      for (int64_t k = e0; k < e1; ++k) acc += (float)w[k] * bf2f(h[(int64_t)col[k] * kF + lane]);
    }
    const uint16_t mb = f2bf(acc / (float)(deg > 0 ? deg : 1));
    Xm[r * kLd + lane] = mb;
    if (m_out != nullptr && v < n) m_out[v * kF + lane] = mb;
  }
  __syncthreads();
  const int i = lane & 15, q = lane >> 4;  // operand row / column, k quarter
  const int r0 = wv * 16;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < kF; ks += 16) {
    const bf16x4 as = ld4(&Xs[(r0 + i) * kLd + ks + 4 * q]);
    const bf16x4 am = ld4(&Xm[(r0 + i) * kLd + ks + 4 * q]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = mfma(as, ld4(&WsT[(16 * t + i) * kLd + ks + 4 * q]), acc[t]);
      acc[t] = mfma(am, ld4(&WnT[(16 * t + i) * kLd + ks + 4 * q]), acc[t]);
    }
  }
  // bias, ReLU, bf16 out: lane holds D[4 q + j][i] of each 16 x 16 tile
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + i;
    const float bc = b[c];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t v = v0 + r0 + 4 * q + j;
      const float z = acc[t][j] + bc;
      if (v < n) out[v * kF + c] = f2bf(z > 0.f ? z : 0.f);
    }
  }
}

// ---------------------------------------------------------------------------
// Backward, part 1: per tile of 64 vertices.
//   dz = g [out > 0]                                     (bf16 in LDS)
//   dh[v] = dz W_self^T          (written, fp32)
//   work[v] = dz W_nb^T / deg    (written, fp32; part 2 sums it over neighbours)
//   dWs += h^T dz, dWn += m^T dz, db += sum dz           (fp32 atomics)
// dz W^T: A = dz rows (four consecutive k = output features), B[k][c] =
// W[c][k] read from W row-major (four consecutive k).  h^T dz: A[i][k] =
// h[k][i] and B[k][c] = dz[k][c] over the tile's vertices k, read from
// transposed tiles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_layer_bwd(int64_t n, const int64_t *row_ptr, const uint16_t *h,
                                                        const uint16_t *m, const uint16_t *out, const uint16_t *Ws,
                                                        const uint16_t *Wn, const float *g, float *dh, float *work,
                                                        float *dWs, float *dWn, float *db) {
  __shared__ __align__(16) uint16_t DZ[kTile * kLd];   // dz[v][c]
  __shared__ __align__(16) uint16_t DZT[kF * kLd];     // dz[v][c] at [c][v]
  __shared__ __align__(16) uint16_t HT[kF * kLd];      // h[v][i] at [i][v]
  __shared__ __align__(16) uint16_t MT[kF * kLd];      // m[v][i] at [i][v]
  __shared__ __align__(16) uint16_t Wsl[kF * kLd];     // W_self[c][k] row-major
  __shared__ __align__(16) uint16_t Wnl[kF * kLd];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t v0 = (int64_t)blockIdx.x * kTile;
  for (int x = threadIdx.x; x < kF * kF; x += kThreads) {
    const int a = x / kF, c = x % kF;
    Wsl[a * kLd + c] = Ws[x];
    Wnl[a * kLd + c] = Wn[x];
  }
  for (int x = threadIdx.x; x < kTile * kF; x += kThreads) {
    const int r = x / kF, c = x % kF;
    const int64_t v = v0 + r;
    uint16_t dzb = 0, hb = 0, mb = 0;
    if (v < n) {
      const float gz = bf2f(out[v * kF + c]) > 0.f ? g[v * kF + c] : 0.f;
      dzb = f2bf(gz);
      hb = h[v * kF + c];
      mb = m[v * kF + c];
    }
    DZ[r * kLd + c] = dzb;
    DZT[c * kLd + r] = dzb;
    HT[c * kLd + r] = hb;
    MT[c * kLd + r] = mb;
  }
  __syncthreads();
  const int i = lane & 15, q = lane >> 4;
  const int r0 = wv * 16;
  // input gradients of rows r0 .. r0 + 15
  {
    f32x4 as[4], an[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) as[t] = an[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kF; ks += 16) {
      const bf16x4 a = ld4(&DZ[(r0 + i) * kLd + ks + 4 * q]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        as[t] = mfma(a, ld4(&Wsl[(16 * t + i) * kLd + ks + 4 * q]), as[t]);
        an[t] = mfma(a, ld4(&Wnl[(16 * t + i) * kLd + ks + 4 * q]), an[t]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t v = v0 + r0 + 4 * q + j;
      if (v >= n) continue;
      const int64_t deg = row_ptr[v + 1] - row_ptr[v];
      const float inv = 1.f / (float)(deg > 0 ? deg : 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        dh[v * kF + 16 * t + i] = as[t][j];
        work[v * kF + 16 * t + i] = an[t][j] * inv;
      }
    }
  }
  // weight gradients: rows r0 .. r0 + 15 of h^T dz and m^T dz
  {
    f32x4 gs[4], gn[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) gs[t] = gn[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kTile; ks += 16) {
      const bf16x4 ah = ld4(&HT[(r0 + i) * kLd + ks + 4 * q]);
      const bf16x4 am = ld4(&MT[(r0 + i) * kLd + ks + 4 * q]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bf16x4 bz = ld4(&DZT[(16 * t + i) * kLd + ks + 4 * q]);
        gs[t] = mfma(ah, bz, gs[t]);
        gn[t] = mfma(am, bz, gn[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = r0 + 4 * q + j, c = 16 * t + i;
        atomicAdd(&dWs[a * kF + c], gs[t][j]);
        atomicAdd(&dWn[a * kF + c], gn[t][j]);
      }
  }
  if (threadIdx.x < kF) {
    float s = 0.f;
    for (int r = 0; r < kTile; ++r) s += bf2f(DZ[r * kLd + threadIdx.x]);
    atomicAdd(&db[threadIdx.x], s);
  }
}

// Backward, part 2: dh[v] += sum_k w_k work[col k] (one wavefront per row,
// lane = feature).
__global__ __launch_bounds__(kThreads) void k_layer_bwd_sum(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                                            const int8_t *w, const float *work, float *dh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * (kThreads / kWave);
  for (int64_t v = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave; v < n; v += stride) {
    float acc = 0.f;
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) acc += (float)w[k] * work[(int64_t)col[k] * kF + lane];
    dh[v * kF + lane] += acc;
  }
}

thread_local char g_err[256];

int launch_error(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return 0;
  snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
  return 8;
}

}  // namespace

extern "C" {

const char *isingWarmLayerLastError(void) { return g_err; }

int isingWarmLayerForward(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                          const uint16_t *h, const uint16_t *W_self, const uint16_t *W_nb, const float *b,
                          uint16_t *out, uint16_t *m_out, void *stream) {
  g_err[0] = 0;
  if (n < 0 || (n > 0 && (row_ptr == nullptr || h == nullptr || W_self == nullptr || W_nb == nullptr ||
                          b == nullptr || out == nullptr)) ||
      (n > 0 && out == h)) {
    snprintf(g_err, sizeof g_err, "invalid argument");
    return 1;
  }
  if (n == 0) return 0;
  const int64_t tiles = (n + kTile - 1) / kTile;
  if (tiles > 0x7FFFFFFF) {
    snprintf(g_err, sizeof g_err, "too many vertices");
    return 1;
  }
  hipLaunchKernelGGL(k_layer_fwd, dim3((unsigned)tiles), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream), n,
                     row_ptr, col, w, h, W_self, W_nb, b, out, m_out);
  return launch_error("layer forward launch");
}

int isingWarmLayerBackward(int64_t n, const int64_t *row_ptr, const int32_t *col, const int8_t *w,
                           const uint16_t *h, const uint16_t *m, const uint16_t *out, const uint16_t *W_self,
                           const uint16_t *W_nb, const float *g, float *dh, float *dW_self, float *dW_nb,
                           float *db, float *work, void *stream) {
  g_err[0] = 0;
  if (n < 0 || (n > 0 && (row_ptr == nullptr || h == nullptr || m == nullptr || out == nullptr ||
                          W_self == nullptr || W_nb == nullptr || g == nullptr || dh == nullptr ||
                          dW_self == nullptr || dW_nb == nullptr || db == nullptr || work == nullptr))) {
    snprintf(g_err, sizeof g_err, "invalid argument");
    return 1;
  }
  if (n == 0) return 0;
  const int64_t tiles = (n + kTile - 1) / kTile;
  if (tiles > 0x7FFFFFFF) {
    snprintf(g_err, sizeof g_err, "too many vertices");
    return 1;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_layer_bwd, dim3((unsigned)tiles), dim3(kThreads), 0, st, n, row_ptr, h, m, out, W_self, W_nb, g,
                     dh, work, dW_self, dW_nb, db);
  int r = launch_error("layer backward launch");
  if (r != 0) return r;
  const int64_t rows = (n + kThreads / kWave - 1) / (kThreads / kWave);
  hipLaunchKernelGGL(k_layer_bwd_sum, dim3((unsigned)(rows < 65536 ? rows : 65536)), dim3(kThreads), 0, st, n,
                     row_ptr, col, w, work, dh);
  return launch_error("layer backward sum launch");
}

}  // extern "C"
