// noalloc.hip -- isingAnnealNoAlloc: the anneal of isingAnneal for callers
// that cannot allocate device or host memory.
//
// isingAnneal keeps each handle's threshold table in device memory that it
// allocates (and regrows) when a schedule is new, staged through pinned host
// memory.  This variant writes the thresholds of the requested sweeps into a
// fixed array of device memory instead, `scratch`, which every call on a GPU
// shares; the anneal kernels then read it exactly as they read the handle's
// table.  Nothing here calls hipMalloc, hipHostMalloc, hipFree or any other
// allocating routine.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "ising_noalloc.h"

// Thresholds of at most ISING_NOALLOC_MAX_SWEEPS sweeps per call (256 KiB
// of device memory per GPU, held until the process ends).
static __device__ __align__(256) uint32_t scratch[ISING_NOALLOC_MAX_SWEEPS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the caller's CurrentDevice guard).  In host code the
// array's name is only a stand-in for the symbol, never a device address.
uint32_t *scratch_ptr(int dev, hipError_t *err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
  }
  return g_scratch_ptr[dev];
}

// T[t - t0] for t in [t0, t0 + count) of the linear schedule from Ts to Te
// over M sweeps: Ts - floor((Ts - Te) t / (M - 1)) (or the mirror image when
// Ts < Te); the product fits 64 bits because both factors are below 2^32.
__global__ void k_linear_thresholds(uint32_t *T, uint32_t ts, uint32_t te, int64_t M, int64_t t0, uint32_t count) {
  const bool down = ts >= te;
  const uint64_t span = down ? (uint64_t)(ts - te) : (uint64_t)(te - ts);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const uint64_t t = (uint64_t)(t0 + i);
    const uint64_t step = M > 1 ? (span * t) / (uint64_t)(M - 1) : 0ull;
    T[i] = down ? ts - (uint32_t)step : ts + (uint32_t)step;
  }
}

// Restores the caller's device on every return path.
class CurrentDevice {
 public:
  explicit CurrentDevice(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) (void)hipSetDevice(dev);
    dev_ = dev;
  }
  ~CurrentDevice() {
    if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1, dev_ = 0;
};

}  // namespace

extern "C" ising_status_t isingAnnealNoAlloc(ising_graph_t g, const ising_schedule_t *s, uint64_t seed,
                                             ising_mode_t mode, int64_t sweep_begin, int64_t sweep_end,
                                             void *stream) {
  internal_clear_error();
  ising_status_t r = internal_check_anneal(g, s, mode, sweep_begin, sweep_end);
  if (r != ISING_OK) return r;
  if (sweep_end - sweep_begin > ISING_NOALLOC_MAX_SWEEPS)
    return internal_fail(ISING_ERR_INVALID_ARGUMENT,
                         "isingAnnealNoAlloc runs at most ISING_NOALLOC_MAX_SWEEPS sweeps per call");
  if (sweep_begin == sweep_end) return ISING_OK;
  CurrentDevice guard(internal_device(g));
  hipError_t e = hipSuccess;
  uint32_t *T = scratch_ptr(internal_device(g), &e);
  if (T == nullptr) return internal_fail(ISING_ERR_DEVICE, std::string("scratch lookup: ") + hipGetErrorString(e));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint32_t count = (uint32_t)(sweep_end - sweep_begin);
  if (s->kind == ISING_SCHED_LINEAR) {
    const int grid = (int)((count + 255u) / 256u);
    hipLaunchKernelGGL(k_linear_thresholds, dim3(grid), dim3(256), 0, st, T, internal_prob_threshold(s->p_start),
                       internal_prob_threshold(s->p_end), s->n_sweeps, sweep_begin, count);
    e = hipGetLastError();
  } else {
    e = hipMemcpyAsync(T, s->thresholds + sweep_begin, sizeof(uint32_t) * count, hipMemcpyDefault, st);
  }
  if (e != hipSuccess) return internal_fail(ISING_ERR_DEVICE, std::string("threshold staging: ") + hipGetErrorString(e));
  return internal_anneal(g, seed, mode, sweep_begin, sweep_end, st, T, sweep_begin);
}
