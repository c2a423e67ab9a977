// kernels.hip -- gfx950 kernels of the Ising max-cut annealer.
//
// The sweep follows the annealed local update of Cook et al. (arXiv
// 1807.10750): each spin takes the value that minimises its local energy
// given its neighbours (Sec. II-A, Eq. 2, with J = -w so that low energy is
// a large cut, Sec. III Eq. 4-5), then flips with the sweep's probability F_p
// (Sec. IV-B, Algorithm 2).  Flip draws are Philox4x32-10 (Salmon et al.,
// SC'11) word 0 at counter {vertex, sweep, replica, 0}, key = seed.
//
// Work is issued colour class by colour class.  In deterministic mode a
// grid barrier separates the classes, which makes the result equal to a
// sequential sweep in (colour, id) order.  In async mode there is no barrier
// inside a sweep: each workgroup refreshes a class's spins right after its
// own share of that class and moves on, so a neighbour's value is from this
// sweep or the previous one, as in the paper's unsynchronised update.
//
// Spin state is an L-bit mask per slot (replica bits) packed in uint32
// words.  When it fits, each workgroup keeps a copy of the whole state in
// LDS and neighbour gathers are LDS reads; the edge stream is read once per
// sweep with 16-byte coalesced loads.  All global spin traffic uses
// agent-scope atomics, which are coherent across the XCDs' L2 caches.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ising {

namespace {

constexpr int kWave = 64;

// Philox4x32-10, word 0 only.
__device__ __forceinline__ uint32_t philox_w0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t a_lo = 0xD2511F53u * c0;
    const uint32_t a_hi = __umulhi(0xD2511F53u, c0);
    const uint32_t b_lo = 0xCD9E8D57u * c2;
    const uint32_t b_hi = __umulhi(0xCD9E8D57u, c2);
    c0 = b_hi ^ c1 ^ k0;
    c1 = b_lo;
    c2 = a_hi ^ c3 ^ k1;
    c3 = a_lo;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c0;
}

__device__ __forceinline__ uint32_t ld_coherent(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_coherent64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int L>
__device__ __forceinline__ uint32_t lmask() {
  return L == 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
}

// Mask of slot s from a word array (LDS or global).
template <int L, typename P>
__device__ __forceinline__ uint32_t mask_of(P words, uint32_t s) {
  const uint32_t bit = s * L;
  return (words[bit >> 5] >> (bit & 31)) & lmask<L>();
}

// Adds the contribution of one edge entry to the L field accumulators.
// pm1: entry = slot | sign; general: slot with separate weight w8.
template <int L, bool PM1, typename P>
__device__ __forceinline__ void accumulate(int32_t (&h)[L], uint32_t x, int32_t w8, P words) {
  if (PM1) {
    const bool valid = x != kSentinel;
    const uint32_t slot = valid ? (x & ~kSignBit) : 0u;
    uint32_t m = mask_of<L>(words, slot);
    if (x & kSignBit) m = ~m;
#pragma unroll
    for (int j = 0; j < L; ++j) h[j] += valid ? (int32_t)(((m >> j) & 1u) << 1) - 1 : 0;
  } else {
    const uint32_t m = mask_of<L>(words, x);
#pragma unroll
    for (int j = 0; j < L; ++j) h[j] += ((m >> j) & 1u) ? w8 : -w8;
  }
}

// Local update (Eq. 2, J = -w, tie keeps) and the annealing flip.
template <int L>
__device__ __forceinline__ uint32_t update_mask(const int32_t (&h)[L], uint32_t own, int32_t v,
                                                uint32_t t, uint32_t T, const AnnealArgs &a) {
  uint32_t nm = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    uint32_t s = (own >> j) & 1u;
    s = h[j] > 0 ? 0u : (h[j] < 0 ? 1u : s);
    if (T != 0u && (uint32_t)j < a.r_count) {
      const uint32_t x = philox_w0((uint32_t)v, t, a.r0 + (uint32_t)j, 0u, a.seed_lo, a.seed_hi);
      s ^= (x < T) ? 1u : 0u;
    }
    nm |= s << j;
  }
  return v >= 0 ? nm : 0u;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Grid-wide barrier of a cooperative launch.  Returns false (and raises the
// error flag) if the other workgroups did not arrive within the poll limit.
__device__ bool grid_barrier(uint32_t *bar, uint32_t target, uint32_t limit) {
  __shared__ uint32_t s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t polls = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          ++polls > limit) {
        __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// ---------------------------------------------------------------------------
// Anneal kernel
// ---------------------------------------------------------------------------
template <int L, bool PM1, bool USE_LDS>
__device__ __forceinline__ void run_slice(const AnnealArgs &a, const Item &it, uint32_t *lds,
                                          int lane, uint32_t t, uint32_t T) {
  const uint32_t slot = it.id * kSliceRows + lane;
  const int32_t v = a.vid[slot];
  int32_t h[L];
#pragma unroll
  for (int j = 0; j < L; ++j) h[j] = 0;
  const uint4 *e = a.entries + it.base4 + lane;
  const uint32_t *wq = PM1 ? nullptr : a.wts4 + it.base4 + lane;
  const uint32_t len4 = it.len4;
#pragma unroll 2
  for (uint32_t q = 0; q < len4; ++q) {
    const uint4 x = e[(size_t)q * kSliceRows];
    const uint32_t wv = PM1 ? 0u : wq[(size_t)q * kSliceRows];
    if (USE_LDS) {
      accumulate<L, PM1>(h, x.x, (int32_t)(int8_t)(wv), lds);
      accumulate<L, PM1>(h, x.y, (int32_t)(int8_t)(wv >> 8), lds);
      accumulate<L, PM1>(h, x.z, (int32_t)(int8_t)(wv >> 16), lds);
      accumulate<L, PM1>(h, x.w, (int32_t)(int8_t)(wv >> 24), lds);
    } else {
      accumulate<L, PM1>(h, x.x, (int32_t)(int8_t)(wv), a.spins);
      accumulate<L, PM1>(h, x.y, (int32_t)(int8_t)(wv >> 8), a.spins);
      accumulate<L, PM1>(h, x.z, (int32_t)(int8_t)(wv >> 16), a.spins);
      accumulate<L, PM1>(h, x.w, (int32_t)(int8_t)(wv >> 24), a.spins);
    }
  }
  const uint32_t own = USE_LDS ? mask_of<L>(lds, slot) : mask_of<L>(a.spins, slot);
  const uint32_t nm = update_mask<L>(h, own, v, t, T, a);
  // A slice's 64 masks fill 2L whole words.
  if (L == 1) {
    const unsigned long long b = __ballot(nm & 1u);
    if (lane == 0) {
      st_coherent64(reinterpret_cast<unsigned long long *>(a.spins) + it.id, b);
      if (USE_LDS) reinterpret_cast<unsigned long long *>(lds)[it.id] = b;
    }
  } else {
    constexpr int P = 32 / L;  // slots per word
    uint32_t val = nm << ((lane % P) * L);
#pragma unroll
    for (int off = 1; off < P; off <<= 1) val |= __shfl_xor(val, off);
    if (lane % P == 0) {
      const uint32_t word = it.id * (2 * L) + lane / P;
      st_coherent(a.spins + word, val);
      if (USE_LDS) lds[word] = val;
    }
  }
}

template <int L, bool PM1, bool USE_LDS>
__device__ __forceinline__ void run_long(const AnnealArgs &a, const Item &it, uint32_t *lds,
                                         int lane, uint32_t t, uint32_t T) {
  const uint32_t slot = it.id;
  const int32_t v = a.vid[slot];
  int32_t h[L];
#pragma unroll
  for (int j = 0; j < L; ++j) h[j] = 0;
  for (uint32_t q = lane; q < it.len4; q += kWave) {
    const uint4 x = a.entries[(size_t)it.base4 + q];
    const uint32_t wv = PM1 ? 0u : a.wts4[(size_t)it.base4 + q];
    if (USE_LDS) {
      accumulate<L, PM1>(h, x.x, (int32_t)(int8_t)(wv), lds);
      accumulate<L, PM1>(h, x.y, (int32_t)(int8_t)(wv >> 8), lds);
      accumulate<L, PM1>(h, x.z, (int32_t)(int8_t)(wv >> 16), lds);
      accumulate<L, PM1>(h, x.w, (int32_t)(int8_t)(wv >> 24), lds);
    } else {
      accumulate<L, PM1>(h, x.x, (int32_t)(int8_t)(wv), a.spins);
      accumulate<L, PM1>(h, x.y, (int32_t)(int8_t)(wv >> 8), a.spins);
      accumulate<L, PM1>(h, x.z, (int32_t)(int8_t)(wv >> 16), a.spins);
      accumulate<L, PM1>(h, x.w, (int32_t)(int8_t)(wv >> 24), a.spins);
    }
  }
#pragma unroll
  for (int j = 0; j < L; ++j) h[j] = wave_sum(h[j]);
  if (lane == 0) {
    const uint32_t own = USE_LDS ? mask_of<L>(lds, slot) : mask_of<L>(a.spins, slot);
    const uint32_t nm = update_mask<L>(h, own, v, t, T, a);
    const uint32_t bit = slot * L;
    const uint32_t change = (own ^ nm) << (bit & 31);
    if (change != 0u) {
      __hip_atomic_fetch_xor(a.spins + (bit >> 5), change, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (USE_LDS) atomicXor(lds + (bit >> 5), change);
    }
  }
}

template <int L, bool PM1, bool USE_LDS>
__global__ __launch_bounds__(kAnnealBlock) void k_anneal(AnnealArgs a) {
  extern __shared__ uint32_t lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int gw = blockIdx.x * (kAnnealBlock / kWave) + (threadIdx.x / kWave);
  const bool multi = gridDim.x > 1;
  if (USE_LDS) {
    const unsigned long long *g64 = reinterpret_cast<const unsigned long long *>(a.spins);
    unsigned long long *l64 = reinterpret_cast<unsigned long long *>(lds);
    for (uint32_t i = threadIdx.x; i < a.n_words / 2; i += blockDim.x) l64[i] = ld_coherent64(g64 + i);
    __syncthreads();
  }
  uint32_t target = 0;
  for (int64_t t = a.t_begin; t < a.t_end; ++t) {
    const uint32_t T = a.thr[t];
    for (int32_t ph = 0; ph < a.n_phases; ++ph) {
      const uint32_t *wp = a.wave_ptr + (size_t)ph * (a.nw + 1) + gw;
      const uint32_t ib = wp[0], ie = wp[1];
      for (uint32_t i = ib; i < ie; ++i) {
        const Item it = a.items[i];
        if (it.kind == kItemSlice)
          run_slice<L, PM1, USE_LDS>(a, it, lds, lane, (uint32_t)t, T);
        else
          run_long<L, PM1, USE_LDS>(a, it, lds, lane, (uint32_t)t, T);
      }
      if (multi) {
        if (!a.async_mode) {
          target += gridDim.x;
          if (!grid_barrier(a.bar, target, a.spin_limit)) return;
        } else {
          __syncthreads();
        }
        if (USE_LDS) {
          // refresh this class's spins from the coherent global state
          const unsigned long long *g64 = reinterpret_cast<const unsigned long long *>(a.spins);
          unsigned long long *l64 = reinterpret_cast<unsigned long long *>(lds);
          const uint32_t b = a.cls_w64[ph], e = a.cls_w64[ph + 1];
          for (uint32_t i = b + threadIdx.x; i < e; i += blockDim.x) l64[i] = ld_coherent64(g64 + i);
        }
        __syncthreads();
      } else {
        // one workgroup: its LDS copy is current; without one, make this
        // phase's global writes visible to the next phase's plain loads
        if (!USE_LDS) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (!USE_LDS) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    if (multi && a.async_mode) {
      // sweeps stay synchronised: nobody starts sweep t+1 before all finished t
      target += gridDim.x;
      if (!grid_barrier(a.bar, target, a.spin_limit)) return;
    }
  }
}

// ---------------------------------------------------------------------------
// Spin initialisation and transfer
// ---------------------------------------------------------------------------
template <int L>
__global__ void k_randomize(uint32_t *spins, const int32_t *vid, uint32_t n_words, uint32_t r0,
                            uint32_t r_count, uint32_t k0, uint32_t k1) {
  constexpr int P = 32 / L;
  for (uint32_t wi = blockIdx.x * blockDim.x + threadIdx.x; wi < n_words; wi += gridDim.x * blockDim.x) {
    uint32_t word = 0;
    for (int i = 0; i < P; ++i) {
      const int32_t v = vid[wi * P + i];
      if (v < 0) continue;
      for (uint32_t j = 0; j < (uint32_t)L && j < r_count; ++j) {
        const uint32_t x = philox_w0((uint32_t)v, 0u, r0 + j, 1u, k0, k1);
        word |= (x >> 31) << (i * L + j);
      }
    }
    spins[wi] = word;
  }
}

template <int L>
__global__ void k_set_spins(uint32_t *spins, const int32_t *vid, uint32_t n_words, const int8_t *src,
                            int64_t n, uint32_t r0, uint32_t r_count) {
  constexpr int P = 32 / L;
  for (uint32_t wi = blockIdx.x * blockDim.x + threadIdx.x; wi < n_words; wi += gridDim.x * blockDim.x) {
    uint32_t word = 0;
    for (int i = 0; i < P; ++i) {
      const int32_t v = vid[wi * P + i];
      if (v < 0) continue;
      for (uint32_t j = 0; j < (uint32_t)L && j < r_count; ++j)
        word |= (src[(int64_t)(r0 + j) * n + v] > 0 ? 1u : 0u) << (i * L + j);
    }
    spins[wi] = word;
  }
}

template <int L>
__global__ void k_get_spins(const uint32_t *spins, const int32_t *vid, uint32_t n_slots, int8_t *dst,
                            int64_t n, uint32_t r0, uint32_t r_count) {
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_slots; s += gridDim.x * blockDim.x) {
    const int32_t v = vid[s];
    if (v < 0) continue;
    const uint32_t m = mask_of<L>(spins, s);
    for (uint32_t j = 0; j < (uint32_t)L && j < r_count; ++j)
      dst[(int64_t)(r0 + j) * n + v] = ((m >> j) & 1u) ? (int8_t)1 : (int8_t)-1;
  }
}

__global__ void k_check_spins(const int8_t *src, int64_t count, uint32_t *flag) {
  uint32_t bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= (src[i] != 1 && src[i] != -1) ? 1u : 0u;
  if (bad) atomicOr(flag, 1u);
}

__global__ void k_cut_finalize(const unsigned long long *sums, int32_t R, int64_t *cut, int64_t *energy) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R; i += gridDim.x * blockDim.x) {
    cut[i] = (int64_t)sums[2 * i + 1] / 2;
    if (energy != nullptr) energy[i] = (int64_t)sums[2 * i] / 2;
  }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t count, uint32_t value) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = value;
}

// ---------------------------------------------------------------------------
// Cut and energy (Eq. 4 and Eq. 5 with J = -w) of one replica bit, summed
// over directed entries (each undirected edge twice).
// ---------------------------------------------------------------------------
template <int L, bool PM1>
__global__ __launch_bounds__(256) void k_cut(CutArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t n_waves = gridDim.x * blockDim.x / kWave;
  long long e_sum = 0, c_sum = 0;
  for (uint32_t i = wave; i < a.n_items; i += n_waves) {
    const Item it = a.items[i];
    const bool slice = it.kind == kItemSlice;
    const uint32_t slot = slice ? it.id * kSliceRows + lane : it.id;
    const uint32_t own = (mask_of<L>(a.spins, slot) >> a.bit) & 1u;
    int32_t e_part = 0, c_part = 0;
    const uint32_t q0 = slice ? 0u : (uint32_t)lane;
    const uint32_t qs = slice ? 1u : (uint32_t)kWave;
    for (uint32_t q = q0; q < it.len4; q += qs) {
      const size_t c = slice ? (size_t)it.base4 + (size_t)q * kSliceRows + lane : (size_t)it.base4 + q;
      const uint4 x4 = a.entries[c];
      const uint32_t wv = PM1 ? 0u : a.wts4[c];
      const uint32_t xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t x = xs[k];
        int32_t w;
        uint32_t nb;
        if (PM1) {
          if (x == kSentinel) continue;
          w = (x & kSignBit) ? -1 : 1;
          nb = x & ~kSignBit;
        } else {
          w = (int32_t)(int8_t)(wv >> (8 * k));
          nb = x;
        }
        const uint32_t other = (mask_of<L>(a.spins, nb) >> a.bit) & 1u;
        e_part += (own == other) ? w : -w;
        c_part += (own != other) ? w : 0;
      }
    }
    e_sum += e_part;
    c_sum += c_part;
  }
  e_sum = wave_sum(e_sum);
  c_sum = wave_sum(c_sum);
  __shared__ long long s_e[4], s_c[4];
  const int wib = threadIdx.x / kWave;
  if (lane == 0) { s_e[wib] = e_sum; s_c[wib] = c_sum; }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long te = 0, tc = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) { te += s_e[i]; tc += s_c[i]; }
    atomicAdd(a.out, (unsigned long long)te);
    atomicAdd(a.out + 1, (unsigned long long)tc);
  }
}

template <typename K>
hipError_t set_lds_limit(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int L, bool PM1, bool USE_LDS>
hipError_t launch_anneal_t(const AnnealArgs &a, int grid, size_t lds_bytes, hipStream_t s) {
  auto kern = k_anneal<L, PM1, USE_LDS>;
  if (USE_LDS) {
    hipError_t e = set_lds_limit(kern, lds_bytes);
    if (e != hipSuccess) return e;
  }
  AnnealArgs copy = a;
  void *args[] = {&copy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(grid), dim3(kAnnealBlock),
                                    args, USE_LDS ? (unsigned)lds_bytes : 0u, s);
}

template <int L, bool PM1, bool USE_LDS>
hipError_t occupancy_t(int *blocks, size_t lds_bytes) {
  auto kern = k_anneal<L, PM1, USE_LDS>;
  if (USE_LDS) {
    hipError_t e = set_lds_limit(kern, lds_bytes);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, reinterpret_cast<const void *>(kern),
                                                      kAnnealBlock, USE_LDS ? lds_bytes : 0);
}

}  // namespace

#define ISING_DISPATCH_L(L_, FN, ...)                    \
  switch (L_) {                                          \
    case 1: return FN<1>(__VA_ARGS__);                   \
    case 2: return FN<2>(__VA_ARGS__);                   \
    case 4: return FN<4>(__VA_ARGS__);                   \
    case 8: return FN<8>(__VA_ARGS__);                   \
    case 16: return FN<16>(__VA_ARGS__);                 \
    case 32: return FN<32>(__VA_ARGS__);                 \
    default: return hipErrorInvalidValue;                \
  }

namespace {
template <int L>
hipError_t anneal_L(const AnnealArgs &a, bool pm1, bool use_lds, int grid, size_t lds, hipStream_t s) {
  if (pm1) return use_lds ? launch_anneal_t<L, true, true>(a, grid, lds, s) : launch_anneal_t<L, true, false>(a, grid, lds, s);
  return use_lds ? launch_anneal_t<L, false, true>(a, grid, lds, s) : launch_anneal_t<L, false, false>(a, grid, lds, s);
}
template <int L>
hipError_t occ_L(bool pm1, bool use_lds, size_t lds, int *blocks) {
  if (pm1) return use_lds ? occupancy_t<L, true, true>(blocks, lds) : occupancy_t<L, true, false>(blocks, lds);
  return use_lds ? occupancy_t<L, false, true>(blocks, lds) : occupancy_t<L, false, false>(blocks, lds);
}
template <int L>
hipError_t randomize_L(uint32_t *spins, const int32_t *vid, uint32_t n_words, uint32_t r0, uint32_t rc,
                       uint64_t seed, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(4096u, (n_words + 255) / 256 + 1);
  hipLaunchKernelGGL(k_randomize<L>, dim3(grid), dim3(256), 0, s, spins, vid, n_words, r0, rc,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}
template <int L>
hipError_t set_L(uint32_t *spins, const int32_t *vid, uint32_t n_words, const int8_t *src, int64_t n,
                 uint32_t r0, uint32_t rc, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(4096u, (n_words + 255) / 256 + 1);
  hipLaunchKernelGGL(k_set_spins<L>, dim3(grid), dim3(256), 0, s, spins, vid, n_words, src, n, r0, rc);
  return hipGetLastError();
}
template <int L>
hipError_t get_L(const uint32_t *spins, const int32_t *vid, uint32_t n_slots, int8_t *dst, int64_t n,
                 uint32_t r0, uint32_t rc, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(4096u, (n_slots + 255) / 256 + 1);
  hipLaunchKernelGGL(k_get_spins<L>, dim3(grid), dim3(256), 0, s, spins, vid, n_slots, dst, n, r0, rc);
  return hipGetLastError();
}
template <int L>
hipError_t cut_L(const CutArgs &a, bool pm1, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(2048u, a.n_items / 4 + 1);
  if (pm1)
    hipLaunchKernelGGL((k_cut<L, true>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_cut<L, false>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_anneal(int L, bool pm1, bool use_lds, const AnnealArgs &a, int grid, size_t lds_bytes,
                         hipStream_t s) {
  ISING_DISPATCH_L(L, anneal_L, a, pm1, use_lds, grid, lds_bytes, s);
}

hipError_t anneal_occupancy(int L, bool pm1, bool use_lds, size_t lds_bytes, int *blocks_per_cu) {
  ISING_DISPATCH_L(L, occ_L, pm1, use_lds, lds_bytes, blocks_per_cu);
}

hipError_t launch_randomize(int L, uint32_t *spins, const int32_t *vid, uint32_t n_words, uint32_t r0,
                            uint32_t r_count, uint64_t seed, hipStream_t s) {
  ISING_DISPATCH_L(L, randomize_L, spins, vid, n_words, r0, r_count, seed, s);
}

hipError_t launch_set_spins(int L, uint32_t *spins, const int32_t *vid, uint32_t n_words, const int8_t *src,
                            int64_t n, uint32_t r0, uint32_t r_count, hipStream_t s) {
  ISING_DISPATCH_L(L, set_L, spins, vid, n_words, src, n, r0, r_count, s);
}

hipError_t launch_get_spins(int L, const uint32_t *spins, const int32_t *vid, uint32_t n_slots, int8_t *dst,
                            int64_t n, uint32_t r0, uint32_t r_count, hipStream_t s) {
  ISING_DISPATCH_L(L, get_L, spins, vid, n_slots, dst, n, r0, r_count, s);
}

hipError_t launch_cut(int L, bool pm1, const CutArgs &a, hipStream_t s) {
  ISING_DISPATCH_L(L, cut_L, a, pm1, s);
}

hipError_t launch_check_spins(const int8_t *src, int64_t count, uint32_t *flag, hipStream_t s) {
  const int grid = (int)std::min<int64_t>(4096, count / 256 + 1);
  hipLaunchKernelGGL(k_check_spins, dim3(grid), dim3(256), 0, s, src, count, flag);
  return hipGetLastError();
}

hipError_t launch_cut_finalize(const unsigned long long *sums, int32_t R, int64_t *cut, int64_t *energy,
                               hipStream_t s) {
  const int grid = (int)std::min<int32_t>(64, R / 256 + 1);
  hipLaunchKernelGGL(k_cut_finalize, dim3(grid), dim3(256), 0, s, sums, R, cut, energy);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t count, uint32_t value, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(1024u, count / 256 + 1);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

}  // namespace ising
