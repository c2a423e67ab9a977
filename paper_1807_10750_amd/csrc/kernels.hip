// kernels.hip -- gfx950 kernels of the Ising max-cut annealer.
//
// The sweep follows the annealed local update of Cook et al. (arXiv
// 1807.10750): each spin takes the value that minimises its local energy
// given its neighbours (Sec. II-A, Eq. 2, with J = -w so that low energy is
// a large cut, Sec. III Eq. 4-5), then flips with the sweep's probability F_p
// (Sec. IV-B, Algorithm 2).  Flip draws come from Philox4x32-10 (Salmon et
// al., SC'11): replica r of vertex v in sweep t uses word (t mod 4) of the
// block at counter {v, t div 4, r, 0}, key = seed, so one block serves four
// consecutive sweeps.
//
// Work is issued in phases, each a run of classes.  In deterministic mode a
// phase is one colour class, which makes the result equal to a sequential
// sweep in (colour, id) order.  In async mode a phase is a run of classes
// (or one near-independent part) with few edges inside, so neighbours inside
// a phase update concurrently and read each other's value from this sweep or
// the previous one, as in the paper's unsynchronised update, while every
// sweep stays synchronised.  Every
// wavefront keeps the loads of its next item in flight while it computes
// the current one.
//
// Spin state is an L-bit mask per slot (replica bits) packed in uint32
// words.  When it fits, each workgroup keeps a copy of the whole state in
// LDS and neighbour gathers are LDS reads; the edge stream is read once per
// sweep with 16-byte coalesced loads, or, with +-1 weights and one replica
// bit per slot, once per call into registers that every wavefront keeps for
// all its sweeps (its items never change within a call).
//
// Phase ends of a multi-workgroup launch with the LDS copy synchronise
// through the data itself.  During the call the spin words live in
// exchange words: word i in bits [31:0] of a 64-bit word, in bits [57:32]
// the number of its bits written so far in the call, and in bits [63:58]
// cover[i], the bits of the word that items write each sweep (32 unless a
// colour class ends inside the word).  A writer adds (new bits - old bits)
// + (bits it covers << 32) in one 64-bit atomic add (its bits are disjoint
// from every other writer's, so the difference replaces exactly them and
// never carries into the count); every covered bit is written once per
// sweep, so after sweep k of the call the count of word i is cover[i] * k
// (an item that writes a word whole stores it outright with that count).
// A phase ends with an arrival of every workgroup, a no-return add on one
// of 128 counters, issued without waiting for its writes to land; once all
// have arrived a workgroup copies the phase's words into
// LDS, and the counts show which words still have a write in flight (those
// are read again).  No store-completion wait, no returned atomic and no
// second counter level sit on that path.  Arrivals also keep every
// workgroup within one phase of the others, so no word is overwritten
// before every workgroup has copied it.  Without the LDS copy, phases end
// with a counter-tree grid barrier and neighbours are read from global
// memory.
// All cross-workgroup spin traffic uses agent-scope atomics, which are
// coherent across the XCDs' L2 caches.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ising {

namespace {

constexpr int kWave = 64;

// Philox4x32-10 (Salmon et al., SC'11): the whole 4-word block.
__device__ __forceinline__ uint4 philox4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    // one 32x32 -> 64 multiply (v_mad_u64_u32) gives both halves of a product
    const uint64_t pa = (uint64_t)0xD2511F53u * c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
    c0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    c1 = (uint32_t)pb;
    c2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c3 = (uint32_t)pa;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t word_of(const uint4 &x, uint32_t i) {
  return i == 0 ? x.x : (i == 1 ? x.y : (i == 2 ? x.z : x.w));
}

__device__ __forceinline__ uint32_t ld_coherent(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_coherent64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Agent-coherent 16-byte load of exchange words 2q and 2q + 1 through a
// buffer resource over the exchange array (cache policy sc1, the one the
// agent-scope loads above get; volatile, so a re-poll is never merged with
// an earlier load; past the array the hardware returns zeros).
constexpr int kCpolSc1Volatile = 16 | (1 << 31);
__device__ __forceinline__ __amdgpu_buffer_rsrc_t xch_rsrc(const unsigned long long *xch, uint32_t n_words) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned long long *>(xch), 0, n_words * 8u, 0x00020000);
}
__device__ __forceinline__ uint4 ld_coherent_pair(__amdgpu_buffer_rsrc_t r, uint32_t q) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, q * 16u, 0, kCpolSc1Volatile));
}
__device__ __forceinline__ uint32_t ld_workgroup(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_coherent(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tables that no kernel writes while it runs (items, wave ranges, class
// word ranges, thresholds) are read through the constant address space, so
// wave-uniform reads become scalar loads.
typedef const __attribute__((address_space(4))) uint32_t ro_u32;
__device__ __forceinline__ uint32_t ro(const uint32_t *p, size_t i) { return ((ro_u32 *)p)[i]; }
__device__ __forceinline__ uint32_t ro(const int32_t *p, size_t i) {
  return ((ro_u32 *)reinterpret_cast<const uint32_t *>(p))[i];
}
// Wave-uniform copy of a value the compiler may hold per lane (a value merged
// after a divergent branch), so that what depends on it stays scalar.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ Item uni(const Item &it) { return Item{uni(it.id), uni(it.base4), uni(it.len4), uni(it.g)}; }

// Item i of a table; the address is made wave-uniform so the read is a
// scalar load (waited for on its own counter, not behind the entry loads).
__device__ __forceinline__ Item ro_item(const Item *p, uint32_t i) {
  const uint64_t addr = reinterpret_cast<uint64_t>(p) + 16ull * i;
  const uint64_t ua = ((uint64_t)uni((uint32_t)(addr >> 32)) << 32) | uni((uint32_t)addr);
  ro_u32 *q = (ro_u32 *)reinterpret_cast<const uint32_t *>(ua);
  return Item{q[0], q[1], q[2], q[3]};
}

template <int L>
__device__ __forceinline__ uint32_t lmask() {
  return L == 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
}

// Mask of slot s from a word array (LDS or global) that starts at spin word woff.
template <int L, typename P>
__device__ __forceinline__ uint32_t mask_of(P words, uint32_t s, uint32_t woff = 0) {
  const uint32_t bit = s * L;
  return (words[(bit >> 5) - woff] >> (bit & 31)) & lmask<L>();
}

// Per-entry field accumulation.  With +-1 weights, c[j] counts the entries
// whose neighbour bit (replica j) differs from the entry's sign bit; the
// field is then 2 c[j] - (entries of the row).  With general weights, c[j]
// sums the weights of the entries whose neighbour bit is set and sw sums all
// weights; the field is 2 c[j] - sw.  Padding entries (layout.h) keep both
// forms exact without a test per entry.
template <int L, int ENC, typename P>
__device__ __forceinline__ void accumulate(int32_t (&c)[L], int32_t &sw, uint32_t x, int32_t wv, P words,
                                           uint32_t woff) {
  const uint32_t slot = ENC == kEncPm1 ? (x & ~kSignBit) : (ENC == kEncW8 ? (x & 0xFFFFFFu) : x);
  const uint32_t word = words[((slot * L) >> 5) - woff];
  // bits [4:0] of the offset operand select the bit; for L = 1 those are slot bits [4:0]
  const uint32_t m = L == 1 ? word : word >> ((slot * L) & 31u);
  const uint32_t off0 = L == 1 ? x : 0u;
  if (ENC == kEncPm1) {
    const uint32_t neg = x >> 31;
#pragma unroll
    for (int j = 0; j < L; ++j) c[j] += (int32_t)(__builtin_amdgcn_ubfe(m, off0 + (uint32_t)j, 1u) ^ neg);
  } else {
    const int32_t w = ENC == kEncW8 ? (int32_t)(int8_t)(x >> 24) : wv;
#pragma unroll
    for (int j = 0; j < L; ++j) c[j] += (int32_t)__builtin_amdgcn_ubfe(m, off0 + (uint32_t)j, 1u) * w;
    sw += w;
  }
}

template <int L, int ENC, typename P>
__device__ __forceinline__ void accumulate4(int32_t (&c)[L], int32_t &sw, const uint4 &x, uint32_t wv, P words,
                                            uint32_t woff) {
  accumulate<L, ENC>(c, sw, x.x, (int32_t)(int8_t)(wv), words, woff);
  accumulate<L, ENC>(c, sw, x.y, (int32_t)(int8_t)(wv >> 8), words, woff);
  accumulate<L, ENC>(c, sw, x.z, (int32_t)(int8_t)(wv >> 16), words, woff);
  accumulate<L, ENC>(c, sw, x.w, (int32_t)(int8_t)(wv >> 24), words, woff);
}

// Register-resident +-1 entries: four 24-bit entries (slot in bits [22:0],
// sign in bit 23) packed in three words, so a chunk takes three registers.
__device__ __forceinline__ uint32_t to24(uint32_t x) { return (x & 0x7FFFFFu) | ((x >> 31) << 23); }
__device__ __forceinline__ void pack24(const uint4 &x, uint32_t *w) {
  const uint32_t p0 = to24(x.x), p1 = to24(x.y), p2 = to24(x.z), p3 = to24(x.w);
  w[0] = p0 | (p1 << 24);
  w[1] = (p1 >> 8) | (p2 << 16);
  w[2] = (p2 >> 16) | (p3 << 8);
}
// The chunk's four gathers are issued together and waited for once (left
// to itself the scheduler waited after each).
template <int L, typename P>
__device__ __forceinline__ void accumulate_packed(int32_t (&c)[L], const uint32_t *w, P words) {
  static_assert(L == 1, "resident chunks serve one replica bit per slot");
  const uint32_t e0 = w[0], e1 = __builtin_amdgcn_alignbit(w[1], w[0], 24),
                 e2 = __builtin_amdgcn_alignbit(w[2], w[1], 16), e3 = w[2] >> 8;
  const uint32_t v0 = words[(e0 & 0x7FFFFFu) >> 5], v1 = words[(e1 & 0x7FFFFFu) >> 5],
                 v2 = words[(e2 & 0x7FFFFFu) >> 5], v3 = words[(e3 & 0x7FFFFFu) >> 5];
  // scheduling groups: the address arithmetic, the four LDS reads, the rest
  __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
  __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
  __builtin_amdgcn_sched_group_barrier(0x002, 16, 0);
  // bits [4:0] of an entry are its slot's bit within the word
  c[0] += (int32_t)((__builtin_amdgcn_ubfe(v0, e0, 1u) ^ ((e0 >> 23) & 1u)) +
                    (__builtin_amdgcn_ubfe(v1, e1, 1u) ^ ((e1 >> 23) & 1u)) +
                    (__builtin_amdgcn_ubfe(v2, e2, 1u) ^ ((e2 >> 23) & 1u)) +
                    (__builtin_amdgcn_ubfe(v3, e3, 1u) ^ ((e3 >> 23) & 1u)));
}

// Local update (Eq. 2 with J = -w, a zero field keeps the spin) of every
// replica bit, then the annealing flips (bit j set = flip replica j).
// Padding slots have only padding entries (whose pairs cancel) and draw no flips.
template <int L>
__device__ __forceinline__ uint32_t update_mask(const int32_t (&h)[L], uint32_t own, uint32_t flips) {
  uint32_t nm = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    uint32_t s = (own >> j) & 1u;
    s = h[j] > 0 ? 0u : (h[j] < 0 ? 1u : s);
    nm |= s << j;
  }
  return (nm ^ flips) & lmask<L>();
}

// Flip thresholds of the Philox block that sweep t draws: word k serves sweep
// 4 (t div 4) + k, zero for the block's sweeps before t or past the call.
// They are uniform over the grid, so one set of scalar loads serves a sweep.
struct Thr4 {
  uint32_t k[4];
};

__device__ __forceinline__ Thr4 sweep_thresholds(const AnnealArgs &a, uint32_t t) {
  const uint32_t b = t >> 2, w = t & 3u;
  Thr4 th;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t tk = 4u * b + (uint32_t)k;
    th.k[k] = ((uint32_t)k >= w && (int64_t)tk < a.t_end) ? ro(a.thr, (size_t)((int64_t)tk - a.thr_base)) : 0u;
  }
  return th;
}

// Flip draws of sweep t (reading: word t mod 4 of the Philox block at counter
// {v, t div 4, r, 0}) against the sweep's thresholds th.  Returns this
// sweep's flip bits; the bits of the block's later sweeps t' < t_end are
// returned in later[0..2] (index t' mod 4 - 1).  With a per-vertex flip
// temperature, slot's threshold is min(2^32 - 1, floor(T m / 8)) for its
// multiplier m.
template <int L>
__device__ __forceinline__ uint32_t draw_flips(int32_t v, uint32_t slot, uint32_t t, const AnnealArgs &a,
                                               const Thr4 &th, uint32_t (&later)[3]) {
  const uint32_t b = t >> 2, w = t & 3u;
  uint32_t Tk[4] = {th.k[0], th.k[1], th.k[2], th.k[3]};
  if (a.scale != nullptr) {
    const uint64_t m = a.scale[slot];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t x = ((uint64_t)Tk[k] * m) >> 3;
      Tk[k] = x > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)x;
    }
  }
  uint32_t now = 0;
  later[0] = later[1] = later[2] = 0u;
  if (v < 0 || (Tk[0] | Tk[1] | Tk[2] | Tk[3]) == 0u) return 0u;
#pragma unroll 1
  for (int j = 0; j < L; ++j) {
    if ((uint32_t)j < a.r_count) {
      const uint4 x = philox4((uint32_t)v, b, a.r0 + (uint32_t)j, 0u, a.seed_lo, a.seed_hi);
      const uint32_t f0 = x.x < Tk[0], f1 = x.y < Tk[1], f2 = x.z < Tk[2], f3 = x.w < Tk[3];
      now |= (w == 0 ? f0 : w == 1 ? f1 : w == 2 ? f2 : f3) << j;
      later[0] |= f1 << j;
      later[1] |= f2 << j;
      later[2] |= f3 << j;
    }
  }
  return now;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// ---------------------------------------------------------------------------
// Grid barrier of a cooperative launch without the LDS copy.  Epochs count
// from 1; no workgroup arrives at epoch k + 1 before epoch k is complete, so
// counters suffice.  Workgroups arrive on one of eight group counters
// (blockIdx mod 8, one per XCD), the last arrival of a group bumps the top
// counter, and epoch k is complete when the top counter reaches k times the
// number of groups.  Neighbour reads are then plain loads, so arrivals are
// agent release fences and waits agent acquire fences.  A poll limit bounds
// every wait; hitting it raises the error flag and every workgroup leaves
// the kernel.
// ---------------------------------------------------------------------------
// LDS words of the phase ends: the verdict of a wait (cleared on failure
// only) and the largest sweep gap this workgroup has seen.
struct BarLds {
  uint32_t ok, gap;
};

__device__ __forceinline__ void bar_arrive(const AnnealArgs &a) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t grp = blockIdx.x & 7u;
    const uint32_t gsize = (gridDim.x - grp + 7u) / 8u;
    const uint32_t old = __hip_atomic_fetch_add(a.bar + kBarGroup + 16 * grp, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if ((old + 1u) % gsize == 0u)
      __hip_atomic_fetch_add(a.bar + kBarTop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Polls-limit test shared by every wait: true when this wait must give up
// (its own limit, or another workgroup raised the error flag).
__device__ __forceinline__ bool give_up(const AnnealArgs &a, uint32_t &polls) {
  if (++polls > a.spin_limit ||
      ((polls & 63u) == 0u && __hip_atomic_load(a.bar + kBarErr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
    __hip_atomic_store(a.bar + kBarErr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return false;
}

// Waits until every workgroup has arrived at barrier epoch `target`.
__device__ __forceinline__ bool bar_wait(const AnnealArgs &a, uint32_t target, BarLds &s) {
  const uint32_t n_grp = gridDim.x < 8u ? gridDim.x : 8u;
  if (threadIdx.x == 0) {
    uint32_t polls = 0;
    while (__hip_atomic_load(a.bar + kBarTop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target * n_grp) {
      if (give_up(a, polls)) {
        s.ok = 0u;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s.ok) != 0u;  // wave-uniform, so loops stay scalar
}

// ---------------------------------------------------------------------------
// Exchange words (multi-workgroup launch with the LDS copy; see the header)
// ---------------------------------------------------------------------------
// Publishes a writer's part of exchange word w: its bits go from ov to nv
// and it covers `cover` bits of the word.  (The writer's own LDS update of
// the word needs no ordering against it: a workgroup copies a phase's
// words into LDS only after a workgroup barrier that follows every item of
// the phase, and the barrier waits for all LDS writes.)
__device__ __forceinline__ void xch_add(const AnnealArgs &a, uint32_t w, uint32_t nv, uint32_t ov, uint32_t cover) {
  const unsigned long long add =
      (unsigned long long)((long long)nv - (long long)ov) + ((unsigned long long)cover << 32);
  __hip_atomic_fetch_add(a.xch + w, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A word that one item writes whole (every sweep, so cover 32): stored
// outright with the count it has after sweep t of the call.
__device__ __forceinline__ void xch_store(const AnnealArgs &a, uint32_t w, uint32_t nv, uint32_t t) {
  const uint32_t k = t - (uint32_t)a.t_begin + 1u;
  st_coherent64(a.xch + w, (unsigned long long)nv | ((unsigned long long)(32u * k) << 32) | (32ull << 58));
}

// Arrival at exchange epoch `epoch` (counted from 1 over the launch) and
// the wait for every workgroup's arrival: once all its wavefronts are past
// the phase, workgroup b adds one to counter b mod 128 (no return), and
// epoch e is complete when counter j reaches e times the number of
// workgroups that use it; thread j of the workgroup polls counter j.
// Adds to one address serialise at the memory side (one counter for the
// whole grid measured twice as slow as eight), hence many counters, each
// on its own page.  ahead_gap: the sweep gap to record if another
// workgroup is seen past this epoch already.
__device__ __forceinline__ bool xch_arrive_wait(const AnnealArgs &a, uint32_t epoch, uint32_t ahead_gap, BarLds &s) {
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t C = kArriveCounters;
  __syncthreads();
  if (tid == 0)
    __hip_atomic_fetch_add(a.bar + kBarArrive + kArriveStride * (blockIdx.x % C), 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (tid < C && tid < gridDim.x) {
    const uint32_t want = epoch * ((gridDim.x - tid + C - 1u) / C);
    uint32_t *cnt = a.bar + kBarArrive + kArriveStride * tid;
    uint32_t polls = 0, c;
    while ((c = ld_coherent(cnt)) < want) {
      if (give_up(a, polls)) {
        s.ok = 0u;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (c > want && ahead_gap > 0u) atomicMax(&s.gap, ahead_gap);
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s.ok) != 0u;
}

// End of phase ph of sweep k (1-based within the call): every workgroup
// arrives, then copies the phase's spin words into LDS; a word whose count
// shows a write still in flight is read again until complete.  With one
// phase per sweep a second arrival follows the copy, so no workgroup writes
// the phase's words of the next sweep before every copy is done (with more
// phases the next arrival implies it).  Each thread keeps XB words in
// flight.  Returns false when a wait gave up.
template <uint32_t XB>
__device__ __forceinline__ bool xch_phase_end(const AnnealArgs &a, uint32_t *lds, int32_t ph, bool last_phase,
                                              uint32_t k, uint32_t &epoch, BarLds &s) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  if (!xch_arrive_wait(a, ++epoch, last_phase ? 1u : 0u, s)) return false;
  // complete: the count (bits [57:32]) equals the cover (bits [63:58]) times k
  auto complete = [k](unsigned long long x) {
    const uint32_t hi = (uint32_t)(x >> 32);
    return (hi & 0x3FFFFFFu) == (hi >> 26) * k;
  };
  bool ok = true;
  // the phase's words come in pairs (its range is whole 64-bit units of the
  // spin state): 16-byte loads, XB / 2 in flight per thread, and an 8-byte
  // LDS write when both words are complete
  constexpr uint32_t XP = XB / 2;
  const uint32_t qb = ro(a.cls_w64, ph), qe = ro(a.cls_w64, ph + 1);
  const __amdgpu_buffer_rsrc_t rs = xch_rsrc(a.xch, a.n_words);
  auto put = [&](uint32_t q, const uint4 &v, uint32_t &pend, uint32_t j) {
    const bool c0 = ((pend >> (2 * j)) & 1u) && complete(((unsigned long long)v.y << 32) | v.x);
    const bool c1 = ((pend >> (2 * j + 1)) & 1u) && complete(((unsigned long long)v.w << 32) | v.z);
    if (c0 && c1) {
      *reinterpret_cast<uint2 *>(lds + 2 * q) = make_uint2(v.x, v.z);
    } else {
      if (c0) lds[2 * q] = v.x;
      if (c1) lds[2 * q + 1] = v.z;
    }
    pend &= ~(((c0 ? 1u : 0u) | (c1 ? 2u : 0u)) << (2 * j));
  };
  for (uint32_t q0 = qb + tid; ok && q0 < qe; q0 += XP * nt) {
    uint4 v[XP];
#pragma unroll
    for (uint32_t j = 0; j < XP; ++j)
      if (q0 + j * nt < qe) v[j] = ld_coherent_pair(rs, q0 + j * nt);
    uint32_t pend = 0;
#pragma unroll
    for (uint32_t j = 0; j < XP; ++j)
      if (q0 + j * nt < qe) {
        pend |= 3u << (2 * j);
        put(q0 + j * nt, v[j], pend, j);
      }
    uint32_t polls = 0;
    while (pend != 0u) {
      if (give_up(a, polls)) {
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
#pragma unroll
      for (uint32_t j = 0; j < XP; ++j)
        if ((pend >> (2 * j)) & 3u) v[j] = ld_coherent_pair(rs, q0 + j * nt);
#pragma unroll
      for (uint32_t j = 0; j < XP; ++j)
        if ((pend >> (2 * j)) & 3u) put(q0 + j * nt, v[j], pend, j);
    }
  }
  if (!ok) s.ok = 0u;
  if (a.n_phases == 1 && !xch_arrive_wait(a, ++epoch, 0u, s)) return false;
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s.ok) != 0u;
}

// ---------------------------------------------------------------------------
// Anneal kernel
// ---------------------------------------------------------------------------
template <int L, int ENC>
struct Fetched {
  static constexpr int KM = kmax_for(L, ENC);
  static constexpr int KW = ENC == kEncWide ? KM : 1;
  uint4 e[KM];
  uint32_t w[KW];  // separate weights (kEncWide only)
  int32_t vid;
  int32_t bias;    // 2 (-h) + odd-degree bit of this lane's row (external field), 0 without one
  uint32_t ownw;   // the coherent spin word holding this lane's row
  uint32_t flipw;  // stored flip bits of this sweep (sweeps not divisible by 4)
};

// Issues every load of one item: this lane's row id, its spin word and its
// share of the sliced-ELL chunks (chunks g, g + G, ...).
// plane: flip plane to read for this item's sweep (-1 when the sweep draws).
// RC > 0: the chunks are register-resident; only the row data is loaded.
// XCH: the spin words live in the exchange words during the call; this
// workgroup's LDS copy always holds its own rows' current bits.
template <int L, int ENC, bool FIELD, int RC = 0, bool XCH = false>
__device__ __forceinline__ void fetch(const AnnealArgs &a, const Item &it_in, int lane, Fetched<L, ENC> &f, int plane,
                                      const uint32_t *lds = nullptr) {
  const Item it = uni(it_in);
  constexpr int KM = Fetched<L, ENC>::KM;
  const uint32_t G = it.g, gs = (uint32_t)__builtin_ctz(G), ks = 6u - gs;
  const uint32_t r = (uint32_t)lane >> gs, gl = (uint32_t)lane & (G - 1u);
  const uint32_t slot = it.id + r;
  // the caller id only keys the Philox draws.  With resident state
  // (RC > 0) compute loads these itself: a prefetched register would make
  // every item wait for all earlier stores (one counter covers loads and
  // stores), also in sweeps that load nothing.
  f.vid = RC == 0 && plane < 0 ? a.vid[slot] : 0;
  f.bias = FIELD && RC == 0 ? a.bias[slot] : 0;
  // Only this item (so this workgroup) writes its row's spin and flip bits,
  // and only those bits are used: workgroup-scope loads are enough.
  f.ownw = RC > 0 ? 0u : (XCH ? lds[(slot * L) >> 5] : ld_workgroup(a.spins + ((slot * L) >> 5)));
  f.flipw = RC == 0 && plane >= 0 ? ld_workgroup(a.flips + (size_t)plane * a.n_words + ((slot * L) >> 5)) : 0u;
  // the item's block starts at a wave-uniform address; offsets inside it fit 32 bits
  const uint4 *blk = a.entries + it.base4;
  const uint32_t *wblk = ENC == kEncWide ? a.wts4 + it.base4 : nullptr;
#pragma unroll
  for (int k = 0; k < (RC > 0 ? 0 : KM); ++k) {
    const uint32_t q = gl + (uint32_t)k * G;
    if (q < it.len4) {
      const uint32_t idx = (q << ks) + r;
      f.e[k] = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(blk) + idx * 16u);
      if (ENC == kEncWide)
        f.w[k < Fetched<L, ENC>::KW ? k : 0] =
            *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(wblk) + idx * 4u);
    }
  }
}

// Per-lane state of a wavefront whose items stay the same for a whole call
// (one replica bit per slot).  Item j of the wavefront's sweep order (all
// phases) keeps this lane's row spin in bit j of own and the flip bits of
// the three sweeps after a drawing sweep in bits 3j .. 3j + 2 of flip: only
// that item writes the row, so the registers hold the current values and a
// sweep loads no spin or flip words.  cr is the next item's first chunk
// register, j the next item's index.
struct ResState {
  uint32_t cr, j, own, flip;
  uint32_t pw;              // exchange word with a pending addition (wave-uniform)
  unsigned long long pv;    // the pending addition, 0 when none
};

// Applies a wavefront's pending addition to its exchange word.
__device__ __forceinline__ void flush_pending(const AnnealArgs &a, ResState &rs, int lane) {
  if (rs.pv != 0ull && lane == 0) {
    __hip_atomic_fetch_add(a.xch + rs.pw, rs.pv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  rs.pv = 0ull;
}

// LDS word of the anneal's mirror array past the spin state that holds 0:
// a resident chunk past a lane's share of its row points all four entries
// (sign 0) at it, so it adds nothing to the count and needs no test.
constexpr uint32_t kZeroWord = (uint32_t)(kLdsBudget / 4) + 1u;
static_assert(kZeroWord * 32u < (1u << 23), "the zero word must be addressable by a 24-bit entry");

// Register-resident chunks of one item (+-1 entries): this lane's chunks
// g, g + G, ... go to registers rw[3 cr ...] onwards, packed by pack24; cr
// advances by the item's chunks per lane, ceil(len4 / G), which is the same
// for every lane.  Also loads the row's spin.
template <int RC>
__device__ __forceinline__ void load_resident(const AnnealArgs &a, const Item &it_in, int lane, uint32_t (&rw)[3 * RC],
                                              ResState &rs) {
  const Item it = uni(it_in);
  const uint32_t G = it.g, gs = (uint32_t)__builtin_ctz(G), ks = 6u - gs;
  const uint32_t r = (uint32_t)lane >> gs, gl = (uint32_t)lane & (G - 1u);
  const uint32_t nch = (it.len4 + G - 1u) >> gs;
  const uint4 *blk = a.entries + it.base4;
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    const uint32_t k = (uint32_t)c - rs.cr;
    const uint32_t q = gl + k * G;
    if (k < nch) {
      uint4 x = make_uint4(kZeroWord * 32u, kZeroWord * 32u, kZeroWord * 32u, kZeroWord * 32u);
      if (q < it.len4) x = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(blk) + ((q << ks) + r) * 16u);
      pack24(x, &rw[3 * c]);
    }
  }
  const uint32_t slot = it.id + r;
  const uint32_t ownw = ld_workgroup(a.spins + (slot >> 5));
  rs.own |= ((ownw >> (slot & 31u)) & 1u) << rs.j;
  rs.cr += nch;
  rs.j += 1;
}

// draws: this sweep computes the Philox blocks (t divisible by 4, or the
// first sweep of the call); otherwise the flip bits come from the planes.
// woff: the spin word that lds[0] holds (0 when LDS mirrors the whole state).
// RC > 0: the item's chunks sit in rw from chunk rs->cr on, its spin and
// flip bits in rs (load_resident); rs moves on to the next item.
// XCH: new spin words go to the LDS copy and the exchange words (xch_add)
// instead of the global spin words.
template <int L, int ENC, bool USE_LDS, bool FIELD, int RC = 0, bool XCH = false>
__device__ __forceinline__ void compute(const AnnealArgs &a, const Item &it_in, int lane, const Fetched<L, ENC> &f,
                                        uint32_t *lds, uint32_t t, bool draws, const Thr4 &th, uint32_t woff = 0,
                                        uint32_t *rw = nullptr, ResState *rs = nullptr) {
  static_assert(RC == 0 || L == 1, "resident state holds one replica bit per slot");
  static_assert(RC == 0 || XCH, "resident state publishes through the exchange words");
  static_assert(!XCH || USE_LDS, "the exchange words serve the LDS copy");
  const Item it = uni(it_in);
  constexpr int KM = Fetched<L, ENC>::KM;
  constexpr bool kPm1 = ENC == kEncPm1;
  const uint32_t G = it.g, gs = (uint32_t)__builtin_ctz(G), ks = 6u - gs, K = 64u >> gs;
  const uint32_t r = (uint32_t)lane >> gs, gl = (uint32_t)lane & (G - 1u);
  const uint32_t slot = it.id + r;
  int32_t h[L], sw = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) h[j] = 0;
  if constexpr (RC > 0) {
    const uint32_t nch = (it.len4 + G - 1u) >> gs;
    const uint32_t cb = rs->cr;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      const uint32_t k = (uint32_t)c - cb;
      if (k < nch) {
        // opaque in place: without it the compiler hoists every entry's
        // decoded address out of the sweep loop, three registers per entry
        // (an opaque copy would cost three moves per chunk)
        asm volatile("" : "+v"(rw[3 * c]), "+v"(rw[3 * c + 1]), "+v"(rw[3 * c + 2]));
        accumulate_packed<L>(h, rw + 3 * c, lds);
      }
    }
    rs->cr = cb + nch;
  }
#pragma unroll
  for (int k = 0; k < (RC > 0 ? 0 : KM); ++k) {
    if (gl + (uint32_t)k * G < it.len4) {
      const uint32_t wv = ENC == kEncWide ? f.w[k < Fetched<L, ENC>::KW ? k : 0] : 0u;
      if (USE_LDS)
        accumulate4<L, ENC>(h, sw, f.e[k], wv, lds, woff);
      else
        accumulate4<L, ENC>(h, sw, f.e[k], wv, a.spins, 0u);
    }
  }
  // rows longer than the prefetch depth: the rest of the chunks, four loads in flight
  const uint4 *blk = a.entries + it.base4;
  const uint32_t *wblk = ENC == kEncWide ? a.wts4 + it.base4 : nullptr;
  for (uint32_t q0 = gl + (uint32_t)KM * G; RC == 0 && q0 < it.len4; q0 += 4u * G) {
    uint4 x[4];
    uint32_t wv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t q = q0 + (uint32_t)k * G;
      const uint32_t idx = ((q < it.len4 ? q : q0) << ks) + r;
      x[k] = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(blk) + idx * 16u);
      wv[k] = ENC == kEncWide ? *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(wblk) + idx * 4u)
                              : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (q0 + (uint32_t)k * G < it.len4) {
        if (USE_LDS)
          accumulate4<L, ENC>(h, sw, x[k], wv[k], lds, woff);
        else
          accumulate4<L, ENC>(h, sw, x[k], wv[k], a.spins, 0u);
      }
    }
  }
  for (uint32_t off = 1; off < G; off <<= 1) {
#pragma unroll
    for (int j = 0; j < L; ++j) h[j] += __shfl_xor(h[j], (int)off);
    if (!kPm1) sw += __shfl_xor(sw, (int)off);
  }
  // counts to fields
  const int32_t base = kPm1 ? (int32_t)(it.len4 * 4u) : sw;
#pragma unroll
  for (int j = 0; j < L; ++j) h[j] = 2 * h[j] - base;
  // An external field h enters as -h (the spin follows the sign of
  // h - sum w s).  With +-1 weights a row of odd degree also holds one
  // unpaired pad, which added the row's own spin (+1 or -1) to the count
  // form above; without a field that never changed a decision (the field
  // is odd, hence nonzero), with one it could, so it is taken out here.
  if (FIELD) {
    const int32_t bias = RC > 0 ? a.bias[slot] : f.bias;
    const int32_t hb = bias >> 1;
    const uint32_t odd = kPm1 ? (uint32_t)bias & 1u : 0u;
    const uint32_t own_bits = RC > 0 ? (rs->own >> rs->j) & 1u : (f.ownw >> ((slot * L) & 31u)) & lmask<L>();
#pragma unroll
    for (int j = 0; j < L; ++j) h[j] += hb - (odd ? (int32_t)(((own_bits >> j) & 1u) << 1) - 1 : 0);
  }
  const uint32_t bit0 = slot * L;
  const uint32_t sh = bit0 & 31;
  const uint32_t own = RC > 0 ? (rs->own >> rs->j) & 1u : (f.ownw >> sh) & lmask<L>();
  uint32_t later[3];
  uint32_t flips;
  if (draws)
    flips = draw_flips<L>(RC > 0 ? a.vid[slot] : f.vid, slot, t, a, th, later);
  else if (RC > 0)
    flips = (rs->flip >> (3u * rs->j + (t & 3u) - 1u)) & 1u;  // sweep t's plane is (t mod 4) - 1
  else
    flips = (f.flipw >> sh) & lmask<L>();
  const uint32_t nm = update_mask<L>(h, own, flips);
  if constexpr (RC > 0) {
    const uint32_t jb = rs->j;
    rs->own = (rs->own & ~(1u << jb)) | (nm << jb);
    if (draws) rs->flip = (rs->flip & ~(7u << (3u * jb))) | ((later[0] | (later[1] << 1) | (later[2] << 2)) << (3u * jb));
    rs->j = jb + 1u;
  }
  const bool rep = gl == 0u;
  if (K * L >= 32u) {
    // the item owns whole words
    if (L == 1 && G == 1u) {
      const unsigned long long b = __ballot(nm & 1u);
      if constexpr (XCH) {
        if (lane < 2) {
          const uint32_t w = (it.id >> 5) + (uint32_t)lane;
          const uint32_t nv = (uint32_t)(b >> (32 * lane));
          lds[w] = nv;
          xch_store(a, w, nv, t);
        }
      } else if (lane == 0) {
        st_coherent64(reinterpret_cast<unsigned long long *>(a.spins) + (it.id >> 6), b);
        if (USE_LDS) reinterpret_cast<unsigned long long *>(lds)[(it.id >> 6) - (woff >> 1)] = b;
      }
      if (RC == 0 && draws) {
        const uint32_t first = t & 3u;  // planes first .. 2 hold sweeps first+1 .. 3
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if ((uint32_t)k < first) continue;
          const unsigned long long fb = __ballot(later[k] & 1u);
          if (lane == 0)
            st_coherent64(reinterpret_cast<unsigned long long *>(a.flips + (size_t)k * a.n_words) + (it.id >> 6), fb);
        }
      }
    } else {
      constexpr uint32_t P = 32u / L;  // rows per word
      uint32_t val = rep ? nm << sh : 0u;
      for (uint32_t off = G; off < G * P; off <<= 1) val |= __shfl_xor(val, (int)off);
      if (rep && (r % P) == 0u) {
        if constexpr (XCH) {
          lds[bit0 >> 5] = val;
          xch_store(a, bit0 >> 5, val, t);
        } else {
          st_coherent(a.spins + (bit0 >> 5), val);
          if (USE_LDS) lds[(bit0 >> 5) - woff] = val;
        }
      }
      if (RC == 0 && draws) {
        const uint32_t first = t & 3u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if ((uint32_t)k < first) continue;
          uint32_t fv = rep ? later[k] << sh : 0u;
          for (uint32_t off = G; off < G * P; off <<= 1) fv |= __shfl_xor(fv, (int)off);
          if (rep && (r % P) == 0u) st_coherent(a.flips + (size_t)k * a.n_words + (bit0 >> 5), fv);
        }
      }
    }
  } else {
    // all K rows share one word with other items: the exact change of this
    // item's bits (XOR for the LDS copy, a difference for the exchange word)
    uint32_t chg = rep ? (own ^ nm) << sh : 0u;
    uint32_t nv = XCH && rep ? nm << sh : 0u;
    for (uint32_t off = G; off < 64u; off <<= 1) {
      chg |= __shfl_xor(chg, (int)off);
      if (XCH) nv |= __shfl_xor(nv, (int)off);
    }
    if constexpr (RC > 0) {
      // consecutive items of a wavefront often share the word: their
      // additions are combined into one (the LDS copy changes at once)
      const uint32_t wd = uni(bit0 >> 5), cu = uni(chg), nu = uni(nv);
      if (lane == 0 && cu != 0u) atomicXor(lds + wd, cu);
      if (wd != rs->pw) {
        flush_pending(a, *rs, lane);
        rs->pw = wd;
      }
      rs->pv += (unsigned long long)((long long)nu - (long long)(nu ^ cu)) + ((unsigned long long)(K * L) << 32);
    } else if constexpr (XCH) {
      if (lane == 0) {
        if (chg != 0u) atomicXor(lds + (bit0 >> 5), chg);
        xch_add(a, bit0 >> 5, nv, nv ^ chg, K * L);
      }
    } else if (lane == 0 && chg != 0u) {
      __hip_atomic_fetch_xor(a.spins + (bit0 >> 5), chg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (USE_LDS) atomicXor(lds + ((bit0 >> 5) - woff), chg);
    }
    if (RC == 0 && draws) {
      // this item's bits of the word: clear, then set
      uint32_t span = rep ? lmask<L>() << sh : 0u;
      for (uint32_t off = G; off < 64u; off <<= 1) span |= __shfl_xor(span, (int)off);
      const uint32_t first = t & 3u;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if ((uint32_t)k < first) continue;
        uint32_t fv = rep ? later[k] << sh : 0u;
        for (uint32_t off = G; off < 64u; off <<= 1) fv |= __shfl_xor(fv, (int)off);
        if (lane == 0) {
          uint32_t *w = a.flips + (size_t)k * a.n_words + (bit0 >> 5);
          __hip_atomic_fetch_and(w, ~span, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (fv != 0u) __hip_atomic_fetch_or(w, fv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

// Copies spin words [b, e) (64-bit units) from the coherent global state into
// LDS; the calling threads split the range as (first, stride).  Each thread
// issues up to eight loads before it waits, so a refresh of up to 64 KiB per
// 1024 threads costs one round trip to memory instead of eight.
__device__ __forceinline__ void restage(const AnnealArgs &a, uint32_t *lds, uint32_t b, uint32_t e,
                                        uint32_t first, uint32_t stride) {
  constexpr uint32_t kBatch = 8;
  const unsigned long long *g64 = reinterpret_cast<const unsigned long long *>(a.spins);
  unsigned long long *l64 = reinterpret_cast<unsigned long long *>(lds);
  for (uint32_t i0 = b + first; i0 < e; i0 += kBatch * stride) {
    unsigned long long v[kBatch];
#pragma unroll
    for (uint32_t k = 0; k < kBatch; ++k) {
      const uint32_t i = i0 + k * stride;
      v[k] = i < e ? ld_coherent64(g64 + i) : 0ull;
    }
#pragma unroll
    for (uint32_t k = 0; k < kBatch; ++k) {
      const uint32_t i = i0 + k * stride;
      if (i < e) l64[i] = v[k];
    }
  }
}

// RC > 0: each wavefront keeps its items' +-1 entries in registers for the
// whole call (at most RC chunks per lane), so a sweep reads no edge stream.
template <int L, int ENC, bool USE_LDS, bool FIELD, int RC = 0>
__global__ __launch_bounds__(kAnnealBlock) void k_anneal(AnnealArgs a) {
  static_assert(RC == 0 || (USE_LDS && ENC == kEncPm1), "resident entries need the LDS mirror and +-1 entries");
  // spin mirror (with the zero word of resident chunks after it)
  __shared__ uint32_t mirror[USE_LDS ? kLdsBudget / 4 + 4 : 4];
  __shared__ BarLds s_bar;
  uint32_t *const lds = mirror;
  constexpr int kWaves = kAnnealBlock / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int gw = blockIdx.x * kWaves + wib;
  const bool multi = gridDim.x > 1;
  // Pipeline shape that fits the registers: two items in flight (three
  // buffers), one item in flight unrolled, or one item in flight rolled.
  constexpr bool kDeep = ENC == kEncPm1 && L <= 4 && RC == 0;
  constexpr bool kUnrolled = L <= 4 && RC == 0;
  if (threadIdx.x == 0) {
    s_bar.ok = 1u;
    s_bar.gap = 0u;
  }
  if (USE_LDS) {
    if (RC > 0 && threadIdx.x == 0) mirror[kZeroWord] = 0u;
    restage(a, lds, 0, a.n_words / 2, threadIdx.x, blockDim.x);
  }
  __syncthreads();
  if (a.n_phases <= 0 || a.t_begin >= a.t_end) return;
  // item range of (phase, wavefront): wave_ptr[2 (phase * nw + gw)] .. [+ 1]
  auto range_at = [&](int32_t ph) -> size_t { return ((size_t)ph * (size_t)a.nw + (size_t)gw) * 2; };
  // resident chunks of this wavefront's items, phase by phase in item order
  // (the order the sweeps visit them); cr is the next chunk's register
  uint32_t rw[RC > 0 ? 3 * RC : 3] = {};
  ResState rs{0u, 0u, 0u, 0u, 0u, 0ull};
  if constexpr (RC > 0) {
    for (int32_t ph = 0; ph < a.n_phases; ++ph) {
      const uint32_t b = ro(a.wave_ptr, range_at(ph)), e = ro(a.wave_ptr, range_at(ph) + 1);
      for (uint32_t i = b; i < e; ++i) load_resident<RC>(a, ro_item(a.items, i), lane, rw, rs);
    }
  }
  // sweep t draws Philox blocks when t is divisible by 4 or starts the call;
  // otherwise its flip bits sit in plane (t mod 4) - 1
  auto plane_of = [&](int64_t t) -> int { return (t == a.t_begin || (t & 3) == 0) ? -1 : (int)(t & 3) - 1; };
  uint32_t epoch = 0;
  uint32_t ib = ro(a.wave_ptr, range_at(0)), ie = ro(a.wave_ptr, range_at(0) + 1);
  Fetched<L, ENC> fa, fb, fc;
  Item ita;
  if (ib < ie) {
    ita = ro_item(a.items, ib);
    fetch<L, ENC, FIELD, RC, USE_LDS>(a, ita, lane, fa, plane_of(a.t_begin), lds);
  }
  for (int64_t t = a.t_begin; t < a.t_end; ++t) {
    const int plane = plane_of(t);
    const bool draws = plane < 0;
    const Thr4 th = draws ? sweep_thresholds(a, (uint32_t)t) : Thr4{};
    rs.cr = 0;
    rs.j = 0;
    for (int32_t ph = 0; ph < a.n_phases; ++ph) {
      // vmcnt(0) before the items, where nothing is in flight any more (the
      // phase end copied, and waited for, every word): without it the
      // compiler, unsure whether a load of the phase end is still in flight
      // at the item loop's head, waits there on every item for every
      // earlier memory operation, the previous item's exchange store included.
      if constexpr (RC > 0) __builtin_amdgcn_s_waitcnt(0x0F70);
      // Items of this phase.  On entry fa holds the loads of item ib.  The
      // loop is unrolled by the pipeline depth so the buffers change roles
      // without register copies (a copy would wait for its loads).
      // pre: the metadata of the next item to fetch, read one step before
      // its fetch so the scalar load is not waited for at the fetch
      if (kDeep) {
        // two items ahead: fa, fb, fc in rotation
        Item itb, itc, pre;
        if (ib + 1 < ie) {
          itb = ro_item(a.items, ib + 1);
          fetch<L, ENC, FIELD, RC, USE_LDS>(a, itb, lane, fb, plane, lds);
        }
        if (ib + 2 < ie) pre = ro_item(a.items, ib + 2);
        for (uint32_t i = ib; i < ie; i += 3) {
          if (i + 2 < ie) {
            itc = pre;
            fetch<L, ENC, FIELD, RC, USE_LDS>(a, itc, lane, fc, plane, lds);
            if (i + 3 < ie) pre = ro_item(a.items, i + 3);
          }
          compute<L, ENC, USE_LDS, FIELD, RC, USE_LDS>(a, ita, lane, fa, lds, (uint32_t)t, draws, th, 0u, rw, &rs);
          if (i + 1 >= ie) break;
          if (i + 3 < ie) {
            ita = pre;
            fetch<L, ENC, FIELD, RC, USE_LDS>(a, ita, lane, fa, plane, lds);
            if (i + 4 < ie) pre = ro_item(a.items, i + 4);
          }
          compute<L, ENC, USE_LDS, FIELD, RC, USE_LDS>(a, itb, lane, fb, lds, (uint32_t)t, draws, th, 0u, rw, &rs);
          if (i + 2 >= ie) break;
          if (i + 4 < ie) {
            itb = pre;
            fetch<L, ENC, FIELD, RC, USE_LDS>(a, itb, lane, fb, plane, lds);
            if (i + 5 < ie) pre = ro_item(a.items, i + 5);
          }
          compute<L, ENC, USE_LDS, FIELD, RC, USE_LDS>(a, itc, lane, fc, lds, (uint32_t)t, draws, th, 0u, rw, &rs);
        }
      } else if (kUnrolled) {
        // one item ahead: fa, fb in rotation
        Item itb, pre;
        if (ib + 1 < ie) pre = ro_item(a.items, ib + 1);
        for (uint32_t i = ib; i < ie; i += 2) {
          if (i + 1 < ie) {
            itb = pre;
            fetch<L, ENC, FIELD, RC, USE_LDS>(a, itb, lane, fb, plane, lds);
            if (i + 2 < ie) pre = ro_item(a.items, i + 2);
          }
          compute<L, ENC, USE_LDS, FIELD, RC, USE_LDS>(a, ita, lane, fa, lds, (uint32_t)t, draws, th, 0u, rw, &rs);
          if (i + 1 >= ie) break;
          if (i + 2 < ie) {
            ita = pre;
            fetch<L, ENC, FIELD, RC, USE_LDS>(a, ita, lane, fa, plane, lds);
            if (i + 3 < ie) pre = ro_item(a.items, i + 3);
          }
          compute<L, ENC, USE_LDS, FIELD, RC, USE_LDS>(a, itb, lane, fb, lds, (uint32_t)t, draws, th, 0u, rw, &rs);
        }
      } else {
        // one item ahead, rolled: the copy waits for the next item's loads
        for (uint32_t i = ib; i < ie; ++i) {
          const bool more = i + 1 < ie;
          Item itb;
          if (more) {
            itb = ro_item(a.items, i + 1);
            fetch<L, ENC, FIELD, RC, USE_LDS>(a, itb, lane, fb, plane, lds);
          }
          compute<L, ENC, USE_LDS, FIELD, RC, USE_LDS>(a, ita, lane, fa, lds, (uint32_t)t, draws, th, 0u, rw, &rs);
          if (more) {
            ita = itb;
            fa = fb;
          }
        }
      }
      // a phase's updates are published before it ends
      if constexpr (RC > 0) flush_pending(a, rs, lane);
      // the next phase's item range and first item
      const bool last_phase = ph + 1 == a.n_phases;
      const int32_t nph = last_phase ? 0 : ph + 1;
      const bool done = last_phase && t + 1 == a.t_end;
      const int next_plane = last_phase ? plane_of(t + 1) : plane;
      ib = ro(a.wave_ptr, range_at(nph));
      ie = ro(a.wave_ptr, range_at(nph) + 1);
      if (done) ie = ib;
      if (multi && USE_LDS) {
        // Every sweep stays synchronised and no value older than the
        // previous sweep is read: after phase ph every workgroup copies the
        // phase's words once complete (xch_phase_end).  In deterministic
        // mode a phase is one colour class, so the sweep equals the
        // sequential one in (colour, id) order.  In async mode a phase is a
        // run of classes: a neighbour of an earlier phase is read at its
        // value of this sweep, a neighbour of a later phase at its value of
        // the previous sweep, and a neighbour of the same phase at either
        // (the race of the paper's update; the LDS copy holds its own
        // workgroup's updates at once and the others' from the previous
        // sweep's copy on).
        if (ib < ie) {
          ita = ro_item(a.items, ib);
          fetch<L, ENC, FIELD, RC, USE_LDS>(a, ita, lane, fa, next_plane, lds);
        }
        if (!done && !xch_phase_end<8u>(a, lds, ph, last_phase, (uint32_t)(t - a.t_begin + 1), epoch, s_bar))
          return;
      } else if (multi) {
        // without the LDS copy: a grid barrier ends every phase
        bar_arrive(a);
        if (ib < ie) {
          ita = ro_item(a.items, ib);
          fetch<L, ENC, FIELD, RC, USE_LDS>(a, ita, lane, fa, next_plane, lds);
        }
        ++epoch;
        if (!bar_wait(a, epoch, s_bar)) return;
      } else {
        // one workgroup: its LDS copy is current
        if (ib < ie) {
          ita = ro_item(a.items, ib);
          fetch<L, ENC, FIELD, RC, USE_LDS>(a, ita, lane, fa, next_plane, lds);
        }
        if (!a.async_mode || last_phase) {
          if (!USE_LDS) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __syncthreads();
          if (!USE_LDS) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
    }
    }
  if (threadIdx.x == 0 && s_bar.gap > 0u) atomicMax(a.bar + kBarGap, s_bar.gap);
}

// ---------------------------------------------------------------------------
// Batched anneal: one workgroup per (bin, replica group).  A bin holds whole
// connected components, so it never reads spins outside its own slot range:
// its LDS copy covers only that range and is always current, colour phases
// need only workgroup syncs, and workgroups never wait for each other.  The
// result equals the single-launch anneal of the union graph.
// ---------------------------------------------------------------------------
template <int L, int ENC, int W, bool FIELD>
__global__ __launch_bounds__(W * kWave) void k_anneal_batch(AnnealArgs args) {
  extern __shared__ uint32_t lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const uint32_t bin = blockIdx.x % (uint32_t)args.n_bins;
  const uint32_t grp = blockIdx.x / (uint32_t)args.n_bins;
  AnnealArgs a = args;
  a.spins = args.spins + (size_t)grp * args.n_words;
  a.flips = args.flips + (size_t)grp * 3 * args.n_words;
  a.r0 = grp * (uint32_t)L;
  a.r_count = args.r_total - a.r0 < (uint32_t)L ? args.r_total - a.r0 : (uint32_t)L;
  const uint32_t w0 = ro(args.bin_words, bin), w1 = ro(args.bin_words, bin + 1);
  for (uint32_t i = threadIdx.x; i < w1 - w0; i += blockDim.x) lds[i] = ld_coherent(a.spins + w0 + i);
  __syncthreads();
  if (a.n_phases <= 0 || a.t_begin >= a.t_end) return;
  auto plane_of = [&](int64_t t) -> int { return (t == a.t_begin || (t & 3) == 0) ? -1 : (int)(t & 3) - 1; };
  const uint32_t *wp = a.wave_ptr + (size_t)bin * a.n_phases * (W + 1) + wib;
  uint32_t ib = ro(wp, 0), ie = ro(wp, 1);
  Fetched<L, ENC> fa, fb;
  Item ita;
  if (ib < ie) {
    ita = ro_item(a.items, ib);
    fetch<L, ENC, FIELD>(a, ita, lane, fa, plane_of(a.t_begin));
  }
  for (int64_t t = a.t_begin; t < a.t_end; ++t) {
    const int plane = plane_of(t);
    const Thr4 th = plane < 0 ? sweep_thresholds(a, (uint32_t)t) : Thr4{};
    for (int32_t ph = 0; ph < a.n_phases; ++ph) {
      // one item ahead, unrolled so fa and fb swap roles without copies
      Item itb;
      for (uint32_t i = ib; i < ie; i += 2) {
        if (i + 1 < ie) {
          itb = ro_item(a.items, i + 1);
          fetch<L, ENC, FIELD>(a, itb, lane, fb, plane);
        }
        compute<L, ENC, true, FIELD>(a, ita, lane, fa, lds, (uint32_t)t, plane < 0, th, w0);
        if (i + 1 >= ie) break;
        if (i + 2 < ie) {
          ita = ro_item(a.items, i + 2);
          fetch<L, ENC, FIELD>(a, ita, lane, fa, plane);
        }
        compute<L, ENC, true, FIELD>(a, itb, lane, fb, lds, (uint32_t)t, plane < 0, th, w0);
      }
      const bool last_phase = ph + 1 == a.n_phases;
      const int32_t nph = last_phase ? 0 : ph + 1;
      const bool done = last_phase && t + 1 == a.t_end;
      ib = ro(wp, (size_t)nph * (W + 1));
      ie = ro(wp, (size_t)nph * (W + 1) + 1);
      if (done) ie = ib;
      if (ib < ie) {
        ita = ro_item(a.items, ib);
        fetch<L, ENC, FIELD>(a, ita, lane, fa, last_phase ? plane_of(t + 1) : plane);
      }
      if (!a.async_mode || last_phase) __syncthreads();
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
        const uint32_t r = r0 + j;
        const uint4 x = philox4((uint32_t)v, 0u, r >> 2, 1u, k0, k1);
        word |= (word_of(x, r & 3u) >> 31) << (i * L + j);
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
    const unsigned long long *p = sums + (size_t)kCutStride * i;
    cut[i] = (int64_t)p[1] / 2;
    if (energy != nullptr) energy[i] = (int64_t)p[0] / 2 + (int64_t)p[2];
  }
}

// Best-of-run tracking.  k_best_select compares each replica's cut with its
// best so far (reset: no best yet), records improvements and marks the
// improved replicas in their group's mask; k_best_merge then copies those
// replicas' bits of the spin state into the best state.
__global__ void k_best_select(const unsigned long long *sums, int32_t R, int32_t L, int32_t reset,
                              int64_t *best, int64_t *cut_out, uint32_t *masks) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R; i += gridDim.x * blockDim.x) {
    const int64_t cut = (int64_t)sums[(size_t)kCutStride * i + 1] / 2;
    if (cut_out != nullptr) cut_out[i] = cut;
    if (reset || cut > best[i]) {
      best[i] = cut;
      atomicOr(masks + i / L, 1u << (i % L));
    }
  }
}

__global__ void k_best_merge(const uint32_t *spins, uint32_t *best, const uint32_t *masks, uint32_t n_words,
                             uint32_t total, int32_t L) {
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < total; w += gridDim.x * blockDim.x) {
    const uint32_t m = masks[w / n_words];
    if (m == 0u) continue;
    uint32_t pat = 0;
    for (int32_t k = 0; k < 32; k += L) pat |= m << k;  // the replica bits of every slot in the word
    best[w] = (best[w] & ~pat) | (spins[w] & pat);
  }
}

// Exchange words of one anneal launch: the spin words with zero counts and
// their covers.
__global__ void k_xch_init(const uint32_t *spins, const uint8_t *cover, unsigned long long *xch, uint32_t n_words) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += gridDim.x * blockDim.x)
    xch[i] = (unsigned long long)spins[i] | ((unsigned long long)cover[i] << 58);
}

// The spin words back from the exchange words after the launch.
__global__ void k_xch_fini(const unsigned long long *xch, uint32_t *spins, uint32_t n_words) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += gridDim.x * blockDim.x)
    spins[i] = (uint32_t)xch[i];
}

__global__ void k_fill_u32(uint32_t *p, uint32_t count, uint32_t value) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = value;
}

// ---------------------------------------------------------------------------
// Cut and energy (Eq. 4 and Eq. 5 with J = -w) of one replica bit, summed
// over directed entries (each undirected edge twice).  With +-1 weights a
// wavefront counts with ballots: for each entry position of a chunk, the
// lanes whose entry is a cut edge of weight +1 and those of weight -1 are
// two 64-bit masks, and popc(first) - popc(second) is the wavefront's
// contribution to the cut; the energy follows from the same masks and the
// signs of all real entries.
// ---------------------------------------------------------------------------
template <int L, int ENC>
__global__ __launch_bounds__(256) void k_cut(CutArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t n_waves = gridDim.x * blockDim.x / kWave;
  long long e_sum = 0, c_sum = 0, f_sum = 0;
  for (uint32_t i = wave; i < a.n_items; i += n_waves) {
    const Item it = ro_item(a.items, i);
    const uint32_t G = it.g, K = 64u / G;
    const uint32_t r = (uint32_t)lane / G, gl = (uint32_t)lane & (G - 1u);
    const uint32_t slot = it.id + r;
    const uint32_t own = (mask_of<L>(a.spins, slot) >> a.bit) & 1u;
    // external field energy -h s, once per row (padding rows carry 0)
    if (a.bias != nullptr && gl == 0u) f_sum += (long long)(a.bias[slot] >> 1) * (own ? 1 : -1);
    int32_t e_part = 0, c_part = 0;
    if constexpr (ENC == kEncPm1) {
      // every lane runs the same number of chunk steps (the item's longest
      // share), so the ballots see the whole wavefront; lanes past their
      // share contribute nothing
      const uint32_t steps = (it.len4 + G - 1u) / G;
      for (uint32_t st = 0; st < steps; ++st) {
        const uint32_t q = gl + st * G;
        const bool live = q < it.len4;
        uint4 x4 = make_uint4(slot, slot, slot, slot);  // padding: names the row itself
        if (live) x4 = a.entries[(size_t)it.base4 + (size_t)q * K + r];
        const uint32_t xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t nb = xs[k] & ~kSignBit;
          const bool real = nb != slot;
          const bool neg = (xs[k] & kSignBit) != 0u;
          const bool cut = real && ((mask_of<L>(a.spins, real ? nb : slot) >> a.bit) & 1u) != own;
          // cut edges of weight +1 and -1; real entries of weight +1 and -1
          const long long cp = __popcll(__ballot(cut && !neg)), cn = __popcll(__ballot(cut && neg));
          const long long rp = __popcll(__ballot(real && !neg)), rn = __popcll(__ballot(real && neg));
          if (lane == 0) {
            c_sum += cp - cn;
            // sum of w s s = sum of w over real entries - 2 (sum of w over cut entries)
            e_sum += (rp - rn) - 2 * (cp - cn);
          }
        }
      }
    }
    for (uint32_t q = gl; ENC != kEncPm1 && q < it.len4; q += G) {
      const size_t c = (size_t)it.base4 + (size_t)q * K + r;
      const uint4 x4 = a.entries[c];
      const uint32_t wv = ENC == kEncWide ? a.wts4[c] : 0u;
      const uint32_t xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t x = xs[k];
        int32_t w;
        uint32_t nb;
        if (ENC == kEncPm1) {
          nb = x & ~kSignBit;
          if (nb == slot) continue;  // padding
          w = (x & kSignBit) ? -1 : 1;
        } else if (ENC == kEncW8) {
          w = (int32_t)(int8_t)(x >> 24);
          nb = x & 0xFFFFFFu;
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
  f_sum = wave_sum(f_sum);
  __shared__ long long s_e[4], s_c[4], s_f[4];
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  if (lane == 0) { s_e[wib] = e_sum; s_c[wib] = c_sum; s_f[wib] = f_sum; }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long te = 0, tc = 0, tf = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) { te += s_e[i]; tc += s_c[i]; tf += s_f[i]; }
    atomicAdd(a.out, (unsigned long long)te);
    atomicAdd(a.out + 1, (unsigned long long)tc);
    if (tf != 0) atomicAdd(a.out + 2, (unsigned long long)tf);
  }
}

template <typename K>
hipError_t set_lds_limit(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int L, int ENC, bool USE_LDS, bool FIELD, int RC = 0>
hipError_t launch_anneal_t(const AnnealArgs &a, int grid, size_t lds_bytes, hipStream_t s) {
  auto kern = k_anneal<L, ENC, USE_LDS, FIELD, RC>;
  if (lds_bytes > kLdsBudget) return hipErrorInvalidValue;
  AnnealArgs copy = a;
  void *args[] = {&copy};
  // Under stream capture the launch becomes an ordinary kernel node: the
  // grid never exceeds what the occupancy query says fits at once, and the
  // barrier's poll limit turns a grid that is not co-resident into an error.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return e;
  if (cap == hipStreamCaptureStatusActive) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kAnnealBlock), 0u, s, copy);
    return hipGetLastError();
  }
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(grid), dim3(kAnnealBlock),
                                    args, 0u, s);
}

template <int L, int ENC, int W, bool FIELD>
hipError_t launch_batch_t(const AnnealArgs &a, int grid, size_t lds_bytes, hipStream_t s) {
  auto kern = k_anneal_batch<L, ENC, W, FIELD>;
  hipError_t e = set_lds_limit(kern, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(W * kWave), (unsigned)lds_bytes, s, a);
  return hipGetLastError();
}

// Co-resident workgroups per CU: the lower of the variants with and
// without an external field, so one grid size fits either launch.
template <int L, int ENC, bool USE_LDS>
hipError_t occupancy_t(int *blocks, size_t lds_bytes) {
  if (lds_bytes > kLdsBudget) return hipErrorInvalidValue;
  int b0 = 0, b1 = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &b0, reinterpret_cast<const void *>(k_anneal<L, ENC, USE_LDS, false>), kAnnealBlock, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &b1, reinterpret_cast<const void *>(k_anneal<L, ENC, USE_LDS, true>), kAnnealBlock, 0);
  *blocks = b0 < b1 ? b0 : b1;
  if constexpr (kHasResident<L, ENC, USE_LDS>) {
    // and the register-resident variants
    const void *res[4] = {reinterpret_cast<const void *>(k_anneal<L, ENC, USE_LDS, false, kResChunks>),
                          reinterpret_cast<const void *>(k_anneal<L, ENC, USE_LDS, true, kResChunks>),
                          reinterpret_cast<const void *>(k_anneal<L, ENC, USE_LDS, false, kResChunksSmall>),
                          reinterpret_cast<const void *>(k_anneal<L, ENC, USE_LDS, true, kResChunksSmall>)};
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, res[k], kAnnealBlock, 0);
      *blocks = std::min(*blocks, b0);
    }
  }
  return e;
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
template <int L, int ENC>
hipError_t anneal_LE(const AnnealArgs &a, bool use_lds, int res_chunks, int grid, size_t lds, hipStream_t s) {
  if (res_chunks != 0) {
    if constexpr (kHasResident<L, ENC, true>) {
      if (!use_lds) return hipErrorInvalidValue;
      if (res_chunks == kResChunksSmall)
        return a.bias != nullptr ? launch_anneal_t<L, ENC, true, true, kResChunksSmall>(a, grid, lds, s)
                                 : launch_anneal_t<L, ENC, true, false, kResChunksSmall>(a, grid, lds, s);
      if (res_chunks == kResChunks)
        return a.bias != nullptr ? launch_anneal_t<L, ENC, true, true, kResChunks>(a, grid, lds, s)
                                 : launch_anneal_t<L, ENC, true, false, kResChunks>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
  }
  if (a.bias != nullptr)
    return use_lds ? launch_anneal_t<L, ENC, true, true>(a, grid, lds, s)
                   : launch_anneal_t<L, ENC, false, true>(a, grid, lds, s);
  return use_lds ? launch_anneal_t<L, ENC, true, false>(a, grid, lds, s)
                 : launch_anneal_t<L, ENC, false, false>(a, grid, lds, s);
}
template <int L>
hipError_t anneal_L(const AnnealArgs &a, int enc, bool use_lds, int res_chunks, int grid, size_t lds, hipStream_t s) {
  if (enc == kEncPm1) return anneal_LE<L, kEncPm1>(a, use_lds, res_chunks, grid, lds, s);
  if (enc == kEncW8) return anneal_LE<L, kEncW8>(a, use_lds, res_chunks, grid, lds, s);
  return anneal_LE<L, kEncWide>(a, use_lds, res_chunks, grid, lds, s);
}
template <int L, int ENC>
hipError_t batch_LE(const AnnealArgs &a, int waves, int grid, size_t lds, hipStream_t s) {
  const bool f = a.bias != nullptr;
  switch (waves) {
    case 4: return f ? launch_batch_t<L, ENC, 4, true>(a, grid, lds, s) : launch_batch_t<L, ENC, 4, false>(a, grid, lds, s);
    case 8: return f ? launch_batch_t<L, ENC, 8, true>(a, grid, lds, s) : launch_batch_t<L, ENC, 8, false>(a, grid, lds, s);
    case 16:
      return f ? launch_batch_t<L, ENC, 16, true>(a, grid, lds, s) : launch_batch_t<L, ENC, 16, false>(a, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}
template <int L>
hipError_t batch_L(const AnnealArgs &a, int enc, int waves, int grid, size_t lds, hipStream_t s) {
  if (enc == kEncPm1) return batch_LE<L, kEncPm1>(a, waves, grid, lds, s);
  if (enc == kEncW8) return batch_LE<L, kEncW8>(a, waves, grid, lds, s);
  return batch_LE<L, kEncWide>(a, waves, grid, lds, s);
}
template <int L, int ENC>
hipError_t occ_LE(bool use_lds, size_t lds, int *blocks) {
  return use_lds ? occupancy_t<L, ENC, true>(blocks, lds) : occupancy_t<L, ENC, false>(blocks, lds);
}
template <int L>
hipError_t occ_L(int enc, bool use_lds, size_t lds, int *blocks) {
  if (enc == kEncPm1) return occ_LE<L, kEncPm1>(use_lds, lds, blocks);
  if (enc == kEncW8) return occ_LE<L, kEncW8>(use_lds, lds, blocks);
  return occ_LE<L, kEncWide>(use_lds, lds, blocks);
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
hipError_t cut_L(const CutArgs &a, int enc, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(2048u, a.n_items / 4 + 1);
  if (enc == kEncPm1)
    hipLaunchKernelGGL((k_cut<L, kEncPm1>), dim3(grid), dim3(256), 0, s, a);
  else if (enc == kEncW8)
    hipLaunchKernelGGL((k_cut<L, kEncW8>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_cut<L, kEncWide>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_best(const unsigned long long *sums, int32_t R, int32_t L, int32_t reset, int64_t *best,
                       int64_t *cut_out, uint32_t *masks, const uint32_t *spins, uint32_t *best_spins,
                       uint32_t n_words, int32_t n_groups, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, masks, (uint32_t)n_groups, 0u);
  hipLaunchKernelGGL(k_best_select, dim3((R + 255) / 256), dim3(256), 0, s, sums, R, L, reset, best, cut_out, masks);
  const uint32_t total = n_words * (uint32_t)n_groups;
  const int grid = (int)std::min<uint32_t>(4096u, (total + 255u) / 256u + 1u);
  hipLaunchKernelGGL(k_best_merge, dim3(grid), dim3(256), 0, s, spins, best_spins, masks, n_words, total, L);
  return hipGetLastError();
}

hipError_t launch_anneal(int L, int enc, bool use_lds, int res_chunks, const AnnealArgs &a, int grid,
                         size_t lds_bytes, hipStream_t s) {
  ISING_DISPATCH_L(L, anneal_L, a, enc, use_lds, res_chunks, grid, lds_bytes, s);
}

hipError_t launch_anneal_batch(int L, int enc, int waves, const AnnealArgs &a, int grid, size_t lds_bytes,
                               hipStream_t s) {
  ISING_DISPATCH_L(L, batch_L, a, enc, waves, grid, lds_bytes, s);
}

hipError_t anneal_occupancy(int L, int enc, bool use_lds, size_t lds_bytes, int *blocks_per_cu) {
  ISING_DISPATCH_L(L, occ_L, enc, use_lds, lds_bytes, blocks_per_cu);
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

hipError_t launch_cut(int L, int enc, const CutArgs &a, hipStream_t s) {
  ISING_DISPATCH_L(L, cut_L, a, enc, s);
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

hipError_t launch_xch_init(const uint32_t *spins, const uint8_t *cover, unsigned long long *xch, uint32_t n_words,
                           hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(1024u, n_words / 256 + 1);
  hipLaunchKernelGGL(k_xch_init, dim3(grid), dim3(256), 0, s, spins, cover, xch, n_words);
  return hipGetLastError();
}

hipError_t launch_xch_fini(const unsigned long long *xch, uint32_t *spins, uint32_t n_words, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(1024u, n_words / 256 + 1);
  hipLaunchKernelGGL(k_xch_fini, dim3(grid), dim3(256), 0, s, xch, spins, n_words);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t count, uint32_t value, hipStream_t s) {
  const int grid = (int)std::min<uint32_t>(1024u, count / 256 + 1);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

}  // namespace ising
