// kernels.h -- launchers of the gfx950 kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "layout.h"

namespace ising {

constexpr int kAnnealBlock = 1024;  // 16 wavefronts per workgroup
// Largest spin state the cooperative anneal mirrors in LDS (a static array
// of the kernel: its address is a compile-time constant).
constexpr size_t kLdsBudget = 160 * 1024 - 2048;
// Register-resident entries (cooperative anneal, +-1 weights, one replica
// bit per slot, LDS mirror): chunks of four entries each lane holds, three
// registers per chunk.  Slots must fit the 23 bits of a packed entry.
constexpr int kResChunks = 24;
// A smaller variant for graphs whose wavefronts hold at most this many: the
// registers it leaves free let the phase-end copy keep twice the loads in
// flight.
constexpr int kResChunksSmall = 18;
// Items per wavefront in that variant: each keeps its row spin and three
// flip bits per lane in two registers (one bit and three bits per item).
constexpr int kResMaxItems = 10;
constexpr int64_t kResMaxSlots = int64_t(1) << 23;
template <int L, int ENC, bool USE_LDS>
constexpr bool kHasResident = L == 1 && ENC == kEncPm1 && USE_LDS;

// res_chunks: 0, or the register-resident variant (kResChunksSmall or
// kResChunks); every wavefront's items must then hold at most that many
// chunks per lane in total (ceil(len4 / g) per item).
hipError_t launch_anneal(int L, int enc, bool use_lds, int res_chunks, const AnnealArgs &a, int grid,
                         size_t lds_bytes, hipStream_t s);
// Batched anneal: grid = n_bins x replica groups, waves per workgroup in {4, 8, 16}.
hipError_t launch_anneal_batch(int L, int enc, int waves, const AnnealArgs &a, int grid, size_t lds_bytes,
                               hipStream_t s);
hipError_t anneal_occupancy(int L, int enc, bool use_lds, size_t lds_bytes, int *blocks_per_cu);
hipError_t launch_randomize(int L, uint32_t *spins, const int32_t *vid, uint32_t n_words, uint32_t r0,
                            uint32_t r_count, uint64_t seed, hipStream_t s);
hipError_t launch_set_spins(int L, uint32_t *spins, const int32_t *vid, uint32_t n_words, const int8_t *src,
                            int64_t n, uint32_t r0, uint32_t r_count, hipStream_t s);
hipError_t launch_get_spins(int L, const uint32_t *spins, const int32_t *vid, uint32_t n_slots, int8_t *dst,
                            int64_t n, uint32_t r0, uint32_t r_count, hipStream_t s);
hipError_t launch_cut(int L, int enc, const CutArgs &a, hipStream_t s);
hipError_t launch_check_spins(const int8_t *src, int64_t count, uint32_t *flag, hipStream_t s);
hipError_t launch_cut_finalize(const unsigned long long *sums, int32_t R, int64_t *cut, int64_t *energy,
                               hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t count, uint32_t value, hipStream_t s);
// Exchange words around a launch with the LDS copy: spin words in with zero
// counts and their covers before, spin words out after.
hipError_t launch_xch_init(const uint32_t *spins, const uint8_t *cover, unsigned long long *xch, uint32_t n_words,
                           hipStream_t s);
hipError_t launch_xch_fini(const unsigned long long *xch, uint32_t *spins, uint32_t n_words, hipStream_t s);
// Best-of-run update from the cut sums of every replica (see k_best_select).
hipError_t launch_best(const unsigned long long *sums, int32_t R, int32_t L, int32_t reset, int64_t *best,
                       int64_t *cut_out, uint32_t *masks, const uint32_t *spins, uint32_t *best_spins,
                       uint32_t n_words, int32_t n_groups, hipStream_t s);

}  // namespace ising
