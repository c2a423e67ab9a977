// layout.h -- device-side data layout of an Ising graph handle (internal).
//
// Vertices are renumbered into "slots": colour class by colour class (the
// classes of the greedy colouring that orders the deterministic sweep), each
// class padded to a multiple of 64 slots, and inside a class by decreasing
// degree.  A work item is one wavefront's worth of rows: K = 64 / G
// consecutive slots, G lanes per row, G in {1, 4, 16, 64} chosen from the
// row degree.  Items start at multiples of K.  The item's edge entries form a
// sliced-ELL block: every row is padded to len4 chunks of 4 entries and chunk
// q of row r sits at uint4 index base4 + q * K + r, so lane (r, g) reads
// chunks g, g + G, g + 2G, ... and every wavefront load covers 1 KiB of
// contiguous memory.
// An edge entry is a uint32 in one of three encodings:
//   kEncPm1  (every weight +-1): slot | sign << 31;
//   kEncW8   (fewer than 2^24 slots): slot | weight << 24;
//   kEncWide (otherwise): slot only, plus one int8 weight per entry in a
//            separate stream.
// Padding entries name the row's own slot (graphs have no self-loops, so an
// entry naming its own row is padding and nothing else).  With general
// weights a pad has weight 0.  With +-1 weights the kernel counts the
// entries whose neighbour bit differs from the sign bit, c, and takes the
// field as 2c - (entries in the row, pads included): the pads come in pairs
// (own, +1), (own, -1), which add exactly one to c whatever the spin, and
// an odd number of pads ends with one (own, +1), which adds the row's own
// bit.  For an odd degree that single pad moves the (odd, hence nonzero)
// field by +1 towards the current spin, so the sign of the field, and the
// tie rule, come out as without padding.
//
// Flip draws: one Philox block per (vertex, replica, 4 sweeps).  The sweep
// that computes a block uses its word for itself and stores the flip bits of
// the block's later sweeps in three bit planes laid out like the spin state.
//
// Spins live as an L-bit mask per slot (bit j = replica j of the group,
// 1 = +1), L in {1,2,4,8,16,32}; the masks of 32/L consecutive slots share
// one uint32 word, so the state of n slots is n*L/32 words.  An item with
// K * L >= 32 owns whole words; smaller items share one word with others.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr uint32_t kSignBit = 0x80000000u;

// Chunks of 4 entries each lane prefetches per item; bounds the degree of a
// row handled with G lanes to 4 * kmax * G (longer rows loop).
enum Encoding { kEncPm1 = 0, kEncW8 = 1, kEncWide = 2 };
constexpr int kmax_for(int L, int enc) { return (L >= 16 || enc == kEncWide || (enc == kEncW8 && L >= 2)) ? 2 : 4; }

// One unit of work for one wavefront.
struct Item {
  uint32_t id;     // first slot (a multiple of K = 64 / g)
  uint32_t base4;  // index of the item's first uint4 chunk in the entry stream
  uint32_t len4;   // chunks per row
  uint32_t g;      // lanes per row: 1, 4, 16 or 64
};

// Words of the per-handle flag buffer.
constexpr int kBarTop = 0;       // grid barrier: epochs completed x groups
constexpr int kBarErr = 1;       // set when a poll limit is hit
constexpr int kBarCheck = 2;     // spin-value check result
constexpr int kBarGap = 3;       // largest sweep gap between workgroups seen at a phase end
constexpr int kBarGroup = 16;    // grid barrier: group counter k at kBarGroup + 16 * k, k < 8
// phase-end arrival counters of the exchange words: counter j (workgroups
// b mod 128 = j) at kBarArrive + j * kArriveStride, each in its own page
constexpr int kArriveCounters = 128;
constexpr int kArriveStride = 1088;  // words: 4 KiB + 256 B, so counters fall in different channels
constexpr int kBarArrive = 1024;
constexpr int kBarWords = kBarArrive + kArriveCounters * kArriveStride;
constexpr int kBarMaxGrid = 1024;  // at most one polling thread per workgroup of the grid

// Arguments of the anneal kernel (passed by value).
struct AnnealArgs {
  const uint4 *entries;      // edge stream, uint4 chunks
  const uint32_t *wts4;      // 4 int8 weights per chunk (general weights only)
  const int32_t *vid;        // slot -> caller vertex id, -1 for padding
  const int32_t *bias;       // slot -> 2 (-h) + (degree odd, +-1 encoding) of the external
                             // field (nullptr: no field); see kernels.hip compute()
  const uint8_t *scale;      // slot -> flip-temperature multiplier m in [0, 15]: the slot flips
                             // iff its draw < min(2^32 - 1, T m / 8) (nullptr: m = 8)
  const Item *items;         // all items, phase by phase
  const uint32_t *wave_ptr;  // cooperative: [n_phases][nw][2] item range (begin, end) of each
                             // wavefront; batched: [bins][phases][waves + 1] prefix offsets
  const uint32_t *cls_w64;   // [n_phases + 1] class boundaries in 64-bit words of the spin state
  uint32_t *spins;           // this replica group's spin words
  uint32_t *flips;           // 3 planes of n_words: flip bits of sweeps 4b+1..4b+3
  // exchange words of a launch with an LDS mirror (see kernels.hip): spin word i in bits
  // [31:0] of xch[i], the count of its bits written so far in this call in bits [57:32], the
  // bits of it that items write each sweep in bits [63:58]
  unsigned long long *xch;
  const uint32_t *thr;       // thresholds: sweep t's at thr[t - thr_base]
  int64_t thr_base;
  uint32_t *bar;             // barrier words (see kBar*), error flag
  uint32_t n_words;          // spin words of the group
  int32_t n_phases;
  int32_t nw;                // wavefronts in the grid
  int32_t async_mode;
  int64_t t_begin, t_end;
  uint32_t seed_lo, seed_hi;
  uint32_t r0;               // replica index of bit 0
  uint32_t r_count;          // replicas of the group in use (<= L)
  uint32_t spin_limit;       // polls of a wait before giving up (error flag)
  // batched launch only
  const uint32_t *bin_words; // [n_bins + 1] first 32-bit spin word of each bin
  int32_t n_bins;            // bins (workgroups per replica group)
  uint32_t r_total;          // replicas of the handle
};

// 64-bit sums per replica in the cut buffer (three used).
constexpr int kCutStride = 4;

struct CutArgs {
  const uint4 *entries;
  const uint32_t *wts4;
  const int32_t *vid;
  const Item *items;
  uint32_t n_items;
  const uint32_t *spins;
  const int32_t *bias;       // as in AnnealArgs
  unsigned long long *out;   // [kCutStride]: over directed entries the sums of w s s and of
                             // w [s != s], then the sum over vertices of -h s
  uint32_t bit;              // replica bit inside the mask
};

}  // namespace ising
