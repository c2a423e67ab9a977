// layout.h -- device-side data layout of an Ising graph handle (internal).
//
// Vertices are renumbered into "slots": colour class by colour class (the
// classes of the greedy colouring that orders the deterministic sweep), each
// class padded to a multiple of 64 slots, and inside a class by decreasing
// degree.  Rows are grouped into slices of 64 consecutive slots, one per
// 64-lane wavefront:
//   * a short slice (max degree <= long threshold) is one work item processed
//     lane-per-row from a sliced-ELL edge block: entry q of row i of the
//     slice lives at uint4 chunk (q / 4) * 64 + i, component q % 4, so each
//     wavefront load reads 1 KiB of contiguous memory;
//   * rows of a long slice are one work item each, processed by a whole
//     wavefront that strides the row's contiguous, 4-padded entry list.
// An edge entry is a uint32: the neighbour's slot, and for graphs whose
// weights are all +-1 the weight's sign in bit 31 (padding = kSentinel).
// Other graphs keep slot-only entries plus one int8 weight per entry
// (padding = slot 0 with weight 0).
//
// Spins live as an L-bit mask per slot (bit j = replica j of the group,
// 1 = +1), L in {1,2,4,8,16,32}; the masks of 32/L consecutive slots share
// one uint32 word, so the state of n slots is n*L/32 words.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr uint32_t kSentinel = 0xFFFFFFFFu;
constexpr uint32_t kSignBit = 0x80000000u;
constexpr int kSliceRows = 64;

enum ItemKind : uint32_t { kItemSlice = 0, kItemLong = 1 };

// One unit of work for one wavefront.
struct Item {
  uint32_t id;     // slice: slice index (slots 64*id .. 64*id+63); long: slot of the row
  uint32_t base4;  // index of the item's first uint4 chunk in the entry stream
  uint32_t len4;   // slice: chunks per lane; long: chunks in the row
  uint32_t kind;   // ItemKind
};

// Arguments of the anneal kernel (passed by value).
struct AnnealArgs {
  const uint4 *entries;      // edge stream, uint4 chunks
  const uint32_t *wts4;      // 4 int8 weights per chunk (general weights only)
  const int32_t *vid;        // slot -> caller vertex id, -1 for padding
  const Item *items;         // all items, phase by phase
  const uint32_t *wave_ptr;  // [n_phases][nw + 1] item ranges per global wavefront
  const uint32_t *cls_w64;   // [n_phases + 1] class boundaries in 64-bit words of the spin state
  uint32_t *spins;           // this replica group's spin words
  const uint32_t *thr;       // thresholds, indexed by absolute sweep
  uint32_t *bar;             // [0] barrier counter, [1] error flag
  uint32_t n_words;          // spin words of the group
  int32_t n_phases;
  int32_t nw;                // wavefronts in the grid
  int32_t async_mode;
  int64_t t_begin, t_end;
  uint32_t seed_lo, seed_hi;
  uint32_t r0;               // replica index of bit 0
  uint32_t r_count;          // replicas of the group in use (<= L)
  uint32_t spin_limit;       // barrier polls before giving up (error flag)
};

struct CutArgs {
  const uint4 *entries;
  const uint32_t *wts4;
  const int32_t *vid;
  const Item *items;
  uint32_t n_items;
  const uint32_t *spins;
  unsigned long long *out;   // [2]: sum over directed entries of w s s, of w [s != s]
  uint32_t bit;              // replica bit inside the mask
};

}  // namespace ising
