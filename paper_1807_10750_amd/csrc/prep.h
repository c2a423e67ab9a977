// prep.h -- host preparation of a graph handle: validation, colouring,
// renumbering into slots and the sliced edge layout (internal).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "layout.h"

namespace ising {

// Status values mirror ising_status_t.
enum PrepStatus {
  kPrepOk = 0,
  kPrepArg = 1,
  kPrepGraph = 2,
  kPrepSelfLoop = 3,
  kPrepDuplicate = 4,
  kPrepAsymmetric = 5,
  kPrepOverflow = 6,
  kPrepNoMem = 7,
};

struct HostCSR {
  int64_t n = 0, nnz = 0;
  const int64_t *row_ptr = nullptr;
  const int32_t *col = nullptr;
  const int8_t *w = nullptr;
};

// Checks, in order: structure, self-loops, duplicate neighbours, symmetry of
// (u, v, w), int32 range of every row's sum |w|.  On failure returns the
// status and writes a message naming the offending row and entry.
int validate_graph(const HostCSR &g, int64_t *W_out, std::string *msg);

// Greedy colouring: vertices visited by id (largest_first = false) or by
// (degree desc, id asc); each takes the least colour absent from its
// already-coloured neighbours.
int32_t greedy_coloring(const HostCSR &g, bool largest_first, std::vector<int32_t> *color);

// Near-independent parts for the async sweep (not a colouring): K parts,
// each with at most budget * nnz directed entries inside it, for the
// smallest K reached counting down from max_parts (at most kMaxParts) before
// an attempt fails.  An attempt at K visits vertices by (degree desc, id
// asc), fills parts 0 .. K-2 first fit as independent sets and puts the rest
// in part K-1, then runs annealed local-search passes that move each vertex
// to the part where it has the fewest (weighted) neighbours.  Deterministic.
// Returns K and writes each vertex's part, or 0 (all parts 0) when not even
// max_parts fits.
constexpr int32_t kMaxParts = 16;
constexpr int kPartPasses = 64;
constexpr double kPartT0 = 0.5;
int32_t near_independent_parts(const HostCSR &g, double budget, int32_t max_parts, std::vector<int32_t> *part);

struct HostLayout {
  int64_t n_slots = 0;                 // multiple of 64
  int32_t n_phases = 0;                // colours
  int32_t n_bins = 1;                  // groups of whole components laid out one after another
  int enc = 0;                         // Encoding of the entries
  std::vector<int32_t> vid;            // slot -> vertex (-1 = padding)
  std::vector<int32_t> slot_of;        // vertex -> slot
  std::vector<int64_t> cls_begin;      // [n_bins * n_phases + 1] first slot of class (bin, colour)
  std::vector<uint32_t> entries;       // edge stream, multiple of 4 entries
  std::vector<int8_t> wts;             // per entry (general weights only)
  std::vector<Item> items;             // phase by phase
  std::vector<uint32_t> phase_items;   // [n_bins * n_phases + 1] first item of class (bin, colour)
};

// The entry encoding a graph with n_slots slots gets.
int choose_encoding(const HostCSR &g, int64_t n_slots);

// Connected components (union-find), packed in order of their smallest
// vertex into bins of at most target vertices (a larger component gets a bin
// of its own).  Returns the bin of every vertex; *max_comp = largest component.
std::vector<int32_t> pack_components(const HostCSR &g, int64_t target, int32_t *n_bins, int64_t *max_comp);

// Classes are (bin, colour) pairs, laid out bin by bin (bin_of = NULL: one
// bin).  enc: entry encoding (kEncW8 becomes kEncWide, with its prefetch
// depth, when the padded slot count exceeds 2^24); kmax: chunks each lane
// prefetches (see kmax_for); a row of degree d gets the fewest lanes G with
// d <= (4 * kmax * G) >> bin_shift.
int build_layout(const HostCSR &g, const std::vector<int32_t> &color, int32_t n_colors, const int32_t *bin_of,
                 int32_t n_bins, int enc, int kmax, int bin_shift, HostLayout *out, std::string *msg);

// Phases of an async sweep as runs of consecutive colour classes:
// [out[i], out[i+1]).  A run grows while the undirected edges between its
// own classes stay at most budget * (nnz / 2); vertices joined by such an
// edge update in the same phase and read each other's value from this sweep
// or the previous one.  budget = 0 gives one class per phase, the phases of
// deterministic mode.
std::vector<int32_t> phase_runs(const HostCSR &g, const std::vector<int32_t> &color, int32_t n_colors,
                                double budget);

// Splits each phase's items over nw wavefronts in contiguous runs of about
// equal cost.  rotate_small: a phase with no more items than wavefronts gets
// one item per wavefront, spaced evenly, from a start that moves from phase
// to phase.  Returns [n_phases][nw + 1] item offsets.
std::vector<uint32_t> partition_waves(const HostLayout &L, const std::vector<int32_t> &phase_cls, int32_t nw,
                                      bool rotate_small);

// The per-wavefront item ranges of the cooperative anneal, [n_ph][nw][2]
// (begin, end), from a prefix table of partition_waves: phase p's ranges
// are rotated by a whole number of workgroups, about p * grid / n_ph, so
// that the heavy first items of the phases (each class is sorted by degree,
// descending) land on different wavefronts.
std::vector<uint32_t> rotate_ranges(const std::vector<uint32_t> &prefix, int32_t n_ph, int32_t nw,
                                    int32_t waves_per_block);

// Bits of each 32-bit spin word that items write every sweep: item i
// covers the Lbits bits of each of its K = 64 / g slots, so a word gets 32
// unless the class ends inside it (slots past the class's last item are
// never written).  [n_words] entries, each at most 32.
std::vector<uint8_t> word_cover(const HostLayout &L, int Lbits, uint32_t n_words);

// Largest number of chunks per lane, sum of ceil(len4 / g) over its items,
// that one wavefront's items of all phases hold; *max_items (if not NULL):
// the most items one wavefront has in all phases.  ranges as from
// rotate_ranges.
uint64_t max_wave_chunks(const HostLayout &L, const std::vector<uint32_t> &ranges, int32_t n_ph, int32_t nw,
                         uint64_t *max_items);

// Verifies that every item addresses only memory inside the layout (index
// ranges of entries, slots and spin words) and that every entry decodes to
// the graph's neighbour and weight at its position.  Returns false with a
// message.
bool check_layout(const HostLayout &L, const HostCSR &g, std::string *msg);

}  // namespace ising
