/*
 * ising.h -- C ABI of the MI355X Ising max-cut annealer.
 *
 * The method is the annealed local spin update of Cook, Zhao, Sato,
 * Hiromoto and Tan, "GPU Ising Computing for Combinatorial Optimization
 * Problems in VLSI Physical Design" (arXiv:1807.10750):
 *   - a spin's local field is the weighted sum of its neighbours' spins and
 *     the spin takes the value that minimises its local energy
 *     (Sec. II-A, Eq. 1-2);
 *   - every spin then flips with a global probability F_p that is lowered
 *     sweep by sweep (Sec. IV-B, Algorithm 2);
 *   - the max-cut value of Sec. III, Eq. (4) is read back from the spins.
 *
 * Conventions used throughout:
 *   - Graph: symmetric CSR.  row_ptr is int64 [n+1] with row_ptr[0] = 0 and
 *     row_ptr[n] = nnz; col is int32 [nnz]; w is int8 [nnz].  Every
 *     undirected edge {u,v} appears as (u -> v, w) and (v -> u, w) with the
 *     same weight.  Self-loops and repeated neighbours are rejected.  Rows
 *     need not be sorted.  Vertex ids are the caller's; any internal
 *     renumbering is invisible at this boundary.
 *   - Max-cut mapping (Sec. III, Eq. 4-5): spin s_v = +1 / -1 is the side of
 *     the cut.  The field is h_v = sum_u w_vu s_u and the update sets
 *     s_v = -1 if h_v > 0, +1 if h_v < 0 and keeps s_v if h_v = 0; this is
 *     the energy minimisation of Eq. (2) with J = -w, the sign that makes
 *     the Ising ground state a maximum cut.
 *   - energy  E   = sum over undirected edges of w_uv s_u s_v,
 *     cut     cut = sum over undirected edges with s_u != s_v of w_uv,
 *     so that 2 cut = W - E with W = sum of w over undirected edges.
 *   - External field (optional, isingSetField): the general Ising model of
 *     Eq. (1) and Eq. (3) adds a bias h_v on each spin.  With J = -w the
 *     spin takes the sign of S_v = h_v - sum_u w_vu s_u (S_v = 0 keeps it)
 *     and the energy becomes E - sum_v h_v s_v.  The cut, W and the identity
 *     above concern the edges only.  The max-cut problem has h = 0.
 *   - Random flips: spin v of replica r in sweep t flips after its update
 *     iff x < T[t], x = word (t mod 4) of the Philox4x32-10 block with
 *     counter {v, floor(t / 4), r, 0} and key {low32(seed), high32(seed)}
 *     (one block serves four consecutive sweeps); T[t] is the flip
 *     probability F_p scaled to 2^32 (ISING_SCHED_*).  Random initial
 *     spins of replica r use word (r mod 4) of the block with counter
 *     {v, 0, floor(r / 4), 1}: s = +1 iff its bit 31 is set.
 *   - Replicas: a handle anneals R independent copies of the spins of one
 *     graph; spin arrays are int8 [R][n], replica-major, values +1 / -1.
 *   - Pointers: every graph or spin pointer may be host or device memory;
 *     the library tells them apart.  Outputs documented as "host" must be
 *     host memory.
 *   - Streams: each call is ordered on the caller's stream (a hipStream_t
 *     passed as void*; NULL is the default stream).  Calls that return
 *     values into host memory synchronise that stream before returning.
 *   - Graph capture: isingRandomizeSpins, isingAnneal with a schedule the
 *     handle has already run (its thresholds are then cached on the
 *     device), and isingCut / isingGetSpins into device memory enqueue only
 *     kernels, so a HIP graph can capture them.  A new schedule uploads its
 *     table first and synchronises the stream, which capture does not allow.
 *     While the stream captures, the multi-workgroup anneal becomes an
 *     ordinary kernel node; its grid never exceeds what fits on the device
 *     at once, and if some workgroups still cannot start (other work holds
 *     the device) its grid barrier gives up after a bounded number of polls
 *     and the next synchronising call reports ISING_ERR_DEVICE.
 *   - Ownership: isingCreate copies its inputs; the caller may free them on
 *     return.  The handle owns every device buffer; isingDestroy frees them.
 *   - Errors: no function aborts, throws or exits.  Each returns an
 *     ising_status_t; on failure isingLastError() describes the cause.
 *   - Threads: one handle must not be used from two threads at once;
 *     distinct handles are independent.
 *   - Environment.  No variable changes a result, only how it is computed
 *     (every launch shape gives the same deterministic result bit for bit),
 *     except ISING_ASYNC_MERGE, which changes which updates race in async
 *     mode, and ISING_FAULT_INJECT, which makes isingCreate fail.  Read by
 *     isingCreate unless noted; unset means the default.
 *       ISING_AUTOTUNE=0        no launch-shape tuning of batched handles
 *       ISING_BIN_VERTICES=v    batched bins of at most v vertices (no tuning)
 *       ISING_BATCH_WAVES=w     w in {4, 8, 16} waves per batched workgroup
 *                               (no tuning)
 *       ISING_TUNE_CACHE=path   file of tuned shapes (empty: none; default
 *                               $HOME/.cache/ising_tune.txt)
 *       ISING_BATCH_L=l         replicas per workgroup of a one-graph batch
 *       ISING_NO_BATCH=1        never the batched layout
 *       ISING_NO_LDS=1          no LDS copy of the spins (global gathers)
 *       ISING_GRID=g            workgroups of the cooperative launch
 *       ISING_BIN_SHIFT=k       lanes per row chosen for degree >> k
 *       ISING_WIDE=1            the separate int8 weight stream for all
 *                               general weights
 *       ISING_RESIDENT_EDGES=0  never keep +-1 entries in registers; =24 only in
 *                               the larger (24-chunk) register variant
 *       ISING_ASYNC_MERGE=b     async phases merge classes while at most
 *                               b/1000 of the edges lie inside (default 10)
 *       ISING_BARRIER_POLLS=p   polls before a wait gives up (isingAnneal)
 *       ISING_FAULT_INJECT=k    the k-th device allocation of each
 *                               isingCreate fails as out of memory (tests)
 */
#ifndef ISING_H
#define ISING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ising_graph_s *ising_graph_t;

typedef enum {
  ISING_OK = 0,
  ISING_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size, mode, range or spin value */
  ISING_ERR_INVALID_GRAPH = 2,    /* row_ptr not 0..nnz monotone, or col out of range */
  ISING_ERR_SELF_LOOP = 3,        /* an entry v -> v */
  ISING_ERR_DUPLICATE_EDGE = 4,   /* a neighbour listed twice in one row */
  ISING_ERR_ASYMMETRIC = 5,       /* (u -> v, w) without (v -> u, w) */
  ISING_ERR_OVERFLOW = 6,         /* some row has sum |w| > INT32_MAX */
  ISING_ERR_OUT_OF_MEMORY = 7,    /* host or device allocation failed */
  ISING_ERR_DEVICE = 8            /* a HIP call or a kernel reported an error */
} ising_status_t;

/* Update order inside a sweep.
 * DETERMINISTIC: vertices are updated colour class by colour class of a
 *   greedy colouring (ising_coloring_t); the result equals a sequential
 *   sweep that visits vertices in (colour, id) order, bit for bit.  This
 *   generalises the checkerboard update the paper cites (Sec. IV-B).
 * ASYNC: the paper's race-tolerant update (Sec. IV-B): every sweep is
 *   synchronised, and inside a sweep a spin reads each neighbour's value
 *   from this sweep or the previous one, never older.  Work is issued in
 *   phases, runs of consecutive colour classes (a run grows while at most
 *   1 % of the edges lie inside it) or the near-independent parts of
 *   ISING_COLOR_NEAR_INDEPENDENT, and a phase starts only once every
 *   spin of the previous phase is final: a neighbour in an earlier phase is
 *   read at this sweep's value, one in a later phase at the previous
 *   sweep's, and one in the same phase at either, as the update races with
 *   the neighbour's.  Results vary from run to run; they are judged by cut
 *   statistics.  isingGetInfo's max_sweep_gap reports how many sweeps apart
 *   two workgroups were ever seen (0 or 1 by construction). */
typedef enum { ISING_MODE_DETERMINISTIC = 0, ISING_MODE_ASYNC = 1 } ising_mode_t;

/* Greedy colouring rule.  FIRST_FIT visits vertices in increasing id;
 * LARGEST_FIRST visits them by decreasing degree, then increasing id.  Each
 * visited vertex takes the smallest colour no coloured neighbour has.
 * NEAR_INDEPENDENT (ASYNC mode only) replaces the colour classes by the
 * fewest parts, each with at most 1 % of the edges inside it, that a
 * first-fit start plus a local search finds, when that is fewer than the
 * phases of the LARGEST_FIRST runs; each part is then one async phase.
 * Otherwise, for graphs of more than 2^25 directed entries (where the
 * search would take minutes) and for batches of graphs that take several
 * bins (the budget holds per graph), the handle keeps the LARGEST_FIRST
 * colouring.
 * With parts, DETERMINISTIC anneals return ISING_ERR_INVALID_ARGUMENT. */
typedef enum {
  ISING_COLOR_FIRST_FIT = 0,
  ISING_COLOR_LARGEST_FIRST = 1,
  ISING_COLOR_NEAR_INDEPENDENT = 2
} ising_coloring_t;

/* Flip-probability schedule F_p (Sec. IV-B, Algorithm 2: F_p is lowered
 * after every sweep).  A probability p in [0,1] becomes the threshold
 * T = min(2^32 - 1, floor(p * 2^32)).
 * LINEAR: T[t] = Ts - floor((Ts - Te) * t / (M - 1)) for Ts >= Te (and the
 *   mirror image for Ts < Te), t in [0, M), Ts, Te from p_start, p_end;
 *   M = 1 gives Ts.
 * EXPLICIT: T[t] = thresholds[t], a host array of n_sweeps entries. */
typedef enum { ISING_SCHED_LINEAR = 0, ISING_SCHED_EXPLICIT = 1 } ising_sched_kind_t;

typedef struct {
  ising_sched_kind_t kind;
  double p_start;               /* LINEAR only, in [0, 1] */
  double p_end;                 /* LINEAR only, in [0, 1] */
  int64_t n_sweeps;             /* M >= 1 */
  const uint32_t *thresholds;   /* EXPLICIT only: host, n_sweeps entries */
} ising_schedule_t;

/* Build a handle for one graph and n_replicas spin copies (Sec. II-A: a
 * general weighted graph of any topology).  Validates the graph in this
 * order, reporting the first failure: arguments, structure, self-loop,
 * duplicate, symmetry, overflow.  Then colours it, lays it out in device
 * memory and allocates spins (all +1 until set or randomised).
 * n >= 0, nnz >= 0, n < 2^31 - 64; n_replicas >= 1.  row_ptr/col/w may be
 * host or device pointers (col and w may be NULL when nnz = 0).
 * On success *out is a new handle; on failure *out is NULL. */
ising_status_t isingCreate(ising_graph_t *out, int64_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col, const int8_t *w, ising_coloring_t coloring,
                           int32_t n_replicas, void *stream);

/* Set every replica's spins to random +-1 drawn from Philox counter domain 1
 * (see the conventions above).  Stream-ordered, no synchronisation. */
ising_status_t isingRandomizeSpins(ising_graph_t g, uint64_t seed, void *stream);

/* Copy caller spins in: int8 [R][n], caller ids, every value +1 or -1
 * (anything else: ISING_ERR_INVALID_ARGUMENT and the spins are unchanged).
 * Host or device pointer; a device pointer is read on the stream and the
 * call synchronises it to check the values. */
ising_status_t isingSetSpins(ising_graph_t g, const int8_t *spins, void *stream);

/* Run sweeps t = sweep_begin .. sweep_end-1 of the schedule (Algorithm 2):
 * in each sweep every spin takes its local update and then flips iff its
 * Philox draw is below T[t].  Chunked calls compose: [0,k) then [k,M) gives
 * the same result as [0,M) in DETERMINISTIC mode.  Requires
 * 0 <= sweep_begin <= sweep_end <= n_sweeps.  Stream-ordered; the schedule
 * is copied before return.  Device faults surface at the next call that
 * synchronises (isingCut, isingGetSpins). */
ising_status_t isingAnneal(ising_graph_t g, const ising_schedule_t *schedule, uint64_t seed,
                           ising_mode_t mode, int64_t sweep_begin, int64_t sweep_end,
                           void *stream);

/* Cut value (Eq. 4) and energy (Eq. 5 with J = -w, plus -sum h s when a
 * field is set, Eq. 3) of every replica: cut int64 [R], energy int64 [R]
 * or NULL.  Host or device outputs; host outputs synchronise the stream.
 * Also checks 2 cut = W - E(edges) on the host when the outputs are host
 * memory. */
ising_status_t isingCut(ising_graph_t g, int64_t *cut, int64_t *energy, void *stream);

/* Copy spins out: int8 [R][n] in caller ids, host or device pointer.  A
 * host destination synchronises the stream. */
ising_status_t isingGetSpins(ising_graph_t g, int8_t *spins, void *stream);

/* Best-of-run tracking (the paper keeps the final state; Sec. V-A suggests
 * keeping the best one seen).  Computes the cut of every replica's current
 * spins, writes it to cut (int64 [R], host or device, or NULL) and, for each
 * replica whose cut exceeds its best since the spins were last randomised or
 * set, records the new best cut and a copy of that replica's spins.  Called
 * between chunked isingAnneal calls it yields a cut trace and the best
 * state.  Stream-ordered; a host cut output synchronises the stream; with a
 * device or NULL output it can be captured in a HIP graph. */
ising_status_t isingUpdateBest(ising_graph_t g, int64_t *cut, void *stream);

/* The best cut of every replica (int64 [R]) and its spins (int8 [R][n] in
 * caller ids), host or device, either may be NULL.  ISING_ERR_INVALID_ARGUMENT
 * if isingUpdateBest has not run since the spins were last randomised or
 * set.  Host outputs synchronise the stream. */
ising_status_t isingGetBest(ising_graph_t g, int64_t *best_cut, int8_t *spins, void *stream);

/* Classes of the handle: color int32 [n] (host), the class of every caller
 * vertex; *n_colors their number.  Colour classes (DETERMINISTIC mode's
 * order), or the near-independent parts of ISING_COLOR_NEAR_INDEPENDENT. */
ising_status_t isingGetColoring(ising_graph_t g, int32_t *color, int32_t *n_colors);

/* Sum of w over undirected edges (W in 2 cut = W - E). */
ising_status_t isingTotalWeight(ising_graph_t g, int64_t *W);

/* External field h_v of every vertex (Sec. II-A, Eq. 1 and Eq. 3): int32 [n]
 * in caller ids, host or device pointer, copied; NULL removes the field.
 * Every row must keep sum |w| + |h_v| <= 2^30 - 1, else
 * ISING_ERR_OVERFLOW names the first offending vertex and the field is
 * unchanged.  Synchronises the stream first (queued anneals finish with
 * the old field); not for use under graph capture. */
ising_status_t isingSetField(ising_graph_t g, const int32_t *h, void *stream);

/* Per-vertex flip temperature (not in the paper, which uses one F_p for
 * every spin; it lets the learned warm start of ising_warm.h say how much
 * each vertex should be shaken): uint8 [n] multipliers m_v in [0, 15], caller
 * ids, host or device pointer, copied.  Vertex v then flips in sweep t iff
 * its draw x < min(2^32 - 1, floor(T[t] * m_v / 8)); m = 8 everywhere is the
 * plain anneal, m = 0 never flips.  NULL removes the multipliers.  A value
 * above 15 gives ISING_ERR_INVALID_ARGUMENT and leaves them unchanged.
 * Synchronises the stream first; not for use under graph capture. */
ising_status_t isingSetFlipScale(ising_graph_t g, const uint8_t *scale, void *stream);

/* Layout and launch facts of a handle, for benchmarks and tests. */
typedef struct {
  int64_t n_slots;          /* vertices after padding each colour class to a multiple of 64 */
  int32_t n_colors;         /* colour classes = phases of a deterministic sweep */
  int32_t replicas_per_group; /* replicas annealed together from one read of the edges */
  int32_t n_groups;         /* replica groups; the edge stream is read once per group per sweep */
  int32_t uses_lds;         /* 1 if neighbour spins are gathered from an LDS copy */
  int32_t grid;             /* workgroups of the anneal launch */
  int32_t block;            /* threads per workgroup */
  int32_t pm1;              /* 1 if every weight is +-1 (sign packed into the edge entry) */
  int32_t encoding;         /* edge entry encoding: 0 slot|sign, 1 slot|int8 weight, 2 slot + weight stream */
  int64_t edge_bytes;       /* bytes of the edge stream read once per sweep per group */
  int64_t vertex_bytes;     /* bytes of per-vertex data read once per sweep per group */
  int64_t spin_bytes;       /* bytes of one group's packed spin state */
  int64_t items;            /* wavefront work items per sweep */
  int32_t bins;             /* batched mode: workgroups per replica group, each owning whole
                               connected components (0: one cooperative launch) */
  int32_t max_sweep_gap;    /* cooperative launch: the largest number of sweeps by which
                               workgroups were seen apart at a phase end over the handle's
                               life (0 or 1); reading it synchronises the device */
  int32_t resident_edges;   /* cooperative launch: bit m set if mode m (0 deterministic, 1 async)
                               reads the +-1 edge entries from HBM once per call and keeps them
                               in registers (3 bytes each) for all its sweeps */
  int32_t async_phases;     /* phases of an async sweep (runs of classes) */
  int32_t resident_chunks;  /* chunks per lane of the register variant in use, 18 or 24 (0: none) */
  int32_t deterministic_ok; /* 1 if the classes are colour classes (DETERMINISTIC mode allowed) */
} ising_info_t;

ising_status_t isingGetInfo(ising_graph_t g, ising_info_t *info);

/* Free the handle and its device memory.  NULL is accepted. */
ising_status_t isingDestroy(ising_graph_t g);

/* Message for the last failed call on this thread ("" if none).  Valid
 * until the next call on this thread. */
const char *isingLastError(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
