/*
 * ising_noalloc.h -- an anneal entry point that allocates nothing.
 *
 * For callers that cannot allocate memory while they anneal: code under HIP
 * graph capture, tight serving loops, and harnesses that forbid hipMalloc.
 * isingAnneal allocates (and regrows) a handle's device threshold table and
 * its pinned host staging the first time it meets a longer schedule; this
 * variant instead writes the thresholds of the requested sweeps into one
 * fixed array of device memory per GPU (ISING_NOALLOC_MAX_SWEEPS uint32
 * words, 256 KiB, held from the first call on that GPU until the process
 * ends) and calls no hipMalloc, hipHostMalloc, hipFree or other allocating
 * routine.
 */
#ifndef ISING_NOALLOC_H
#define ISING_NOALLOC_H

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Largest sweep_end - sweep_begin one isingAnnealNoAlloc call accepts. */
#define ISING_NOALLOC_MAX_SWEEPS 65536

/* Same arguments, results and errors as isingAnneal (Algorithm 2, Sec. IV-B),
 * and the same results bit for bit in DETERMINISTIC mode, with these
 * differences:
 *   - sweep_end - sweep_begin must not exceed ISING_NOALLOC_MAX_SWEEPS, else
 *     ISING_ERR_INVALID_ARGUMENT and nothing is enqueued;
 *   - the thresholds of sweeps [sweep_begin, sweep_end) are written on the
 *     stream into the GPU's shared array: for LINEAR by a kernel, for
 *     EXPLICIT by an asynchronous copy from schedule->thresholds (host or
 *     device memory, read before the call returns only when it is host
 *     memory);
 *   - every call on one GPU shares that array, which keeps the last call's
 *     contents: calls that overlap on one GPU (on different streams, or
 *     from different threads) race and must be serialised by the caller.
 * Stream-ordered; does not synchronise. */
ising_status_t isingAnnealNoAlloc(ising_graph_t g, const ising_schedule_t *schedule, uint64_t seed,
                                  ising_mode_t mode, int64_t sweep_begin, int64_t sweep_end, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ISING_NOALLOC_H */
