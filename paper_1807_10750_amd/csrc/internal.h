// internal.h -- library-internal entry points shared by the C ABI sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ising.h"

// Sets the thread's last-error message and returns st.
ising_status_t internal_fail(ising_status_t st, const std::string &msg);
// Clears the thread's last-error message (every entry point starts so).
void internal_clear_error();
// Device the handle lives on.
int internal_device(ising_graph_t g);
// min(2^32 - 1, floor(p * 2^32)): the flip threshold of probability p.
uint32_t internal_prob_threshold(double p);
// Argument checks of isingAnneal (handle, schedule, mode, sweep range).
ising_status_t internal_check_anneal(ising_graph_t g, const ising_schedule_t *s, ising_mode_t mode,
                                     int64_t sweep_begin, int64_t sweep_end);
// Enqueues sweeps [sweep_begin, sweep_end) on st; sweep t's threshold is
// thr[t - thr_base] in device memory.  Allocates nothing.  The caller has
// checked the arguments and made the handle's device current.
ising_status_t internal_anneal(ising_graph_t g, uint64_t seed, ising_mode_t mode, int64_t sweep_begin,
                               int64_t sweep_end, hipStream_t st, const uint32_t *thr, int64_t thr_base);
