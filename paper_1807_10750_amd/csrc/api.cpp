// api.cpp -- the C ABI declared in include/ising.h.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <sys/stat.h>
#include <tuple>
#include <vector>

#include "internal.h"
#include "ising.h"
#include "kernels.h"
#include "prep.h"

using namespace ising;

namespace {

thread_local std::string g_last_error;

ising_status_t fail(ising_status_t st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

ising_status_t hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? ISING_ERR_OUT_OF_MEMORY : ISING_ERR_DEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                   \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)


bool is_device_ptr(const void *p) {
  if (p == nullptr) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

int64_t env_int(const char *name, int64_t dflt) {
  const char *s = std::getenv(name);
  if (s == nullptr || *s == 0) return dflt;
  return std::strtoll(s, nullptr, 10);
}

// Edges allowed inside one async phase, in units of 0.1 % of all edges.
constexpr int64_t kAsyncMergeBudget = 10;
// largest graph (directed entries) the near-independent part search runs on
// (about 8 s on the host for 8M entries)
constexpr int64_t kPartSearchMaxEntries = int64_t(1) << 25;

int pow2_at_least(int x) {
  int p = 1;
  while (p < x && p < 32) p <<= 1;
  return p;
}

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) (void)hipSetDevice(dev);
    dev_ = dev;
  }
  ~DeviceGuard() {
    if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1, dev_ = 0;
};

}  // namespace

struct ising_graph_s {
  int device = 0;
  int64_t n = 0, nnz = 0;
  int32_t R = 1;
  int32_t n_colors = 0;
  std::vector<int32_t> color;
  bool proper_classes = true;  // classes are colour classes (false: near-independent parts)
  int64_t W = 0;
  HostLayout lay;            // host copy (entries/wts released after upload)
  int64_t entry_bytes = 0;   // edge stream bytes per sweep (entries + weights)
  int L = 1, n_groups = 1;
  uint32_t n_words = 0;      // spin words per group
  bool use_lds = false;
  size_t lds_bytes = 0;
  int grid = 1, nw = 16;
  // device buffers
  void *d_entries = nullptr;
  uint32_t *d_wts4 = nullptr;
  int32_t *d_vid = nullptr;
  Item *d_items = nullptr;
  uint32_t *d_wave_ptr[2] = {nullptr, nullptr};  // per mode: [phases][nw][2] item ranges
  // exchange words of a launch with the LDS copy (kernels.hip): [n_words]
  // words and the bits each word's items write per sweep
  unsigned long long *d_xch = nullptr;
  uint8_t *d_cover = nullptr;
  uint32_t *d_flips = nullptr;                   // 3 flip planes per replica group
  // batched mode: one workgroup per (bin of whole components, replica group)
  bool batch = false;
  int batch_waves = 4;
  size_t batch_lds = 0;
  uint32_t *d_bin_wave_ptr = nullptr;            // [n_bins][colours][waves + 1]
  uint32_t *d_bin_words = nullptr;               // [n_bins + 1]
  int res_edges[2] = {0, 0};  // per mode: chunks of the register-resident variant (0: entries streamed)
  uint32_t *d_cls_w64[2] = {nullptr, nullptr};   // per mode: phase -> spin word range
  int32_t n_phases[2] = {0, 0};
  uint32_t *d_spins = nullptr;
  uint32_t *d_thr = nullptr;
  int64_t thr_cap = 0;
  uint32_t *d_bar = nullptr;   // barrier counters, error and spin-check flags (kBar*)
  unsigned long long *d_cut = nullptr;
  int8_t *d_stage = nullptr;
  // external field: sum |w| of every row (the field contract) and -h per slot
  std::vector<uint32_t> row_abs;
  std::vector<uint32_t> degree;
  int32_t *d_bias = nullptr;
  bool has_field = false;
  // per-vertex flip-temperature multipliers per slot (isingSetFlipScale)
  uint8_t *d_scale = nullptr;
  bool has_scale = false;
  // best-of-run state (isingUpdateBest): best cut per replica, the spins it
  // was seen with, per-group improvement masks, a scratch cut array
  int64_t *d_best_cut = nullptr;
  uint32_t *d_best_spins = nullptr;
  uint32_t *d_best_mask = nullptr;
  int64_t *d_cutvals = nullptr;
  bool best_reset = true;  // no best recorded since the spins were last set
  bool best_any = false;   // some update ran since
  // schedule cache
  bool thr_valid = false;
  double ps = -1, pe = -1;
  int64_t M = 0;
  uint32_t *h_thr = nullptr;   // pinned staging of the thresholds
  int64_t h_thr_cap = 0;
};

namespace {

// Failure injection for tests of the error paths: with ISING_FAULT_INJECT =
// k >= 1, the k-th device allocation of each isingCreate call fails as if
// the device were out of memory (counted per thread from the call's start).
thread_local int64_t g_alloc_count = 0;
thread_local int64_t g_alloc_fail_at = 0;

template <typename T>
ising_status_t dev_alloc(T **p, size_t bytes, const char *what) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (g_alloc_fail_at > 0 && ++g_alloc_count == g_alloc_fail_at) return hip_fail(hipErrorOutOfMemory, what);
  hipError_t e = hipMalloc(reinterpret_cast<void **>(p), bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, what);
  }
  return ISING_OK;
}

void free_all(ising_graph_s *g) {
  void *bufs[] = {g->d_entries, g->d_wts4, g->d_vid, g->d_items, g->d_wave_ptr[0], g->d_wave_ptr[1],
                  g->d_cls_w64[0], g->d_cls_w64[1], g->d_xch, g->d_cover, g->d_flips,
                  g->d_bin_wave_ptr, g->d_bin_words,
                  g->d_spins, g->d_thr, g->d_bar, g->d_cut, g->d_stage, g->d_bias,
                  g->d_best_cut, g->d_best_spins, g->d_best_mask, g->d_cutvals, g->d_scale};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (g->h_thr) (void)hipHostFree(g->h_thr);
}

// Copies an array given by a host or device pointer into a host vector.
template <typename T>
ising_status_t fetch(std::vector<T> *dst, const T *src, int64_t count, const char *what) {
  try {
    dst->resize((size_t)count);
  } catch (const std::bad_alloc &) {
    return fail(ISING_ERR_OUT_OF_MEMORY, std::string("host allocation failed for ") + what);
  }
  if (count == 0) return ISING_OK;
  if (is_device_ptr(src)) {
    HIP_TRY(hipMemcpy(dst->data(), src, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost), what);
  } else {
    std::memcpy(dst->data(), src, sizeof(T) * (size_t)count);
  }
  return ISING_OK;
}

ising_status_t upload(void *dst, const void *src, size_t bytes, const char *what) {
  if (bytes == 0) return ISING_OK;
  HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), what);
  return ISING_OK;
}

// Thresholds T[t] of a linear schedule (see ising.h).
uint32_t prob_threshold(double p) {
  const double x = p * 4294967296.0;  // exact scaling by 2^32
  return x >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)x;
}

void linear_thresholds(double ps, double pe, int64_t M, uint32_t *T) {
  const uint32_t a = prob_threshold(ps), b = prob_threshold(pe);
  const bool down = a >= b;
  const uint64_t span = down ? (uint64_t)(a - b) : (uint64_t)(b - a);
  for (int64_t t = 0; t < M; ++t) {
    uint64_t step = 0;
    if (M > 1) step = (uint64_t)(((unsigned __int128)span * (uint64_t)t) / (uint64_t)(M - 1));
    T[t] = down ? a - (uint32_t)step : a + (uint32_t)step;
  }
}

ising_status_t ensure_thresholds(ising_graph_s *g, const ising_schedule_t *s, hipStream_t st) {
  const bool cached = s->kind == ISING_SCHED_LINEAR && g->thr_valid && g->ps == s->p_start &&
                      g->pe == s->p_end && g->M == s->n_sweeps;
  if (cached) return ISING_OK;
  // previous anneals on this stream may still read the old table
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s->n_sweeps > g->thr_cap) {
    if (g->d_thr) (void)hipFree(g->d_thr);
    g->d_thr = nullptr;
    g->thr_cap = 0;
    ising_status_t r = dev_alloc(&g->d_thr, sizeof(uint32_t) * (size_t)s->n_sweeps, "threshold table");
    if (r != ISING_OK) return r;
    g->thr_cap = s->n_sweeps;
  }
  if (s->n_sweeps > g->h_thr_cap) {
    if (g->h_thr) (void)hipHostFree(g->h_thr);
    g->h_thr = nullptr;
    g->h_thr_cap = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&g->h_thr), sizeof(uint32_t) * (size_t)s->n_sweeps),
            "pinned threshold staging");
    g->h_thr_cap = s->n_sweeps;
  }
  if (s->kind == ISING_SCHED_LINEAR)
    linear_thresholds(s->p_start, s->p_end, s->n_sweeps, g->h_thr);
  else
    std::memcpy(g->h_thr, s->thresholds, sizeof(uint32_t) * (size_t)s->n_sweeps);
  HIP_TRY(hipMemcpyAsync(g->d_thr, g->h_thr, sizeof(uint32_t) * (size_t)s->n_sweeps, hipMemcpyHostToDevice, st),
          "threshold upload");
  g->thr_valid = s->kind == ISING_SCHED_LINEAR;
  g->ps = s->p_start;
  g->pe = s->p_end;
  g->M = s->n_sweeps;
  return ISING_OK;
}

uint32_t group_r_count(const ising_graph_s *g, int grp) {
  const int r0 = grp * g->L;
  return (uint32_t)std::min(g->L, g->R - r0);
}

ising_status_t check_flags(ising_graph_s *g, hipStream_t st) {
  uint32_t flags[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(flags, g->d_bar, sizeof flags, hipMemcpyDeviceToHost, st), "flag readback");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (flags[kBarErr] != 0) return fail(ISING_ERR_DEVICE, "an anneal grid barrier timed out");
  return ISING_OK;
}

// Launch-shape tuning of the batched anneal: waves per workgroup.  Choices
// are cached for the process by a key of the handle's shape, so handles of
// the same shape are timed once.
typedef std::tuple<int32_t, int64_t, int64_t, int32_t, int32_t, int32_t, size_t> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune_cache;

// The batched anneal: one workgroup per (bin, replica group).
hipError_t launch_batch(const ising_graph_s *g, AnnealArgs a, int waves, hipStream_t st) {
  a.n_bins = g->lay.n_bins;
  return launch_anneal_batch(g->L, g->lay.enc, waves, a, g->lay.n_bins * g->n_groups, g->batch_lds, st);
}

// Times a short deterministic anneal of the handle with each candidate wave
// table and returns the index of the fastest.  The spins and flip planes
// are clobbered; the caller resets them.
ising_status_t time_batch_shapes(ising_graph_s *g, const std::vector<std::vector<uint32_t>> &tables,
                                 const int *waves, hipStream_t st, int *best, float *best_ms_out) {
  constexpr int kSweeps = 8;
  uint32_t *d_tab = nullptr, *d_thr = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  size_t cap = 0;
  for (const auto &t : tables) cap = std::max(cap, t.size());
  ising_status_t r = dev_alloc(&d_tab, sizeof(uint32_t) * cap, "tuning table");
  if (r == ISING_OK) r = dev_alloc(&d_thr, sizeof(uint32_t) * kSweeps, "tuning thresholds");
  std::vector<uint32_t> thr(kSweeps);
  for (int t = 0; t < kSweeps; ++t) thr[t] = (uint32_t)(0x0A000000u - 0x01000000u * (uint32_t)t);
  if (r == ISING_OK) r = upload(d_thr, thr.data(), sizeof(uint32_t) * kSweeps, "tuning threshold upload");
  if (r == ISING_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    r = fail(ISING_ERR_DEVICE, "hipEventCreate");
  float best_ms = 0.f;
  *best = 0;
  for (size_t c = 0; r == ISING_OK && c < tables.size(); ++c) {
    hipError_t e = hipMemcpyAsync(d_tab, tables[c].data(), sizeof(uint32_t) * tables[c].size(),
                                  hipMemcpyHostToDevice, st);
    AnnealArgs a{};
    a.entries = reinterpret_cast<const uint4 *>(g->d_entries);
    a.wts4 = g->d_wts4;
    a.vid = g->d_vid;
    a.items = g->d_items;
    a.thr = d_thr;
    a.bar = g->d_bar;
    a.n_words = g->n_words;
    a.seed_lo = 1u;
    a.spin_limit = 1000000;
    a.spins = g->d_spins;
    a.flips = g->d_flips;
    a.wave_ptr = d_tab;
    a.bin_words = g->d_bin_words;
    a.n_bins = g->lay.n_bins;
    a.n_phases = g->n_colors;
    a.r_total = (uint32_t)g->R;
    a.t_begin = 0;
    a.t_end = kSweeps;
    float ms = 0.f;
    // the first launch warms caches and code; the second is timed
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      if (rep == 1) e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = launch_batch(g, a, waves[c], st);
      if (rep == 1 && e == hipSuccess) e = hipEventRecord(e1, st);
    }
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) r = hip_fail(e, "launch-shape tuning");
    if (r == ISING_OK && (c == 0 || ms < best_ms)) {
      best_ms = ms;
      *best = (int)c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d_tab) (void)hipFree(d_tab);
  if (d_thr) (void)hipFree(d_thr);
  if (best_ms_out != nullptr) *best_ms_out = best_ms;
  return r;
}

// Options of one handle build.  bin_target: vertices per bin of the batched
// layout (0: ISING_BIN_VERTICES, default 4096); waves: wavefronts per
// workgroup of the batched launch (0: ISING_BATCH_WAVES, else timed);
// tuned_ms (out, may be NULL): the 8-sweep time of the timed choice, or -1.
struct CreateOpts {
  int64_t bin_target = 0;
  int waves = 0;
  float *tuned_ms = nullptr;
};

// The persisted choices of the batched launch shape: one line per input
// shape, "n nnz replicas coloring bin_target waves", in the file named by
// ISING_TUNE_CACHE (empty: none), else $HOME/.cache/ising_tune.txt.
std::string tune_cache_path() {
  const char *e = std::getenv("ISING_TUNE_CACHE");
  if (e != nullptr) return std::string(e);
  const char *home = std::getenv("HOME");
  if (home == nullptr || *home == 0) return std::string();
  return std::string(home) + "/.cache/ising_tune.txt";
}

bool tune_cache_get(int64_t n, int64_t nnz, int32_t R, int coloring, int64_t *target, int *waves) {
  const std::string path = tune_cache_path();
  if (path.empty()) return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE *f = std::fopen(path.c_str(), "r");
  if (f == nullptr) return false;
  long long a, b, t;
  int c, d, wv;
  bool found = false;
  while (std::fscanf(f, "%lld %lld %d %d %lld %d", &a, &b, &c, &d, &t, &wv) == 6)
    if (a == n && b == nnz && c == R && d == coloring && t > 0 && (wv == 4 || wv == 8 || wv == 16)) {
      *target = t;
      *waves = wv;
      found = true;  // the last matching line wins
    }
  std::fclose(f);
  return found;
}

void tune_cache_put(int64_t n, int64_t nnz, int32_t R, int coloring, int64_t target, int waves) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE *f = std::fopen(path.c_str(), "a");
  if (f == nullptr) {
    // the default directory may not exist yet
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    f = std::fopen(path.c_str(), "a");
  }
  if (f == nullptr) return;  // not persisted; the choice still holds for this handle
  std::fprintf(f, "%lld %lld %d %d %lld %d\n", (long long)n, (long long)nnz, R, coloring, (long long)target, waves);
  std::fclose(f);
}

ising_status_t create_impl(ising_graph_t *out, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                           const int8_t *w, ising_coloring_t coloring, int32_t n_replicas, void *stream,
                           const CreateOpts &opt);

}  // namespace

ising_status_t internal_fail(ising_status_t st, const std::string &msg) { return fail(st, msg); }

void internal_clear_error() { g_last_error.clear(); }

int internal_device(ising_graph_t g) { return g->device; }

uint32_t internal_prob_threshold(double p) { return prob_threshold(p); }

ising_status_t internal_check_anneal(ising_graph_t g, const ising_schedule_t *s, ising_mode_t mode,
                                     int64_t sweep_begin, int64_t sweep_end) {
  if (g == nullptr || s == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  if (mode != ISING_MODE_DETERMINISTIC && mode != ISING_MODE_ASYNC)
    return fail(ISING_ERR_INVALID_ARGUMENT, "unknown mode");
  if (mode == ISING_MODE_DETERMINISTIC && !g->proper_classes)
    return fail(ISING_ERR_INVALID_ARGUMENT,
                "deterministic mode needs colour classes; this handle holds near-independent parts (async only)");
  if (s->n_sweeps < 1 || s->n_sweeps > ((int64_t)1 << 32))
    return fail(ISING_ERR_INVALID_ARGUMENT, "n_sweeps must be in [1, 2^32]");
  if (s->kind == ISING_SCHED_LINEAR) {
    if (!(s->p_start >= 0.0 && s->p_start <= 1.0 && s->p_end >= 0.0 && s->p_end <= 1.0))
      return fail(ISING_ERR_INVALID_ARGUMENT, "probabilities must lie in [0, 1]");
  } else if (s->kind == ISING_SCHED_EXPLICIT) {
    if (s->thresholds == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "thresholds is NULL");
  } else {
    return fail(ISING_ERR_INVALID_ARGUMENT, "unknown schedule kind");
  }
  if (sweep_begin < 0 || sweep_begin > sweep_end || sweep_end > s->n_sweeps)
    return fail(ISING_ERR_INVALID_ARGUMENT, "need 0 <= sweep_begin <= sweep_end <= n_sweeps");
  return ISING_OK;
}

// Launches sweeps [sweep_begin, sweep_end) with the threshold of sweep t at
// thr[t - thr_base]; allocates nothing.
ising_status_t internal_anneal(ising_graph_t g, uint64_t seed, ising_mode_t mode, int64_t sweep_begin,
                               int64_t sweep_end, hipStream_t st, const uint32_t *thr, int64_t thr_base) {
  AnnealArgs a{};
  a.entries = reinterpret_cast<const uint4 *>(g->d_entries);
  a.wts4 = g->d_wts4;
  a.vid = g->d_vid;
  a.bias = g->has_field ? g->d_bias : nullptr;
  a.scale = g->has_scale ? g->d_scale : nullptr;
  a.items = g->d_items;
  const int m = mode == ISING_MODE_ASYNC ? 1 : 0;
  a.wave_ptr = g->d_wave_ptr[m];
  a.cls_w64 = g->d_cls_w64[m];
  a.thr = thr;
  a.thr_base = thr_base;
  a.bar = g->d_bar;
  a.n_words = g->n_words;
  a.n_phases = g->n_phases[m];
  a.nw = g->nw;
  a.async_mode = mode == ISING_MODE_ASYNC ? 1 : 0;
  a.seed_lo = (uint32_t)seed;
  a.seed_hi = (uint32_t)(seed >> 32);
  a.spin_limit = (uint32_t)std::max<int64_t>(1000, env_int("ISING_BARRIER_POLLS", 20000000));
  if (g->batch) {
    a.spins = g->d_spins;
    a.flips = g->d_flips;
    a.wave_ptr = g->d_bin_wave_ptr;
    a.bin_words = g->d_bin_words;
    a.n_bins = g->lay.n_bins;
    a.n_phases = g->n_colors;
    a.r_total = (uint32_t)g->R;
    a.t_begin = sweep_begin;
    a.t_end = sweep_end;
    HIP_TRY(launch_batch(g, a, g->batch_waves, st), "batched anneal launch");
    return ISING_OK;
  }
  // Counts within one launch.  Exchange words (launch with the LDS copy; one
  // workgroup uses them too, without waiting on them): a word's count
  // reaches 32 times the sweeps, kept below 2^26.  Arrival counters:
  // epochs (phases, at least two per sweep) times at most 1024 workgroups,
  // kept below 2^31; without the LDS copy the barrier's top counter reaches
  // epochs times at most 8 groups.
  const bool xch = g->use_lds;
  int64_t chunk = sweep_end - sweep_begin;
  if (xch) chunk = std::min<int64_t>(chunk, (int64_t)1 << 20);
  if (g->grid > 1)
    chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, ((int64_t)1 << 30) / (1024 * std::max(2, a.n_phases))));
  a.xch = g->d_xch;
  for (int grp = 0; grp < g->n_groups; ++grp) {
    a.spins = g->d_spins + (size_t)grp * g->n_words;
    a.flips = g->d_flips + (size_t)grp * 3 * g->n_words;
    a.r0 = (uint32_t)(grp * g->L);
    a.r_count = group_r_count(g, grp);
    for (int64_t t0 = sweep_begin; t0 < sweep_end; t0 += chunk) {
      a.t_begin = t0;
      a.t_end = std::min(sweep_end, t0 + chunk);
      HIP_TRY(launch_fill_u32(g->d_bar + kBarTop, 1, 0u, st), "barrier reset");
      HIP_TRY(launch_fill_u32(g->d_bar + kBarGroup, 16 * 8, 0u, st), "barrier reset");
      if (xch) HIP_TRY(launch_fill_u32(g->d_bar + kBarArrive, kArriveCounters * kArriveStride, 0u, st), "arrival reset");
      if (xch) HIP_TRY(launch_xch_init(a.spins, g->d_cover, g->d_xch, g->n_words, st), "exchange words");
      HIP_TRY(launch_anneal(g->L, g->lay.enc, g->use_lds, g->res_edges[m], a, g->grid, g->lds_bytes, st),
              "anneal launch");
      if (xch) HIP_TRY(launch_xch_fini(g->d_xch, a.spins, g->n_words, st), "exchange words");
    }
  }
  return ISING_OK;
}

namespace {

ising_status_t create_impl(ising_graph_t *out, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                           const int8_t *w, ising_coloring_t coloring, int32_t n_replicas, void *stream,
                           const CreateOpts &opt) {
  g_last_error.clear();
  if (opt.tuned_ms != nullptr) *opt.tuned_ms = -1.f;
  if (out == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (n < 0 || nnz < 0 || n >= (int64_t)0x7FFFFFFF - 64)
    return fail(ISING_ERR_INVALID_ARGUMENT, "n or nnz out of range");
  if (row_ptr == nullptr || (nnz > 0 && (col == nullptr || w == nullptr)))
    return fail(ISING_ERR_INVALID_ARGUMENT, "graph pointer is NULL");
  if (n_replicas < 1) return fail(ISING_ERR_INVALID_ARGUMENT, "n_replicas < 1");
  if (coloring != ISING_COLOR_FIRST_FIT && coloring != ISING_COLOR_LARGEST_FIRST &&
      coloring != ISING_COLOR_NEAR_INDEPENDENT)
    return fail(ISING_ERR_INVALID_ARGUMENT, "unknown colouring");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (is_device_ptr(row_ptr) || is_device_ptr(col) || is_device_ptr(w)) {
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
  std::vector<int64_t> rp;
  std::vector<int32_t> cl;
  std::vector<int8_t> wt;
  ising_status_t r;
  if ((r = fetch(&rp, row_ptr, n + 1, "row_ptr")) != ISING_OK) return r;
  if ((r = fetch(&cl, col, nnz, "col")) != ISING_OK) return r;
  if ((r = fetch(&wt, w, nnz, "w")) != ISING_OK) return r;
  HostCSR csr;
  csr.n = n;
  csr.nnz = nnz;
  csr.row_ptr = rp.data();
  csr.col = cl.data();
  csr.w = wt.data();

  ising_graph_s *g = new (std::nothrow) ising_graph_s();
  if (g == nullptr) return fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed");
  g_alloc_count = 0;
  g_alloc_fail_at = std::max<int64_t>(0, env_int("ISING_FAULT_INJECT", 0));
  auto bail = [&](ising_status_t s) {
    free_all(g);
    delete g;
    g_alloc_fail_at = 0;
    return s;
  };
  g->n = n;
  g->nnz = nnz;
  g->R = n_replicas;
  if (hipGetDevice(&g->device) != hipSuccess) return bail(fail(ISING_ERR_DEVICE, "no HIP device"));
  std::string msg;
  int v = validate_graph(csr, &g->W, &msg);
  if (v != kPrepOk) return bail(fail((ising_status_t)v, msg));
  try {
    g->row_abs.assign((size_t)n, 0u);
    g->degree.assign((size_t)n, 0u);
    for (int64_t u = 0; u < n; ++u) {
      g->degree[(size_t)u] = (uint32_t)(csr.row_ptr[u + 1] - csr.row_ptr[u]);
      int64_t a = 0;
      for (int64_t k = csr.row_ptr[u]; k < csr.row_ptr[u + 1]; ++k) a += csr.w[k] < 0 ? -(int64_t)csr.w[k] : csr.w[k];
      g->row_abs[(size_t)u] = (uint32_t)a;  // validated: at most INT32_MAX
    }
  } catch (const std::bad_alloc &) {
    return bail(fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed for the row sums"));
  }
  // budget of edges inside one async phase (ISING_ASYNC_MERGE, in units of
  // 0.1 % of the edges)
  const double merge_budget = 0.001 * (double)std::max<int64_t>(0, env_int("ISING_ASYNC_MERGE", kAsyncMergeBudget));
  try {
    g->n_colors = greedy_coloring(csr, coloring != ISING_COLOR_FIRST_FIT, &g->color);
  } catch (const std::bad_alloc &) {
    return bail(fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed while colouring"));
  }
  // Batched mode: a graph made of many small components (a batch of graphs)
  // runs one workgroup per bin of whole components, with no grid barriers.
  std::vector<int32_t> bin_of;
  int32_t n_bins = 1;
  int64_t max_bin_slots = 0;
  const bool allow_lds = env_int("ISING_NO_LDS", 0) == 0;
  if (allow_lds && env_int("ISING_NO_BATCH", 0) == 0 && n > 0) {
    int64_t max_comp = 0;
    try {
      const int64_t target = opt.bin_target > 0 ? opt.bin_target : env_int("ISING_BIN_VERTICES", 4096);
      bin_of = pack_components(csr, std::max<int64_t>(64, target), &n_bins, &max_comp);
    } catch (const std::bad_alloc &) {
      return bail(fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed while finding components"));
    }
    // a batch of small graphs, or one small graph whose replicas spread over workgroups
    g->batch = max_comp <= 16384 && (n_bins >= 2 || n_replicas >= 2);
    if (g->batch) {
      std::vector<int64_t> cnt((size_t)n_bins * g->n_colors, 0);
      for (int64_t v = 0; v < n; ++v) ++cnt[(size_t)bin_of[v] * g->n_colors + g->color[v]];
      for (int32_t b = 0; b < n_bins; ++b) {
        int64_t slots = 0;
        for (int32_t c = 0; c < g->n_colors; ++c) slots += (cnt[(size_t)b * g->n_colors + c] + 63) / 64 * 64;
        max_bin_slots = std::max(max_bin_slots, slots);
      }
    }
  }
  if (!g->batch) {
    bin_of.clear();
    n_bins = 1;
  }
  // Near-independent parts for one graph (a cooperative launch, or the one
  // bin of a batched launch): fewer async phases than the largest-first
  // colouring's runs, each within the same budget; otherwise the colouring
  // stays.  Not for batches of several bins (the budget holds per graph),
  // nor above kPartSearchMaxEntries entries, where the search would take
  // minutes.
  if (coloring == ISING_COLOR_NEAR_INDEPENDENT && n > 0 && nnz <= kPartSearchMaxEntries && n_bins == 1) {
    try {
      const int32_t runs = (int32_t)phase_runs(csr, g->color, g->n_colors, merge_budget).size() - 1;
      std::vector<int32_t> part;
      const int32_t K = near_independent_parts(csr, merge_budget, runs - 1, &part);
      if (K > 0) {
        g->color.swap(part);
        g->n_colors = K;
        g->proper_classes = false;
        if (g->batch) {
          std::vector<int64_t> cnt((size_t)K, 0);
          for (int64_t v = 0; v < n; ++v) ++cnt[(size_t)g->color[v]];
          max_bin_slots = 0;
          for (int64_t c : cnt) max_bin_slots += (c + 63) / 64 * 64;
        }
      }
    } catch (const std::bad_alloc &) {
      return bail(fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed while searching parts"));
    }
  }
  // replica packing: as many replicas per pass as fit an LDS copy of the state
  int64_t n_slots = 0;
  std::vector<int64_t> class_size(g->n_colors, 0);
  for (int64_t v = 0; v < n; ++v) ++class_size[g->color[v]];
  for (int64_t c : class_size) n_slots += (c + 63) / 64 * 64;
  int L = pow2_at_least(n_replicas);
  // one small graph: one replica per workgroup, so replicas run in parallel
  if (g->batch && n_bins == 1) L = (int)std::min<int64_t>(L, std::max<int64_t>(1, env_int("ISING_BATCH_L", 1)));
  const size_t budget = g->batch ? (size_t)64 * 1024 : kLdsBudget;
  const int64_t lds_slots = g->batch ? max_bin_slots : n_slots;
  auto state_bytes = [&](int l) { return (size_t)lds_slots * (size_t)l / 8; };
  while (allow_lds && L > 1 && state_bytes(L) > budget) L >>= 1;
  g->use_lds = allow_lds && state_bytes(L) <= budget;
  if (!g->use_lds) L = pow2_at_least(n_replicas);
  const int bin_shift = (int)std::min<int64_t>(8, std::max<int64_t>(0, env_int("ISING_BIN_SHIFT", 0)));
  int enc = choose_encoding(csr, n_slots);
  if (enc == kEncW8 && env_int("ISING_WIDE", 0) != 0) enc = kEncWide;
  v = build_layout(csr, g->color, g->n_colors, g->batch ? bin_of.data() : nullptr, n_bins, enc, kmax_for(L, enc),
                   bin_shift, &g->lay, &msg);
  if (v != kPrepOk) return bail(fail((ising_status_t)v, msg));
  if (!check_layout(g->lay, csr, &msg)) return bail(fail(ISING_ERR_DEVICE, "internal layout check: " + msg));
  HostLayout &lay = g->lay;
  g->L = L;
  g->n_groups = (n_replicas + L - 1) / L;
  g->n_words = (uint32_t)((size_t)lay.n_slots * (size_t)L / 32);
  g->lds_bytes = g->use_lds && !g->batch ? std::max<size_t>((size_t)n_slots * L / 8, 16) : 0;

  // grid: enough workgroups for the largest colour class, at most what is co-resident
  int per_cu = 0;
  {
    hipError_t e = anneal_occupancy(L, lay.enc, g->use_lds, g->lds_bytes, &per_cu);
    if (e != hipSuccess) return bail(hip_fail(e, "occupancy query"));
  }
  hipDeviceProp_t prop;
  {
    hipError_t e = hipGetDeviceProperties(&prop, g->device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDeviceProperties"));
  }
  const int waves_per_block = kAnnealBlock / 64;
  const int max_grid = std::max(1, per_cu) * prop.multiProcessorCount;
  uint32_t max_phase = 0;
  for (int32_t p = 0; p < lay.n_phases; ++p)
    max_phase = std::max(max_phase, lay.phase_items[p + 1] - lay.phase_items[p]);
  int grid = (int)std::min<int64_t>(max_grid, std::max<int64_t>(1, (max_phase + waves_per_block - 1) / waves_per_block));
  if ((int64_t)lay.items.size() <= 4 * waves_per_block) grid = 1;  // no grid barriers for tiny graphs
  const int64_t want = env_int("ISING_GRID", 0);
  if (want > 0) grid = (int)std::min<int64_t>(want, max_grid);
  grid = std::min(grid, kBarMaxGrid);  // the grid barrier polls one flag per workgroup
  g->grid = grid;
  g->nw = grid * waves_per_block;
  // phase tables: deterministic = one colour class per phase; async merges
  // consecutive classes while the edges inside a phase stay within the budget
  std::vector<uint32_t> wave_ptr[2], cls_w64[2];
  for (int m = 0; m < 2; ++m) {
    std::vector<int32_t> pc;
    if (m == 0) {
      for (int32_t c = 0; c <= g->n_colors; ++c) pc.push_back(c);
    } else {
      try {
        pc = phase_runs(csr, g->color, g->n_colors, merge_budget);
      } catch (const std::bad_alloc &) {
        return bail(fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed while building phases"));
      }
    }
    g->n_phases[m] = (int32_t)pc.size() - 1;
    wave_ptr[m] = rotate_ranges(partition_waves(lay, pc, g->nw, true), g->n_phases[m], g->nw, waves_per_block);
    // register-resident entries when every wavefront's items fit them
    // (the smaller variant when it is enough; ISING_RESIDENT_EDGES=24 takes
    // the larger one, =0 neither)
    const int64_t res_knob = env_int("ISING_RESIDENT_EDGES", 1);
    if (!g->batch && g->use_lds && L == 1 && lay.enc == kEncPm1 && lay.n_slots <= kResMaxSlots && res_knob != 0) {
      uint64_t items = 0;
      const uint64_t chunks = max_wave_chunks(lay, wave_ptr[m], g->n_phases[m], g->nw, &items);
      if (items <= (uint64_t)kResMaxItems)
        g->res_edges[m] = chunks <= (uint64_t)kResChunksSmall && res_knob != kResChunks ? kResChunksSmall
                          : chunks <= (uint64_t)kResChunks                              ? kResChunks
                                                                                        : 0;
    }
    cls_w64[m].resize(pc.size());
    for (size_t p = 0; p < pc.size(); ++p) cls_w64[m][p] = (uint32_t)((uint64_t)lay.cls_begin[pc[p]] * L / 64);
  }

  // batched mode tables
  // one wave table per candidate launch shape (waves per workgroup); the
  // tuner below keeps one of them
  static const int kWaveChoices[3] = {4, 8, 16};
  std::vector<std::vector<uint32_t>> bin_wave_ptrs;
  std::vector<uint32_t> bin_words;
  int tune_forced = 0;
  if (g->batch) {
    tune_forced = opt.waves > 0 ? opt.waves : (int)env_int("ISING_BATCH_WAVES", 0);
    if (tune_forced != 0 && tune_forced != 4 && tune_forced != 8 && tune_forced != 16) tune_forced = 4;
    if (tune_forced == 0 && env_int("ISING_AUTOTUNE", 1) == 0) tune_forced = 4;
    const int32_t nc = g->n_colors;
    bin_words.resize((size_t)n_bins + 1);
    size_t max_words = 0;
    bin_wave_ptrs.resize(3);
    for (int32_t b = 0; b < n_bins; ++b) {
      std::vector<int32_t> pc((size_t)nc + 1);
      for (int32_t c = 0; c <= nc; ++c) pc[c] = b * nc + c;
      for (int k = 0; k < 3; ++k) {
        if (tune_forced != 0 && kWaveChoices[k] != tune_forced) continue;
        const std::vector<uint32_t> wp = partition_waves(lay, pc, kWaveChoices[k], false);
        bin_wave_ptrs[k].insert(bin_wave_ptrs[k].end(), wp.begin(), wp.end());
      }
      bin_words[b] = (uint32_t)((uint64_t)lay.cls_begin[(size_t)b * nc] * L / 32);
      const uint64_t end = (uint64_t)lay.cls_begin[(size_t)(b + 1) * nc] * L / 32;
      max_words = std::max<size_t>(max_words, (size_t)(end - bin_words[b]));
    }
    bin_words[n_bins] = (uint32_t)((uint64_t)lay.n_slots * L / 32);
    g->batch_lds = std::max<size_t>(max_words * 4, 16);
  }

  // device buffers
  const size_t entry_b = lay.entries.size() * sizeof(uint32_t);
  g->entry_bytes = (int64_t)entry_b + (int64_t)lay.wts.size();
  if ((r = dev_alloc(&g->d_entries, entry_b, "edge stream")) != ISING_OK) return bail(r);
  if ((r = upload(g->d_entries, lay.entries.data(), entry_b, "edge stream upload")) != ISING_OK) return bail(r);
  if (lay.enc == kEncWide) {
    if ((r = dev_alloc(&g->d_wts4, lay.wts.size(), "weights")) != ISING_OK) return bail(r);
    if ((r = upload(g->d_wts4, lay.wts.data(), lay.wts.size(), "weights upload")) != ISING_OK) return bail(r);
  }
  if ((r = dev_alloc(&g->d_vid, sizeof(int32_t) * lay.vid.size(), "slot table")) != ISING_OK) return bail(r);
  if ((r = upload(g->d_vid, lay.vid.data(), sizeof(int32_t) * lay.vid.size(), "slot upload")) != ISING_OK) return bail(r);
  if ((r = dev_alloc(&g->d_items, sizeof(Item) * lay.items.size(), "items")) != ISING_OK) return bail(r);
  if ((r = upload(g->d_items, lay.items.data(), sizeof(Item) * lay.items.size(), "items upload")) != ISING_OK) return bail(r);
  for (int m = 0; m < 2; ++m) {
    if ((r = dev_alloc(&g->d_wave_ptr[m], sizeof(uint32_t) * wave_ptr[m].size(), "wave table")) != ISING_OK) return bail(r);
    if ((r = upload(g->d_wave_ptr[m], wave_ptr[m].data(), sizeof(uint32_t) * wave_ptr[m].size(), "wave upload")) != ISING_OK)
      return bail(r);
    if ((r = dev_alloc(&g->d_cls_w64[m], sizeof(uint32_t) * cls_w64[m].size(), "class table")) != ISING_OK) return bail(r);
    if ((r = upload(g->d_cls_w64[m], cls_w64[m].data(), sizeof(uint32_t) * cls_w64[m].size(), "class upload")) != ISING_OK)
      return bail(r);
  }
  if ((r = dev_alloc(&g->d_spins, sizeof(uint32_t) * (size_t)g->n_words * g->n_groups, "spins")) != ISING_OK) return bail(r);
  if (g->use_lds && !g->batch) {
    // exchange words: one replica group at a time (groups run one after another)
    std::vector<uint8_t> cover;
    try {
      cover = word_cover(lay, L, g->n_words);
    } catch (const std::bad_alloc &) {
      return bail(fail(ISING_ERR_OUT_OF_MEMORY, "host allocation failed for the word cover"));
    }
    if ((r = dev_alloc(&g->d_xch, sizeof(unsigned long long) * g->n_words, "exchange words")) != ISING_OK) return bail(r);
    if ((r = dev_alloc(&g->d_cover, cover.size(), "word cover")) != ISING_OK) return bail(r);
    if ((r = upload(g->d_cover, cover.data(), cover.size(), "word cover upload")) != ISING_OK) return bail(r);
  }
  if ((r = dev_alloc(&g->d_flips, sizeof(uint32_t) * 3 * (size_t)g->n_words * g->n_groups, "flip planes")) != ISING_OK)
    return bail(r);
  if (g->batch) {
    if ((r = dev_alloc(&g->d_bin_words, sizeof(uint32_t) * bin_words.size(), "bin word table")) != ISING_OK) return bail(r);
    if ((r = upload(g->d_bin_words, bin_words.data(), sizeof(uint32_t) * bin_words.size(), "bin word upload")) != ISING_OK)
      return bail(r);
  }
  if ((r = dev_alloc(&g->d_bar, sizeof(uint32_t) * kBarWords, "flags")) != ISING_OK) return bail(r);
  if ((r = dev_alloc(&g->d_cut, sizeof(unsigned long long) * kCutStride * (size_t)n_replicas, "cut")) != ISING_OK)
    return bail(r);
  if ((r = dev_alloc(&g->d_stage, (size_t)n * (size_t)n_replicas, "spin staging")) != ISING_OK) return bail(r);
  if (g->batch) {
    // launch shape: forced, cached for this shape, or timed now
    int pick = 0;
    for (int k = 0; k < 3; ++k)
      if (kWaveChoices[k] == tune_forced) pick = k;
    if (tune_forced == 0) {
      const TuneKey key{g->lay.n_bins, (int64_t)lay.items.size(), (int64_t)lay.n_slots, g->L, g->n_groups,
                        lay.enc, g->batch_lds};
      bool cached = false;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
          pick = it->second;
          cached = true;
        }
      }
      if (!cached) {
        hipError_t e = launch_fill_u32(g->d_spins, g->n_words * (uint32_t)g->n_groups, 0xFFFFFFFFu, st);
        if (e != hipSuccess) return bail(hip_fail(e, "initialising spins"));
        if ((r = time_batch_shapes(g, bin_wave_ptrs, kWaveChoices, st, &pick, opt.tuned_ms)) != ISING_OK)
          return bail(r);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = pick;
      }
    }
    g->batch_waves = kWaveChoices[pick];
    const std::vector<uint32_t> &tab = bin_wave_ptrs[pick];
    if ((r = dev_alloc(&g->d_bin_wave_ptr, sizeof(uint32_t) * tab.size(), "bin wave table")) != ISING_OK)
      return bail(r);
    if ((r = upload(g->d_bin_wave_ptr, tab.data(), sizeof(uint32_t) * tab.size(), "bin wave upload")) != ISING_OK)
      return bail(r);
  }
  {
    hipError_t e = launch_fill_u32(g->d_spins, g->n_words * (uint32_t)g->n_groups, 0xFFFFFFFFu, st);
    if (e == hipSuccess) e = launch_fill_u32(g->d_bar, kBarWords, 0u, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(hip_fail(e, "initialising spins"));
  }
  // the edge stream is on the device now; keep only what later calls need
  std::vector<uint32_t>().swap(lay.entries);
  std::vector<int8_t>().swap(lay.wts);
  g_alloc_fail_at = 0;
  *out = g;
  return ISING_OK;
}

}  // namespace

extern "C" {

const char *isingLastError(void) { return g_last_error.c_str(); }

// The autotuner of the batched launch: for a graph that takes the batched
// layout, handles are built with bins of 1024, 2048 and 4096 vertices, each
// timing 4, 8 and 16 wavefronts per workgroup over 8 sweeps, and the fastest
// (bins, waves) is kept, persisted per input shape (tune_cache_*), so that
// later processes build it directly.  ISING_BIN_VERTICES or
// ISING_BATCH_WAVES force a choice, ISING_AUTOTUNE=0 turns tuning off.
ising_status_t isingCreate(ising_graph_t *out, int64_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col, const int8_t *w, ising_coloring_t coloring,
                           int32_t n_replicas, void *stream) {
  const bool tune = env_int("ISING_AUTOTUNE", 1) != 0 && std::getenv("ISING_BIN_VERTICES") == nullptr &&
                    std::getenv("ISING_BATCH_WAVES") == nullptr;
  CreateOpts opt;
  if (!tune) return create_impl(out, n, nnz, row_ptr, col, w, coloring, n_replicas, stream, opt);
  int64_t target = 0;
  int waves = 0;
  if (tune_cache_get(n, nnz, n_replicas, (int)coloring, &target, &waves)) {
    opt.bin_target = target;
    opt.waves = waves;
    return create_impl(out, n, nnz, row_ptr, col, w, coloring, n_replicas, stream, opt);
  }
  // the default bins first; a graph that does not take the batched layout ends here
  float best_ms = -1.f;
  opt.bin_target = 4096;
  opt.tuned_ms = &best_ms;
  ising_status_t r = create_impl(out, n, nnz, row_ptr, col, w, coloring, n_replicas, stream, opt);
  if (r != ISING_OK || !(*out)->batch || best_ms < 0.f) return r;
  int64_t best_target = 4096;
  int best_waves = (*out)->batch_waves;
  for (int64_t t : {2048, 1024}) {
    ising_graph_t h = nullptr;
    float ms = -1.f;
    CreateOpts o;
    o.bin_target = t;
    o.tuned_ms = &ms;
    if (create_impl(&h, n, nnz, row_ptr, col, w, coloring, n_replicas, stream, o) != ISING_OK) {
      g_last_error.clear();  // a candidate that cannot be built is skipped
      continue;
    }
    if (h->batch && ms >= 0.f && ms < best_ms) {
      best_ms = ms;
      best_target = t;
      best_waves = h->batch_waves;
    }
    DeviceGuard guard(h->device);
    free_all(h);
    delete h;
  }
  tune_cache_put(n, nnz, n_replicas, (int)coloring, best_target, best_waves);
  if (best_target == 4096) return ISING_OK;
  {
    DeviceGuard guard((*out)->device);
    free_all(*out);
    delete *out;
  }
  *out = nullptr;
  opt.bin_target = best_target;
  opt.waves = best_waves;
  opt.tuned_ms = nullptr;
  return create_impl(out, n, nnz, row_ptr, col, w, coloring, n_replicas, stream, opt);
}

ising_status_t isingDestroy(ising_graph_t g) {
  g_last_error.clear();
  if (g == nullptr) return ISING_OK;
  DeviceGuard guard(g->device);
  free_all(g);
  delete g;
  return ISING_OK;
}

ising_status_t isingGetInfo(ising_graph_t g, ising_info_t *info) {
  g_last_error.clear();
  if (g == nullptr || info == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  info->n_slots = g->lay.n_slots;
  info->n_colors = g->n_colors;
  info->replicas_per_group = g->L;
  info->n_groups = g->n_groups;
  info->uses_lds = g->use_lds ? 1 : 0;
  info->grid = g->batch ? g->lay.n_bins * g->n_groups : g->grid;
  info->block = g->batch ? 64 * g->batch_waves : kAnnealBlock;
  info->bins = g->batch ? g->lay.n_bins : 0;
  info->max_sweep_gap = 0;
  if (!g->batch && g->grid > 1) {
    // read after the work queued on every stream of the device
    uint32_t gap = 0;
    DeviceGuard guard(g->device);
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(hipMemcpy(&gap, g->d_bar + kBarGap, sizeof gap, hipMemcpyDeviceToHost), "gap readback");
    info->max_sweep_gap = (int32_t)gap;
  }
  info->resident_edges = (g->res_edges[0] ? 1 : 0) | (g->res_edges[1] ? 2 : 0);
  info->resident_chunks = std::max(g->res_edges[0], g->res_edges[1]);
  info->async_phases = g->batch ? g->n_colors : g->n_phases[1];
  info->deterministic_ok = g->proper_classes ? 1 : 0;
  info->pm1 = g->lay.enc == kEncPm1 ? 1 : 0;
  info->encoding = g->lay.enc;
  info->edge_bytes = g->entry_bytes;
  info->vertex_bytes = (int64_t)g->lay.n_slots * 4;
  info->spin_bytes = (int64_t)g->n_words * 4;
  info->items = (int64_t)g->lay.items.size();
  return ISING_OK;
}

ising_status_t isingTotalWeight(ising_graph_t g, int64_t *W) {
  g_last_error.clear();
  if (g == nullptr || W == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  *W = g->W;
  return ISING_OK;
}

constexpr int64_t kFieldMax = (1LL << 30) - 1;  // bound on sum |w| + |h| per row

ising_status_t isingSetField(ising_graph_t g, const int32_t *h, void *stream) {
  g_last_error.clear();
  if (g == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL handle");
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // anneals already queued on the stream may still read the old field
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (h == nullptr) {
    g->has_field = false;
    return ISING_OK;
  }
  std::vector<int32_t> hv;
  ising_status_t r = fetch(&hv, h, g->n, "field");
  if (r != ISING_OK) return r;
  for (int64_t v = 0; v < g->n; ++v) {
    const int64_t a = (int64_t)g->row_abs[(size_t)v] + (hv[(size_t)v] < 0 ? -(int64_t)hv[(size_t)v] : hv[(size_t)v]);
    if (a > kFieldMax)
      return fail(ISING_ERR_OVERFLOW, "vertex " + std::to_string(v) + ": sum |w| + |h| exceeds 2^30 - 1");
  }
  // per slot: 2 (-h) plus, with +-1 weights, the parity of the degree (the
  // kernel takes the unpaired pad of an odd row back out of its field)
  std::vector<int32_t> bias((size_t)g->lay.n_slots, 0);
  for (int64_t v = 0; v < g->n; ++v)
    bias[(size_t)g->lay.slot_of[(size_t)v]] =
        -2 * hv[(size_t)v] + (g->lay.enc == kEncPm1 ? (int32_t)(g->degree[(size_t)v] & 1u) : 0);
  if (g->d_bias == nullptr && (r = dev_alloc(&g->d_bias, sizeof(int32_t) * bias.size(), "field")) != ISING_OK)
    return r;
  if ((r = upload(g->d_bias, bias.data(), sizeof(int32_t) * bias.size(), "field upload")) != ISING_OK) return r;
  g->has_field = true;
  return ISING_OK;
}

ising_status_t isingSetFlipScale(ising_graph_t g, const uint8_t *scale, void *stream) {
  g_last_error.clear();
  if (g == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL handle");
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // anneals already queued on the stream may still read the old multipliers
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (scale == nullptr) {
    g->has_scale = false;
    return ISING_OK;
  }
  std::vector<uint8_t> m;
  ising_status_t r = fetch(&m, scale, g->n, "flip scale");
  if (r != ISING_OK) return r;
  for (int64_t v = 0; v < g->n; ++v)
    if (m[(size_t)v] > 15)
      return fail(ISING_ERR_INVALID_ARGUMENT, "vertex " + std::to_string(v) + ": flip scale above 15");
  std::vector<uint8_t> per_slot((size_t)g->lay.n_slots, 0);
  for (int64_t v = 0; v < g->n; ++v) per_slot[(size_t)g->lay.slot_of[(size_t)v]] = m[(size_t)v];
  if (g->d_scale == nullptr && (r = dev_alloc(&g->d_scale, per_slot.size(), "flip scale")) != ISING_OK) return r;
  if ((r = upload(g->d_scale, per_slot.data(), per_slot.size(), "flip scale upload")) != ISING_OK) return r;
  g->has_scale = true;
  return ISING_OK;
}

ising_status_t isingGetColoring(ising_graph_t g, int32_t *color, int32_t *n_colors) {
  g_last_error.clear();
  if (g == nullptr || n_colors == nullptr || (color == nullptr && g->n > 0))
    return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  if (g->n > 0) std::memcpy(color, g->color.data(), sizeof(int32_t) * (size_t)g->n);
  *n_colors = g->n_colors;
  return ISING_OK;
}

ising_status_t isingRandomizeSpins(ising_graph_t g, uint64_t seed, void *stream) {
  g_last_error.clear();
  if (g == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL handle");
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int grp = 0; grp < g->n_groups; ++grp) {
    HIP_TRY(launch_randomize(g->L, g->d_spins + (size_t)grp * g->n_words, g->d_vid, g->n_words,
                             (uint32_t)(grp * g->L), group_r_count(g, grp), seed, st),
            "randomize launch");
  }
  g->best_reset = true;
  return ISING_OK;
}

ising_status_t isingSetSpins(ising_graph_t g, const int8_t *spins, void *stream) {
  g_last_error.clear();
  if (g == nullptr || (spins == nullptr && g->n > 0)) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  if (g->n == 0) return ISING_OK;
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t count = g->n * (int64_t)g->R;
  const int8_t *src = spins;
  if (is_device_ptr(spins)) {
    HIP_TRY(launch_fill_u32(g->d_bar + kBarCheck, 1, 0u, st), "flag reset");
    HIP_TRY(launch_check_spins(spins, count, g->d_bar + kBarCheck, st), "spin check launch");
    uint32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, g->d_bar + kBarCheck, sizeof bad, hipMemcpyDeviceToHost, st), "flag readback");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (bad) return fail(ISING_ERR_INVALID_ARGUMENT, "spin values must be +1 or -1");
  } else {
    for (int64_t i = 0; i < count; ++i)
      if (spins[i] != 1 && spins[i] != -1)
        return fail(ISING_ERR_INVALID_ARGUMENT, "spin value at index " + std::to_string(i) + " is not +1 or -1");
    HIP_TRY(hipMemcpyAsync(g->d_stage, spins, (size_t)count, hipMemcpyHostToDevice, st), "spin upload");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    src = g->d_stage;
  }
  for (int grp = 0; grp < g->n_groups; ++grp)
    HIP_TRY(launch_set_spins(g->L, g->d_spins + (size_t)grp * g->n_words, g->d_vid, g->n_words, src, g->n,
                             (uint32_t)(grp * g->L), group_r_count(g, grp), st),
            "set-spins launch");
  g->best_reset = true;
  return ISING_OK;
}

ising_status_t isingGetSpins(ising_graph_t g, int8_t *spins, void *stream) {
  g_last_error.clear();
  if (g == nullptr || (spins == nullptr && g->n > 0)) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  if (g->n == 0) return ISING_OK;
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool dev = is_device_ptr(spins);
  int8_t *dst = dev ? spins : g->d_stage;
  for (int grp = 0; grp < g->n_groups; ++grp)
    HIP_TRY(launch_get_spins(g->L, g->d_spins + (size_t)grp * g->n_words, g->d_vid, (uint32_t)g->lay.n_slots,
                             dst, g->n, (uint32_t)(grp * g->L), group_r_count(g, grp), st),
            "get-spins launch");
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(spins, g->d_stage, (size_t)(g->n * g->R), hipMemcpyDeviceToHost, st), "spin readback");
    return check_flags(g, st);
  }
  return ISING_OK;
}

ising_status_t isingAnneal(ising_graph_t g, const ising_schedule_t *s, uint64_t seed, ising_mode_t mode,
                           int64_t sweep_begin, int64_t sweep_end, void *stream) {
  g_last_error.clear();
  ising_status_t r = internal_check_anneal(g, s, mode, sweep_begin, sweep_end);
  if (r != ISING_OK) return r;
  if (sweep_begin == sweep_end || g->n == 0) return ISING_OK;
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((r = ensure_thresholds(g, s, st)) != ISING_OK) return r;
  return internal_anneal(g, seed, mode, sweep_begin, sweep_end, st, g->d_thr, 0);
}

// Per replica: the sums over directed entries of w s s and of w [s != s],
// and the field energy, into g->d_cut (kCutStride words each).
ising_status_t cut_sums(ising_graph_s *g, hipStream_t st) {
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(g->d_cut), 2 * kCutStride * (uint32_t)g->R, 0u, st),
          "cut reset");
  for (int grp = 0; grp < g->n_groups; ++grp)
    for (uint32_t j = 0; j < group_r_count(g, grp); ++j) {
      CutArgs c{};
      c.entries = reinterpret_cast<const uint4 *>(g->d_entries);
      c.wts4 = g->d_wts4;
      c.vid = g->d_vid;
      c.items = g->d_items;
      c.n_items = (uint32_t)g->lay.items.size();
      c.spins = g->d_spins + (size_t)grp * g->n_words;
      c.bias = g->has_field ? g->d_bias : nullptr;
      c.out = g->d_cut + kCutStride * (size_t)(grp * g->L + j);
      c.bit = j;
      if (c.n_items > 0) HIP_TRY(launch_cut(g->L, g->lay.enc, c, st), "cut launch");
    }
  return ISING_OK;
}

ising_status_t isingUpdateBest(ising_graph_t g, int64_t *cut, void *stream) {
  g_last_error.clear();
  if (g == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL handle");
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  ising_status_t r = ISING_OK;
  if (g->d_best_cut == nullptr) {
    if ((r = dev_alloc(&g->d_best_cut, sizeof(int64_t) * (size_t)g->R, "best cuts")) != ISING_OK) return r;
    if ((r = dev_alloc(&g->d_best_spins, sizeof(uint32_t) * (size_t)g->n_words * g->n_groups, "best spins")) !=
        ISING_OK)
      return r;
    if ((r = dev_alloc(&g->d_best_mask, sizeof(uint32_t) * (size_t)g->n_groups, "best masks")) != ISING_OK) return r;
    if ((r = dev_alloc(&g->d_cutvals, sizeof(int64_t) * (size_t)g->R, "cut values")) != ISING_OK) return r;
  }
  const bool dev_out = cut != nullptr && is_device_ptr(cut);
  if ((r = cut_sums(g, st)) != ISING_OK) return r;
  int64_t *out = dev_out ? cut : g->d_cutvals;
  HIP_TRY(launch_best(g->d_cut, g->R, g->L, g->best_reset ? 1 : 0, g->d_best_cut, out, g->d_best_mask, g->d_spins,
                      g->d_best_spins, g->n_words, g->n_groups, st),
          "best-of-run update");
  g->best_reset = false;
  g->best_any = true;
  if (cut != nullptr && !dev_out) {
    HIP_TRY(hipMemcpyAsync(cut, g->d_cutvals, sizeof(int64_t) * (size_t)g->R, hipMemcpyDeviceToHost, st),
            "cut readback");
    return check_flags(g, st);
  }
  return ISING_OK;
}

ising_status_t isingGetBest(ising_graph_t g, int64_t *best_cut, int8_t *spins, void *stream) {
  g_last_error.clear();
  if (g == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL handle");
  if (!g->best_any || g->best_reset)
    return fail(ISING_ERR_INVALID_ARGUMENT, "no best recorded since the spins were last set");
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  bool sync = false;
  if (best_cut != nullptr) {
    const bool dev = is_device_ptr(best_cut);
    HIP_TRY(hipMemcpyAsync(best_cut, g->d_best_cut, sizeof(int64_t) * (size_t)g->R,
                           dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st),
            "best cut copy");
    sync = sync || !dev;
  }
  if (spins != nullptr && g->n > 0) {
    const bool dev = is_device_ptr(spins);
    int8_t *dst = dev ? spins : g->d_stage;
    for (int grp = 0; grp < g->n_groups; ++grp)
      HIP_TRY(launch_get_spins(g->L, g->d_best_spins + (size_t)grp * g->n_words, g->d_vid, (uint32_t)g->lay.n_slots,
                               dst, g->n, (uint32_t)(grp * g->L), group_r_count(g, grp), st),
              "best spins");
    if (!dev) {
      HIP_TRY(hipMemcpyAsync(spins, g->d_stage, (size_t)g->n * (size_t)g->R, hipMemcpyDeviceToHost, st),
              "best spins readback");
      sync = true;
    }
  }
  if (sync) HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  return ISING_OK;
}

ising_status_t isingCut(ising_graph_t g, int64_t *cut, int64_t *energy, void *stream) {
  g_last_error.clear();
  if (g == nullptr || cut == nullptr) return fail(ISING_ERR_INVALID_ARGUMENT, "NULL argument");
  DeviceGuard guard(g->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool dev_cut = is_device_ptr(cut);
  const bool dev_e = energy != nullptr && is_device_ptr(energy);
  if (energy != nullptr && dev_cut != dev_e)
    return fail(ISING_ERR_INVALID_ARGUMENT, "cut and energy must both be host or both be device memory");
  {
    ising_status_t r = cut_sums(g, st);
    if (r != ISING_OK) return r;
  }
  if (dev_cut) {
    HIP_TRY(launch_cut_finalize(g->d_cut, g->R, cut, energy, st), "cut finalize");
    return ISING_OK;
  }
  std::vector<unsigned long long> sums(kCutStride * (size_t)g->R);
  HIP_TRY(hipMemcpyAsync(sums.data(), g->d_cut, sizeof(unsigned long long) * sums.size(), hipMemcpyDeviceToHost, st),
          "cut readback");
  {
    ising_status_t r = check_flags(g, st);
    if (r != ISING_OK) return r;
  }
  for (int32_t i = 0; i < g->R; ++i) {
    const unsigned long long *p = sums.data() + (size_t)kCutStride * i;
    const int64_t e_dir = (int64_t)p[0], c_dir = (int64_t)p[1], F = (int64_t)p[2];
    if ((e_dir & 1) || (c_dir & 1)) return fail(ISING_ERR_DEVICE, "cut sums over directed edges are odd");
    const int64_t E = e_dir / 2, C = c_dir / 2;
    if (2 * C != g->W - E) return fail(ISING_ERR_DEVICE, "cut/energy identity 2 cut = W - E failed");
    cut[i] = C;
    if (energy) energy[i] = E + F;
  }
  return ISING_OK;
}

}  // extern "C"
