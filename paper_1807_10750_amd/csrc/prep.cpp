// prep.cpp -- host preparation of a graph handle (see prep.h).
#include "prep.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <new>

namespace ising {

namespace {

std::string at(int64_t row, int64_t k) {
  char buf[96];
  if (k >= 0)
    std::snprintf(buf, sizeof buf, "row %lld entry %lld", (long long)row, (long long)k);
  else
    std::snprintf(buf, sizeof buf, "row %lld", (long long)row);
  return buf;
}

}  // namespace

int validate_graph(const HostCSR &g, int64_t *W_out, std::string *msg) {
  const int64_t n = g.n, nnz = g.nnz;
  const int64_t *rp = g.row_ptr;
  const int32_t *col = g.col;
  const int8_t *w = g.w;
  // structure
  if (rp[0] != 0) { *msg = "row_ptr[0] != 0 (" + at(0, -1) + ")"; return kPrepGraph; }
  for (int64_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) { *msg = "row_ptr decreases at " + at(v, -1); return kPrepGraph; }
  if (rp[n] != nnz) { *msg = "row_ptr[n] != nnz (" + at(n, -1) + ")"; return kPrepGraph; }
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k)
      if (col[k] < 0 || col[k] >= n) { *msg = "column out of range at " + at(v, k); return kPrepGraph; }
  // self-loops
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k)
      if (col[k] == v) { *msg = "self-loop at " + at(v, k); return kPrepSelfLoop; }
  try {
    // duplicate neighbours: stamp[u] = v + 1 once u has been seen in row v
    std::vector<int64_t> stamp(n, 0);
    for (int64_t v = 0; v < n; ++v)
      for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
        if (stamp[col[k]] == v + 1) { *msg = "duplicate neighbour at " + at(v, k); return kPrepDuplicate; }
        stamp[col[k]] = v + 1;
      }
    // symmetry: the transpose lists, for each row v, the (x, w) with x -> v.
    // Entry (v -> u, w) has its reverse iff (u, w) is in transpose row v.
    std::vector<int64_t> tp(n + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) ++tp[col[k] + 1];
    for (int64_t v = 0; v < n; ++v) tp[v + 1] += tp[v];
    std::vector<int32_t> tsrc(nnz);
    std::vector<int8_t> tw(nnz);
    {
      std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
      for (int64_t v = 0; v < n; ++v)
        for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
          int64_t pos = fill[col[k]]++;
          tsrc[pos] = (int32_t)v;
          tw[pos] = w[k];
        }
    }
    std::vector<int16_t> mark_w(n, 0);
    std::fill(stamp.begin(), stamp.end(), 0);
    for (int64_t v = 0; v < n; ++v) {
      for (int64_t q = tp[v]; q < tp[v + 1]; ++q) {
        stamp[tsrc[q]] = v + 1;
        mark_w[tsrc[q]] = tw[q];
      }
      for (int64_t k = rp[v]; k < rp[v + 1]; ++k)
        if (stamp[col[k]] != v + 1 || mark_w[col[k]] != w[k]) {
          *msg = "edge without an equal-weight reverse at " + at(v, k);
          return kPrepAsymmetric;
        }
    }
  } catch (const std::bad_alloc &) {
    *msg = "host allocation failed during validation";
    return kPrepNoMem;
  }
  // field range
  for (int64_t v = 0; v < n; ++v) {
    int64_t s = 0;
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) s += w[k] < 0 ? -(int64_t)w[k] : (int64_t)w[k];
    if (s > (int64_t)std::numeric_limits<int32_t>::max()) {
      *msg = "sum of |w| exceeds INT32_MAX at " + at(v, -1);
      return kPrepOverflow;
    }
  }
  int64_t W = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k)
      if (col[k] > v) W += w[k];
  *W_out = W;
  return kPrepOk;
}

int32_t greedy_coloring(const HostCSR &g, bool largest_first, std::vector<int32_t> *color) {
  const int64_t n = g.n;
  const int64_t *rp = g.row_ptr;
  color->assign(n, -1);
  std::vector<int32_t> visit(n);
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) maxdeg = std::max(maxdeg, rp[v + 1] - rp[v]);
  if (largest_first) {
    // counting sort by degree, descending; ids ascending inside a degree
    std::vector<int64_t> start(maxdeg + 2, 0);
    for (int64_t v = 0; v < n; ++v) ++start[maxdeg - (rp[v + 1] - rp[v]) + 1];
    for (int64_t d = 0; d <= maxdeg; ++d) start[d + 1] += start[d];
    for (int64_t v = 0; v < n; ++v) visit[start[maxdeg - (rp[v + 1] - rp[v])]++] = (int32_t)v;
  } else {
    for (int64_t v = 0; v < n; ++v) visit[v] = (int32_t)v;
  }
  std::vector<int64_t> taken(maxdeg + 2, -1);
  int32_t n_colors = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = visit[i];
    const int64_t deg = rp[v + 1] - rp[v];
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t c = (*color)[g.col[k]];
      if (c >= 0 && c <= deg) taken[c] = v;
    }
    int32_t c = 0;
    while (taken[c] == v) ++c;
    (*color)[v] = c;
    n_colors = std::max(n_colors, c + 1);
  }
  return n_colors;
}

int32_t near_independent_parts(const HostCSR &g, double budget, int32_t max_parts, std::vector<int32_t> *part) {
  const int64_t n = g.n;
  const int64_t *rp = g.row_ptr;
  std::vector<int32_t> &pt = *part;
  pt.assign(n, 0);
  max_parts = std::min(max_parts, kMaxParts);
  // visit order: degree descending, id ascending
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) maxdeg = std::max(maxdeg, rp[v + 1] - rp[v]);
  std::vector<int32_t> visit(n);
  {
    std::vector<int64_t> start(maxdeg + 2, 0);
    for (int64_t v = 0; v < n; ++v) ++start[maxdeg - (rp[v + 1] - rp[v]) + 1];
    for (int64_t d = 0; d <= maxdeg; ++d) start[d + 1] += start[d];
    for (int64_t v = 0; v < n; ++v) visit[start[maxdeg - (rp[v + 1] - rp[v])]++] = (int32_t)v;
  }
  // directed entries allowed inside one part (an undirected edge is two)
  const double limit = budget * (double)g.nnz;
  // one attempt at K parts, left in pt; true when every part fits
  auto attempt = [&](int32_t K) {
    // first fit into parts 0 .. K-2, which start out independent; a vertex
    // with a neighbour in each of them goes to part K-1
    pt.assign(n, -1);
    for (int64_t i = 0; i < n; ++i) {
      const int32_t v = visit[i];
      uint32_t used = 0;
      for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
        const int32_t q = pt[g.col[k]];
        if (q >= 0) used |= 1u << q;
      }
      int32_t q = 0;
      while (q < K - 1 && (used >> q) & 1u) ++q;
      pt[v] = q;
    }
    int64_t inside[kMaxParts] = {};
    for (int64_t v = 0; v < n; ++v)
      for (int64_t k = rp[v]; k < rp[v + 1]; ++k) inside[pt[v]] += pt[g.col[k]] == pt[v] ? 1 : 0;
    auto worst = [&]() {
      int64_t m = 0;
      for (int32_t q = 0; q < K; ++q) m = std::max(m, inside[q]);
      return m;
    };
    // local search: each vertex in turn moves to the part where it has the
    // fewest neighbours, counted with a weight per part that grows while the
    // part holds more inside edges than the mean.  When no part is better, a
    // random other part is taken with probability exp(-d / T) (d: the
    // weighted increase), T falling linearly to 0 over kPartPasses passes
    // (annealing, with a fixed-seed xorshift).  It stops once every part
    // fits, or after kPartPasses passes, or half way when the fullest part
    // has never come within twice the limit.
    double wt[kMaxParts];
    for (int32_t q = 0; q < K; ++q) wt[q] = 1.0;
    uint64_t rng = 0x9E3779B97F4A7C15ull ^ (uint64_t)K;
    auto next = [&]() {
      rng ^= rng << 13;
      rng ^= rng >> 7;
      rng ^= rng << 17;
      return rng;
    };
    int64_t best = worst();
    for (int pass = 0; pass < kPartPasses && (double)worst() > limit; ++pass) {
      if (pass >= kPartPasses / 2 && (double)best > 2.0 * limit) break;
      const double T = kPartT0 * (1.0 - (double)pass / kPartPasses);
      for (int64_t i = 0; i < n; ++i) {
        const int32_t v = visit[i];
        int64_t cnt[kMaxParts] = {};
        for (int64_t k = rp[v]; k < rp[v + 1]; ++k) ++cnt[pt[g.col[k]]];
        const int32_t cur = pt[v];
        int32_t to = cur;
        for (int32_t q = 0; q < K; ++q)
          if (wt[q] * (double)cnt[q] < wt[to] * (double)cnt[to]) to = q;
        if (to == cur && K > 1) {
          const int32_t q = (int32_t)(next() % (uint64_t)K);
          const double d = wt[q] * (double)cnt[q] - wt[cur] * (double)cnt[cur];
          const double u = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
          if (q != cur && (d <= 0.0 || (T > 0.0 && u < std::exp(-d / T)))) to = q;
        }
        if (to != cur) {
          inside[cur] -= 2 * cnt[cur];
          inside[to] += 2 * cnt[to];
          pt[v] = to;
        }
      }
      double mean = 0.0;
      for (int32_t q = 0; q < K; ++q) mean += (double)inside[q] / K;
      for (int32_t q = 0; q < K; ++q) wt[q] *= (double)inside[q] > mean ? 1.05 : 0.97;
      best = std::min(best, worst());
    }
    return (double)worst() <= limit;
  };
  // from max_parts down while the parts still fit
  int32_t found = 0;
  std::vector<int32_t> keep;
  for (int32_t K = max_parts; K >= 1; --K) {
    if (!attempt(K)) break;
    found = K;
    keep.swap(pt);
  }
  if (found > 0) pt.swap(keep);
  else pt.assign(n, 0);
  return found;
}

int choose_encoding(const HostCSR &g, int64_t n_slots) {
  bool pm1 = true;
  for (int64_t k = 0; k < g.nnz; ++k)
    if (g.w[k] != 1 && g.w[k] != -1) { pm1 = false; break; }
  if (pm1) return kEncPm1;
  return n_slots <= ((int64_t)1 << 24) ? kEncW8 : kEncWide;
}

std::vector<int32_t> pack_components(const HostCSR &g, int64_t target, int32_t *n_bins, int64_t *max_comp) {
  const int64_t n = g.n;
  // union-find over the edges
  std::vector<int32_t> parent(n);
  for (int64_t v = 0; v < n; ++v) parent[v] = (int32_t)v;
  auto find = [&](int32_t x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  };
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = g.row_ptr[v]; k < g.row_ptr[v + 1]; ++k) {
      const int32_t a = find((int32_t)v), b = find(g.col[k]);
      if (a != b) parent[a < b ? b : a] = a < b ? a : b;
    }
  // components in order of their smallest vertex, packed greedily into bins
  std::vector<int64_t> comp_size(n, 0);
  for (int64_t v = 0; v < n; ++v) ++comp_size[find((int32_t)v)];
  std::vector<int32_t> bin_of_root(n, -1), bin(n);
  int32_t nb = 0;
  int64_t fill = 0, biggest = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t r = find((int32_t)v);
    if (bin_of_root[r] < 0) {
      const int64_t c = comp_size[r];
      biggest = std::max(biggest, c);
      if (nb == 0 || fill + c > target) {
        ++nb;
        fill = 0;
      }
      bin_of_root[r] = nb - 1;
      fill += c;
    }
    bin[v] = bin_of_root[r];
  }
  *n_bins = nb;
  *max_comp = biggest;
  return bin;
}

int build_layout(const HostCSR &g, const std::vector<int32_t> &color, int32_t n_colors, const int32_t *bin_of,
                 int32_t n_bins, int enc, int kmax, int bin_shift, HostLayout *out, std::string *msg) {
  HostLayout &L = *out;
  const int64_t n = g.n;
  const int64_t *rp = g.row_ptr;
  try {
    L.enc = enc;
    L.n_phases = n_colors;
    L.n_bins = std::max(1, n_bins);
    // classes are (bin, colour) pairs: key = bin * n_colors + colour
    const int64_t n_cls = (int64_t)L.n_bins * n_colors;
    auto key = [&](int64_t v) { return (bin_of ? (int64_t)bin_of[v] * n_colors : 0) + color[v]; };
    // vertices of each class, by (degree desc, id asc)
    std::vector<int64_t> cnt(n_cls + 1, 0);
    for (int64_t v = 0; v < n; ++v) ++cnt[key(v) + 1];
    for (int64_t c = 0; c < n_cls; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> byc(n);
    {
      std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
      for (int64_t v = 0; v < n; ++v) byc[fill[key(v)]++] = (int32_t)v;
    }
    auto deg = [&](int32_t v) { return rp[v + 1] - rp[v]; };
    for (int64_t c = 0; c < n_cls; ++c)
      std::stable_sort(byc.begin() + cnt[c], byc.begin() + cnt[c + 1],
                       [&](int32_t a, int32_t b) { return deg(a) > deg(b); });
    // slots: each class padded to a multiple of 64
    L.cls_begin.assign(n_cls + 1, 0);
    for (int64_t c = 0; c < n_cls; ++c) {
      const int64_t size = cnt[c + 1] - cnt[c];
      L.cls_begin[c + 1] = L.cls_begin[c] + (size + 63) / 64 * 64;
    }
    L.n_slots = L.cls_begin[n_cls];
    if (L.n_slots >= (int64_t)0x7FFFFFFF) { *msg = "too many vertices"; return kPrepArg; }
    // slot | weight << 24 holds slots below 2^24 only; padding classes to 64
    // slots (per bin) can push the count past it, so the choice is checked
    // against the final count
    if (L.enc == kEncW8 && L.n_slots > ((int64_t)1 << 24)) {
      L.enc = kEncWide;
      kmax = kmax_for(1, kEncWide);
    }
    L.vid.assign(L.n_slots, -1);
    L.slot_of.assign(n, -1);
    for (int64_t c = 0; c < n_cls; ++c)
      for (int64_t i = cnt[c]; i < cnt[c + 1]; ++i) {
        const int64_t slot = L.cls_begin[c] + (i - cnt[c]);
        L.vid[slot] = byc[i];
        L.slot_of[byc[i]] = (int32_t)slot;
      }
    // Items: walk each class's rows (degree descending).  An item starting
    // at class position pos takes G lanes per row, the smallest G in
    // {1, 4, 16, 64} whose prefetch depth covers the first (largest) row's
    // degree, widened until K = 64 / G divides pos; it spans K rows.
    L.items.clear();
    L.phase_items.assign(n_cls + 1, 0);
    uint64_t chunks = 0;  // uint4 chunks allocated so far
    auto lanes_for = [&](int64_t d) -> uint32_t {
      for (uint32_t lanes = 1; lanes < 64; lanes *= 4)
        if (d <= ((4 * (int64_t)kmax * (int64_t)lanes) >> bin_shift)) return lanes;
      return 64;
    };
    for (int64_t c = 0; c < n_cls; ++c) {
      const int64_t size = cnt[c + 1] - cnt[c];
      for (int64_t pos = 0; pos < size;) {
        const int32_t first = L.vid[L.cls_begin[c] + pos];
        const int64_t dmax = deg(first);
        uint32_t lanes = lanes_for(dmax);
        while (pos % (64 / lanes) != 0) lanes *= 4;
        const uint32_t K = 64 / lanes;
        const uint64_t len4 = (uint64_t)(dmax + 3) / 4;
        L.items.push_back(Item{(uint32_t)(L.cls_begin[c] + pos), (uint32_t)chunks, (uint32_t)len4, lanes});
        chunks += len4 * K;
        pos += K;
        if (chunks >= (uint64_t)0xFFFFFFFFu) { *msg = "edge stream too large"; return kPrepArg; }
      }
      L.phase_items[c + 1] = (uint32_t)L.items.size();
    }
    // fill the entry stream; padding names the row's own slot (see layout.h)
    L.entries.assign(chunks * 4, 0u);
    if (L.enc == kEncWide) L.wts.assign(chunks * 4, 0);
    for (const Item &it : L.items) {
      const uint32_t K = 64 / it.g;
      for (uint32_t r = 0; r < K; ++r) {
        const int64_t slot = (int64_t)it.id + r;
        if (slot >= L.n_slots) break;
        const int32_t v = L.vid[slot];
        const int64_t deg = v < 0 ? 0 : rp[v + 1] - rp[v];
        for (int64_t q = 0; q < (int64_t)it.len4 * 4; ++q) {
          const uint64_t pos = ((uint64_t)it.base4 + (uint64_t)(q / 4) * K + r) * 4 + (q % 4);
          if (q >= deg) {
            const bool odd = ((q - deg) & 1) != 0;
            L.entries[pos] = (uint32_t)slot | (L.enc == kEncPm1 && odd ? kSignBit : 0u);
            continue;
          }
          const int64_t k = rp[v] + q;
          const uint32_t nb = (uint32_t)L.slot_of[g.col[k]];
          if (L.enc == kEncPm1) {
            L.entries[pos] = nb | (g.w[k] < 0 ? kSignBit : 0u);
          } else if (L.enc == kEncW8) {
            L.entries[pos] = nb | ((uint32_t)(uint8_t)g.w[k] << 24);
          } else {
            L.entries[pos] = nb;
            L.wts[pos] = g.w[k];
          }
        }
      }
    }
  } catch (const std::bad_alloc &) {
    *msg = "host allocation failed while building the layout";
    return kPrepNoMem;
  }
  return kPrepOk;
}

std::vector<int32_t> phase_runs(const HostCSR &g, const std::vector<int32_t> &color, int32_t n_colors,
                                double budget) {
  std::vector<int32_t> out{0};
  if (n_colors <= 0) {
    out.push_back(0);
    return out;
  }
  // vertices grouped by colour
  std::vector<int64_t> start((size_t)n_colors + 1, 0);
  for (int64_t v = 0; v < g.n; ++v) ++start[(size_t)color[v] + 1];
  for (int32_t c = 0; c < n_colors; ++c) start[c + 1] += start[c];
  std::vector<int32_t> byc((size_t)g.n);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t v = 0; v < g.n; ++v) byc[(size_t)fill[color[v]]++] = (int32_t)v;
  }
  const double limit = budget * (double)(g.nnz / 2);
  int32_t first = 0;  // first class of the open run
  int64_t inside = 0; // undirected edges inside the open run
  for (int32_t c = 1; c < n_colors; ++c) {
    // edges from class c into the open run's classes (all of them lower)
    int64_t add = 0;
    for (int64_t i = start[c]; i < start[c + 1]; ++i) {
      const int32_t v = byc[(size_t)i];
      for (int64_t k = g.row_ptr[v]; k < g.row_ptr[v + 1]; ++k) {
        const int32_t cu = color[g.col[k]];
        add += (cu >= first && cu < c) ? 1 : 0;
      }
    }
    if (budget > 0.0 && (double)(inside + add) <= limit) {
      inside += add;
    } else {
      out.push_back(c);
      first = c;
      inside = 0;
    }
  }
  out.push_back(n_colors);
  return out;
}

std::vector<uint32_t> partition_waves(const HostLayout &L, const std::vector<int32_t> &phase_cls, int32_t nw,
                                      bool rotate_small) {
  const int32_t n_ph = (int32_t)phase_cls.size() - 1;
  std::vector<uint32_t> out((size_t)n_ph * (nw + 1));
  uint64_t rot = 0;
  for (int32_t p = 0; p < n_ph; ++p) {
    const uint32_t b = L.phase_items[phase_cls[p]], e = L.phase_items[phase_cls[p + 1]];
    const int32_t nwp = nw;  // waves that share the phase
    uint32_t *o = &out[(size_t)p * (nw + 1)];
    const uint32_t n = e - b;
    if (rotate_small && n > 0 && n <= (uint32_t)nwp) {
      // one item per wavefront, item j on wavefront k + j s: the start k
      // moves from phase to phase so that no wavefront collects the first
      // item of every small phase
      const uint32_t s = (uint32_t)nwp / n, k = (uint32_t)(rot % s);
      rot += n;
      for (int32_t w = 0; w <= nw; ++w) {
        const uint32_t before = w <= (int32_t)k ? 0u : std::min<uint32_t>(n, ((uint32_t)w - k + s - 1) / s);
        o[w] = b + before;
      }
      o[nw] = e;
      continue;
    }
    std::vector<uint64_t> prefix(e - b + 1, 0);
    for (uint32_t i = b; i < e; ++i) {
      const Item &it = L.items[i];
      // a fixed share for the item's latency chain plus its entries
      const uint64_t cost = 512 + (uint64_t)it.len4 * 4 * (64 / it.g);
      prefix[i - b + 1] = prefix[i - b] + cost;
    }
    const uint64_t total = prefix.back();
    uint32_t j = 0;
    for (int32_t w = 0; w <= nw; ++w) {
      if (w >= nwp) {
        o[w] = e;
        continue;
      }
      // first item whose cost prefix reaches w/nwp of the phase
      const unsigned __int128 goal = (unsigned __int128)total * (uint64_t)w;
      while (j < e - b && (unsigned __int128)prefix[j] * (uint64_t)nwp < goal) ++j;
      o[w] = b + j;
    }
    o[nw] = e;
  }
  return out;
}

std::vector<uint32_t> rotate_ranges(const std::vector<uint32_t> &prefix, int32_t n_ph, int32_t nw,
                                    int32_t waves_per_block) {
  std::vector<uint32_t> out((size_t)n_ph * nw * 2);
  const int32_t grid = std::max(1, nw / std::max(1, waves_per_block));
  for (int32_t p = 0; p < n_ph; ++p) {
    // phase p starts at workgroup rot, so phases spread their heads
    const int32_t rot = (int32_t)(((int64_t)p * grid) / std::max(1, n_ph)) * waves_per_block;
    const uint32_t *o = &prefix[(size_t)p * (nw + 1)];
    for (int32_t w = 0; w < nw; ++w) {
      const int32_t j = ((w - rot) % nw + nw) % nw;
      out[((size_t)p * nw + w) * 2] = o[j];
      out[((size_t)p * nw + w) * 2 + 1] = o[j + 1];
    }
  }
  return out;
}

uint64_t max_wave_chunks(const HostLayout &L, const std::vector<uint32_t> &ranges, int32_t n_ph, int32_t nw,
                         uint64_t *max_items) {
  uint64_t most = 0, items = 0;
  for (int32_t w = 0; w < nw; ++w) {
    uint64_t sum = 0, cnt = 0;
    for (int32_t p = 0; p < n_ph; ++p)
      for (uint32_t i = ranges[((size_t)p * nw + w) * 2]; i < ranges[((size_t)p * nw + w) * 2 + 1]; ++i) {
        sum += (L.items[i].len4 + L.items[i].g - 1) / L.items[i].g;
        ++cnt;
      }
    most = std::max(most, sum);
    items = std::max(items, cnt);
  }
  if (max_items != nullptr) *max_items = items;
  return most;
}

std::vector<uint8_t> word_cover(const HostLayout &L, int Lbits, uint32_t n_words) {
  std::vector<uint8_t> cover(n_words, 0);
  for (const Item &it : L.items) {
    const uint64_t b0 = (uint64_t)it.id * (uint64_t)Lbits, b1 = b0 + (uint64_t)(64 / it.g) * (uint64_t)Lbits;
    for (uint64_t bit = b0; bit < b1;) {
      const uint64_t w = bit >> 5, end = std::min<uint64_t>(b1, (w + 1) << 5);
      if (w < n_words) cover[w] = (uint8_t)(cover[w] + (end - bit));
      bit = end;
    }
  }
  return cover;
}

bool check_layout(const HostLayout &L, const HostCSR &g, std::string *msg) {
  const uint64_t chunks = L.entries.size() / 4;
  for (size_t i = 0; i < L.items.size(); ++i) {
    const Item &it = L.items[i];
    const bool g_ok = it.g == 1 || it.g == 4 || it.g == 16 || it.g == 64;
    const uint32_t K = g_ok ? 64 / it.g : 1;
    const bool ok = g_ok && it.id % K == 0 && (int64_t)it.id + K <= L.n_slots &&
                    (uint64_t)it.base4 + (uint64_t)it.len4 * K <= chunks && L.vid[it.id] >= 0;
    if (!ok) {
      *msg = "layout item " + std::to_string(i) + " out of range";
      return false;
    }
  }
  // Every entry decodes to what the graph says: entry q of a vertex's row is
  // its q-th CSR neighbour with that weight, every later entry is padding on
  // its own slot (+-1 padding: pairs of opposite signs plus at most one
  // unsigned entry), and a padding row holds padding only.
  std::vector<uint8_t> seen((size_t)L.n_slots, 0);
  for (size_t i = 0; i < L.items.size(); ++i) {
    const Item &it = L.items[i];
    const uint32_t K = 64 / it.g;
    for (uint32_t r = 0; r < K; ++r) {
      const uint32_t own = it.id + r;
      const int32_t v = L.vid[own];
      const int64_t deg = v < 0 ? 0 : g.row_ptr[v + 1] - g.row_ptr[v];
      if (seen[own]++ != 0 || deg > (int64_t)it.len4 * 4) {
        *msg = "layout row of slot " + std::to_string(own) + " is listed twice or too short";
        return false;
      }
      int64_t pad_plus = 0, pad_minus = 0;
      for (uint64_t q = 0; q < (uint64_t)it.len4 * 4; ++q) {
        const uint64_t pos = ((uint64_t)it.base4 + (q / 4) * K + r) * 4 + (q % 4);
        const uint32_t x = L.entries[pos];
        const uint32_t slot = L.enc == kEncPm1 ? (x & ~kSignBit) : (L.enc == kEncW8 ? (x & 0xFFFFFFu) : x);
        const int32_t wt = L.enc == kEncPm1 ? ((x & kSignBit) ? -1 : 1)
                                            : (L.enc == kEncW8 ? (int32_t)(int8_t)(x >> 24) : (int32_t)L.wts[pos]);
        bool ok;
        if ((int64_t)q < deg) {
          const int64_t k = g.row_ptr[v] + (int64_t)q;
          ok = (int64_t)slot < L.n_slots && slot != own && L.vid[slot] == g.col[k] && wt == (int32_t)g.w[k];
        } else {
          ok = slot == own && (L.enc == kEncPm1 || wt == 0);
          if (ok) (wt < 0 ? pad_minus : pad_plus) += 1;
        }
        if (!ok) {
          *msg = "layout entry " + std::to_string(pos) + " does not match the graph";
          return false;
        }
      }
      if (L.enc == kEncPm1 && pad_plus != pad_minus && pad_plus != pad_minus + 1) {
        *msg = "layout padding of item " + std::to_string(i) + " is unbalanced";
        return false;
      }
    }
  }
  for (int64_t s = 0; s < L.n_slots; ++s)
    if (L.vid[s] >= 0 && !seen[(size_t)s]) {
      *msg = "layout slot " + std::to_string(s) + " has no row";
      return false;
    }
  for (int64_t p = 0; p < (int64_t)L.n_bins * L.n_phases; ++p)
    if (L.cls_begin[p] % 64 != 0 || L.phase_items[p] > L.phase_items[p + 1]) {
      *msg = "layout class table inconsistent";
      return false;
    }
  return true;
}

}  // namespace ising
