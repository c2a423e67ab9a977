// Exercises the host preparation of a graph handle (validation, colouring,
// components, layout, phase and wavefront tables, word cover) on seeded
// random graphs, for a build with AddressSanitizer and UBSan.  Exits nonzero
// on a broken invariant; the sanitizers abort on a memory or UB error.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "prep.h"

using namespace ising;

namespace {

struct Graph {
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<int8_t> w;
  HostCSR csr() const {
    HostCSR g;
    g.n = n;
    g.nnz = (int64_t)col.size();
    g.row_ptr = rp.data();
    g.col = col.data();
    g.w = w.data();
    return g;
  }
};

// Random simple graph: n vertices, about m edges, a few hubs, weights from
// the given set, stored symmetrically.
Graph random_graph(int64_t n, int64_t m, int hubs, bool pm1, uint32_t seed) {
  std::mt19937 rng(seed);
  std::vector<std::vector<std::pair<int32_t, int8_t>>> adj((size_t)n);
  auto add = [&](int32_t u, int32_t v) {
    if (u == v) return;
    for (auto &e : adj[(size_t)u])
      if (e.first == v) return;
    int8_t w = pm1 ? (rng() & 1 ? 1 : -1) : (int8_t)((int)(rng() % 255) - 127);
    if (w == 0) w = 1;
    adj[(size_t)u].push_back({v, w});
    adj[(size_t)v].push_back({u, w});
  };
  for (int64_t k = 0; k < m; ++k) add((int32_t)(rng() % n), (int32_t)(rng() % n));
  for (int h = 0; h < hubs && n > 1; ++h)
    for (int64_t k = 0; k < n / 3; ++k) add((int32_t)h, (int32_t)(rng() % n));
  Graph g;
  g.n = n;
  g.rp.assign((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    g.rp[(size_t)v + 1] = g.rp[(size_t)v] + (int64_t)adj[(size_t)v].size();
    for (auto &e : adj[(size_t)v]) {
      g.col.push_back(e.first);
      g.w.push_back(e.second);
    }
  }
  return g;
}

int failures = 0;
void expect(bool ok, const std::string &what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what.c_str());
    ++failures;
  }
}

void exercise(const Graph &G0, bool batched, int L) {
  HostCSR g = G0.csr();
  int64_t W = 0;
  std::string msg;
  expect(validate_graph(g, &W, &msg) == kPrepOk, "valid graph accepted: " + msg);
  for (int lf = 0; lf < 2; ++lf) {
    std::vector<int32_t> color;
    const int32_t nc = greedy_coloring(g, lf != 0, &color);
    for (int64_t v = 0; v < g.n; ++v)
      for (int64_t k = g.row_ptr[v]; k < g.row_ptr[v + 1]; ++k)
        expect(color[(size_t)v] != color[(size_t)g.col[k]], "proper colouring");
    std::vector<int32_t> bin_of;
    int32_t n_bins = 1;
    if (batched) {
      int64_t max_comp = 0;
      bin_of = pack_components(g, 64, &n_bins, &max_comp);
    }
    const int enc = choose_encoding(g, g.n + 64 * (int64_t)nc);
    HostLayout lay;
    const int v = build_layout(g, color, nc, batched ? bin_of.data() : nullptr, n_bins, enc, kmax_for(L, enc), 0,
                               &lay, &msg);
    expect(v == kPrepOk, "layout built: " + msg);
    if (v != kPrepOk) continue;
    expect(check_layout(lay, g, &msg), "layout check: " + msg);
    const uint32_t n_words = (uint32_t)(lay.n_slots * L / 32);
    const std::vector<uint8_t> cover = word_cover(lay, L, n_words);
    uint64_t covered = 0;
    for (uint8_t c : cover) {
      expect(c <= 32, "cover at most 32");
      covered += c;
    }
    uint64_t want = 0;
    for (const Item &it : lay.items) want += (uint64_t)(64 / it.g) * (uint64_t)L;
    expect(covered == want, "cover sums the items' bits");
    for (double budget : {0.0, 0.01, 0.5}) {
      const std::vector<int32_t> pc = phase_runs(g, color, nc, budget);
      const int32_t n_ph = (int32_t)pc.size() - 1;
      expect(pc.front() == 0 && pc.back() == nc, "phase runs cover the classes");
      for (int32_t nw : {16, 64, 1024}) {
        const std::vector<uint32_t> pre = partition_waves(lay, pc, nw, true);
        const std::vector<uint32_t> ranges = rotate_ranges(pre, n_ph, nw, 16);
        uint64_t items = 0;
        (void)max_wave_chunks(lay, ranges, n_ph, nw, &items);
        uint64_t total = 0;
        for (int32_t p = 0; p < n_ph; ++p)
          for (int32_t w = 0; w < nw; ++w)
            total += ranges[((size_t)p * nw + w) * 2 + 1] - ranges[((size_t)p * nw + w) * 2];
        if (!batched) expect(total == lay.items.size(), "every item in one wavefront range");
      }
    }
  }
}

// Near-independent parts: every part within the budget, the fewest parts
// the search finds (one fewer finds none), the same result on a second call.
void parts(const Graph &G0) {
  HostCSR g = G0.csr();
  for (double budget : {0.0, 0.01, 0.05}) {
    std::vector<int32_t> pt, again;
    const int32_t K = near_independent_parts(g, budget, kMaxParts, &pt);
    expect(K >= 1 || g.nnz > 0, "an empty graph is one part");
    if (K == 0) continue;
    std::vector<int64_t> inside((size_t)K, 0);
    for (int64_t v = 0; v < g.n; ++v) {
      expect(pt[(size_t)v] >= 0 && pt[(size_t)v] < K, "part in range");
      for (int64_t k = g.row_ptr[v]; k < g.row_ptr[v + 1]; ++k)
        inside[(size_t)pt[(size_t)v]] += pt[(size_t)v] == pt[(size_t)g.col[k]] ? 1 : 0;
    }
    for (int32_t q = 0; q < K; ++q) expect((double)inside[(size_t)q] <= budget * (double)g.nnz, "part within budget");
    if (K > 1) expect(near_independent_parts(g, budget, K - 1, &again) == 0, "no fewer parts found");
    expect(near_independent_parts(g, budget, K, &again) == K && again == pt, "same parts again");
  }
}

Graph from_edges(int64_t n, const std::vector<std::pair<int32_t, int32_t>> &edges) {
  std::vector<std::vector<int32_t>> adj((size_t)n);
  for (auto &e : edges) {
    adj[(size_t)e.first].push_back(e.second);
    adj[(size_t)e.second].push_back(e.first);
  }
  Graph g;
  g.n = n;
  g.rp.assign((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    g.rp[(size_t)v + 1] = g.rp[(size_t)v] + (int64_t)adj[(size_t)v].size();
    for (int32_t u : adj[(size_t)v]) {
      g.col.push_back(u);
      g.w.push_back(1);
    }
  }
  return g;
}

void parts_known() {
  std::vector<int32_t> pt;
  // with no edge allowed inside a part: a triangle needs 3, an even cycle 2
  expect(near_independent_parts(from_edges(3, {{0, 1}, {1, 2}, {2, 0}}).csr(), 0.0, 16, &pt) == 3, "triangle: 3 parts");
  std::vector<std::pair<int32_t, int32_t>> cyc;
  for (int32_t v = 0; v < 10; ++v) cyc.push_back({v, (v + 1) % 10});
  expect(near_independent_parts(from_edges(10, cyc).csr(), 0.0, 16, &pt) == 2, "even cycle: 2 parts");
  // a triangle with a third of its edges allowed inside a part: 2 parts
  expect(near_independent_parts(from_edges(3, {{0, 1}, {1, 2}, {2, 0}}).csr(), 1.0 / 3.0, 16, &pt) == 2,
         "triangle, one edge allowed: 2 parts");
  // K_5 with no edge allowed cannot be split into 4
  std::vector<std::pair<int32_t, int32_t>> k5;
  for (int32_t a = 0; a < 5; ++a)
    for (int32_t b = a + 1; b < 5; ++b) k5.push_back({a, b});
  expect(near_independent_parts(from_edges(5, k5).csr(), 0.0, 4, &pt) == 0, "K5: not 4 parts");
  expect(near_independent_parts(from_edges(5, k5).csr(), 0.0, 16, &pt) == 5, "K5: 5 parts");
  expect(near_independent_parts(from_edges(4, {}).csr(), 0.0, 16, &pt) == 1, "no edges: 1 part");
}

void bad_inputs() {
  // structure, self-loop, duplicate, asymmetry, overflow: each reported
  Graph g = random_graph(50, 120, 0, true, 7);
  int64_t W = 0;
  std::string msg;
  {
    Graph b = g;
    b.rp[10] = b.rp[11] + 1;
    expect(validate_graph(b.csr(), &W, &msg) == kPrepGraph, "non-monotone row_ptr");
  }
  {
    Graph b = g;
    b.col[0] = 0;  // the first entry of row 0 names row 0 itself
    expect(validate_graph(b.csr(), &W, &msg) != kPrepOk, "self-loop rejected");
  }
  {
    Graph b = g;
    if (b.rp[1] - b.rp[0] >= 2) {
      b.col[1] = b.col[0];
      expect(validate_graph(b.csr(), &W, &msg) != kPrepOk, "duplicate rejected");
    }
  }
  {
    Graph b = g;
    b.w[0] = (int8_t)(b.w[0] == 1 ? -1 : 1);
    expect(validate_graph(b.csr(), &W, &msg) == kPrepAsymmetric, "asymmetric weight rejected");
  }
  {
    Graph b = g;
    b.col[3] = 1000;
    expect(validate_graph(b.csr(), &W, &msg) == kPrepGraph, "column out of range");
  }
}

}  // namespace

int main() {
  bad_inputs();
  exercise(random_graph(0, 0, 0, true, 1), false, 1);
  exercise(random_graph(1, 0, 0, true, 1), false, 1);
  exercise(random_graph(700, 2000, 2, true, 2), false, 1);
  exercise(random_graph(700, 2000, 2, false, 3), false, 4);
  exercise(random_graph(3000, 9000, 3, true, 4), false, 32);
  exercise(random_graph(2000, 1500, 0, true, 5), true, 8);  // many components
  parts(random_graph(0, 0, 0, true, 1));
  parts(random_graph(700, 2000, 2, true, 2));
  parts(random_graph(3000, 9000, 3, true, 4));
  parts(random_graph(2000, 1500, 0, true, 5));
  parts_known();
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("prep driver ok\n");
  return 0;
}
