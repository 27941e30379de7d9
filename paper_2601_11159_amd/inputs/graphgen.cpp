// Seeded synthetic graph generators for resistance-distance workloads.
//
// This file holds graph construction only (sampling, de-duplication, largest
// connected component, relabelling). It contains none of the resistance
// distance arithmetic and is shared, as an input source, by the CPU oracle and
// the GPU path alike.
//
// Random numbers come from a counter-based generator: the SplitMix64 output
// function (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) applied to a (seed, stream, index) counter, so a
// draw depends only on its index and results do not depend on the thread
// count.
//
// Every generator returns an undirected simple graph as canonical edges
// (u < v), sorted by (u, v), restricted to the largest connected component and
// relabelled 0..n'-1 in increasing original id order.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>
#include <parallel/algorithm>
#include <omp.h>

namespace {

inline uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Counter-based draw: independent of evaluation order.
inline uint64_t draw_u64(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t k = splitmix_out(seed * 0x9e3779b97f4a7c15ULL + stream + 0x632be59bd9b4e019ULL);
  return splitmix_out(k + (idx + 1) * 0x9e3779b97f4a7c15ULL);
}

// Uniform in [0, 1).
inline double draw_unit(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(draw_u64(seed, stream, idx) >> 11) * 0x1.0p-53;
}

// Uniform in (0, 1].
inline double draw_unit_pos(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)((draw_u64(seed, stream, idx) >> 11) + 1) * 0x1.0p-53;
}

struct KeyIdx {
  uint64_t key;
  uint64_t idx;
  bool operator<(const KeyIdx& o) const { return key < o.key || (key == o.key && idx < o.idx); }
};

inline uint64_t pack(uint32_t a, uint32_t b) {
  uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  return ((uint64_t)lo << 32) | hi;
}

struct Graph {
  int64_t n = 0;
  std::vector<uint64_t> keys;  // canonical packed (u<v), sorted
};

// Union-find with path halving; union by smaller root id keeps it deterministic.
int64_t uf_find(std::vector<int64_t>& p, int64_t x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

// Keep the largest connected component (ties: the one holding the smallest id)
// and relabel its nodes 0..n'-1 in increasing original id order.
void keep_lcc(Graph& g) {
  const int64_t n = g.n;
  std::vector<int64_t> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  for (uint64_t k : g.keys) {
    int64_t a = uf_find(parent, (int64_t)(k >> 32)), b = uf_find(parent, (int64_t)(k & 0xffffffffULL));
    if (a != b) {
      if (a < b) parent[b] = a; else parent[a] = b;
    }
  }
  std::vector<int64_t> size(n, 0);
  for (int64_t i = 0; i < n; ++i) size[uf_find(parent, i)]++;
  int64_t best = 0;
  for (int64_t i = 0; i < n; ++i)
    if (size[i] > size[best]) best = i;
  std::vector<int64_t> newid(n, -1);
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i)
    if (uf_find(parent, i) == best) newid[i] = c++;
  size_t w = 0;
  for (size_t e = 0; e < g.keys.size(); ++e) {
    uint64_t k = g.keys[e];
    int64_t a = newid[k >> 32], b = newid[k & 0xffffffffULL];
    if (a >= 0 && b >= 0) g.keys[w++] = ((uint64_t)a << 32) | (uint64_t)b;  // monotone relabel keeps order
  }
  g.keys.resize(w);
  g.n = c;
}

// Sort (key, first draw index) records and keep one record per key with its
// smallest index.
void dedupe_keep_first(std::vector<KeyIdx>& v) {
  __gnu_parallel::sort(v.begin(), v.end());
  size_t w = 0;
  for (size_t i = 0; i < v.size(); ++i)
    if (w == 0 || v[w - 1].key != v[i].key) v[w++] = v[i];
  v.resize(w);
}

}  // namespace

extern "C" {

struct gg_graph {
  Graph g;
};

// 0 on success, nonzero on bad arguments or allocation failure.

int gg_grid(int32_t nx, int32_t ny, gg_graph** out) {
  if (nx < 1 || ny < 1 || (int64_t)nx * ny > (1LL << 31) - 1) return 1;
  try {
    gg_graph* h = new gg_graph();
    h->g.n = (int64_t)nx * ny;
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        uint32_t id = (uint32_t)(y * nx + x);
        if (x + 1 < nx) h->g.keys.push_back(pack(id, id + 1));
        if (y + 1 < ny) h->g.keys.push_back(pack(id, (uint32_t)(id + nx)));
      }
    std::sort(h->g.keys.begin(), h->g.keys.end());
    *out = h;
    return 0;
  } catch (const std::bad_alloc&) {
    return 2;
  }
}

// Road-like graph: an N x N four-neighbour grid, each edge deleted with
// probability p_del, plus round(frac_short * kept) shortcut draws, each joining
// a uniform node to the node at a uniform offset (dx, dy) with
// 2 <= |dx| + |dy| <= max_len, clipped to the grid; duplicates are merged and
// the largest connected component is kept.
int gg_road_like(int32_t N, double p_del, double frac_short, int32_t max_len, uint64_t seed,
                 gg_graph** out) {
  if (N < 2 || p_del < 0 || p_del >= 1 || frac_short < 0 || max_len < 2 ||
      (int64_t)N * N > (1LL << 31) - 1)
    return 1;
  try {
    gg_graph* h = new gg_graph();
    Graph& g = h->g;
    g.n = (int64_t)N * N;
    const int64_t nh = (int64_t)(N - 1) * N;  // horizontal edges, then the same count of vertical
    std::vector<uint8_t> keep(2 * nh);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < 2 * nh; ++e) keep[e] = draw_unit(seed, 2, (uint64_t)e) >= p_del;
    int64_t kept = 0;
    for (int64_t e = 0; e < 2 * nh; ++e) kept += keep[e];
    g.keys.reserve(kept + (size_t)(frac_short * kept) + 16);
    for (int64_t e = 0; e < 2 * nh; ++e) {
      if (!keep[e]) continue;
      uint32_t a, b;
      if (e < nh) {  // horizontal: row y, column x in [0, N-1)
        int64_t y = e / (N - 1), x = e % (N - 1);
        a = (uint32_t)(y * N + x);
        b = a + 1;
      } else {
        int64_t f = e - nh, y = f / N, x = f % N;  // vertical: y in [0, N-1)
        a = (uint32_t)(y * N + x);
        b = (uint32_t)(a + N);
      }
      g.keys.push_back(pack(a, b));
    }
    std::vector<std::pair<int, int>> offs;
    for (int dy = -max_len; dy <= max_len; ++dy)
      for (int dx = -max_len; dx <= max_len; ++dx) {
        int l = std::abs(dx) + std::abs(dy);
        if (l >= 2 && l <= max_len) offs.push_back({dx, dy});
      }
    const int64_t nshort = (int64_t)std::llround(frac_short * (double)kept);
    for (int64_t j = 0; j < nshort; ++j) {
      int64_t node = (int64_t)(draw_unit(seed, 3, 2 * (uint64_t)j) * (double)g.n);
      if (node >= g.n) node = g.n - 1;
      size_t oi = (size_t)(draw_unit(seed, 3, 2 * (uint64_t)j + 1) * (double)offs.size());
      if (oi >= offs.size()) oi = offs.size() - 1;
      int64_t x = node % N, y = node / N;
      int64_t tx = std::min<int64_t>(N - 1, std::max<int64_t>(0, x + offs[oi].first));
      int64_t ty = std::min<int64_t>(N - 1, std::max<int64_t>(0, y + offs[oi].second));
      int64_t t = ty * N + tx;
      if (t != node) g.keys.push_back(pack((uint32_t)node, (uint32_t)t));
    }
    __gnu_parallel::sort(g.keys.begin(), g.keys.end());
    g.keys.erase(std::unique(g.keys.begin(), g.keys.end()), g.keys.end());
    keep_lcc(g);
    *out = h;
    return 0;
  } catch (const std::bad_alloc&) {
    return 2;
  }
}

// Chung-Lu power-law graph. Node weights w_i = w_min * U_i^(-1/(gamma-1)),
// w_min = mean_deg (gamma-2)/(gamma-1), capped at sqrt(n mean_deg) and rescaled
// to mean mean_deg. Edge draws pick both endpoints independently with
// probability proportional to w; loops are discarded and draws continue until
// round(n mean_deg / 2) distinct edges exist, keeping the first ones in draw
// order. The largest connected component is kept.
int gg_chung_lu(int64_t n, double gamma, double mean_deg, uint64_t seed, gg_graph** out) {
  if (n < 2 || n > (1LL << 31) - 1 || gamma <= 2.0 || mean_deg <= 0) return 1;
  const int64_t m_target = (int64_t)std::llround((double)n * mean_deg / 2.0);
  if (m_target < 1 || (double)m_target > 0.5 * (double)n * (double)(n - 1) * 0.5) return 1;
  try {
    gg_graph* h = new gg_graph();
    Graph& g = h->g;
    g.n = n;
    std::vector<double> w(n);
    const double wmin = mean_deg * (gamma - 2.0) / (gamma - 1.0);
    const double cap = std::sqrt((double)n * mean_deg);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double x = wmin * std::pow(draw_unit_pos(seed, 1, (uint64_t)i), -1.0 / (gamma - 1.0));
      w[i] = x < cap ? x : cap;
    }
    double sum = 0;
    for (int64_t i = 0; i < n; ++i) sum += w[i];
    const double scale = mean_deg * (double)n / sum;
    std::vector<double> cum(n);
    double acc = 0;
    for (int64_t i = 0; i < n; ++i) {
      acc += w[i] * scale;
      cum[i] = acc;
    }
    const double total = acc;
    auto pick = [&](uint64_t idx) -> uint32_t {
      double x = draw_unit(seed, 4, idx) * total;
      int64_t k = std::upper_bound(cum.begin(), cum.end(), x) - cum.begin();
      return (uint32_t)(k < n ? k : n - 1);
    };
    std::vector<KeyIdx> rec;
    uint64_t drawn = 0;
    for (;;) {
      int64_t need = m_target - (int64_t)rec.size();
      uint64_t M = (uint64_t)((double)need * 1.15) + 1024;
      size_t base = rec.size();
      rec.resize(base + M);
#pragma omp parallel for schedule(static)
      for (int64_t j = 0; j < (int64_t)M; ++j) {
        uint64_t d = drawn + (uint64_t)j;
        uint32_t a = pick(2 * d), b = pick(2 * d + 1);
        rec[base + j] = KeyIdx{a == b ? ~0ULL : pack(a, b), d};
      }
      drawn += M;
      dedupe_keep_first(rec);
      if (!rec.empty() && rec.back().key == ~0ULL) rec.pop_back();  // loops
      if ((int64_t)rec.size() >= m_target) break;
    }
    if ((int64_t)rec.size() > m_target) {
      std::nth_element(rec.begin(), rec.begin() + m_target, rec.end(),
                       [](const KeyIdx& a, const KeyIdx& b) { return a.idx < b.idx; });
      rec.resize(m_target);
    }
    g.keys.resize(rec.size());
    for (size_t i = 0; i < rec.size(); ++i) g.keys[i] = rec[i].key;
    std::vector<KeyIdx>().swap(rec);
    __gnu_parallel::sort(g.keys.begin(), g.keys.end());
    keep_lcc(g);
    *out = h;
    return 0;
  } catch (const std::bad_alloc&) {
    return 2;
  }
}

// Log-normal edge weights exp(mu + sigma Z), Z standard normal by Box-Muller
// (Box & Muller, 1958), one pair of uniforms per edge index.
int gg_lognormal(int64_t m, double mu, double sigma, uint64_t seed, float* out) {
  if (m < 0 || !out) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    double u1 = draw_unit_pos(seed, 5, 2 * (uint64_t)e), u2 = draw_unit(seed, 5, 2 * (uint64_t)e + 1);
    double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    out[e] = (float)std::exp(mu + sigma * z);
  }
  return 0;
}

int64_t gg_num_nodes(const gg_graph* h) { return h ? h->g.n : -1; }
int64_t gg_num_edges(const gg_graph* h) { return h ? (int64_t)h->g.keys.size() : -1; }

void gg_copy_edges(const gg_graph* h, int32_t* u, int32_t* v) {
  const int64_t m = (int64_t)h->g.keys.size();
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    u[e] = (int32_t)(h->g.keys[e] >> 32);
    v[e] = (int32_t)(h->g.keys[e] & 0xffffffffULL);
  }
}

void gg_free(gg_graph* h) { delete h; }

}  // extern "C"
