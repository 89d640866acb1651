// Seeded synthetic graph generators.
//
// This module only synthesises inputs: it holds none of the partitioning
// method's arithmetic and is shared by the GPU library's tests/benchmarks and
// by the CPU oracle's tests.  Every draw comes from a counter-based hash
// (MurmurHash3's 64-bit finaliser, public domain) of (seed, stream, counter),
// so a graph is a pure function of its parameters and the seed, independent of
// thread count.
//
// Output is a canonical symmetric CSR: xadj (u64, n+1), adjncy (u32), rows
// sorted ascending, no self-loops, no duplicate entries; optional int32 edge
// weights (symmetric).  Node weights are always unit (the paper's synthetic
// graph classes are unweighted, Appendix C table).
//
// Models (textbook definitions):
//   grid  : 2D 4-neighbour lattice, node id = r*cols + c.
//   rmat  : R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each of ef*2^scale
//           draws descends `scale` quadrant levels with probabilities
//           (a, b, c, d); self-loops dropped, symmetrised, deduplicated.
//   er    : Erdos-Renyi G(n, m): the first m distinct unordered pairs in draw
//           order, each draw a uniform ordered pair with u != v.
//   rgg   : random geometric graph in [0,1)^2 with radius r; node ids in
//           cell-major order of a grid with cells of side >= r; edge weight
//           1 + floor(8 (1 - d/r)) in {1..9}.
//   planted: planted partition (Condon & Karp's planted l-partition model,
//           drawn as a multigraph): n nodes in b contiguous groups; each of
//           d n / 2 draws picks u uniformly and v uniformly inside u's group
//           with probability f_in, else uniformly in the graph; self-loops
//           dropped, symmetrised, deduplicated.
//   chung_lu: Chung-Lu graph with a power-law expected-degree sequence
//           w_i proportional to (i + 1)^(-1 / (gamma - 1)), scaled to average
//           degree d; each of d n / 2 draws picks both endpoints with
//           probability proportional to w (inverse CDF on the prefix sums);
//           self-loops dropped, symmetrised, deduplicated.
#include <algorithm>
#include <parallel/algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

inline uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

// Draw number `ctr` of stream `stream` under `seed`.
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t s = fmix64(seed ^ 0x6a09e667f3bcc909ULL);
  s = fmix64(s ^ (stream * 0x9e3779b97f4a7c15ULL));
  return fmix64(s ^ ctr);
}

// Uniform integer in [0, n) by the multiply-shift map of the top 32 bits.
inline uint64_t bounded(uint64_t h, uint64_t n) {
  return ((h >> 32) * n) >> 32;
}

struct Csr {
  uint64_t n = 0;
  std::vector<uint64_t> xadj;
  std::vector<uint32_t> adj;
  std::vector<int32_t> w;  // empty => unit weights
};

// Build a canonical CSR from directed entries (already containing both
// directions).  Rows are sorted; duplicate (u,v) entries are merged keeping
// the first weight (generators only produce equal duplicates).
void build_csr(uint64_t n, const std::vector<uint64_t>& src, const std::vector<uint32_t>& dst,
               const std::vector<int32_t>* wt, Csr& out) {
  const size_t M = src.size();
  std::vector<uint64_t> deg(n + 1, 0);
  for (size_t e = 0; e < M; ++e) deg[src[e] + 1]++;
  for (uint64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  std::vector<uint32_t> adj(M);
  std::vector<int32_t> w(wt ? M : 0);
  {
    std::vector<uint64_t> fill(deg.begin(), deg.end() - 1);
    for (size_t e = 0; e < M; ++e) {
      uint64_t p = fill[src[e]]++;
      adj[p] = dst[e];
      if (wt) w[p] = (*wt)[e];
    }
  }
  // sort + dedup each row (parallel over rows)
  std::vector<uint64_t> newdeg(n + 1, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < (int64_t)n; ++u) {
    uint64_t b = deg[u], e = deg[u + 1];
    if (wt) {
      std::vector<std::pair<uint32_t, int32_t>> row(e - b);
      for (uint64_t i = b; i < e; ++i) row[i - b] = {adj[i], w[i]};
      std::stable_sort(row.begin(), row.end(),
                       [](const auto& x, const auto& y) { return x.first < y.first; });
      uint64_t k = 0;
      for (uint64_t i = 0; i < row.size(); ++i) {
        if (k > 0 && row[k - 1].first == row[i].first) continue;
        row[k++] = row[i];
      }
      for (uint64_t i = 0; i < k; ++i) {
        adj[b + i] = row[i].first;
        w[b + i] = row[i].second;
      }
      newdeg[u + 1] = k;
    } else {
      std::sort(adj.begin() + b, adj.begin() + e);
      uint64_t k = std::unique(adj.begin() + b, adj.begin() + e) - (adj.begin() + b);
      newdeg[u + 1] = k;
    }
  }
  out.n = n;
  out.xadj.assign(n + 1, 0);
  for (uint64_t i = 0; i < n; ++i) out.xadj[i + 1] = out.xadj[i] + newdeg[i + 1];
  out.adj.resize(out.xadj[n]);
  if (wt) out.w.resize(out.xadj[n]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < (int64_t)n; ++u) {
    uint64_t b = deg[u], k = newdeg[u + 1], o = out.xadj[u];
    std::memcpy(&out.adj[o], &adj[b], k * sizeof(uint32_t));
    if (wt) std::memcpy(&out.w[o], &w[b], k * sizeof(int32_t));
  }
}

void gen_grid(uint64_t rows, uint64_t cols, Csr& out) {
  const uint64_t n = rows * cols;
  out.n = n;
  out.xadj.assign(n + 1, 0);
  for (uint64_t r = 0; r < rows; ++r)
    for (uint64_t c = 0; c < cols; ++c) {
      uint64_t d = (r > 0) + (c > 0) + (c + 1 < cols) + (r + 1 < rows);
      out.xadj[r * cols + c + 1] = d;
    }
  for (uint64_t i = 0; i < n; ++i) out.xadj[i + 1] += out.xadj[i];
  out.adj.resize(out.xadj[n]);
  for (uint64_t r = 0; r < rows; ++r)
    for (uint64_t c = 0; c < cols; ++c) {
      uint64_t id = r * cols + c, p = out.xadj[id];
      if (r > 0) out.adj[p++] = (uint32_t)(id - cols);
      if (c > 0) out.adj[p++] = (uint32_t)(id - 1);
      if (c + 1 < cols) out.adj[p++] = (uint32_t)(id + 1);
      if (r + 1 < rows) out.adj[p++] = (uint32_t)(id + cols);
    }
}

void gen_rmat(uint32_t scale, uint64_t ef, double a, double b, double c, uint64_t seed, Csr& out) {
  const uint64_t n = 1ULL << scale;
  const uint64_t draws = ef * n;
  // quadrant thresholds on a 32-bit uniform
  const uint64_t ta = (uint64_t)std::floor(a * 4294967296.0);
  const uint64_t tb = (uint64_t)std::floor((a + b) * 4294967296.0);
  const uint64_t tc = (uint64_t)std::floor((a + b + c) * 4294967296.0);
  std::vector<uint64_t> su(draws);
  std::vector<uint32_t> sv(draws);
  std::vector<uint8_t> keep(draws);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)draws; ++e) {
    uint64_t u = 0, v = 0;
    for (uint32_t l = 0; l < scale; ++l) {
      uint64_t p = draw(seed, 1 + l, (uint64_t)e) >> 32;
      uint64_t ub = 0, vb = 0;
      if (p < ta) {
      } else if (p < tb) {
        vb = 1;
      } else if (p < tc) {
        ub = 1;
      } else {
        ub = 1;
        vb = 1;
      }
      u = (u << 1) | ub;
      v = (v << 1) | vb;
    }
    su[e] = u;
    sv[e] = (uint32_t)v;
    keep[e] = (u != v);
  }
  std::vector<uint64_t> src;
  std::vector<uint32_t> dst;
  size_t cnt = 0;
  for (uint64_t e = 0; e < draws; ++e) cnt += keep[e];
  src.reserve(2 * cnt);
  dst.reserve(2 * cnt);
  for (uint64_t e = 0; e < draws; ++e) {
    if (!keep[e]) continue;
    src.push_back(su[e]);
    dst.push_back(sv[e]);
    src.push_back(sv[e]);
    dst.push_back((uint32_t)su[e]);
  }
  su.clear();
  su.shrink_to_fit();
  build_csr(n, src, dst, nullptr, out);
}

void gen_er(uint64_t n, uint64_t m, uint64_t seed, Csr& out) {
  // First m distinct unordered pairs in draw order.
  uint64_t D = m + m / 64 + 1024;
  std::vector<std::pair<uint64_t, uint64_t>> kv;  // (pair key, first draw index)
  for (;;) {
    std::vector<uint64_t> key(D);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)D; ++e) {
      uint64_t u = bounded(draw(seed, 101, (uint64_t)e), n);
      uint64_t v = bounded(draw(seed, 102, (uint64_t)e), n);
      if (u == v) {
        key[e] = UINT64_MAX;
      } else {
        uint64_t lo = std::min(u, v), hi = std::max(u, v);
        key[e] = lo * n + hi;
      }
    }
    kv.resize(D);
    for (uint64_t e = 0; e < D; ++e) kv[e] = {key[e], e};
    // (key, draw index) pairs are distinct: any sort gives this order
    __gnu_parallel::sort(kv.begin(), kv.end());
    size_t k = 0;
    for (size_t i = 0; i < kv.size(); ++i) {
      if (kv[i].first == UINT64_MAX) break;
      if (k > 0 && kv[k - 1].first == kv[i].first) continue;  // keeps the smallest draw index
      kv[k++] = kv[i];
    }
    kv.resize(k);
    if (k >= m) break;
    D = D + D / 2;
  }
  // keep the m pairs with the smallest first-draw index
  std::nth_element(kv.begin(), kv.begin() + (m - 1), kv.end(),
                   [](const auto& x, const auto& y) { return x.second < y.second; });
  kv.resize(m);
  std::vector<uint64_t> src(2 * m);
  std::vector<uint32_t> dst(2 * m);
  for (uint64_t i = 0; i < m; ++i) {
    uint64_t lo = kv[i].first / n, hi = kv[i].first % n;
    src[2 * i] = lo;
    dst[2 * i] = (uint32_t)hi;
    src[2 * i + 1] = hi;
    dst[2 * i + 1] = (uint32_t)lo;
  }
  kv.clear();
  kv.shrink_to_fit();
  build_csr(n, src, dst, nullptr, out);
}

void sym_dedup(uint64_t n, const std::vector<uint64_t>& u, const std::vector<uint64_t>& v,
               Csr& out) {
  std::vector<uint64_t> src;
  std::vector<uint32_t> dst;
  src.reserve(2 * u.size());
  dst.reserve(2 * u.size());
  for (size_t e = 0; e < u.size(); ++e) {
    if (u[e] == v[e]) continue;
    src.push_back(u[e]);
    dst.push_back((uint32_t)v[e]);
    src.push_back(v[e]);
    dst.push_back((uint32_t)u[e]);
  }
  build_csr(n, src, dst, nullptr, out);
}

void gen_planted(uint64_t n, uint64_t groups, double avg_degree, double f_in, uint64_t seed,
                 Csr& out) {
  const uint64_t draws = (uint64_t)(avg_degree * (double)n / 2.0);
  const uint64_t t_in = (uint64_t)std::floor(f_in * 4294967296.0);
  std::vector<uint64_t> su(draws), sv(draws);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)draws; ++e) {
    const uint64_t u = bounded(draw(seed, 201, (uint64_t)e), n);
    uint64_t v;
    if ((draw(seed, 202, (uint64_t)e) >> 32) < t_in) {
      const uint64_t g = u * groups / n;                      // u's group
      const uint64_t lo = (g * n + groups - 1) / groups;      // first node of the group
      const uint64_t hi = ((g + 1) * n + groups - 1) / groups;
      v = lo + bounded(draw(seed, 203, (uint64_t)e), hi - lo);
    } else {
      v = bounded(draw(seed, 203, (uint64_t)e), n);
    }
    su[e] = u;
    sv[e] = v;
  }
  sym_dedup(n, su, sv, out);
}

void gen_chung_lu(uint64_t n, double avg_degree, double gamma, uint64_t seed, Csr& out) {
  std::vector<double> cdf(n + 1, 0.0);
  const double ex = -1.0 / (gamma - 1.0);
  for (uint64_t i = 0; i < n; ++i) cdf[i + 1] = cdf[i] + std::pow((double)(i + 1), ex);
  const double total = cdf[n];
  const uint64_t draws = (uint64_t)(avg_degree * (double)n / 2.0);
  std::vector<uint64_t> su(draws), sv(draws);
  auto pick = [&](uint64_t h) {
    // uniform in [0, total) from the top 53 bits; first i with cdf[i + 1] > x
    const double x = (double)(h >> 11) * (1.0 / 9007199254740992.0) * total;
    uint64_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) / 2;
      if (cdf[mid] <= x) lo = mid;
      else hi = mid;
    }
    return lo;
  };
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)draws; ++e) {
    su[e] = pick(draw(seed, 301, (uint64_t)e));
    sv[e] = pick(draw(seed, 302, (uint64_t)e));
  }
  sym_dedup(n, su, sv, out);
}

// Random geometric graph.  Distances in binary64 with no contraction
// (this file is compiled with -ffp-contract=off).
void gen_rgg(uint64_t n, double r, uint64_t seed, Csr& out) {
  std::vector<double> px(n), py(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    px[i] = (double)(draw(seed, 201, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    py[i] = (double)(draw(seed, 202, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
  }
  uint64_t G = (uint64_t)std::floor(1.0 / r);
  if (G < 1) G = 1;
  auto cell_of = [&](double x) {
    uint64_t c = (uint64_t)(x * (double)G);
    return c >= G ? G - 1 : c;
  };
  // counting sort of points by cell (cy, cx), stable in draw index
  std::vector<uint64_t> cstart(G * G + 1, 0);
  std::vector<uint64_t> cellid(n);
  for (uint64_t i = 0; i < n; ++i) {
    cellid[i] = cell_of(py[i]) * G + cell_of(px[i]);
    cstart[cellid[i] + 1]++;
  }
  for (uint64_t c = 0; c < G * G; ++c) cstart[c + 1] += cstart[c];
  std::vector<uint64_t> perm(n);  // new id -> draw index
  {
    std::vector<uint64_t> fill(cstart.begin(), cstart.end() - 1);
    for (uint64_t i = 0; i < n; ++i) perm[fill[cellid[i]]++] = i;
  }
  std::vector<double> x(n), y(n);
  for (uint64_t j = 0; j < n; ++j) {
    x[j] = px[perm[j]];
    y[j] = py[perm[j]];
  }
  px.clear();
  py.clear();
  // new ids are contiguous per cell: cell c holds ids [cstart[c], cstart[c+1])
  std::vector<uint64_t> deg(n + 1, 0);
  auto for_nbrs = [&](uint64_t j, auto&& f) {
    uint64_t c = cellid[perm[j]];
    int64_t cy = (int64_t)(c / G), cx = (int64_t)(c % G);
    for (int64_t dy = -1; dy <= 1; ++dy)
      for (int64_t dx = -1; dx <= 1; ++dx) {
        int64_t ny = cy + dy, nx = cx + dx;
        if (ny < 0 || nx < 0 || ny >= (int64_t)G || nx >= (int64_t)G) continue;
        uint64_t cc = (uint64_t)ny * G + (uint64_t)nx;
        for (uint64_t q = cstart[cc]; q < cstart[cc + 1]; ++q) {
          if (q == j) continue;
          double ddx = x[j] - x[q];
          double ddy = y[j] - y[q];
          double d2 = ddx * ddx;
          double t = ddy * ddy;
          d2 = d2 + t;
          double d = std::sqrt(d2);
          if (d < r) f(q, d);
        }
      }
  };
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t j = 0; j < (int64_t)n; ++j) {
    uint64_t cnt = 0;
    for_nbrs((uint64_t)j, [&](uint64_t, double) { cnt++; });
    deg[j + 1] = cnt;
  }
  for (uint64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  out.n = n;
  out.xadj = deg;
  out.adj.resize(deg[n]);
  out.w.resize(deg[n]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t j = 0; j < (int64_t)n; ++j) {
    std::vector<std::pair<uint32_t, int32_t>> row;
    for_nbrs((uint64_t)j, [&](uint64_t q, double d) {
      double f = 1.0 - d / r;
      int32_t w = 1 + (int32_t)std::floor(8.0 * f);
      row.push_back({(uint32_t)q, w});
    });
    std::sort(row.begin(), row.end());
    uint64_t o = deg[j];
    for (size_t i = 0; i < row.size(); ++i) {
      out.adj[o + i] = row[i].first;
      out.w[o + i] = row[i].second;
    }
  }
}

}  // namespace

extern "C" {

// Opaque handle holding a generated graph until the caller copies it out.
void* gg_grid(uint64_t rows, uint64_t cols) {
  Csr* g = new Csr();
  gen_grid(rows, cols, *g);
  return g;
}
void* gg_rmat(uint32_t scale, uint64_t ef, double a, double b, double c, uint64_t seed) {
  Csr* g = new Csr();
  gen_rmat(scale, ef, a, b, c, seed, *g);
  return g;
}
void* gg_er(uint64_t n, uint64_t m, uint64_t seed) {
  Csr* g = new Csr();
  gen_er(n, m, seed, *g);
  return g;
}
void* gg_planted(uint64_t n, uint64_t groups, double avg_degree, double f_in, uint64_t seed) {
  Csr* g = new Csr();
  gen_planted(n, groups, avg_degree, f_in, seed, *g);
  return g;
}
void* gg_chung_lu(uint64_t n, double avg_degree, double gamma, uint64_t seed) {
  Csr* g = new Csr();
  gen_chung_lu(n, avg_degree, gamma, seed, *g);
  return g;
}
void* gg_rgg(uint64_t n, double r, uint64_t seed) {
  Csr* g = new Csr();
  gen_rgg(n, r, seed, *g);
  return g;
}
uint64_t gg_n(void* h) { return ((Csr*)h)->n; }
uint64_t gg_nnz(void* h) { return ((Csr*)h)->adj.size(); }
int gg_weighted(void* h) { return ((Csr*)h)->w.empty() ? 0 : 1; }
void gg_copy(void* h, uint64_t* xadj, uint32_t* adjncy, int32_t* adjwgt) {
  Csr* g = (Csr*)h;
  std::memcpy(xadj, g->xadj.data(), g->xadj.size() * sizeof(uint64_t));
  std::memcpy(adjncy, g->adj.data(), g->adj.size() * sizeof(uint32_t));
  if (adjwgt && !g->w.empty()) std::memcpy(adjwgt, g->w.data(), g->w.size() * sizeof(int32_t));
}
void gg_free(void* h) { delete (Csr*)h; }
}
