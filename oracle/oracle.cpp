// CPU oracle for "Linear-Time Multilevel Graph Partitioning via Edge
// Sparsification" (arXiv 2504.17615).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
// this file; only the tests, the smoke check and the benchmark's CPU-baseline
// leg do.  It shares no code, header, table or helper with the GPU library.
//
// It is deliberately plain and slow: std::sort / std::nth_element as the only
// library steps, every quantity recomputed from its definition.  It runs
// single-threaded unless or_set_threads asks for more: then the per-node
// rating pass of label propagation, the rows of a contraction and the cut sum
// are spread over OpenMP threads.  Every parallel step only reads state fixed
// before it and its outputs are merged in a fixed order (or sorted by a total
// order), so results do not depend on the thread count.  It follows the
// paper's steps in the paper's order:
//
//   * size-constrained label propagation (Sec. 3, KaMinPar paragraph; the
//     clustering rule of Sec. 4.1), with the cluster weight limit
//     U = c(V)/(160k) and the 2.5x node-reduction cap (Sec. 4.3);
//   * 2-hop clustering through favourite clusters, including isolated nodes
//     (Sec. 4.1, Theorem 1 and the paragraph after its proof);
//   * contraction (Sec. 2, "Multilevel Graph Partitioning");
//   * Algorithm 1 (coarsening with sparsification): the budget m_hat, the
//     trigger |E'| > rho * m_hat, and weighted threshold sampling
//     (Sec. 4.2, "Weighted Threshold Sampling");
//   * termination at 160k nodes or when the shrink factor is too small
//     (Sec. 4.3);
//   * recursive bipartitioning of the coarsest graph (Sec. 4.3);
//   * uncoarsening: projection and size-constrained LP refinement with the
//     block weight limit L_max (Sec. 2 and Sec. 3).
//
// Where the paper leaves a choice open the oracle takes one fixed reading
// (visit order, tie-breaking, admission under concurrent moves, packing in
// 2-hop clustering, rounding, exact-size sampling, the bipartitioner).  Each
// reading is stated at the point where it is used.
//
// Randomness: every choice is a counter-based hash
//   H(seed, tag, x1..xj):  s = mix(seed); s = mix(s ^ tag); s = mix(s ^ xi) ...
// where mix is the SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <initializer_list>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

int g_threads = 1;  // OpenMP threads of the parallel steps (1 = plain loops)

int thread_id() {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- hashing --
uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t H(uint64_t seed, uint64_t tag, std::initializer_list<uint64_t> xs) {
  uint64_t s = mix(seed);
  s = mix(s ^ tag);
  for (uint64_t x : xs) s = mix(s ^ x);
  return s;
}

enum : uint64_t {
  TAG_SUB = 1, TAG_TIE = 2, TAG_ADM = 3, TAG_FAV = 4, TAG_TWOHOP = 5, TAG_SPARS = 6,
  TAG_IP = 7, TAG_RSUB = 8, TAG_RTIE = 9, TAG_RADM = 10,
  TAG_FFSTART = 11, TAG_FFDRAW = 12, TAG_FFBREAK = 13, TAG_FFCLAIM = 14
};

const uint32_t ISO = 0xFFFFFFFFu;  // favourite of an isolated node: after every label

// ------------------------------------------------------------------ graph --
// G = (V, E, c, omega), Sec. 2.  Symmetric CSR: every undirected edge {u,v}
// is stored as the two entries (u,v) and (v,u) with equal weight.
struct Graph {
  uint64_t n = 0;
  std::vector<uint64_t> xadj;
  std::vector<uint32_t> adj;
  std::vector<int64_t> ew;  // omega per entry
  std::vector<int64_t> nw;  // c per node
  uint64_t deg(uint64_t u) const { return xadj[u + 1] - xadj[u]; }
  uint64_t m() const { return adj.size() / 2; }  // undirected edge count |E|
  int64_t total_weight() const {
    int64_t s = 0;
    for (int64_t c : nw) s += c;
    return s;
  }
};

}  // namespace

extern "C" {

// Plain-data view used at the ctypes boundary.  Weights are int64; a NULL
// weight pointer means unit weights.
typedef struct {
  uint64_t n;
  const uint64_t* xadj;
  const uint32_t* adjncy;
  const int64_t* vwgt;
  const int64_t* adjwgt;
} or_graph;

typedef struct {
  uint32_t tau_e_num, tau_e_den;  // edge threshold tau_e (1/2)
  uint32_t tau_d_num, tau_d_den;  // density threshold tau_d (1/2)
  uint32_t rho_num, rho_den;      // minimum reduction factor rho (4)
  uint32_t sampler;               // 0 = weighted threshold sampling (exact size), 1 = uniform
                                  // random sampling, 2 = off, 3 = weighted threshold sampling
                                  // with independent coins for the edges of weight omega_t,
                                  // 4 / 5 = threshold sampling over Forest Fire / Weighted
                                  // Forest Fire burn scores (exact size)
  uint32_t clim;                  // C in U = c(V)/(C k) and the stop size C k (160)
  uint32_t shrink_num, shrink_den;  // node reduction cap 5/2 (2.5x)
  uint32_t lp_rounds, ref_rounds, subrounds;  // 5, 5, 4
  uint32_t max_levels;            // 64
  uint32_t stop_num, stop_den;    // stop when stop_den*n' > stop_num*n (19/20)
  uint32_t ff_p_num, ff_p_den;    // Forest Fire: break probability after a burn (3/5)
  uint32_t ff_nu_num, ff_nu_den;  // Forest Fire: burn ratio nu (1/2)
} or_params;

typedef struct {
  uint64_t n, m;           // this level
  uint64_t m_prime;        // |E'| before sparsification (== m if not triggered)
  uint64_t m_hat;          // budget
  uint32_t triggered;
  uint32_t lp_rounds;      // LP rounds run while clustering the previous level
  uint32_t twohop;         // 2-hop clustering ran on the previous level
  uint32_t pad;
  int64_t w_t;             // threshold weight omega_t (0 if not triggered)
  uint64_t n_gt, n_eq;     // |E'^>|, |E'^=| (undirected)
  uint64_t nclusters_lp;   // clusters after LP (before 2-hop)
} or_level_info;

typedef struct {
  int64_t cut;
  int64_t max_block_weight;
  int64_t lmax;
  uint32_t levels;
  uint32_t pad;
} or_result;

}  // extern "C"

namespace {

Graph from_view(const or_graph* v) {
  Graph g;
  g.n = v->n;
  g.xadj.assign(v->xadj, v->xadj + v->n + 1);
  uint64_t M = g.xadj[g.n];
  g.adj.assign(v->adjncy, v->adjncy + M);
  g.ew.resize(M);
  for (uint64_t e = 0; e < M; ++e) g.ew[e] = v->adjwgt ? v->adjwgt[e] : 1;
  g.nw.resize(g.n);
  for (uint64_t u = 0; u < g.n; ++u) g.nw[u] = v->vwgt ? v->vwgt[u] : 1;
  return g;
}

// ------------------------------------------------- label propagation (LP) --
// Size-constrained label propagation (Sec. 3): each node moves to the
// adjacent cluster (block) K with the most neighbours such that
// c(K) + c(u) <= cap; rounds until a round without moves or a round limit.
//
// Readings fixed here:
//  * "most neighbours" under edge weights: the rating r(K) is the sum of
//    omega(u,v) over neighbours v in K (equals the neighbour count at level 1
//    with unit weights);
//  * visit order: each round is S synchronous sub-rounds; node u is active in
//    sub-round floor(hi32(H(SUB, level, r, u)) * S / 2^32); ratings, labels and
//    cluster weights are those at the start of the sub-round; isolated nodes
//    are never active;
//  * target choice: best rating among K != label(u) with W(K) + c(u) <= cap,
//    ties by smaller H(TIE, level, r, u, K), then smaller K; u becomes a
//    candidate only if r(K) > r(own cluster);
//  * concurrent moves: per target K, candidates ordered by (gain desc,
//    hi32(H(ADM, level, r, u)) asc, u asc); the longest prefix with
//    W_start(K) + sum c <= cap is admitted (departures are not credited, so
//    no cluster or block ever exceeds cap); admitted moves are applied
//    together.
struct LpSetup {
  uint64_t seed;
  uint64_t tag_sub, tag_tie, tag_adm;
  uint64_t level;
  int64_t cap;
  uint32_t rounds, subrounds;
  bool shrink_stop;  // stop once shrink_num * |C| <= shrink_den * n
  uint32_t shrink_num, shrink_den;
};

struct Cand {
  uint32_t u, tgt;
  int64_t gain;
  uint32_t hadm;
};

uint32_t subround_of(uint64_t seed, uint64_t tag, uint64_t level, uint64_t r, uint64_t u,
                     uint32_t S) {
  uint64_t h = H(seed, tag, {level, r, u});
  return (uint32_t)(((h >> 32) * (uint64_t)S) >> 32);
}

// Returns the number of rounds run.  label/W are updated in place;
// *moves_total gets the number of applied moves.

uint32_t label_propagation(const Graph& g, std::vector<uint32_t>& label, std::vector<int64_t>& W,
                           const LpSetup& cfg, uint64_t* moves_total) {
  const uint64_t n = g.n;
  const int T = g_threads;
  std::vector<std::vector<int64_t>> ratings(T, std::vector<int64_t>(W.size(), 0));
  std::vector<std::vector<uint32_t>> touch(T);
  std::vector<std::vector<Cand>> tcands(T);
  uint64_t moves = 0;
  uint32_t rounds_run = 0;
  bool stop = false;
  for (uint32_t r = 0; r < cfg.rounds && !stop; ++r) {
    rounds_run = r + 1;
    uint64_t moved_this_round = 0;
    for (uint32_t s = 0; s < cfg.subrounds && !stop; ++s) {
      // --- rating phase: state frozen at the start of the sub-round; each
      // thread rates its share of the nodes into its own table
#pragma omp parallel for num_threads(T) schedule(dynamic, 1024)
      for (uint64_t u = 0; u < n; ++u) {
        std::vector<int64_t>& rating = ratings[thread_id()];
        std::vector<uint32_t>& touched = touch[thread_id()];
        if (g.deg(u) == 0) continue;
        if (subround_of(cfg.seed, cfg.tag_sub, cfg.level, r, u, cfg.subrounds) != s) continue;
        touched.clear();
        for (uint64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
          uint32_t K = label[g.adj[e]];
          if (rating[K] == 0) touched.push_back(K);
          rating[K] += g.ew[e];
        }
        const uint32_t own = label[u];
        const int64_t r_own = rating[own];
        bool have = false;
        uint32_t best = 0;
        int64_t best_r = 0;
        uint64_t best_h = 0;
        for (uint32_t K : touched) {
          if (K == own) continue;
          if (W[K] + g.nw[u] > cfg.cap) continue;
          uint64_t h = H(cfg.seed, cfg.tag_tie, {cfg.level, (uint64_t)r, u, (uint64_t)K});
          bool better;
          if (!have) better = true;
          else if (rating[K] != best_r) better = rating[K] > best_r;
          else if (h != best_h) better = h < best_h;
          else better = K < best;
          if (better) {
            have = true;
            best = K;
            best_r = rating[K];
            best_h = h;
          }
        }
        if (have && best_r > r_own) {
          uint32_t hadm = (uint32_t)(H(cfg.seed, cfg.tag_adm, {cfg.level, (uint64_t)r, u}) >> 32);
          tcands[thread_id()].push_back({(uint32_t)u, best, best_r - r_own, hadm});
        }
        for (uint32_t K : touched) rating[K] = 0;
      }
      std::vector<Cand> cands;
      for (auto& tc : tcands) {
        cands.insert(cands.end(), tc.begin(), tc.end());
        tc.clear();
      }
      // --- admission: per target, the longest prefix of (gain desc, hadm asc,
      // u asc) order with W_start(K) + sum c <= cap (departures not credited)
      std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) {
        if (a.tgt != b.tgt) return a.tgt < b.tgt;
        if (a.gain != b.gain) return a.gain > b.gain;
        if (a.hadm != b.hadm) return a.hadm < b.hadm;
        return a.u < b.u;
      });
      std::vector<Cand> admitted;
      for (size_t i = 0; i < cands.size();) {
        size_t j = i;
        while (j < cands.size() && cands[j].tgt == cands[i].tgt) ++j;
        const int64_t room = cfg.cap - W[cands[i].tgt];  // W is still W_start
        int64_t acc = 0;
        for (size_t p = i; p < j; ++p) {
          int64_t c = g.nw[cands[p].u];
          if (acc + c > room) break;  // longest prefix only
          acc += c;
          admitted.push_back(cands[p]);
        }
        i = j;
      }
      // --- apply all admitted moves together
      for (const Cand& c : admitted) {
        W[label[c.u]] -= g.nw[c.u];
        W[c.tgt] += g.nw[c.u];
        label[c.u] = c.tgt;
      }
      moves += admitted.size();
      moved_this_round += admitted.size();
      if (cfg.shrink_stop) {
        uint64_t ncl = 0;
        for (int64_t w : W) ncl += (w > 0);
        if ((u128)cfg.shrink_num * ncl <= (u128)cfg.shrink_den * n) stop = true;
      }
    }
    if (moved_this_round == 0) break;
  }
  if (moves_total) *moves_total = moves;
  return rounds_run;
}

uint64_t count_clusters(const std::vector<uint32_t>& label, uint64_t n) {
  std::vector<uint8_t> used(n, 0);
  for (uint32_t K : label) used[K] = 1;
  uint64_t c = 0;
  for (uint8_t x : used) c += x;
  return c;
}

// ------------------------------------------------------- 2-hop clustering --
// Sec. 4.1: a singleton cluster S = {v} gets a favourite cluster K_S among
// its adjacent clusters; singletons with the same favourite are merged while
// the weight limit allows.  Isolated nodes are clustered with each other
// (paragraph after Theorem 1's proof).
//
// Readings: every singleton lighter than U takes part (a node of weight >= U
// fits with no other node).  Favourite = adjacent cluster with the largest
// rating, ties by smaller H(FAV, level, v, K) then smaller K; isolated
// singletons share the favourite ISO (after all labels).  Singletons are
// ordered by (fav, c(v), hi32(H(TWOHOP, level, v)), v) and each favourite
// segment is packed next-fit in that order: a node joins the group opened
// last if the group's weight plus c(v) stays <= U, otherwise it opens a new
// group (label of a joiner := label of its group's first node).  Ascending
// weight keeps Theorem 1's premise: a light singleton (c <= U/2) is left
// alone only when every later node of its segment is heavier than U/2, so at
// most one light singleton per favourite stays unmerged.  Joins are taken in
// that global order and at most |C| - ceil(shrink_den * n / shrink_num) of
// them are applied (the 2.5x cap, Sec. 4.3).  Returns the number of joins.
uint64_t two_hop(const Graph& g, std::vector<uint32_t>& label, uint64_t nclusters, int64_t U,
                 uint64_t seed, uint64_t level, uint32_t shrink_num, uint32_t shrink_den) {
  const uint64_t n = g.n;
  std::vector<uint64_t> size(n, 0);
  for (uint64_t u = 0; u < n; ++u) size[label[u]]++;
  struct S {
    uint32_t fav;
    int64_t c;
    uint32_t h;
    uint32_t v;
  };
  std::vector<S> singles;
  std::vector<int64_t> rating(n, 0);
  std::vector<uint32_t> touched;
  for (uint64_t v = 0; v < n; ++v) {
    if (size[label[v]] != 1) continue;
    if (g.nw[v] >= U) continue;  // fits with no other node
    uint32_t fav = ISO;
    if (g.deg(v) > 0) {
      touched.clear();
      for (uint64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
        uint32_t K = label[g.adj[e]];
        if (rating[K] == 0) touched.push_back(K);
        rating[K] += g.ew[e];
      }
      bool have = false;
      int64_t best_r = 0;
      uint64_t best_h = 0;
      for (uint32_t K : touched) {
        uint64_t h = H(seed, TAG_FAV, {level, v, (uint64_t)K});
        bool better;
        if (!have) better = true;
        else if (rating[K] != best_r) better = rating[K] > best_r;
        else if (h != best_h) better = h < best_h;
        else better = K < fav;
        if (better) {
          have = true;
          fav = K;
          best_r = rating[K];
          best_h = h;
        }
      }
      for (uint32_t K : touched) rating[K] = 0;
    }
    uint32_t h = (uint32_t)(H(seed, TAG_TWOHOP, {level, v}) >> 32);
    singles.push_back({fav, g.nw[v], h, (uint32_t)v});
  }
  std::sort(singles.begin(), singles.end(), [](const S& a, const S& b) {
    if (a.fav != b.fav) return a.fav < b.fav;
    if (a.c != b.c) return a.c < b.c;
    if (a.h != b.h) return a.h < b.h;
    return a.v < b.v;
  });
  // the cap keeps |C| >= ceil(shrink_den * n / shrink_num)
  uint64_t floor_clusters = (uint64_t)(((u128)shrink_den * n + shrink_num - 1) / shrink_num);
  uint64_t P = nclusters > floor_clusters ? nclusters - floor_clusters : 0;
  uint64_t merged = 0;
  for (size_t i = 0; i < singles.size() && merged < P;) {
    size_t j = i;
    while (j < singles.size() && singles[j].fav == singles[i].fav) ++j;
    uint32_t leader = singles[i].v;
    int64_t group_w = singles[i].c;
    for (size_t p = i + 1; p < j && merged < P; ++p) {
      if (group_w + singles[p].c <= U) {  // joins the open group
        label[singles[p].v] = label[leader];
        group_w += singles[p].c;
        ++merged;
      } else {  // opens a new group
        leader = singles[p].v;
        group_w = singles[p].c;
      }
    }
    i = j;
  }
  return merged;
}

// ------------------------------------------------------------ contraction --
// Sec. 2: cluster C_i becomes coarse node c_i with c(c_i) = c(C_i); clusters
// C_i != C_j joined by edges get the coarse edge of weight omega(E_ij).
// Reading: coarse ids are the ranks of the used labels in ascending label
// order; rows are sorted ascending.
Graph contract(const Graph& g, const std::vector<uint32_t>& label, std::vector<uint32_t>& map) {
  const uint64_t n = g.n;
  std::vector<uint8_t> used(n, 0);
  for (uint64_t u = 0; u < n; ++u) used[label[u]] = 1;
  std::vector<uint32_t> cid(n, 0);
  uint64_t nc = 0;
  for (uint64_t K = 0; K < n; ++K)
    if (used[K]) cid[K] = (uint32_t)nc++;
  map.assign(n, 0);
  for (uint64_t u = 0; u < n; ++u) map[u] = cid[label[u]];
  Graph c;
  c.n = nc;
  c.nw.assign(nc, 0);
  for (uint64_t u = 0; u < n; ++u) c.nw[map[u]] += g.nw[u];
  // members of each coarse node
  std::vector<uint64_t> mstart(nc + 1, 0);
  for (uint64_t u = 0; u < n; ++u) mstart[map[u] + 1]++;
  for (uint64_t x = 0; x < nc; ++x) mstart[x + 1] += mstart[x];
  std::vector<uint32_t> members(n);
  {
    std::vector<uint64_t> fill(mstart.begin(), mstart.end() - 1);
    for (uint64_t u = 0; u < n; ++u) members[fill[map[u]]++] = (uint32_t)u;
  }
  // coarse rows in T contiguous ranges of x, each range built by one thread
  // into its own arrays, joined in range order
  const int T = g_threads;
  std::vector<std::vector<uint32_t>> radj(T);
  std::vector<std::vector<int64_t>> rew(T);
  std::vector<uint64_t> rowlen(nc, 0);
#pragma omp parallel for num_threads(T) schedule(static, 1)
  for (int t = 0; t < T; ++t) {
    std::vector<std::pair<uint32_t, int64_t>> row;
    for (uint64_t x = nc * t / T; x < nc * (t + 1) / T; ++x) {
      row.clear();
      for (uint64_t i = mstart[x]; i < mstart[x + 1]; ++i) {
        uint32_t u = members[i];
        for (uint64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
          uint32_t y = map[g.adj[e]];
          if (y != x) row.push_back({y, g.ew[e]});
        }
      }
      std::sort(row.begin(), row.end(),
                [](const auto& a, const auto& b) { return a.first < b.first; });
      for (size_t i = 0; i < row.size();) {
        size_t j = i;
        int64_t w = 0;
        while (j < row.size() && row[j].first == row[i].first) w += row[j++].second;
        radj[t].push_back(row[i].first);
        rew[t].push_back(w);
        rowlen[x]++;
        i = j;
      }
    }
  }
  c.xadj.assign(nc + 1, 0);
  for (uint64_t x = 0; x < nc; ++x) c.xadj[x + 1] = c.xadj[x] + rowlen[x];
  for (int t = 0; t < T; ++t) {
    c.adj.insert(c.adj.end(), radj[t].begin(), radj[t].end());
    c.ew.insert(c.ew.end(), rew[t].begin(), rew[t].end());
  }
  return c;
}

// ----------------------------------------------------------- edge budget --
// Algorithm 1: m_hat = min{tau_e |E_i|, tau_d |E_i|/|V_i| |V_{i+1}|}; the
// sparsifier runs iff |E'_{i+1}| > rho * m_hat.  Reading: rational tau and
// rho, floors, exact integer arithmetic, undirected edge counts.
uint64_t edge_budget(uint64_t m, uint64_t n, uint64_t n_next, const or_params& p) {
  u128 a = (u128)p.tau_e_num * m / p.tau_e_den;
  u128 b = (u128)p.tau_d_num * m * n_next / ((u128)p.tau_d_den * n);
  return (uint64_t)(a < b ? a : b);
}

bool budget_triggers(uint64_t m_prime, uint64_t m_hat, const or_params& p) {
  if (p.sampler == 2) return false;
  return (u128)m_prime * p.rho_den > (u128)p.rho_num * m_hat;
}

// --------------------------------------------------- threshold sampling --
// Sec. 4.2, Weighted Threshold Sampling: omega_t is the weight of the
// m_hat-th heaviest edge; edges lighter than omega_t are dropped, heavier ones
// kept, and edges of weight omega_t are sampled to reach m_hat.
// Reading: the sample of E'^= is exact-size: the r = m_hat - |E'^>| edges
// {a<b} with the smallest (H(SPARS, level, a, b), a, b) are kept, so
// |E_{i+1}| = m_hat.  `level` is the index of the level being created.
struct SparsStats {
  int64_t w_t = 0;
  uint64_t n_gt = 0, n_eq = 0;
};

// Sec. 4.2, Uniform Random Sampling: every edge is kept independently with
// probability m_hat / |E'|; the mode with coins for E'^= keeps each edge of
// weight omega_t with probability (m_hat - |E'^>|) / |E'^=| (the paper's
// literal rule).  Reading: the coin of edge {a<b} is H(SPARS, level, a, b)
// read as a uniform 64-bit fraction, and the edge is kept iff
// floor(H * N / 2^64) < r, i.e. with probability r / N up to 2^-64.
uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) >> 64); }

// Sec. 4.2, (Weighted) Forest Fire sampling, and the appendix's WFF
// algorithm: fires start at random nodes; a node reached by a fire burns a
// geometric number of its not-yet-visited neighbours (a break with
// probability p after each burn), each drawn with probability proportional
// to its edge weight among the unvisited ones (Weighted), or uniformly; every
// burn adds one to the edge's score; fires are scheduled while the burns so
// far are at most nu |E|.
// Readings (deterministic, for a data-parallel fire):
//  * fire f starts at floor(H(FFSTART, level, f) * n / 2^64); its visited set
//    starts empty (the start node is not in it, as in the appendix);
//  * a fire advances one frontier at a time: every node u of frontier l
//    draws against the visited set as it was when frontier l began; its j-th
//    draw picks, in ascending neighbour order, the entry at which the summed
//    weight of the still-candidate entries exceeds
//    floor(H(FFDRAW, level, f, l, u, j) * W / 2^64) (W = their total; unit
//    weights for Forest Fire), removes it from u's candidates and breaks
//    iff H(FFBREAK, level, f, l, u, j) < floor(p 2^64);
//  * several frontier nodes may draw the same neighbour v: the draw with the
//    smallest (floor(H(FFCLAIM, level, f, l, v, u) / 2^32), u) burns, the
//    others burn nothing; v joins the visited set and the next frontier;
//  * fire f runs iff the burns of fires 0..f-1 are at most nu |E| (exact
//    rational test), so the result does not depend on how many fires run
//    side by side;
//  * the score of an undirected edge is the number of burns of either of its
//    two entries.
// Returns the score of every entry (equal for the two entries of an edge).
struct FireStats {
  uint64_t fires = 0, burns = 0;
};

void default_params(or_params* p);

std::vector<int64_t> fire_scores(const Graph& g, uint64_t seed, uint64_t level, bool weighted,
                                 const or_params& p, FireStats* fs) {
  const uint64_t n = g.n, m = g.m();
  std::vector<int64_t> burns(g.adj.size(), 0);
  FireStats st;
  if (n == 0 || m == 0) {
    if (fs) *fs = st;
    return burns;
  }
  // break iff H < floor(p 2^64); p >= 1 always breaks
  const bool always = p.ff_p_num >= p.ff_p_den;
  const uint64_t pthr = always ? 0 : (uint64_t)(((u128)p.ff_p_num << 64) / p.ff_p_den);
  std::vector<uint8_t> visited(n);
  for (uint64_t f = 0; (u128)st.burns * p.ff_nu_den <= (u128)p.ff_nu_num * m; ++f) {
    std::fill(visited.begin(), visited.end(), 0);
    std::vector<uint32_t> frontier{(uint32_t)mulhi64(H(seed, TAG_FFSTART, {level, f}), n)};
    for (uint64_t l = 0; !frontier.empty(); ++l) {
      // draws of every frontier node against the visited set of this frontier
      struct Claim {
        uint64_t key;  // the claim hash's upper 32 bits
        uint32_t u;
        uint64_t e;
      };
      std::vector<std::pair<uint32_t, Claim>> claims;  // (v, claim)
      for (uint32_t u : frontier) {
        std::vector<uint64_t> cand;  // entries of u's row to unvisited nodes, row order
        for (uint64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
          if (!visited[g.adj[e]]) cand.push_back(e);
        for (uint64_t j = 0; !cand.empty(); ++j) {
          int64_t W = 0;
          for (uint64_t e : cand) W += weighted ? g.ew[e] : 1;
          const uint64_t R = mulhi64(H(seed, TAG_FFDRAW, {level, f, l, (uint64_t)u, j}), (uint64_t)W);
          size_t pick = 0;
          for (int64_t acc = 0; pick < cand.size(); ++pick) {
            acc += weighted ? g.ew[cand[pick]] : 1;
            if ((uint64_t)acc > R) break;
          }
          const uint64_t e = cand[pick];
          const uint32_t v = g.adj[e];
          claims.push_back(
              {v, Claim{H(seed, TAG_FFCLAIM, {level, f, l, (uint64_t)v, (uint64_t)u}) >> 32, u, e}});
          cand.erase(cand.begin() + pick);
          if (always || H(seed, TAG_FFBREAK, {level, f, l, (uint64_t)u, j}) < pthr) break;
        }
      }
      // one burn per claimed node: the smallest (key, u)
      std::sort(claims.begin(), claims.end(), [](const auto& a, const auto& b) {
        if (a.first != b.first) return a.first < b.first;
        if (a.second.key != b.second.key) return a.second.key < b.second.key;
        return a.second.u < b.second.u;
      });
      std::vector<uint32_t> next;
      for (size_t i = 0; i < claims.size(); ++i) {
        if (i > 0 && claims[i].first == claims[i - 1].first) continue;
        burns[claims[i].second.e] += 1;
        st.burns += 1;
        visited[claims[i].first] = 1;
        next.push_back(claims[i].first);
      }
      frontier.swap(next);
    }
    st.fires = f + 1;
  }
  // score of an edge: burns of both its entries (rows are sorted)
  std::vector<int64_t> score(g.adj.size(), 0);
  for (uint64_t u = 0; u < n; ++u)
    for (uint64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
      const uint32_t v = g.adj[e];
      const auto first = g.adj.begin() + g.xadj[v], last = g.adj.begin() + g.xadj[v + 1];
      const uint64_t r = (uint64_t)(std::lower_bound(first, last, (uint32_t)u) - g.adj.begin());
      score[e] = burns[e] + burns[r];
    }
  if (fs) *fs = st;
  return score;
}

Graph sparsify(const Graph& g, uint64_t m_hat, uint64_t seed, uint64_t level, uint32_t sampler,
               SparsStats* st, const or_params* fp = nullptr, FireStats* fst = nullptr) {
  // selection key of an edge: its weight, or its fire score (samplers 4, 5)
  struct E {
    uint32_t a, b;
    int64_t w, key;
  };
  std::vector<int64_t> score;
  if (sampler == 4 || sampler == 5) {
    or_params dp;
    if (!fp) default_params(&dp);
    score = fire_scores(g, seed, level, sampler == 5, fp ? *fp : dp, fst);
  }
  std::vector<E> edges;
  for (uint64_t a = 0; a < g.n; ++a)
    for (uint64_t e = g.xadj[a]; e < g.xadj[a + 1]; ++e)
      if (a < g.adj[e]) edges.push_back({(uint32_t)a, g.adj[e], g.ew[e], score.empty() ? g.ew[e] : score[e]});
  std::vector<uint8_t> keep(edges.size(), 0);
  SparsStats s;
  if (sampler == 1) {
    const uint64_t mp = edges.size();
    for (size_t i = 0; i < edges.size(); ++i) {
      const uint64_t h = H(seed, TAG_SPARS, {level, (uint64_t)edges[i].a, (uint64_t)edges[i].b});
      if (mulhi64(h, mp) < m_hat) keep[i] = 1;
    }
  } else if (m_hat > 0 && !edges.empty()) {
    std::vector<int64_t> ws(edges.size());
    for (size_t i = 0; i < edges.size(); ++i) ws[i] = edges[i].key;
    std::nth_element(ws.begin(), ws.begin() + (m_hat - 1), ws.end(), std::greater<int64_t>());
    s.w_t = ws[m_hat - 1];
    std::vector<std::pair<uint64_t, size_t>> eq;  // (hash, edge index); edges listed by (a, b)
    for (size_t i = 0; i < edges.size(); ++i) {
      if (edges[i].key > s.w_t) {
        keep[i] = 1;
        s.n_gt++;
      } else if (edges[i].key == s.w_t) {
        s.n_eq++;
        eq.push_back({H(seed, TAG_SPARS, {level, (uint64_t)edges[i].a, (uint64_t)edges[i].b}), i});
      }
    }
    uint64_t r = m_hat - s.n_gt;
    if (sampler == 3) {
      for (const auto& q : eq)
        if (mulhi64(q.first, s.n_eq) < r) keep[q.second] = 1;
    } else {
      // edge indices increase with (a, b), so (hash, index) orders by (hash, a, b)
      std::sort(eq.begin(), eq.end());
      for (uint64_t j = 0; j < r; ++j) keep[eq[j].second] = 1;
    }
  }
  if (st) *st = s;
  Graph out;
  out.n = g.n;
  out.nw = g.nw;
  std::vector<uint64_t> deg(g.n + 1, 0);
  for (size_t i = 0; i < edges.size(); ++i)
    if (keep[i]) {
      deg[edges[i].a + 1]++;
      deg[edges[i].b + 1]++;
    }
  for (uint64_t u = 0; u < g.n; ++u) deg[u + 1] += deg[u];
  out.xadj = deg;
  out.adj.resize(deg[g.n]);
  out.ew.resize(deg[g.n]);
  std::vector<uint64_t> fill(deg.begin(), deg.end() - 1);
  for (size_t i = 0; i < edges.size(); ++i)
    if (keep[i]) {
      uint64_t p = fill[edges[i].a]++;
      out.adj[p] = edges[i].b;
      out.ew[p] = edges[i].w;
      p = fill[edges[i].b]++;
      out.adj[p] = edges[i].a;
      out.ew[p] = edges[i].w;
    }
  // rows sorted by neighbour (pairs were emitted in (a, b) order, so row a
  // gets b ascending after its smaller neighbours; sort to be plain about it)
  for (uint64_t u = 0; u < g.n; ++u) {
    std::vector<std::pair<uint32_t, int64_t>> row;
    for (uint64_t e = out.xadj[u]; e < out.xadj[u + 1]; ++e) row.push_back({out.adj[e], out.ew[e]});
    std::sort(row.begin(), row.end());
    for (size_t i = 0; i < row.size(); ++i) {
      out.adj[out.xadj[u] + i] = row[i].first;
      out.ew[out.xadj[u] + i] = row[i].second;
    }
  }
  return out;
}

// -------------------------------------------------------------- hierarchy --
struct Hierarchy {
  std::vector<Graph> levels;              // G_1 .. G_l
  std::vector<std::vector<uint32_t>> maps;  // maps[i]: G_{i+1} node of each G_i node (0-based i)
  std::vector<or_level_info> info;
};

void default_params(or_params* p) {
  p->tau_e_num = 1; p->tau_e_den = 2;
  p->tau_d_num = 1; p->tau_d_den = 2;
  p->rho_num = 4; p->rho_den = 1;
  p->sampler = 0;
  p->clim = 160;
  p->shrink_num = 5; p->shrink_den = 2;
  p->lp_rounds = 5; p->ref_rounds = 5; p->subrounds = 4;
  p->max_levels = 64;
  p->stop_num = 19; p->stop_den = 20;
  p->ff_p_num = 3; p->ff_p_den = 5;
  p->ff_nu_num = 1; p->ff_nu_den = 2;
}

int64_t cluster_limit(int64_t cV, uint32_t k, const or_params& p) {
  // U = c(V) / (160 k), Sec. 4.3; floored, at least 1
  int64_t U = (int64_t)((u128)cV / ((u128)p.clim * k));
  return U < 1 ? 1 : U;
}

// One coarsening step of Algorithm 1's loop body up to (excluding) the
// sparsification decision: cluster G_i and contract.
struct Step {
  std::vector<uint32_t> label;
  uint32_t lp_rounds = 0;
  uint64_t nclusters_lp = 0;
  bool twohop = false;
  uint64_t nclusters = 0;
};

Step cluster_level(const Graph& g, int64_t U, uint64_t seed, uint64_t level, const or_params& p) {
  Step st;
  st.label.resize(g.n);
  std::vector<int64_t> W(g.n);
  for (uint64_t u = 0; u < g.n; ++u) {
    st.label[u] = (uint32_t)u;
    W[u] = g.nw[u];
  }
  LpSetup cfg{seed, TAG_SUB, TAG_TIE, TAG_ADM, level, U, p.lp_rounds, p.subrounds,
              true, p.shrink_num, p.shrink_den};
  st.lp_rounds = label_propagation(g, st.label, W, cfg, nullptr);
  st.nclusters_lp = count_clusters(st.label, g.n);
  st.nclusters = st.nclusters_lp;
  // 2-hop clustering when LP reduced the node count by less than 2x (Sec. 3)
  if (2 * st.nclusters > g.n) {
    st.twohop = true;
    uint64_t merged = two_hop(g, st.label, st.nclusters, U, seed, level, p.shrink_num, p.shrink_den);
    st.nclusters -= merged;
  }
  return st;
}

Hierarchy coarsen(const Graph& g1, uint32_t k, uint64_t seed, const or_params& p) {
  Hierarchy h;
  h.levels.push_back(g1);
  or_level_info i1{};
  i1.n = g1.n;
  i1.m = g1.m();
  i1.m_prime = i1.m;
  h.info.push_back(i1);
  const int64_t U = cluster_limit(g1.total_weight(), k, p);
  uint64_t i = 1;
  // Algorithm 1: while G_i is not small enough (more than C k nodes)
  while ((u128)h.levels.back().n > (u128)p.clim * k && i < p.max_levels) {
    const Graph& gi = h.levels.back();
    Step st = cluster_level(gi, U, seed, i, p);
    std::vector<uint32_t> map;
    Graph gp = contract(gi, st.label, map);
    // shrink factor too small: discard G' and stop (Sec. 4.3)
    if ((u128)p.stop_den * gp.n > (u128)p.stop_num * gi.n) break;
    or_level_info li{};
    li.n = gp.n;
    li.m_prime = gp.m();
    li.m_hat = edge_budget(gi.m(), gi.n, gp.n, p);
    li.lp_rounds = st.lp_rounds;
    li.twohop = st.twohop;
    li.nclusters_lp = st.nclusters_lp;
    if (budget_triggers(li.m_prime, li.m_hat, p)) {
      SparsStats ss;
      Graph gs = sparsify(gp, li.m_hat, seed, i + 1, p.sampler, &ss, &p);
      li.triggered = 1;
      li.w_t = ss.w_t;
      li.n_gt = ss.n_gt;
      li.n_eq = ss.n_eq;
      gp = std::move(gs);
    }
    li.m = gp.m();
    h.maps.push_back(std::move(map));
    h.levels.push_back(std::move(gp));
    h.info.push_back(li);
    ++i;
  }
  return h;
}

// ------------------------------------------------- initial partitioning --
// Sec. 4.3: recursive bipartitioning of the coarsest graph.  Reading: greedy
// graph growing.  For a node set S that gets blocks [off, off + kS):
// k1 = ceil(kS/2), target T1 = ceil(c(S) k1 / kS).  A BFS over G[S] starts at
// the unvisited node of S with the smallest (H(IP, level, off, kS, u), u);
// a popped node joins part 1 iff w1 + c(v) <= T1 and only joined nodes expand
// (neighbours in ascending order); when the queue runs dry the next start is
// taken; growing stops at w1 = T1 or when S is exhausted.  Part 1 recurses on
// [off, off+k1), the rest on [off+k1, off+kS).
void bisect(const Graph& g, const std::vector<uint32_t>& S, uint32_t kS, uint32_t off,
            uint64_t seed, uint64_t level, std::vector<uint32_t>& block,
            std::vector<uint32_t>& inset, uint32_t& stamp) {
  if (S.empty()) return;
  if (kS == 1) {
    for (uint32_t v : S) block[v] = off;
    return;
  }
  const uint32_t k1 = (kS + 1) / 2;
  int64_t cS = 0;
  for (uint32_t v : S) cS += g.nw[v];
  const int64_t T1 = (int64_t)(((u128)cS * k1 + kS - 1) / kS);
  const uint32_t my = ++stamp;
  for (uint32_t v : S) inset[v] = my;
  std::vector<std::pair<uint64_t, uint32_t>> order;
  for (uint32_t v : S) order.push_back({H(seed, TAG_IP, {level, (uint64_t)off, (uint64_t)kS, (uint64_t)v}), v});
  std::sort(order.begin(), order.end());
  std::vector<uint8_t> visited(g.n, 0), part1(g.n, 0);
  int64_t w1 = 0;
  size_t ptr = 0;
  while (w1 < T1) {
    while (ptr < order.size() && visited[order[ptr].second]) ++ptr;
    if (ptr == order.size()) break;
    std::deque<uint32_t> q;
    visited[order[ptr].second] = 1;
    q.push_back(order[ptr].second);
    while (!q.empty() && w1 < T1) {
      uint32_t v = q.front();
      q.pop_front();
      if (w1 + g.nw[v] > T1) continue;  // does not fit: stays in part 2, not expanded
      part1[v] = 1;
      w1 += g.nw[v];
      for (uint64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
        uint32_t x = g.adj[e];
        if (inset[x] == my && !visited[x]) {
          visited[x] = 1;
          q.push_back(x);
        }
      }
    }
  }
  std::vector<uint32_t> S1, S2;
  for (uint32_t v : S) (part1[v] ? S1 : S2).push_back(v);
  bisect(g, S1, k1, off, seed, level, block, inset, stamp);
  bisect(g, S2, kS - k1, off + k1, seed, level, block, inset, stamp);
}

std::vector<uint32_t> initial_partition(const Graph& g, uint32_t k, uint64_t seed, uint64_t level) {
  std::vector<uint32_t> block(g.n, 0), inset(g.n, 0), S(g.n);
  for (uint64_t v = 0; v < g.n; ++v) S[v] = (uint32_t)v;
  uint32_t stamp = 0;
  bisect(g, S, k, 0, seed, level, block, inset, stamp);
  return block;
}

// ------------------------------------------------------------- refinement --
// Sec. 3: in uncoarsening, LP starts from the projected partition, labels are
// blocks and the size constraint is L_max.  Same rule as clustering with its
// own hash tags, R_r rounds, no node-reduction stop and no 2-hop step.
uint64_t refine(const Graph& g, std::vector<uint32_t>& block, uint32_t k, int64_t lmax,
                uint64_t seed, uint64_t level, const or_params& p) {
  std::vector<int64_t> BW(k, 0);
  for (uint64_t u = 0; u < g.n; ++u) BW[block[u]] += g.nw[u];
  LpSetup cfg{seed, TAG_RSUB, TAG_RTIE, TAG_RADM, level, lmax, p.ref_rounds, p.subrounds,
              false, p.shrink_num, p.shrink_den};
  uint64_t moves = 0;
  label_propagation(g, block, BW, cfg, &moves);
  return moves;
}

// L_max = (1 + eps) * ceil(c(V)/k), Sec. 2; floored, evaluated in binary64.
int64_t balance_limit(int64_t cV, uint32_t k, double eps) {
  int64_t avg = (cV + (int64_t)k - 1) / (int64_t)k;
  return (int64_t)std::floor((1.0 + eps) * (double)avg);
}

// cut(Pi) = sum over i<j of omega(E_ij), Sec. 2.
void evaluate(const Graph& g, const std::vector<uint32_t>& block, uint32_t k, int64_t* cut,
              int64_t* maxbw) {
  int64_t c = 0;
#pragma omp parallel for num_threads(g_threads) reduction(+ : c)
  for (uint64_t u = 0; u < g.n; ++u)
    for (uint64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
      if (u < g.adj[e] && block[u] != block[g.adj[e]]) c += g.ew[e];
  std::vector<int64_t> BW(k, 0);
  for (uint64_t u = 0; u < g.n; ++u) BW[block[u]] += g.nw[u];
  *cut = c;
  *maxbw = k ? *std::max_element(BW.begin(), BW.end()) : 0;
}

struct Handle {
  Graph g;
  Hierarchy h;
};

}  // namespace

// =========================================================== C interface ===
extern "C" {

// Threads of the parallel steps (1 = single-threaded, the default); returns
// the number in effect (1 when built without OpenMP).
int or_set_threads(int threads) {
#ifdef _OPENMP
  g_threads = threads < 1 ? 1 : threads;
#else
  (void)threads;
  g_threads = 1;
#endif
  return g_threads;
}

uint64_t or_hash(uint64_t seed, uint64_t tag, uint32_t nx, const uint64_t* xs) {
  uint64_t s = mix(seed);
  s = mix(s ^ tag);
  for (uint32_t i = 0; i < nx; ++i) s = mix(s ^ xs[i]);
  return s;
}

uint64_t or_mix(uint64_t z) { return mix(z); }


void or_default_params(or_params* p) { default_params(p); }

// Graph handles --------------------------------------------------------------
void* or_graph_new(const or_graph* v) {
  Handle* h = new Handle();
  h->g = from_view(v);
  return h;
}
void or_free(void* h) { delete (Handle*)h; }
uint64_t or_g_n(void* h) { return ((Handle*)h)->g.n; }
uint64_t or_g_nnz(void* h) { return ((Handle*)h)->g.adj.size(); }
void or_g_copy(void* hp, uint64_t* xadj, uint32_t* adj, int64_t* vwgt, int64_t* adjwgt) {
  const Graph& g = ((Handle*)hp)->g;
  std::memcpy(xadj, g.xadj.data(), (g.n + 1) * sizeof(uint64_t));
  std::memcpy(adj, g.adj.data(), g.adj.size() * sizeof(uint32_t));
  if (vwgt) std::memcpy(vwgt, g.nw.data(), g.n * sizeof(int64_t));
  if (adjwgt) std::memcpy(adjwgt, g.ew.data(), g.ew.size() * sizeof(int64_t));
}

// One LP clustering + 2-hop step on a graph (level index `level`).
// label_out[n]; stats_out = {lp_rounds, nclusters_lp, twohop, nclusters}.
void or_cluster(const or_graph* v, int64_t U, uint64_t seed, uint64_t level, const or_params* p,
                uint32_t* label_out, uint64_t* stats_out) {
  Graph g = from_view(v);
  Step st = cluster_level(g, U, seed, level, *p);
  std::memcpy(label_out, st.label.data(), g.n * sizeof(uint32_t));
  stats_out[0] = st.lp_rounds;
  stats_out[1] = st.nclusters_lp;
  stats_out[2] = st.twohop;
  stats_out[3] = st.nclusters;
}

// LP only (no 2-hop): labels/weights in-out, for step-level tests.
uint32_t or_label_propagation(const or_graph* v, uint32_t* label, int64_t* W, uint64_t nW,
                              int64_t cap, uint64_t seed, uint64_t level, uint32_t refine_tags,
                              uint32_t rounds, uint32_t subrounds, uint32_t shrink_stop,
                              uint64_t* moves) {
  Graph g = from_view(v);
  std::vector<uint32_t> lab(label, label + g.n);
  std::vector<int64_t> w(W, W + nW);
  LpSetup cfg{seed,
              refine_tags ? (uint64_t)TAG_RSUB : (uint64_t)TAG_SUB,
              refine_tags ? (uint64_t)TAG_RTIE : (uint64_t)TAG_TIE,
              refine_tags ? (uint64_t)TAG_RADM : (uint64_t)TAG_ADM,
              level, cap, rounds, subrounds, shrink_stop != 0, 5, 2};
  uint32_t r = label_propagation(g, lab, w, cfg, moves);
  std::memcpy(label, lab.data(), g.n * sizeof(uint32_t));
  std::memcpy(W, w.data(), nW * sizeof(int64_t));
  return r;
}

// (Weighted) Forest Fire scores of every entry of a graph (canonical rows);
// stats_out = {fires run, burns}.
void or_fire_scores(const or_graph* v, uint64_t seed, uint64_t level, uint32_t weighted,
                    uint32_t p_num, uint32_t p_den, uint32_t nu_num, uint32_t nu_den,
                    int64_t* scores_out, uint64_t* stats_out) {
  Graph g = from_view(v);
  or_params p;
  default_params(&p);
  p.ff_p_num = p_num, p.ff_p_den = p_den, p.ff_nu_num = nu_num, p.ff_nu_den = nu_den;
  FireStats fs;
  std::vector<int64_t> sc = fire_scores(g, seed, level, weighted != 0, p, &fs);
  std::memcpy(scores_out, sc.data(), sc.size() * sizeof(int64_t));
  stats_out[0] = fs.fires;
  stats_out[1] = fs.burns;
}

// Contract a clustering; returns a graph handle, map_out[n].
void* or_contract(const or_graph* v, const uint32_t* label, uint32_t* map_out) {
  Graph g = from_view(v);
  std::vector<uint32_t> lab(label, label + g.n), map;
  Handle* h = new Handle();
  h->g = contract(g, lab, map);
  std::memcpy(map_out, map.data(), g.n * sizeof(uint32_t));
  return h;
}

uint64_t or_edge_budget(uint64_t m, uint64_t n, uint64_t n_next, const or_params* p) {
  return edge_budget(m, n, n_next, *p);
}
int or_budget_triggers(uint64_t m_prime, uint64_t m_hat, const or_params* p) {
  return budget_triggers(m_prime, m_hat, *p) ? 1 : 0;
}

// Sparsify to m_hat with the given sampler (0, 1, 3, or 4 / 5 for the
// (Weighted) Forest Fire scores under p's fire parameters, defaults when p
// is NULL); stats_out = {w_t, n_gt, n_eq} (zeros for uniform sampling).
void* or_sparsify(const or_graph* v, uint64_t m_hat, uint64_t seed, uint64_t level,
                  uint32_t sampler, const or_params* p, int64_t* stats_out) {
  Graph g = from_view(v);
  SparsStats s;
  Handle* h = new Handle();
  h->g = sparsify(g, m_hat, seed, level, sampler, &s, p);
  stats_out[0] = s.w_t;
  stats_out[1] = (int64_t)s.n_gt;
  stats_out[2] = (int64_t)s.n_eq;
  return h;
}

// Hierarchy ------------------------------------------------------------------
void* or_coarsen(const or_graph* v, uint32_t k, uint64_t seed, const or_params* p) {
  Handle* h = new Handle();
  h->g = from_view(v);
  h->h = coarsen(h->g, k, seed, *p);
  return h;
}
uint32_t or_h_levels(void* hp) { return (uint32_t)((Handle*)hp)->h.levels.size(); }
void or_h_info(void* hp, uint32_t lvl, or_level_info* out) { *out = ((Handle*)hp)->h.info[lvl]; }
uint64_t or_h_n(void* hp, uint32_t lvl) { return ((Handle*)hp)->h.levels[lvl].n; }
uint64_t or_h_nnz(void* hp, uint32_t lvl) { return ((Handle*)hp)->h.levels[lvl].adj.size(); }
// lvl is 0-based; map (for lvl < levels-1) gives the node of level lvl+1.
void or_h_copy(void* hp, uint32_t lvl, uint64_t* xadj, uint32_t* adj, int64_t* vwgt,
               int64_t* adjwgt, uint32_t* map) {
  Handle* h = (Handle*)hp;
  const Graph& g = h->h.levels[lvl];
  std::memcpy(xadj, g.xadj.data(), (g.n + 1) * sizeof(uint64_t));
  std::memcpy(adj, g.adj.data(), g.adj.size() * sizeof(uint32_t));
  if (vwgt) std::memcpy(vwgt, g.nw.data(), g.n * sizeof(int64_t));
  if (adjwgt) std::memcpy(adjwgt, g.ew.data(), g.ew.size() * sizeof(int64_t));
  if (map && lvl + 1 < h->h.levels.size())
    std::memcpy(map, h->h.maps[lvl].data(), g.n * sizeof(uint32_t));
}

void or_initial_partition(const or_graph* v, uint32_t k, uint64_t seed, uint64_t level,
                          uint32_t* block_out) {
  Graph g = from_view(v);
  std::vector<uint32_t> b = initial_partition(g, k, seed, level);
  std::memcpy(block_out, b.data(), g.n * sizeof(uint32_t));
}

uint64_t or_refine(const or_graph* v, uint32_t* block, uint32_t k, int64_t lmax, uint64_t seed,
                   uint64_t level, const or_params* p) {
  Graph g = from_view(v);
  std::vector<uint32_t> b(block, block + g.n);
  uint64_t moves = refine(g, b, k, lmax, seed, level, *p);
  std::memcpy(block, b.data(), g.n * sizeof(uint32_t));
  return moves;
}

int64_t or_balance_limit(int64_t cV, uint32_t k, double eps) { return balance_limit(cV, k, eps); }

void or_evaluate(const or_graph* v, const uint32_t* block, uint32_t k, int64_t* cut,
                 int64_t* maxbw) {
  Graph g = from_view(v);
  std::vector<uint32_t> b(block, block + g.n);
  evaluate(g, b, k, cut, maxbw);
}

// Full partition: coarsen, initial partitioning on G_l, then refine and
// project level by level.  Phase times (ns) in times_out[3] =
// {coarsen, initial, refine} when non-NULL.
void or_partition(const or_graph* v, uint32_t k, double eps, uint64_t seed, const or_params* p,
                  uint32_t* block_out, or_result* res, int64_t* times_out);

}  // extern "C"

#include <chrono>

extern "C" void or_partition(const or_graph* v, uint32_t k, double eps, uint64_t seed,
                             const or_params* p, uint32_t* block_out, or_result* res,
                             int64_t* times_out) {
  using clk = std::chrono::steady_clock;
  Graph g1 = from_view(v);
  auto t0 = clk::now();
  Hierarchy h = coarsen(g1, k, seed, *p);
  auto t1 = clk::now();
  const uint32_t L = (uint32_t)h.levels.size();
  const int64_t lmax = balance_limit(g1.total_weight(), k, eps);
  std::vector<uint32_t> block = initial_partition(h.levels[L - 1], k, seed, L);
  auto t2 = clk::now();
  for (uint32_t i = L; i >= 1; --i) {
    const Graph& gi = h.levels[i - 1];
    refine(gi, block, k, lmax, seed, i, *p);
    if (i > 1) {
      const std::vector<uint32_t>& map = h.maps[i - 2];
      std::vector<uint32_t> fine(h.levels[i - 2].n);
      for (uint64_t u = 0; u < fine.size(); ++u) fine[u] = block[map[u]];
      block.swap(fine);
    }
  }
  auto t3 = clk::now();
  std::memcpy(block_out, block.data(), g1.n * sizeof(uint32_t));
  evaluate(g1, block, k, &res->cut, &res->max_block_weight);
  res->lmax = lmax;
  res->levels = L;
  if (times_out) {
    times_out[0] = std::chrono::duration_cast<std::chrono::nanoseconds>(t1 - t0).count();
    times_out[1] = std::chrono::duration_cast<std::chrono::nanoseconds>(t2 - t1).count();
    times_out[2] = std::chrono::duration_cast<std::chrono::nanoseconds>(t3 - t2).count();
  }
}
