// Size-constrained label propagation on the GPU: rating, sub-round bucketing
// and capacity admission.  Used for clustering (labels = clusters, cap = U),
// for the favourite clusters of 2-hop clustering and for refinement
// (labels = blocks, cap = L_max).
//
// Rule (Sec. 3 and Sec. 4.1, with the synchronous reading): in a sub-round
// every active node u rates the labels of its neighbours,
// r(K) = sum of omega(u,v) over neighbours v with label K, and proposes the
// best K != label(u) with W(K) + c(u) <= cap (ties: smaller
// H(TIE, level, round, u, K), then smaller K) if r(K) > r(label(u)).
// Per target the proposals are ordered by (gain desc, hi32 H(ADM, level,
// round, u) asc, u asc) and the longest prefix that fits cap - W_start(K) is
// admitted; all admitted moves are applied together.
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>

#include <hip/hip_ext.h>

#include "kernels.h"
#include "profiler.h"

namespace lmgp {

namespace {

struct Best {
  int64_t r;
  uint64_t h;
  uint32_t K;
};

LMGP_D bool better(int64_t ar, uint64_t ah, uint32_t aK, const Best& b) {
  if (ar != b.r) return ar > b.r;
  if (ah != b.h) return ah < b.h;
  return aK < b.K;
}

template <int WIDTH>
LMGP_D void reduce_best(Best& b, int64_t& r_own) {
#pragma unroll
  for (int d = WIDTH / 2; d > 0; d >>= 1) {
    int64_t orr = __shfl_xor(b.r, d, WIDTH);
    uint64_t oh = __shfl_xor(b.h, d, WIDTH);
    uint32_t oK = __shfl_xor(b.K, d, WIDTH);
    int64_t oo = __shfl_xor(r_own, d, WIDTH);
    if (better(orr, oh, oK, b)) b = Best{orr, oh, oK};
    r_own = oo > r_own ? oo : r_own;
  }
}

// Lane groups of at most 16 lanes reduce with DPP moves inside a 16-lane row
// instead of LDS-routed shuffles.  Stage s pairs each lane with a partner in
// the other half of its 2^(s+1)-lane block: stages 0 and 1 are the quad
// permutes i^1 and i^2, stage 2 the half-row mirror (i <-> 7 - i), stage 3 the
// row mirror (i <-> 15 - i).  The halves agree after the earlier stages, so
// after stages 0 .. log2(G) - 1 of an all-reduce (an associative, commutative
// operation) every lane of an aligned G-lane group holds the group's result.
// Every lane of the wave must take part.
template <int S>
LMGP_D uint32_t dpp_partner(uint32_t v) {
  constexpr int ctrl = S == 0 ? 0xB1 : S == 1 ? 0x4E : S == 2 ? 0x141 : 0x140;
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xF, 0xF, false);
}
template <int S>
LMGP_D uint64_t dpp_partner64(uint64_t v) {
  return (uint64_t)dpp_partner<S>((uint32_t)v) | ((uint64_t)dpp_partner<S>((uint32_t)(v >> 32)) << 32);
}

template <int S, int G>
LMGP_D void dpp_best_stage(Best& b, bool r32) {
  if constexpr ((1 << S) < G) {
    const int64_t orr = r32 ? (int64_t)dpp_partner<S>((uint32_t)b.r)
                            : (int64_t)dpp_partner64<S>((uint64_t)b.r);
    const uint64_t oh = dpp_partner64<S>(b.h);
    const uint32_t oK = dpp_partner<S>(b.K);
    if (better(orr, oh, oK, b)) b = Best{orr, oh, oK};
  }
}

// As reduce_best for a group whose own-label rating is already known to every
// lane; with r32 (every rating below 2^32) the ratings cross lanes as 32-bit
// words.
template <int WIDTH>
LMGP_D void reduce_best_only(Best& b, bool r32) {
  if constexpr (WIDTH <= 16) {
    dpp_best_stage<0, WIDTH>(b, r32);
    dpp_best_stage<1, WIDTH>(b, r32);
    dpp_best_stage<2, WIDTH>(b, r32);
    dpp_best_stage<3, WIDTH>(b, r32);
    return;
  }
#pragma unroll
  for (int d = WIDTH / 2; d > 0; d >>= 1) {
    const int64_t orr = r32 ? (int64_t)(uint32_t)__shfl_xor((uint32_t)b.r, d, WIDTH)
                            : __shfl_xor(b.r, d, WIDTH);
    const uint64_t oh = __shfl_xor(b.h, d, WIDTH);
    const uint32_t oK = __shfl_xor(b.K, d, WIDTH);
    if (better(orr, oh, oK, b)) b = Best{orr, oh, oK};
  }
}

// Consider table slot (K, r) for node u.
LMGP_D void consider(const RateArgs& a, uint32_t K, int64_t r, uint32_t own, int64_t cu,
                     int64_t cap, uint64_t pre_u, uint64_t label_base, Best& best,
                     int64_t& r_own) {
  if (K == own) {
    r_own = r;
    return;
  }
  if (a.mode == MODE_LP && a.W[K] + cu > cap) return;
  if (r < best.r) return;
  uint64_t h = hash_add(pre_u, (uint64_t)K - label_base);
  if (better(r, h, K, best)) best = Best{r, h, K};
}

// As consider, with W[K] already loaded by the caller (wk; unused for the own
// label and in MODE_FAV), so that a thread can issue its W gathers together.
LMGP_D void consider_w(const RateArgs& a, uint32_t K, int64_t r, uint32_t own, int64_t cu,
                       int64_t cap, int64_t wk, uint64_t pre_u, uint64_t label_base, Best& best,
                       int64_t& r_own) {
  if (K == own) {
    r_own = r;
    return;
  }
  if (a.mode == MODE_LP && wk + cu > cap) return;
  if (r < best.r) return;
  uint64_t h = hash_add(pre_u, (uint64_t)K - label_base);
  if (better(r, h, K, best)) best = Best{r, h, K};
}

// Candidate slots are dense: the node at position idx of the rated list owns
// slot idx and marks it empty (tgt = EMPTY_KEY) when it proposes no move, so
// that no global counter is needed.
LMGP_D void no_cand(const RateArgs& a, uint32_t idx) {
  if (a.mode == MODE_LP) a.cands[idx].tgt = EMPTY_KEY;
}

LMGP_D void emit(const RateArgs& a, uint32_t idx, uint32_t u, const GraphDesc& gd,
                 const Best& best, int64_t r_own, int64_t cu) {
  if (a.mode == MODE_FAV) {
    a.fav[u] = best.r > 0 ? best.K : EMPTY_KEY;
    return;
  }
  if (!(best.r > r_own)) {
    a.cands[idx].tgt = EMPTY_KEY;
  } else {
    const uint32_t i = idx;
    Cand c;
    c.u = u;
    c.tgt = best.K;
    c.gain = best.r - r_own;
    a.cands[i] = c;
    if (!a.few && !a.trial) {
      atomicAdd((unsigned long long*)&a.tally[best.K].demand, (unsigned long long)cu);
      atomicAdd(&a.tally[best.K].ntgt, 1u);
    }
  }
}

// Open addressing with linear probing.  The probe loop has a single exit
// (the slot holding K, claimed or found) and the add follows it, so that a
// wave's divergent probes cost few scalar mask updates per step.
template <int T>
LMGP_D void lds_insert(uint32_t* key, unsigned long long* val, uint32_t K, uint64_t w) {
  constexpr int LOGT = __builtin_ctz(T);
  uint32_t s = (K * 0x9E3779B1u) >> (32 - LOGT);
  bool hit;
  do {
    const uint32_t prev = atomicCAS(&key[s], EMPTY_KEY, K);
    hit = prev == EMPTY_KEY || prev == K;
    s = hit ? s : (s + 1) & (T - 1);
  } while (!hit);
  atomicAdd(&val[s], (unsigned long long)w);
}

// Table of 2^logt slots (logt >= 1): runtime-sized variant.
LMGP_D void lds_insert_n(uint32_t* key, unsigned long long* val, uint32_t K, uint64_t w,
                         int logt) {
  const uint32_t mask = (1u << logt) - 1;
  uint32_t s = (K * 0x9E3779B1u) >> (32 - logt);
  bool hit;
  do {
    const uint32_t prev = atomicCAS(&key[s], EMPTY_KEY, K);
    hit = prev == EMPTY_KEY || prev == K;
    s = hit ? s : (s + 1) & mask;
  } while (!hit);
  atomicAdd(&val[s], (unsigned long long)w);
}

template <int G>
LMGP_D int64_t group_sum(int64_t v) {
  if constexpr (G <= 16) {
    if constexpr (G > 1) v += (int64_t)dpp_partner64<0>((uint64_t)v);
    if constexpr (G > 2) v += (int64_t)dpp_partner64<1>((uint64_t)v);
    if constexpr (G > 4) v += (int64_t)dpp_partner64<2>((uint64_t)v);
    if constexpr (G > 8) v += (int64_t)dpp_partner64<3>((uint64_t)v);
    return v;
  }
#pragma unroll
  for (int d = G / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, G);
  return v;
}

// Lane groups of G lanes (G <= 64) rate one node each; degree <= 2G, table 4G.
// Entries whose label is the node's own label are summed in registers and
// inserted once per group: in refinement and in settled clusters most
// neighbours share that label, and their LDS atomics would all hit one slot.
// Every lane-group class uses 1024 LDS slots per 256-thread block (256 / G
// groups of 4G slots), and so do the two smallest block classes (one node
// per block, 512 or 1024 slots): all eight share one launch (k_rate_groups).
constexpr int GROUP_SLOTS = 1024;

// Label of a neighbour (the byte copy when the labels fit in one).
LMGP_D uint32_t nbr_label(const RateArgs& a, uint32_t v) {
  return a.label8 ? (uint32_t)a.label8[v] : a.label[v];
}

// Planned launch: node count and list range from the sub-round's plan.
LMGP_D void resolve_plan(RateArgs& r) {
  if (!r.plan) return;
  const SubPlan& p = *r.plan;
  uint32_t cnt = 0;
  for (int c = r.plan_c0; c <= r.plan_c1; ++c) cnt += p.cnt[c];
  r.count = cnt;
  r.list = r.list + p.lbase + p.off[r.plan_c0];
  if (r.cands) r.cands = r.cands + p.off[r.plan_c0];
}

// The best of a lane group's eligible slots (el: label, rating), as the
// lexicographic order of `better` picks it: the group's highest rating
// first, then the smallest (tie hash, label) among the slots that reach it.
// Only those slots hash their label (a slot below the maximum cannot win,
// whatever its hash).  {0, 0, 0} when no slot is eligible.  Every lane of the
// wave takes part (shuffles).
template <int G, int SPL>
LMGP_D Best group_best(const bool* el, const uint32_t* Ks, const int64_t* rs, uint64_t pre_u,
                       uint64_t label_base, bool r32) {
  int64_t rm = 0;
#pragma unroll
  for (int j = 0; j < SPL; ++j) rm = el[j] && rs[j] > rm ? rs[j] : rm;
  if constexpr (G <= 16) {
    auto stage = [&](auto sc) {
      constexpr int S = decltype(sc)::value;
      if constexpr ((1 << S) < G) {
        const int64_t o = r32 ? (int64_t)dpp_partner<S>((uint32_t)rm)
                              : (int64_t)dpp_partner64<S>((uint64_t)rm);
        rm = o > rm ? o : rm;
      }
    };
    stage(std::integral_constant<int, 0>());
    stage(std::integral_constant<int, 1>());
    stage(std::integral_constant<int, 2>());
    stage(std::integral_constant<int, 3>());
  } else {
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) {
      const int64_t o =
          r32 ? (int64_t)(uint32_t)__shfl_xor((uint32_t)rm, d, G) : __shfl_xor(rm, d, G);
      rm = o > rm ? o : rm;
    }
  }
  Best b{0, 0, 0};
#pragma unroll
  for (int j = 0; j < SPL; ++j) {
    if (el[j] && rs[j] == rm) {
      const uint64_t h = hash_add(pre_u, (uint64_t)Ks[j] - label_base);
      if (b.r == 0 || h < b.h || (h == b.h && Ks[j] < b.K)) b = Best{rm, h, Ks[j]};
    }
  }
  reduce_best_only<G>(b, r32);
  return b;
}

// Graph of node u; ONE: a single graph (index 0), so that its descriptor is
// read with scalar loads.
template <bool ONE>
LMGP_D uint32_t graph_at(const uint32_t* gid, uint64_t u) {
  return ONE ? 0u : graph_of(gid, u);
}

template <int G, int EWK, bool ONE>
LMGP_D void rate_group(const RateArgs& a, uint32_t* skey, unsigned long long* sval,
                       uint64_t blk) {
  constexpr int T = 4 * G;
  constexpr int GPB = 256 / G;
  static_assert(GPB * T == GROUP_SLOTS, "group tables fill the block's slots");
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  uint32_t* key = skey + grp * T;
  unsigned long long* val = sval + grp * T;
  const uint64_t idx = blk * GPB + grp;
  bool valid = idx < a.count;
  const uint32_t u = valid ? a.list[idx] : 0u;
  // a graph may stop in the middle of a round (its flag is cleared on the device)
  if (valid && !a.gd[graph_at<ONE>(a.gid, u)].active) valid = false;
#pragma unroll
  for (int s = gl; s < T; s += G) {
    key[s] = EMPTY_KEY;
    val[s] = 0;
  }
  wave_sync();
  uint64_t beg = 0, end = 0;
  uint32_t own = EMPTY_KEY;
  if (valid) {
    beg = a.xadj[u];
    end = a.xadj[u + 1];
    own = a.label[u];
  }
  int64_t acc = 0;
  {
    // degree <= 2G: at most two entries per lane, loads issued together
    // (past the row end the loads repeat the row's first entry, a valid
    // address, and are masked: no branch around them)
    const uint64_t e0 = beg + gl, e1 = e0 + G;
    const uint64_t f0 = e0 < end ? e0 : beg, f1 = e1 < end ? e1 : beg;
    const uint32_t v0 = a.adj[f0], v1 = a.adj[f1];
    const int64_t w0 = edge_w<EWK>(a.ew, f0), w1 = edge_w<EWK>(a.ew, f1);
    const uint32_t l0 = nbr_label(a, v0), l1 = nbr_label(a, v1);
    const uint32_t K0 = e0 < end ? l0 : EMPTY_KEY;
    const uint32_t K1 = e1 < end ? l1 : EMPTY_KEY;
    acc += (K0 != EMPTY_KEY && K0 == own ? w0 : 0) + (K1 != EMPTY_KEY && K1 == own ? w1 : 0);
    if (K0 != EMPTY_KEY && K0 != own) lds_insert<T>(key, val, K0, (uint64_t)w0);
    if (K1 != EMPTY_KEY && K1 != own) lds_insert<T>(key, val, K1, (uint64_t)w1);
  }
  acc = group_sum<G>(acc);
  if (gl == 0 && acc > 0) lds_insert<T>(key, val, own, (uint64_t)acc);
  wave_sync();
  int64_t r_own = 0;
  GraphDesc gd{};
  int64_t cu = 0;
  // Clustering: the best label ignoring the capacity first (a rated node is
  // lighter than the cap, so only the labels' weights can exclude one); if
  // it fits, it is the best of the labels that fit, and the group read one
  // cluster weight instead of one per label (the random gathers that count
  // where labels are scattered).  Otherwise, and in refinement (where the
  // best block is often full), the table is evaluated with every label's
  // weight.
  constexpr int SPL = T / G;  // slots per lane
  uint32_t Ks[SPL];
  int64_t rs[SPL];
  bool el[SPL];
#pragma unroll
  for (int j = 0; j < SPL; ++j) Ks[j] = EMPTY_KEY, rs[j] = 0;
  uint64_t pre_u = 0;
  const bool first = a.mode == MODE_LP && a.phase == 0;
  const bool r32 = a.packed != 0;
  if (valid) {
    gd = a.gd[graph_at<ONE>(a.gid, u)];
    cu = a.nw[u];
    pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      Ks[j] = key[gl + j * G];
      rs[j] = (int64_t)val[gl + j * G];
    }
  }
  Best best{0, 0, 0};
  if (first || a.mode != MODE_LP) {
    const bool fits = valid && (a.mode != MODE_LP || cu <= gd.cap);
#pragma unroll
    for (int j = 0; j < SPL; ++j) el[j] = fits && Ks[j] != EMPTY_KEY && Ks[j] != own;
    best = group_best<G, SPL>(el, Ks, rs, pre_u, gd.label_base, r32);
  }
  // the whole group holds the same best: the check and the evaluation with
  // weights are uniform within it
  const bool redo = valid && a.mode == MODE_LP &&
                    (!first || (best.r > 0 && a.W[best.K] + cu > gd.cap));
  if (__ballot(redo)) {
    int64_t wk[SPL];
#pragma unroll
    for (int j = 0; j < SPL; ++j)
      wk[j] = (redo && Ks[j] != EMPTY_KEY && Ks[j] != own) ? a.W[Ks[j]] : 0;
#pragma unroll
    for (int j = 0; j < SPL; ++j)
      el[j] = redo && Ks[j] != EMPTY_KEY && Ks[j] != own && wk[j] + cu <= gd.cap;
    const Best nb = group_best<G, SPL>(el, Ks, rs, pre_u, gd.label_base, r32);
    if (redo) best = nb;
  }
  r_own = acc;
  if (gl == 0 && idx < a.count) {
    if (valid) emit(a, (uint32_t)idx, u, gd, best, r_own, cu);
    else no_cand(a, (uint32_t)idx);  // graph stopped
  }
}


// One 256-thread block per node of degree <= 2^(LOGT-1), LDS table of 2^LOGT
// slots (load <= 1/2).  Own-label entries are summed in registers.
struct BlockScratch {
  Best sb[NWAVE];
  int64_t so[NWAVE];
  int64_t sm[NWAVE];
};

template <int EWK, int LOGT, bool ONE>
LMGP_D void rate_block(const RateArgs& a, uint32_t* key, unsigned long long* val,
                       BlockScratch& bs, uint64_t idx) {
  constexpr int T = 1 << LOGT;
  constexpr int logt = LOGT;
  Best* sb = bs.sb;
  int64_t* so = bs.so;
  int64_t* sm = bs.sm;
  if (idx >= a.count) return;
  const uint32_t u = a.list[idx];
  if (!a.gd[graph_at<ONE>(a.gid, u)].active) {
    if (threadIdx.x == 0) no_cand(a, (uint32_t)idx);
    return;
  }
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  for (int s = threadIdx.x; s < T; s += 256) {
    key[s] = EMPTY_KEY;
    val[s] = 0;
  }
  __syncthreads();
  const uint32_t own = a.label[u];
  int64_t acc = 0;
  constexpr int U = 8;  // entries per thread whose loads are issued together
  for (uint64_t e0 = beg + threadIdx.x; e0 < end; e0 += (uint64_t)U * 256) {
    uint32_t v[U], K[U];
    int64_t w[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint64_t e = e0 + (uint64_t)j * 256;
      v[j] = e < end ? a.adj[e] : 0u;
      w[j] = e < end ? edge_w<EWK>(a.ew, e) : 0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) K[j] = e0 + (uint64_t)j * 256 < end ? a.label[v[j]] : EMPTY_KEY;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (K[j] == EMPTY_KEY) continue;
      if (K[j] == own) acc += w[j];
      else lds_insert_n(key, val, K[j], (uint64_t)w[j], logt);
    }
  }
  int64_t acc_tot;
  (void)block_exclusive_scan(acc, sm, acc_tot);
  if (threadIdx.x == 0 && acc_tot > 0) lds_insert_n(key, val, own, (uint64_t)acc_tot, logt);
  __syncthreads();
  const GraphDesc gd = a.gd[graph_at<ONE>(a.gid, u)];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  constexpr int SB = 8;  // slots per thread whose W gathers are issued together
  for (int s0 = threadIdx.x; s0 < T; s0 += SB * 256) {
    uint32_t Ks[SB];
    int64_t wk[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) Ks[j] = s0 + j * 256 < T ? key[s0 + j * 256] : EMPTY_KEY;
#pragma unroll
    for (int j = 0; j < SB; ++j)
      wk[j] = (Ks[j] != EMPTY_KEY && Ks[j] != own && a.mode == MODE_LP) ? a.W[Ks[j]] : 0;
#pragma unroll
    for (int j = 0; j < SB; ++j)
      if (Ks[j] != EMPTY_KEY)
        consider_w(a, Ks[j], (int64_t)val[s0 + j * 256], own, cu, gd.cap, wk[j], pre_u,
                   gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sb[w] = best;
    so[w] = r_own;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NWAVE; ++i) {
      if (better(sb[i].r, sb[i].h, sb[i].K, best)) best = sb[i];
      r_own = so[i] > r_own ? so[i] : r_own;
    }
    emit(a, (uint32_t)idx, u, gd, best, r_own, cu);
  }
}

template <int EWK, int LOGT>
__global__ __launch_bounds__(256) void k_rate_block(RateArgs a0) {
  __shared__ uint32_t key[1 << LOGT];
  __shared__ unsigned long long val[1 << LOGT];
  __shared__ BlockScratch bs;
  RateArgs a = a0;
  resolve_plan(a);
  rate_block<EWK, LOGT, false>(a, key, val, bs, blockIdx.x);
}

// The classes 0..7 in one launch: block b belongs to the class c
// with split.bstart[c] <= b < split.bstart[c + 1]; each class has its own
// list range (and candidate slots) at split.off[c].
template <int EWK>
__global__ __launch_bounds__(256) void k_rate_groups(RateArgs a, GroupSplit split) {
  __shared__ uint32_t skey[GROUP_SLOTS];
  __shared__ unsigned long long sval[GROUP_SLOTS];
  __shared__ BlockScratch bs;
  const uint32_t b = blockIdx.x;
  // planned launch: the split comes from the device and the grid is an upper bound
  const GroupSplit& sp = a.plan ? a.plan->gs : split;
  if (b >= sp.bstart[GROUP_CLASSES]) return;
  int c = 0;
#pragma unroll
  for (int q = 1; q < GROUP_CLASSES; ++q)
    if (b >= sp.bstart[q]) c = q;
  RateArgs r = a;
  r.plan = nullptr;
  r.list = a.list + (a.plan ? a.plan->lbase : 0u) + sp.off[c];
  if (a.mode == MODE_LP) r.cands = a.cands + sp.off[c];
  r.count = sp.count[c];
  const uint64_t blk = b - sp.bstart[c];
  // one graph (uniform over the launch): its descriptor at a constant index
  auto classes = [&](auto one) {
    constexpr bool ONE = decltype(one)::value;
    switch (c) {
      case 0: rate_group<2, EWK, ONE>(r, skey, sval, blk); break;
      case 1: rate_group<4, EWK, ONE>(r, skey, sval, blk); break;
      case 2: rate_group<8, EWK, ONE>(r, skey, sval, blk); break;
      case 3: rate_group<16, EWK, ONE>(r, skey, sval, blk); break;
      case 4: rate_group<32, EWK, ONE>(r, skey, sval, blk); break;
      case 5: rate_group<64, EWK, ONE>(r, skey, sval, blk); break;
      case 6: rate_block<EWK, 9, ONE>(r, skey, sval, bs, blk); break;  // whole block per node
      default: rate_block<EWK, 10, ONE>(r, skey, sval, bs, blk); break;
    }
  };
  if (a.gid) classes(std::false_type());
  else classes(std::true_type());
}

constexpr unsigned long long EMPTY_SLOT = ~0ull;  // packed slot: label EMPTY_KEY

// Packed LDS table: label in the high half of a slot, rating in the low half
// (valid when every rating fits in 32 bits).  The compare-and-swap claims an
// empty slot with the first rating or returns the occupant; the loop's only
// exit is the slot of K, and the add for a found slot follows it.
template <int T>
LMGP_D void lds_add_packed(unsigned long long* tab, uint32_t K, unsigned long long w) {
  constexpr int LOGT = __builtin_ctz(T);
  const unsigned long long mine = ((unsigned long long)K << 32) | w;
  uint32_t s = (K * 0x9E3779B1u) >> (32 - LOGT);
  unsigned long long prev;
  bool hit;
  do {
    prev = atomicCAS(&tab[s], EMPTY_SLOT, mine);
    hit = prev == EMPTY_SLOT || (uint32_t)(prev >> 32) == K;
    s = hit ? s : (s + 1) & (T - 1);
  } while (!hit);
  if (prev != EMPTY_SLOT) atomicAdd(&tab[s], w);
}

// Runtime-sized variant of lds_add_packed: 2^logt slots.
LMGP_D void lds_add_packed_n(unsigned long long* tab, uint32_t K, unsigned long long w, int logt) {
  const uint32_t mask = (1u << logt) - 1;
  const unsigned long long mine = ((unsigned long long)K << 32) | w;
  uint32_t s = (K * 0x9E3779B1u) >> (32 - logt);
  unsigned long long prev;
  bool hit;
  do {
    prev = atomicCAS(&tab[s], EMPTY_SLOT, mine);
    hit = prev == EMPTY_SLOT || (uint32_t)(prev >> 32) == K;
    s = hit ? s : (s + 1) & mask;
  } while (!hit);
  if (prev != EMPTY_SLOT) atomicAdd(&tab[s], w);
}

// One block of NT threads per node, packed LDS table of 2^LOGT slots: 8192
// slots for degree <= 6144 (load <= 3/4, two 1024-thread blocks fit a CU),
// 16384 for degree <= 8192; with packed ratings the block classes use it too
// (2048 slots / 256 threads, 4096 slots / 512 threads: half the LDS of a
// key + value table, so twice the nodes in flight per CU).  Own-label entries
// are summed in registers.
template <int EWK, int LOGT, int NT>
__global__ __launch_bounds__(NT) void k_rate_big(RateArgs a0) {
  constexpr int NW = NT / WAVE;
  constexpr int T = 1 << LOGT;
  constexpr int logt = LOGT;
  __shared__ unsigned long long tab[T];
  __shared__ Best sb[NW];
  __shared__ int64_t so[NW];
  __shared__ int64_t sm[NW];
  RateArgs a = a0;
  resolve_plan(a);
  const uint64_t idx = blockIdx.x;
  if (idx >= a.count) return;
  const uint32_t u = a.list[idx];
  if (!a.gd[graph_of(a.gid, u)].active) {
    if (threadIdx.x == 0) no_cand(a, (uint32_t)idx);
    return;
  }
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  for (int s = threadIdx.x; s < T; s += NT) tab[s] = EMPTY_SLOT;
  __syncthreads();
  const uint32_t own = a.label[u];
  int64_t acc = 0;
  constexpr int U = 8;  // entries per thread whose loads are issued together
  // 32-bit offsets into the row (a block-uniform base): the loads take a
  // scalar base and one vector offset
  const uint32_t deg = (uint32_t)(end - beg);
  const uint32_t* arow = a.adj + beg;
  const void* wrow = edge_row<EWK>(a.ew, beg);
  for (uint32_t o0 = threadIdx.x; o0 < deg; o0 += (uint32_t)(U * NT)) {
    uint32_t v[U], K[U];
    int64_t w[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint32_t o = o0 + (uint32_t)(j * NT);
      v[j] = o < deg ? arow[o] : 0u;
      w[j] = o < deg ? edge_w<EWK>(wrow, o) : 0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) K[j] = o0 + (uint32_t)(j * NT) < deg ? a.label[v[j]] : EMPTY_KEY;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (K[j] == EMPTY_KEY) continue;
      if (K[j] == own) acc += w[j];
      else lds_add_packed_n(tab, K[j], (unsigned long long)w[j], logt);
    }
  }
  int64_t acc_tot;
  (void)block_exclusive_scan<int64_t, NW>(acc, sm, acc_tot);
  if (threadIdx.x == 0 && acc_tot > 0) lds_add_packed_n(tab, own, (unsigned long long)acc_tot, logt);
  __syncthreads();
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  constexpr int SB = 8;  // slots per thread whose W gathers are issued together
  for (int s0 = threadIdx.x; s0 < T; s0 += SB * NT) {
    unsigned long long v[SB];
    int64_t wk[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) v[j] = s0 + j * NT < T ? tab[s0 + j * NT] : EMPTY_SLOT;
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      const uint32_t K = (uint32_t)(v[j] >> 32);
      wk[j] = (v[j] != EMPTY_SLOT && K != own && a.mode == MODE_LP) ? a.W[K] : 0;
    }
#pragma unroll
    for (int j = 0; j < SB; ++j)
      if (v[j] != EMPTY_SLOT)
        consider_w(a, (uint32_t)(v[j] >> 32), (int64_t)(v[j] & 0xFFFFFFFFull), own, cu, gd.cap,
                   wk[j], pre_u, gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sb[w] = best;
    so[w] = r_own;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NW; ++i) {
      if (better(sb[i].r, sb[i].h, sb[i].K, best)) best = sb[i];
      r_own = so[i] > r_own ? so[i] : r_own;
    }
    emit(a, (uint32_t)idx, u, gd, best, r_own, cu);
  }
}

// Refinement with few labels (blocks, at most FEW_LABELS): nodes of the block
// and big-block classes rate into a dense LDS row indexed by the label, with
// no hashing and no probing; NT threads per node.
// P: ratings fit in 32 bits (RateArgs.packed), the row holds 32-bit counters.
template <bool P>
using RowCount = typename std::conditional<P, uint32_t, unsigned long long>::type;

template <int EWK, int NT, bool P>
__global__ __launch_bounds__(NT) void k_rate_dense(RateArgs a0) {
  constexpr int NW = NT / WAVE;
  using CT = RowCount<P>;
  __shared__ CT tab[FEW_LABELS];
  __shared__ Best sb[NW];
  __shared__ int64_t so[NW];
  __shared__ int64_t sm[NW];
  RateArgs a = a0;
  resolve_plan(a);
  const uint64_t idx = blockIdx.x;
  if (idx >= a.count) return;
  const uint32_t u = a.list[idx];
  if (!a.gd[graph_of(a.gid, u)].active) {
    if (threadIdx.x == 0) no_cand(a, (uint32_t)idx);
    return;
  }
  const uint32_t few = a.few;
  for (uint32_t t = threadIdx.x; t < few; t += NT) tab[t] = 0;
  __syncthreads();
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  const uint32_t own = a.label[u];
  int64_t acc = 0;
  constexpr int U = 8;
  const uint32_t deg = (uint32_t)(end - beg);
  const uint32_t* arow = a.adj + beg;
  const void* wrow = edge_row<EWK>(a.ew, beg);
  for (uint32_t o0 = threadIdx.x; o0 < deg; o0 += (uint32_t)(U * NT)) {
    uint32_t v[U], K[U];
    int64_t w[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint32_t o = o0 + (uint32_t)(j * NT);
      v[j] = o < deg ? arow[o] : 0u;
      w[j] = o < deg ? edge_w<EWK>(wrow, o) : 0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) K[j] = o0 + (uint32_t)(j * NT) < deg ? a.label[v[j]] : EMPTY_KEY;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (K[j] == EMPTY_KEY) continue;
      if (K[j] == own) acc += w[j];
      else atomicAdd(&tab[K[j]], (CT)w[j]);
    }
  }
  int64_t acc_tot;
  (void)block_exclusive_scan<int64_t, NW>(acc, sm, acc_tot);
  if (threadIdx.x == 0) tab[own] += (CT)acc_tot;
  __syncthreads();
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (uint32_t t = threadIdx.x; t < few; t += NT) {
    const int64_t r = (int64_t)tab[t];
    if (r == 0) continue;  // not adjacent (edge weights are positive)
    const int64_t wk = t != own ? a.W[t] : 0;
    consider_w(a, t, r, own, cu, gd.cap, wk, pre_u, gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  const int wv = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sb[wv] = best;
    so[wv] = r_own;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NW; ++q) {
      if (better(sb[q].r, sb[q].h, sb[q].K, best)) best = sb[q];
      r_own = so[q] > r_own ? so[q] : r_own;
    }
    emit(a, (uint32_t)idx, u, gd, best, r_own, cu);
  }
}

// Refinement with few labels, one wavefront per node (the two smallest
// dense classes): each wave rates its node into a dense LDS row of its own,
// so no wave waits at a block barrier and one node's evaluation overlaps the
// other waves' loads.  RW_WAVES rows of `few` counters per block, in
// dynamic LDS.
template <int EWK, bool P>
__global__ __launch_bounds__(RW_WAVES * WAVE) void k_rate_rows(RateArgs a0) {
  using CT = RowCount<P>;
  extern __shared__ __align__(8) unsigned char rw_raw[];
  CT* rw_tab = reinterpret_cast<CT*>(rw_raw);
  RateArgs a = a0;
  resolve_plan(a);
  const int wv = threadIdx.x / WAVE, ln = lane_id();
  const uint64_t idx = (uint64_t)blockIdx.x * RW_WAVES + wv;
  if (idx >= a.count) return;  // whole waves leave: nothing below waits on the block
  const uint32_t u = a.list[idx];
  const uint32_t g = graph_of(a.gid, u);
  if (!a.gd[g].active) {
    if (ln == 0) no_cand(a, (uint32_t)idx);
    return;
  }
  const uint32_t few = a.few;
  CT* tab = rw_tab + (size_t)wv * few;
  for (uint32_t t = ln; t < few; t += WAVE) tab[t] = 0;
  wave_sync();
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  const uint32_t own = a.label[u];
  int64_t acc = 0;
  constexpr int U = 8;
  for (uint64_t e0 = beg + ln; e0 < end; e0 += (uint64_t)U * WAVE) {
    uint32_t v[U], K[U];
    int64_t w[U];
    // past the row end the loads repeat the row's first entry (these rows are
    // never empty) and are masked below
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint64_t e = e0 + (uint64_t)j * WAVE;
      const uint64_t f = e < end ? e : beg;
      v[j] = a.adj[f];
      w[j] = edge_w<EWK>(a.ew, f);
    }
#pragma unroll
    for (int j = 0; j < U; ++j) K[j] = a.label[v[j]];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (e0 + (uint64_t)j * WAVE >= end) continue;
      if (K[j] == own) acc += w[j];
      else atomicAdd(&tab[K[j]], (CT)w[j]);
    }
  }
  acc = group_sum<WAVE>(acc);
  if (ln == 0 && acc > 0) atomicAdd(&tab[own], (CT)acc);
  wave_sync();
  const GraphDesc gd = a.gd[g];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (uint32_t t = ln; t < few; t += WAVE) {
    const int64_t r = (int64_t)tab[t];
    if (r == 0) continue;  // not adjacent (edge weights are positive)
    const int64_t wk = t != own ? a.W[t] : 0;
    consider_w(a, t, r, own, cu, gd.cap, wk, pre_u, gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  if (ln == 0) emit(a, (uint32_t)idx, u, gd, best, r_own, cu);
}

// ------------------------------------------------- hub nodes (degree > 2048) --
// A hub's rating table lives in global memory; its adjacency is split into
// chunks of HUB_CHUNK entries rated by separate blocks, and its table into
// chunks of HUB_SLOTS slots evaluated by separate blocks, so that a few hubs
// still spread over the whole GPU.
constexpr int HUB_CHUNK = 2048;
constexpr int HUB_SLOTS = 4096;

struct HubArgs {
  RateArgs a;
  const uint64_t* toff;  // table offset of hub i (c + 1 entries)
  const uint64_t* coff;  // first insert chunk of hub i
  const uint64_t* soff;  // first slot chunk of hub i
  uint64_t slots;        // total table slots
  struct Partial* part;  // one per slot chunk
};

struct Partial {
  int64_t r;
  uint64_t h;
  uint32_t K;
  uint32_t pad;
  int64_t r_own;
};

LMGP_D uint32_t find_hub(const uint64_t* off, uint32_t c, uint64_t b) {
  uint32_t lo = 0, hi = c;  // off[lo] <= b < off[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

LMGP_D bool hub_active(const RateArgs& a, uint32_t u) {
  return a.gd[graph_of(a.gid, u)].active;
}

__global__ void k_hub_clear(HubArgs h) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < h.slots; i += stride) {
    if (h.a.packed) {
      h.a.gtab[i] = EMPTY_SLOT;
    } else {
      h.a.gkeys[i] = EMPTY_KEY;
      h.a.gvals[i] = 0;
    }
  }
}

// Add w to label K of a global table of T slots (T a power of two).
LMGP_D void hub_add(const RateArgs& a, uint64_t base, uint64_t T, uint32_t K,
                    unsigned long long w) {
  uint64_t s = ((uint64_t)K * 0x9E3779B97F4A7C15ull) & (T - 1);
  if (a.packed) {
    // one 64-bit word per slot: label in the high half, rating in the low half
    unsigned long long* tab = a.gtab + base;
    while (true) {
      unsigned long long cur = tab[s];
      if (cur == EMPTY_SLOT) {
        cur = atomicCAS(&tab[s], EMPTY_SLOT, ((unsigned long long)K << 32) | w);
        if (cur == EMPTY_SLOT) return;
      }
      if ((uint32_t)(cur >> 32) == K) {
        atomicAdd(&tab[s], w);
        return;
      }
      s = (s + 1) & (T - 1);
    }
  }
  uint32_t* key = a.gkeys + base;
  unsigned long long* val = (unsigned long long*)(a.gvals + base);
  while (true) {
    const uint32_t prev = atomicCAS(&key[s], EMPTY_KEY, K);
    if (prev == EMPTY_KEY || prev == K) {
      atomicAdd(&val[s], w);
      return;
    }
    s = (s + 1) & (T - 1);
  }
}

// Each block sums its chunk per label in LDS first, then adds the distinct
// labels to the hub's global table (neighbours of a coarse hub share few
// labels, so this removes most same-address global atomics).
template <int EWK>
__global__ __launch_bounds__(256) void k_hub_insert(HubArgs h) {
  constexpr int LT = 2 * HUB_CHUNK;
  __shared__ uint32_t lk[LT];
  __shared__ unsigned long long lv[LT];
  const RateArgs& a = h.a;
  const uint32_t i = find_hub(h.coff, a.count, blockIdx.x);
  const uint32_t u = a.list[i];
  if (!hub_active(a, u)) return;
  for (int s = threadIdx.x; s < LT; s += 256) {
    lk[s] = EMPTY_KEY;
    lv[s] = 0;
  }
  __syncthreads();
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  const uint64_t c0 = beg + (uint64_t)(blockIdx.x - h.coff[i]) * HUB_CHUNK;
  const uint64_t c1 = c0 + HUB_CHUNK < end ? c0 + HUB_CHUNK : end;
  for (uint64_t e = c0 + threadIdx.x; e < c1; e += 256)
    lds_insert<LT>(lk, lv, a.label[a.adj[e]], (uint64_t)edge_w<EWK>(a.ew, e));
  __syncthreads();
  const uint64_t T = h.toff[i + 1] - h.toff[i];
  for (int ls = threadIdx.x; ls < LT; ls += 256) {
    const uint32_t K = lk[ls];
    if (K != EMPTY_KEY) hub_add(a, h.toff[i], T, K, lv[ls]);
  }
}

__global__ __launch_bounds__(256) void k_hub_eval(HubArgs h) {
  __shared__ Best sb[NWAVE];
  __shared__ int64_t so[NWAVE];
  const RateArgs& a = h.a;
  const uint32_t i = find_hub(h.soff, a.count, blockIdx.x);
  const uint32_t u = a.list[i];
  if (!hub_active(a, u)) return;
  const uint64_t T = h.toff[i + 1] - h.toff[i];
  const uint32_t* key = a.gkeys + h.toff[i];
  const unsigned long long* val = (const unsigned long long*)(a.gvals + h.toff[i]);
  const unsigned long long* tab = a.gtab + h.toff[i];
  const uint64_t s0 = (uint64_t)(blockIdx.x - h.soff[i]) * HUB_SLOTS;
  const uint64_t s1 = s0 + HUB_SLOTS < T ? s0 + HUB_SLOTS : T;
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const uint32_t own = a.label[u];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (uint64_t s = s0 + threadIdx.x; s < s1; s += 256) {
    uint32_t K;
    int64_t r;
    if (a.packed) {
      const unsigned long long v = tab[s];
      K = (uint32_t)(v >> 32);
      r = (int64_t)(v & 0xFFFFFFFFull);
    } else {
      K = key[s];
      r = (int64_t)val[s];
    }
    if (K != EMPTY_KEY) consider(a, K, r, own, cu, gd.cap, pre_u, gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sb[w] = best;
    so[w] = r_own;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NWAVE; ++q) {
      if (better(sb[q].r, sb[q].h, sb[q].K, best)) best = sb[q];
      r_own = so[q] > r_own ? so[q] : r_own;
    }
    h.part[blockIdx.x] = Partial{best.r, best.h, best.K, 0, r_own};
  }
}

__global__ void k_hub_final(HubArgs h) {
  const RateArgs& a = h.a;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.count) return;
  const uint32_t u = a.list[i];
  if (!hub_active(a, u)) {
    no_cand(a, i);
    return;
  }
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (uint64_t p = h.soff[i]; p < h.soff[i + 1]; ++p) {
    const Partial q = h.part[p];
    if (better(q.r, q.h, q.K, best)) best = Best{q.r, q.h, q.K};
    r_own = q.r_own > r_own ? q.r_own : r_own;
  }
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  emit(a, i, u, gd, best, r_own, a.nw[u]);
}

// Label-range partitioned hub rating (packed ratings only): the labels of hub
// i are split into P_i hash ranges of about HUB_RANGE entries; block j of hub i
// scans the whole adjacency and aggregates only labels of range j in a packed
// LDS table, so no global atomics are needed.  Probing is bounded: a range
// that does not fit raises `overflow` and the caller recomputes the hubs with
// the global tables (same ratings, same result).
constexpr int HUB_RANGE = 12288;

LMGP_D uint32_t label_range(uint32_t K, uint32_t P) {
  uint32_t h = K * 0x9E3779B1u;
  h ^= h >> 15;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  return (uint32_t)(((uint64_t)h * P) >> 32);
}

template <int T>
LMGP_D bool lds_add_bounded(unsigned long long* tab, uint32_t K, unsigned long long w) {
  constexpr int LOGT = __builtin_ctz(T);
  const unsigned long long mine = ((unsigned long long)K << 32) | w;
  uint32_t s = (K * 0x9E3779B1u) >> (32 - LOGT);
  unsigned long long prev;
  bool hit;
  int probe = 0;
  do {
    prev = atomicCAS(&tab[s], EMPTY_SLOT, mine);
    hit = prev == EMPTY_SLOT || (uint32_t)(prev >> 32) == K;
    s = hit ? s : (s + 1) & (T - 1);
  } while (!hit && ++probe < T);
  if (hit && prev != EMPTY_SLOT) atomicAdd(&tab[s], w);
  return hit;
}

template <int EWK>
__global__ __launch_bounds__(1024) void k_hub_range(HubArgs h, uint32_t* ovl, int force_overflow) {
  constexpr int T = BIG_TABLE;
  constexpr int NW = 1024 / WAVE;
  __shared__ unsigned long long tab[T];
  __shared__ Best sb[NW];
  __shared__ int64_t so[NW];
  __shared__ int sfull;
  const RateArgs& a = h.a;
  if (blockIdx.x >= h.soff[a.count]) return;  // the grid is an upper bound
  const uint32_t i = find_hub(h.soff, a.count, blockIdx.x);
  const uint32_t u = a.list[i];
  if (!hub_active(a, u)) return;
  const uint32_t P = (uint32_t)(h.soff[i + 1] - h.soff[i]);
  const uint32_t j = (uint32_t)(blockIdx.x - h.soff[i]);
  for (int s = threadIdx.x; s < T; s += 1024) tab[s] = EMPTY_SLOT;
  if (threadIdx.x == 0) sfull = force_overflow;
  __syncthreads();
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  bool ok = true;
  constexpr int U = 4;
  for (uint64_t e0 = beg + threadIdx.x; e0 < end && ok; e0 += (uint64_t)U * 1024) {
    uint32_t v[U], K[U];
    int64_t w[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint64_t e = e0 + (uint64_t)q * 1024;
      v[q] = e < end ? a.adj[e] : 0u;
      w[q] = e < end ? edge_w<EWK>(a.ew, e) : 0;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) K[q] = e0 + (uint64_t)q * 1024 < end ? a.label[v[q]] : EMPTY_KEY;
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (ok && K[q] != EMPTY_KEY && label_range(K[q], P) == j)
        ok = lds_add_bounded<T>(tab, K[q], (unsigned long long)w[q]);
  }
  if (!ok) sfull = 1;
  __syncthreads();
  if (sfull) {  // recomputed by k_hub_repair
    if (threadIdx.x == 0) ovl[1 + atomicAdd(&ovl[0], 1u)] = blockIdx.x;
    return;
  }
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const uint32_t own = a.label[u];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (int s = threadIdx.x; s < T; s += 1024) {
    const unsigned long long v = tab[s];
    if (v != EMPTY_SLOT)
      consider(a, (uint32_t)(v >> 32), (int64_t)(v & 0xFFFFFFFFull), own, cu, gd.cap, pre_u,
               gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sb[w] = best;
    so[w] = r_own;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NW; ++q) {
      if (better(sb[q].r, sb[q].h, sb[q].K, best)) best = sb[q];
      r_own = so[q] > r_own ? so[q] : r_own;
    }
    h.part[blockIdx.x] = Partial{best.r, best.h, best.K, 0, r_own};
  }
}

// A second, independent split of a range's labels (repair passes).
LMGP_D uint32_t label_subrange(uint32_t K, uint32_t R) {
  uint32_t x = K * 0x85EBCA77u + 0x27D4EB2Fu;
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  return (uint32_t)(((uint64_t)x * R) >> 32);
}

// Ranges whose labels did not fit the LDS table: each is recomputed by one
// block in R2 passes, pass q aggregating the labels of sub-range q of the
// range (R2 doubles until every pass fits), so the result is exact without a
// host round trip.  Ranges almost never overflow (about HUB_RANGE entries
// for 16384 slots); the loop is for exactness.
template <int EWK>
__global__ __launch_bounds__(1024) void k_hub_repair(HubArgs h, const uint32_t* ovl) {
  constexpr int T = BIG_TABLE;
  constexpr int NW = 1024 / WAVE;
  __shared__ unsigned long long tab[T];
  __shared__ Best sb[NW];
  __shared__ int64_t so[NW];
  __shared__ int sfull;
  const RateArgs& a = h.a;
  const uint32_t nov = ovl[0];
  for (uint32_t o = blockIdx.x; o < nov; o += gridDim.x) {
    const uint32_t b = ovl[1 + o];
    const uint32_t i = find_hub(h.soff, a.count, b);
    const uint32_t u = a.list[i];
    const uint32_t P = (uint32_t)(h.soff[i + 1] - h.soff[i]);
    const uint32_t j = (uint32_t)(b - h.soff[i]);
    const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
    const GraphDesc gd = a.gd[graph_of(a.gid, u)];
    const uint32_t own = a.label[u];
    const int64_t cu = a.nw[u];
    const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
    Best best{0, 0, 0};
    int64_t r_own = 0;
    for (uint32_t R2 = (uint32_t)ceil_div(end - beg, T / 2);; R2 *= 2) {
      Best bb{0, 0, 0};
      int64_t ro = 0;
      bool failed = false;
      for (uint32_t q2 = 0; q2 < R2 && !failed; ++q2) {
        for (int s = threadIdx.x; s < T; s += 1024) tab[s] = EMPTY_SLOT;
        if (threadIdx.x == 0) sfull = 0;
        __syncthreads();
        bool ok = true;
        for (uint64_t e = beg + threadIdx.x; e < end && ok; e += 1024) {
          const uint32_t K = a.label[a.adj[e]];
          if (label_range(K, P) != j || label_subrange(K, R2) != q2) continue;
          ok = lds_add_bounded<T>(tab, K, (unsigned long long)edge_w<EWK>(a.ew, e));
        }
        if (!ok) sfull = 1;
        __syncthreads();
        failed = sfull != 0;  // uniform: read after the barrier
        if (!failed)
          for (int s = threadIdx.x; s < T; s += 1024) {
            const unsigned long long v = tab[s];
            if (v != EMPTY_SLOT)
              consider(a, (uint32_t)(v >> 32), (int64_t)(v & 0xFFFFFFFFull), own, cu, gd.cap,
                       pre_u, gd.label_base, bb, ro);
          }
        __syncthreads();
      }
      if (!failed) {
        best = bb;
        r_own = ro;
        break;
      }
    }
    reduce_best<WAVE>(best, r_own);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
      sb[w] = best;
      so[w] = r_own;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < NW; ++q) {
        if (better(sb[q].r, sb[q].h, sb[q].K, best)) best = sb[q];
        r_own = so[q] > r_own ? so[q] : r_own;
      }
      h.part[b] = Partial{best.r, best.h, best.K, 0, r_own};
    }
    __syncthreads();
  }
}

struct HubRanges {
  const uint64_t* xadj;
  const uint32_t* list;
  LMGP_D uint64_t operator()(uint64_t i) const {
    const uint32_t u = list[i];
    return ceil_div(xadj[u + 1] - xadj[u], HUB_RANGE);
  }
};

struct HubTable {
  const uint64_t* xadj;
  const uint32_t* list;
  LMGP_D uint64_t operator()(uint64_t i) const {
    const uint32_t u = list[i];
    const uint64_t d = xadj[u + 1] - xadj[u];
    uint64_t T = 1;
    while (T < 2 * d) T <<= 1;
    return T;
  }
};
struct HubChunks {
  const uint64_t* xadj;
  const uint32_t* list;
  LMGP_D uint64_t operator()(uint64_t i) const {
    const uint32_t u = list[i];
    return ceil_div(xadj[u + 1] - xadj[u], HUB_CHUNK);
  }
};
struct HubSlotChunks {
  const uint64_t* xadj;
  const uint32_t* list;
  LMGP_D uint64_t operator()(uint64_t i) const {
    const uint32_t u = list[i];
    const uint64_t d = xadj[u + 1] - xadj[u];
    uint64_t T = 1;
    while (T < 2 * d) T <<= 1;
    return ceil_div(T, HUB_SLOTS);
  }
};

// Profiler family of a rating launch: phase, degree class, edge-weight type
// (e.g. "cl_rate_block_i64" for clustering, "rf_" refinement, "fv_" 2-hop
// favourites).
std::string rate_name(int phase, int cls, int ewk, bool few, bool packed) {
  // "<phase>:<kernel>": the kernel part is the HIP kernel's template name, so
  // that event timings line up with a kernel trace; the hub class brackets
  // several kernels and is named rate_hubs
  static const char* ph[3] = {"cl:", "rf:", "fv:"};
  const int w = ewk;
  std::string k;
  if (phase == 1 && few && cls >= CLASS_BLOCK && cls < CLASS_BLOCK + 2)
    k = "k_rate_rows<" + std::to_string(w) + (packed ? ", true>" : ", false>");
  else if (phase == 1 && few && cls >= CLASS_BLOCK && cls < CLASS_GLOBAL)
    k = "k_rate_dense<" + std::to_string(w) + ", " + (cls < CLASS_BIG ? "256, " : "1024, ") +
        (packed ? "true>" : "false>");
  else if (cls < CLASS_BLOCK) k = "k_rate_group<" + std::to_string(class_group(cls)) + ", " + std::to_string(w) + ">";
  else if (cls < CLASS_BIG && !(packed && cls >= CLASS_BLOCK + 2))
    k = "k_rate_block<" + std::to_string(w) + ", " + std::to_string(class_table_log(cls)) + ">";
  else if (cls < CLASS_GLOBAL)
    k = "k_rate_big<" + std::to_string(w) + ", " + std::to_string(class_table_log(cls)) + ", " +
        (cls == CLASS_BLOCK + 2 ? "256>" : cls == CLASS_BLOCK + 3 ? "512>" : "1024>");
  else k = "rate_hubs<" + std::to_string(w) + ">";
  return std::string(ph[phase]) + k;
}

// Algorithmic bytes of rating `count` nodes with `degsum` entries: per node the
// two offsets, its list slot, label and weight (32 B); per entry the neighbour
// id, its label (`label_bytes`: 1 where the kernel gathers the byte copy of
// the blocks, else 4) and the edge weight (if stored).
uint64_t rate_bytes(int ewk, uint64_t count, uint64_t degsum, uint64_t label_bytes = 4) {
  const uint64_t bw = ewk == EW_UNIT ? 0 : ewk == EW_I32 ? 4 : 8;
  return 32 * count + (4 + label_bytes + bw) * degsum;
}

template <int EWK>
void launch_groups_t(const RateArgs& a, const uint32_t* count, const uint32_t* off,
                     uint64_t degsum, hipStream_t s) {
  GroupSplit split{};
  uint32_t blocks = 0, total = 0;
  for (int c = 0; c < GROUP_CLASSES; ++c) {
    split.bstart[c] = blocks;
    split.off[c] = off[c];
    split.count[c] = count[c];
    blocks += c < CLASS_BLOCK ? grid_for(count[c], 256 / class_group(c)) : count[c];
    total += count[c];
  }
  split.bstart[GROUP_CLASSES] = blocks;
  if (!blocks) return;
  const char* ph[3] = {"cl:", "rf:", "fv:"};
  ProfLaunch prof((std::string(ph[a.phase]) + "k_rate_groups<" + std::to_string(EWK) + ">").c_str(),
                  rate_bytes(EWK, total, degsum, a.label8 ? 1 : 4));
  launch_k(k_rate_groups<EWK>, dim3(blocks), dim3(256), s, prof.start(), prof.stop(), a, split);
  LAUNCH_CHECK();
}

template <int EWK>
void launch_rate_t(int cls, const RateArgs& a, hipStream_t s) {
  if (a.count == 0) return;
  // single-kernel classes: the launch timestamps its own start and end
  const bool few = a.few && a.few <= FEW_LABELS && a.mode == MODE_LP;
  ProfLaunch prof(rate_name(a.phase, cls, EWK, few, a.packed != 0).c_str(),
                  rate_bytes(EWK, a.count, a.degsum));
  const hipEvent_t e0 = prof.start(), e1 = prof.stop();
  if (cls < CLASS_BLOCK) {
    throw InvalidArg("lane-group classes are launched by launch_rate_groups");
  } else if (a.few && a.few <= FEW_LABELS && a.mode == MODE_LP && cls < CLASS_GLOBAL) {
    const dim3 rgrid((uint32_t)ceil_div(a.count, RW_WAVES)), rblk(RW_WAVES * WAVE);
    const uint32_t rlds = (uint32_t)(RW_WAVES * a.few * (a.packed ? 4 : 8));
    if (cls < CLASS_BLOCK + 2) {
      if (a.packed) launch_k_lds(k_rate_rows<EWK, true>, rgrid, rblk, rlds, s, e0, e1, a);
      else launch_k_lds(k_rate_rows<EWK, false>, rgrid, rblk, rlds, s, e0, e1, a);
    } else if (cls < CLASS_BIG) {
      if (a.packed) launch_k(k_rate_dense<EWK, 256, true>, dim3(a.count), dim3(256), s, e0, e1, a);
      else launch_k(k_rate_dense<EWK, 256, false>, dim3(a.count), dim3(256), s, e0, e1, a);
    } else {
      if (a.packed) launch_k(k_rate_dense<EWK, 1024, true>, dim3(a.count), dim3(1024), s, e0, e1, a);
      else launch_k(k_rate_dense<EWK, 1024, false>, dim3(a.count), dim3(1024), s, e0, e1, a);
    }
  } else if (cls < CLASS_BIG && a.packed && cls >= CLASS_BLOCK + 2) {
    if (cls == CLASS_BLOCK + 2)
      launch_k(k_rate_big<EWK, 11, 256>, dim3(a.count), dim3(256), s, e0, e1, a);
    else
      launch_k(k_rate_big<EWK, 12, 512>, dim3(a.count), dim3(512), s, e0, e1, a);
  } else if (cls < CLASS_BIG) {
    const dim3 grid(a.count), blk(256);
    switch (cls - CLASS_BLOCK) {
      case 0: case 1: throw InvalidArg("block classes 6, 7 are launched by launch_rate_groups");
      case 2: launch_k(k_rate_block<EWK, 11>, grid, blk, s, e0, e1, a); break;
      default: launch_k(k_rate_block<EWK, 12>, grid, blk, s, e0, e1, a); break;
    }
  } else if (is_big_class(cls)) {
    if (!a.packed) throw InvalidArg("big-block class needs packed ratings");
    const dim3 grid(a.count), blk(1024);
    if (cls == CLASS_BIG) launch_k(k_rate_big<EWK, 13, 1024>, grid, blk, s, e0, e1, a);
    else launch_k(k_rate_big<EWK, 14, 1024>, grid, blk, s, e0, e1, a);
  } else {
    throw InvalidArg("hub class needs launch_rate_hubs");
  }
  LAUNCH_CHECK();
}

// Few labels (refinement with at most FEW_LABELS blocks): a hub's ratings
// are a dense row of `few` entries in global memory.  Each block rates a chunk
// of HUB_CHUNK entries into per-wave dense LDS rows (a chunk's labels fall on
// few addresses, so each wave keeps its own copy), merges the copies and adds
// its non-zero ratings to the hub's row.
template <int EWK>
__global__ __launch_bounds__(256) void k_hub_few_insert(HubArgs h, unsigned long long* rows) {
  __shared__ unsigned long long tab[NWAVE * FEW_LABELS];
  const RateArgs& a = h.a;
  const uint32_t few = a.few;
  const uint64_t b = blockIdx.x;
  if (b >= h.coff[a.count]) return;  // the grid is an upper bound
  for (uint32_t t = threadIdx.x; t < NWAVE * few; t += 256) tab[t] = 0;
  __syncthreads();
  const uint32_t i = find_hub(h.coff, a.count, b);
  const uint32_t u = a.list[i];
  if (!hub_active(a, u)) return;  // uniform over the block
  const uint64_t beg = a.xadj[u] + (b - h.coff[i]) * HUB_CHUNK;
  const uint64_t lim = a.xadj[u + 1];
  const uint64_t end = beg + HUB_CHUNK < lim ? beg + HUB_CHUNK : lim;
  unsigned long long* mt = tab + (threadIdx.x / WAVE) * few;
  constexpr int U = HUB_CHUNK / 256;
  uint32_t v[U];
  int64_t w[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const uint64_t e = beg + (uint64_t)j * 256 + threadIdx.x;
    v[j] = e < end ? a.adj[e] : 0u;
    w[j] = e < end ? edge_w<EWK>(a.ew, e) : 0;
  }
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const uint64_t e = beg + (uint64_t)j * 256 + threadIdx.x;
    if (e < end) atomicAdd(&mt[nbr_label(a, v[j])], (unsigned long long)w[j]);
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < few; t += 256) {
    unsigned long long sum = 0;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) sum += tab[q * few + t];
    if (sum) atomicAdd(&rows[(uint64_t)i * few + t], sum);
  }
}

// One block per hub: the best label of its dense row.
__global__ __launch_bounds__(256) void k_hub_few_final(HubArgs h, const unsigned long long* rows) {
  __shared__ Best sb[NWAVE];
  __shared__ int64_t so[NWAVE];
  const RateArgs& a = h.a;
  const uint32_t i = blockIdx.x;
  const uint32_t u = a.list[i];
  if (!hub_active(a, u)) {
    if (threadIdx.x == 0) no_cand(a, i);
    return;
  }
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const uint32_t own = a.label[u];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (uint32_t t = threadIdx.x; t < a.few; t += 256) {
    const int64_t r = (int64_t)rows[(uint64_t)i * a.few + t];
    if (r == 0) continue;  // not adjacent (edge weights are positive)
    const int64_t wk = (t != own && a.mode == MODE_LP) ? a.W[t] : 0;
    consider_w(a, t, r, own, cu, gd.cap, wk, pre_u, gd.label_base, best, r_own);
  }
  reduce_best<WAVE>(best, r_own);
  const int wv = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sb[wv] = best;
    so[wv] = r_own;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NWAVE; ++q) {
      if (better(sb[q].r, sb[q].h, sb[q].K, best)) best = sb[q];
      r_own = so[q] > r_own ? so[q] : r_own;
    }
    emit(a, i, u, gd, best, r_own, cu);
  }
}

template <int EWK>
void launch_hubs_t(const RateArgs& ra, Pool& pool, hipStream_t s) {
  const uint32_t c = ra.count;
  ProfScope prof(rate_name(ra.phase, CLASS_GLOBAL, EWK, false, false).c_str(),
                 rate_bytes(EWK, ra.count, ra.degsum, ra.label8 ? 1 : 4), s);
  // LMGP_HUB_TABLES=global forces the chunked global-table path (taken when
  // ratings do not fit 32 bits); =repair makes every label range report an
  // overflow so that k_hub_repair computes all of them (both used by tests)
  const char* force = std::getenv("LMGP_HUB_TABLES");
  if (ra.few && ra.few <= FEW_LABELS && ra.mode == MODE_LP &&
      !(force && std::strcmp(force, "global") == 0)) {
    // dense rows of `few` ratings; the chunk grid is an upper bound (blocks
    // past the last chunk exit), so no host round trip is needed
    DBuf<uint64_t> coff(&pool, s, c + 1);
    exclusive_scan(HubChunks{ra.xadj, ra.list}, c, coff.get(), true, pool, s);
    DBuf<unsigned long long> rows(&pool, s, (uint64_t)c * ra.few);
    rows.zero();
    HubArgs h{};
    h.a = ra;
    h.coff = coff.get();
    const uint64_t nchunks = ra.degsum / HUB_CHUNK + c;
    k_hub_few_insert<EWK><<<(unsigned)nchunks, 256, 0, s>>>(h, rows.get());
    LAUNCH_CHECK();
    k_hub_few_final<<<c, 256, 0, s>>>(h, rows.get());
    LAUNCH_CHECK();
    return;
  }
  // refinement labels are blocks: few distinct labels per hub, so the chunked
  // global tables see few atomics and re-reading the adjacency per range would
  // cost more
  const bool ranges =
      ra.packed && ra.phase != 1 && !(force && std::strcmp(force, "global") == 0);
  if (ranges) {
    // label-range partitioning in LDS; ranges that overflow their table are
    // recomputed on the device (k_hub_repair), so no host round trip is needed
    DBuf<uint64_t> roff(&pool, s, c + 1);
    exclusive_scan(HubRanges{ra.xadj, ra.list}, c, roff.get(), true, pool, s);
    // sum over hubs of ceil(d / HUB_RANGE) <= degsum / HUB_RANGE + c
    const uint64_t nr = ra.degsum / HUB_RANGE + c;
    DBuf<Partial> part(&pool, s, nr);
    DBuf<uint32_t> ovl(&pool, s, nr + 1);
    device_zero(ovl.get(), sizeof(uint32_t), s);
    HubArgs h{};
    h.a = ra;
    h.soff = roff.get();
    h.part = part.get();
    const int force_ovf = force && std::strcmp(force, "repair") == 0;
    k_hub_range<EWK><<<(unsigned)nr, 1024, 0, s>>>(h, ovl.get(), force_ovf);
    LAUNCH_CHECK();
    k_hub_repair<EWK><<<64, 1024, 0, s>>>(h, ovl.get());
    LAUNCH_CHECK();
    k_hub_final<<<grid_for(c, 64), 64, 0, s>>>(h);
    LAUNCH_CHECK();
    return;
  }
  DBuf<uint64_t> toff(&pool, s, c + 1), coff(&pool, s, c + 1), soff(&pool, s, c + 1);
  exclusive_scan(HubTable{ra.xadj, ra.list}, c, toff.get(), true, pool, s);
  exclusive_scan(HubChunks{ra.xadj, ra.list}, c, coff.get(), true, pool, s);
  exclusive_scan(HubSlotChunks{ra.xadj, ra.list}, c, soff.get(), true, pool, s);
  uint64_t tot[3] = {0, 0, 0};
  read_now(&tot[0], toff.get() + c, 8, s);
  read_now(&tot[1], coff.get() + c, 8, s);
  read_now(&tot[2], soff.get() + c, 8, s);
  DBuf<uint32_t> keys;
  DBuf<int64_t> vals;
  DBuf<unsigned long long> tab;
  if (ra.packed) {
    tab.reset(&pool, s, tot[0]);
  } else {
    keys.reset(&pool, s, tot[0]);
    vals.reset(&pool, s, tot[0]);
  }
  DBuf<Partial> part(&pool, s, tot[2]);
  HubArgs h;
  h.a = ra;
  h.a.gkeys = keys.get();
  h.a.gvals = vals.get();
  h.a.gtab = tab.get();
  h.toff = toff.get();
  h.coff = coff.get();
  h.soff = soff.get();
  h.slots = tot[0];
  h.part = part.get();
  unsigned gc = grid_for(tot[0], 256);
  k_hub_clear<<<gc > 4096 ? 4096 : gc, 256, 0, s>>>(h);
  LAUNCH_CHECK();
  k_hub_insert<EWK><<<(unsigned)tot[1], 256, 0, s>>>(h);
  LAUNCH_CHECK();
  k_hub_eval<<<(unsigned)tot[2], 256, 0, s>>>(h);
  LAUNCH_CHECK();
  k_hub_final<<<grid_for(c, 64), 64, 0, s>>>(h);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------- bucketing --
// The descriptor fields bucketing reads.  A single graph's (gid NULL) are
// loaded once per thread, with scalar loads; a union reads its graph's.
struct BucketGd {
  uint64_t node_base, pre_sub;
  int64_t cap;
  uint32_t active, subrounds;
};
LMGP_D BucketGd bucket_gd(const GraphDesc& d) {
  return BucketGd{d.node_base, d.pre_sub, d.cap, d.active, d.subrounds};
}
LMGP_D BucketGd bucket_gd0(const BucketArgs& a) {
  return a.gid ? BucketGd{0, 0, 0, 0, 1} : bucket_gd(a.gd[0]);
}

LMGP_D int bucket_of(const BucketArgs& a, uint64_t u, const BucketGd& g0) {
  // boundary refinement: interior nodes cost one byte
  if (a.mode == 0 && a.only && !a.only[u]) return -1;
  const BucketGd gd = a.gid ? bucket_gd(a.gd[a.gid[u]]) : g0;
  if (!gd.active) return -1;
  const uint64_t d = a.xadj[u + 1] - a.xadj[u];
  if (d == 0) return -1;
  if (a.mode == 0) {
    // a node at least as heavy as the capacity can join no label (every
    // adjacent label weighs at least one), so rating it cannot produce a move
    if (a.nw[u] >= gd.cap) return -1;
    // listed nodes (ids) are those of sub-round only_sub already
    const uint32_t sr =
        a.ids ? a.only_sub : subround_of(hash_add(gd.pre_sub, u - gd.node_base), gd.subrounds);
    if (a.only && sr != a.only_sub) return -1;
    return (int)(sr * NCLASS + class_of(d, a.cuts));
  }
  // 2-hop: singletons lighter than the cap, with neighbours
  if (a.csize[a.label[u]] != 1) return -1;
  if (a.nw[u] >= gd.cap) return -1;
  return class_of(d, a.cuts);
}

__global__ __launch_bounds__(256) void k_bucket_count(BucketArgs a) {
  const BucketGd g0 = bucket_gd0(a);
  __shared__ uint32_t h[MAX_BUCKETS];
  __shared__ unsigned long long hd[MAX_BUCKETS];
  for (uint32_t i = threadIdx.x; i < a.nbuckets; i += 256) {
    h[i] = 0;
    hd[i] = 0;
  }
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t cnt = a.ids ? *a.nids : a.n;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const uint64_t u = a.ids ? a.ids[i] : i;
    int b = bucket_of(a, u, g0);
    if (a.bkt) a.bkt[u] = b >= 0 ? (uint8_t)b : (uint8_t)0xFF;
    if (b >= 0) {
      atomicAdd(&h[b], 1u);
      if (a.degs_all || b % NCLASS == CLASS_GLOBAL)
        atomicAdd(&hd[b], (unsigned long long)(a.xadj[u + 1] - a.xadj[u]));
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < a.nbuckets; i += 256)
    if (h[i]) {
      atomicAdd(&a.counts[i], (unsigned long long)h[i]);
      if (a.degs) atomicAdd(&a.degs[i], hd[i]);
    }
}

__global__ void k_bucket_offsets(BucketArgs a) {
  // nbuckets <= MAX_BUCKETS: one wave scans them in chunks of 64
  uint32_t run = 0;
  for (uint32_t i0 = 0; i0 < a.nbuckets; i0 += WAVE) {
    const uint32_t i = i0 + lane_id();
    const uint32_t c = i < a.nbuckets ? (uint32_t)a.counts[i] : 0u;
    const uint32_t inc = wave_inclusive_scan(c);
    if (i < a.nbuckets) {
      a.offs[i] = run + inc - c;
      a.fill[i] = 0;
    }
    run += __shfl(inc, WAVE - 1);
  }
}

// One thread per sub-round: the launch plan the host derives from the bucket
// counts in an unplanned round (launch_groups_t, rate_classes).
__global__ void k_lp_plan(const unsigned long long* counts, const uint32_t* offs, uint32_t S,
                          int dense, SubPlan* plan) {
  const uint32_t sr = threadIdx.x;
  if (sr >= S) return;
  SubPlan p{};
  const uint32_t* o = offs + sr * NCLASS;
  p.lbase = o[0];
  uint32_t total = 0;
  for (int c = 0; c < NCLASS; ++c) {
    p.cnt[c] = (uint32_t)counts[sr * NCLASS + c];
    p.off[c] = o[c] - o[0];
    total += p.cnt[c];
  }
  p.total = total;
  const int nsmall = dense ? CLASS_BLOCK : GROUP_CLASSES;
  uint32_t blocks = 0;
  for (int c = 0; c < GROUP_CLASSES; ++c) {
    const uint32_t n = c < nsmall ? p.cnt[c] : 0u;
    p.gs.bstart[c] = blocks;
    p.gs.off[c] = p.off[c];
    p.gs.count[c] = n;
    const uint32_t per = c < CLASS_BLOCK ? 256u / (uint32_t)class_group(c) : 1u;
    blocks += (n + per - 1) / per;
  }
  p.gs.bstart[GROUP_CLASSES] = blocks;
  plan[sr] = p;
}

// Each block takes 2048 consecutive nodes, counts them per bucket in LDS and
// reserves its range of every bucket with one atomic (order inside a bucket
// does not affect any result).
constexpr int BK_ITEMS = 8;

__global__ __launch_bounds__(256) void k_bucket_scatter(BucketArgs a) {
  const BucketGd g0 = bucket_gd0(a);
  __shared__ uint32_t cnt[MAX_BUCKETS], base[MAX_BUCKETS];
  // node range: one tile per block; node list: tiles grid-strided over its
  // device-side length
  const uint64_t total = a.ids ? *a.nids : a.n;
  const uint64_t tile = 256 * BK_ITEMS;
  const uint64_t step = a.ids ? (uint64_t)gridDim.x * tile : total + tile;
  for (uint64_t b0 = (uint64_t)blockIdx.x * tile; b0 < total; b0 += step) {
    for (uint32_t i = threadIdx.x; i < a.nbuckets; i += 256) cnt[i] = 0;
    __syncthreads();
    int bk[BK_ITEMS];
    uint32_t lp[BK_ITEMS], uu[BK_ITEMS];
#pragma unroll
    for (int j = 0; j < BK_ITEMS; ++j) {
      const uint64_t i = b0 + (uint64_t)j * 256 + threadIdx.x;
      uu[j] = i < total ? (a.ids ? a.ids[i] : (uint32_t)i) : 0u;
      if (a.bkt) {
        const uint8_t v = i < total ? a.bkt[uu[j]] : (uint8_t)0xFF;
        bk[j] = v == 0xFF ? -1 : (int)v;
      } else {
        bk[j] = i < total ? bucket_of(a, uu[j], g0) : -1;
      }
      lp[j] = bk[j] >= 0 ? atomicAdd(&cnt[bk[j]], 1u) : 0u;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < a.nbuckets; i += 256)
      if (cnt[i]) base[i] = atomicAdd(&a.fill[i], cnt[i]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BK_ITEMS; ++j)
      if (bk[j] >= 0) a.list[a.offs[bk[j]] + base[bk[j]] + lp[j]] = uu[j];
    __syncthreads();  // cnt and base are rewritten by the next tile
  }
}

// The flagged nodes of sub-round only_sub, listed in ascending order (the
// rating kernels read the rows of nearby nodes together): block b takes a
// contiguous chunk of 8-byte flag words (most words of a boundary are zero
// and cost one load), k_sub_count counts its nodes, k_sub_write adds the
// counts of the blocks before it and writes them.
constexpr unsigned SUB_BLOCKS = SUB_LIST_BLOCKS;

// bit i: node w * 8 + i is flagged and in sub-round only_sub
LMGP_D uint32_t sub_select(const BucketArgs& a, const uint8_t* flag, uint64_t w,
                           const BucketGd& g0) {
  uint64_t bits = ((const uint64_t*)flag)[w];
  uint32_t sel = 0;
  while (bits) {
    const int byte = __builtin_ctzll(bits) >> 3;
    bits &= ~(0xFFull << (byte * 8));
    const uint64_t u = w * 8 + (uint64_t)byte;
    if (u >= a.n) break;
    const BucketGd gd = a.gid ? bucket_gd(a.gd[a.gid[u]]) : g0;
    if (subround_of(hash_add(gd.pre_sub, u - gd.node_base), gd.subrounds) == a.only_sub)
      sel |= 1u << byte;
  }
  return sel;
}

// words [w0, w1) of block b, split into 256 contiguous runs
LMGP_D void sub_chunk(uint64_t words, uint64_t& w0, uint64_t& w1) {
  const uint64_t per = (words + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = b0 + per < words ? b0 + per : words;
  const uint64_t tper = (per + 255) / 256;
  w0 = b0 + (uint64_t)threadIdx.x * tper;
  w1 = w0 + tper;
  if (w0 > b1) w0 = b1;
  if (w1 > b1) w1 = b1;
}

__global__ __launch_bounds__(256) void k_sub_count(BucketArgs a, const uint8_t* flag,
                                                   uint32_t* block_cnt, uint8_t* wsel) {
  __shared__ uint32_t sm[NWAVE];
  uint64_t w0, w1;
  sub_chunk((a.n + 7) / 8, w0, w1);
  uint32_t c = 0;
  const BucketGd g0 = bucket_gd0(a);
  for (uint64_t w = w0; w < w1; ++w) {
    const uint32_t sel = sub_select(a, flag, w, g0);
    wsel[w] = (uint8_t)sel;  // read back by k_sub_write
    c += (uint32_t)__popc(sel);
  }
  const uint32_t tot = block_reduce_sum(c, sm);
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_sub_write(BucketArgs a, const uint8_t* wsel,
                                                   const uint32_t* block_cnt, uint32_t* ids,
                                                   unsigned long long* nids) {
  __shared__ uint32_t sm[NWAVE];
  uint32_t before = 0;
  for (uint32_t b = threadIdx.x; b < blockIdx.x; b += 256) before += block_cnt[b];
  before = block_reduce_sum(before, sm);
  uint64_t w0, w1;
  sub_chunk((a.n + 7) / 8, w0, w1);
  uint32_t c = 0;
  for (uint64_t w = w0; w < w1; ++w) c += (uint32_t)__popc(wsel[w]);
  uint32_t tot;
  uint64_t at = before + block_exclusive_scan(c, sm, tot);
  for (uint64_t w = w0; w < w1; ++w) {
    uint32_t sel = wsel[w];
    while (sel) {
      const int byte = __builtin_ctz(sel);
      sel &= sel - 1;
      ids[at++] = (uint32_t)(w * 8 + (uint64_t)byte);
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *nids = before + tot;
}

// ------------------------------------------------------------- admission --
LMGP_D uint32_t cand_graph(const AdmitArgs& a, uint32_t u) { return graph_of(a.gid, u); }

// A graph's sub-round made a move: only "any move" is read (a round without
// moves ends the graph's LP), so the counter is a flag.  One add per wave on
// a single address would serialise (tens of thousands per launch); a load
// that already sees the flag skips the store.
LMGP_D void mark_moved(const AdmitArgs& a, uint32_t g) {
  if (__hip_atomic_load(&a.moves[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    __hip_atomic_store(&a.moves[g], (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Few labels (refinement): per-target demand and candidate count from
// block-privatised LDS histograms, one global atomic per block and target.
constexpr int ADM_ITEMS = 8;

__global__ __launch_bounds__(256) void k_adm_count_few(AdmitArgs a) {
  __shared__ unsigned long long sd[FEW_LABELS];
  __shared__ uint32_t sn[FEW_LABELS];
  for (uint32_t t = threadIdx.x; t < a.few; t += 256) {
    sd[t] = 0;
    sn[t] = 0;
  }
  __syncthreads();
  const uint32_t nc = a.plan ? a.plan->total : a.max_cands;
  const uint64_t b0 = (uint64_t)blockIdx.x * 256 * ADM_ITEMS;
#pragma unroll
  for (int j = 0; j < ADM_ITEMS; ++j) {
    const uint64_t i = b0 + (uint64_t)j * 256 + threadIdx.x;
    if (i < nc && a.cands[i].tgt != EMPTY_KEY) {
      const Cand c = a.cands[i];
      atomicAdd(&sd[c.tgt], (unsigned long long)a.nw[c.u]);
      atomicAdd(&sn[c.tgt], 1u);
    }
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < a.few; t += 256)
    if (sn[t]) {
      atomicAdd((unsigned long long*)&a.tally[t].demand, sd[t]);
      atomicAdd(&a.tally[t].ntgt, sn[t]);
    }
}

// Few labels: as k_adm_classify, with the segment slots of a block's
// overflowing candidates reserved by one atomic per block and target.
__global__ __launch_bounds__(256) void k_adm_classify_few(AdmitArgs a) {
  __shared__ uint32_t cnt[FEW_LABELS], base[FEW_LABELS];
  const int64_t cap0 = a.gid ? 0 : a.gd[0].cap;  // a single graph's, one scalar load
  for (uint32_t t = threadIdx.x; t < a.few; t += 256) cnt[t] = 0;
  __syncthreads();
  const uint32_t nc = a.plan ? a.plan->total : a.max_cands;
  const uint64_t b0 = (uint64_t)blockIdx.x * 256 * ADM_ITEMS;
  uint32_t tg[ADM_ITEMS], lp[ADM_ITEMS];
#pragma unroll
  for (int j = 0; j < ADM_ITEMS; ++j) {
    const uint64_t i = b0 + (uint64_t)j * 256 + threadIdx.x;
    tg[j] = EMPTY_KEY;
    if (i < nc && a.cands[i].tgt == EMPTY_KEY) {
      a.adm[i] = 0;
    } else if (i < nc) {
      const Cand c = a.cands[i];
      const int64_t cap = a.gid ? a.gd[a.gid[c.u]].cap : cap0;
      if (a.W[c.tgt] + a.tally[c.tgt].demand <= cap) {
        a.adm[i] = 1;
      } else {
        a.adm[i] = 0;
        tg[j] = c.tgt;
        lp[j] = atomicAdd(&cnt[c.tgt], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < a.few; t += 256)
    if (cnt[t]) {
      const uint32_t p = atomicAdd(&a.tally[t].fill, cnt[t]);
      base[t] = p;
      if (p == 0) {
        a.segbase[t] = atomicAdd(a.ovtotal, a.tally[t].ntgt);
        a.ovtgts[atomicAdd(a.ovcount, 1u)] = t;
      }
    }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ADM_ITEMS; ++j)
    if (tg[j] != EMPTY_KEY) a.cpos[b0 + (uint64_t)j * 256 + threadIdx.x] = base[tg[j]] + lp[j];
}

// Few labels without cluster bookkeeping (refinement): apply the admitted
// moves; label weight changes are summed per block in LDS.
__global__ __launch_bounds__(256) void k_adm_apply_few(AdmitArgs a) {
  __shared__ long long dw[FEW_LABELS];
  __shared__ uint64_t smv[NWAVE];
  for (uint32_t t = threadIdx.x; t < a.few; t += 256) {
    dw[t] = 0;
    if (blockIdx.x == 0) {  // per-target scratch for the next sub-round
      a.tally[t] = LabelTally{0, 0, 0};
    }
  }
  __syncthreads();
  const uint32_t nc = a.plan ? a.plan->total : a.max_cands;
  const uint64_t b0 = (uint64_t)blockIdx.x * 256 * ADM_ITEMS;
  uint64_t mv = 0;
#pragma unroll
  for (int j = 0; j < ADM_ITEMS; ++j) {
    const uint64_t i = b0 + (uint64_t)j * 256 + threadIdx.x;
    if (i < nc && a.adm[i]) {
      const Cand c = a.cands[i];
      const uint32_t own = a.label[c.u];
      const long long cu = a.nw[c.u];
      a.label[c.u] = c.tgt;
      if (a.label8) a.label8[c.u] = (uint8_t)c.tgt;
      atomicAdd((unsigned long long*)&dw[c.tgt], (unsigned long long)cu);
      atomicAdd((unsigned long long*)&dw[own], (unsigned long long)(-cu));
      if (a.gid) mark_moved(a, a.gid[c.u]);
      else ++mv;
    }
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < a.few; t += 256)
    if (dw[t]) atomicAdd((unsigned long long*)&a.Wmut[t], (unsigned long long)dw[t]);
  if (!a.gid) {
    uint64_t tot;
    (void)block_exclusive_scan(mv, smv, tot);
    if (threadIdx.x == 0 && tot) mark_moved(a, 0);
  }
  // every kernel of this admission that reads the overflow counters has run
  if (a.clear_ov && blockIdx.x == 0 && threadIdx.x == 0) a.ovtotal[0] = 0, a.ovcount[0] = 0;
}

__global__ void k_adm_reset_few(AdmitArgs a) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < a.few; t += gridDim.x * blockDim.x) {
    a.tally[t] = LabelTally{0, 0, 0};
  }
}

__global__ __launch_bounds__(256) void k_adm_classify(AdmitArgs a) {
  const uint32_t nc = a.plan ? a.plan->total : a.max_cands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const Cand c = a.cands[i];
  if (c.tgt == EMPTY_KEY) {
    a.adm[i] = 0;
    return;
  }
  const int64_t cap = a.gid ? a.gd[a.gid[c.u]].cap : a.gd[0].cap;
  const uint32_t t = c.tgt;
  const LabelTally tl = a.tally[t];
  if (a.W[t] + tl.demand <= cap) {
    a.adm[i] = 1;  // everything aimed at t fits
    return;
  }
  a.adm[i] = 0;
  const uint32_t p = atomicAdd(&a.tally[t].fill, 1u);
  a.cpos[i] = p;
  if (p == 0) {
    a.segbase[t] = atomicAdd(a.ovtotal, tl.ntgt);
    a.ovtgts[atomicAdd(a.ovcount, 1u)] = t;
  }
}

__global__ __launch_bounds__(256) void k_adm_scatter(AdmitArgs a) {
  const uint32_t nc = a.plan ? a.plan->total : a.max_cands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc || a.adm[i]) return;
  const uint32_t t = a.cands[i].tgt;
  if (t != EMPTY_KEY) a.seg[a.segbase[t] + a.cpos[i]] = i;
}

// Admission order key: (gain desc, hadm asc, u asc) as two uint64 words, hadm
// the upper 32 bits of H(seed, ADM|RADM, level, round, u).
LMGP_D void cand_key(const AdmitArgs& a, const Cand& c, uint64_t& hi, uint64_t& lo) {
  const GraphDesc& gd = a.gd[graph_of(a.gid, c.u)];
  const uint32_t hadm = (uint32_t)(hash_add(gd.pre_adm, (uint64_t)c.u - gd.node_base) >> 32);
  hi = (uint64_t)INT64_MAX - (uint64_t)c.gain;
  lo = ((uint64_t)hadm << 32) | c.u;
}
LMGP_D bool key_less(uint64_t ahi, uint64_t alo, uint64_t bhi, uint64_t blo) {
  return ahi < bhi || (ahi == bhi && alo < blo);
}

// Segments of at most 64 candidates: one wave, bitonic sort in registers.
LMGP_D void seg_waves(const AdmitArgs& a, uint32_t wid, uint32_t waves) {
  const uint32_t nt = *a.ovcount;
  const int l = lane_id();
  for (uint32_t j = wid; j < nt; j += waves) {
    const uint32_t t = a.ovtgts[j];
    const uint32_t size = a.tally[t].ntgt;
    if (size > WAVE) continue;
    const uint32_t base = a.segbase[t];
    const bool valid = (uint32_t)l < size;
    uint32_t ci = valid ? a.seg[base + l] : 0u;
    uint64_t khi = ~0ull, klo = ~0ull;
    int64_t w = 0;
    if (valid) {
      Cand c = a.cands[ci];
      cand_key(a, c, khi, klo);
      w = a.nw[c.u];
    }
    for (int k = 2; k <= WAVE; k <<= 1) {
      for (int j2 = k >> 1; j2 > 0; j2 >>= 1) {
        const int partner = (j2 == (k >> 1)) ? (l ^ (k - 1)) : (l ^ j2);
        uint64_t ohi = __shfl(khi, partner);
        uint64_t olo = __shfl(klo, partner);
        uint32_t oci = __shfl(ci, partner);
        int64_t ow = __shfl(w, partner);
        const bool o_less = key_less(ohi, olo, khi, klo);
        const bool take = (l < partner) ? o_less : key_less(khi, klo, ohi, olo);
        if (take) {
          khi = ohi, klo = olo, ci = oci, w = ow;
        }
      }
    }
    const int64_t incl = wave_inclusive_scan(w);
    const uint32_t u0 = a.cands[a.seg[base]].u;
    const int64_t room = a.gd[cand_graph(a, u0)].cap - a.W[t];
    if (khi != ~0ull && incl <= room) a.adm[ci] = 1;
  }
}

template <int NW = NWAVE>
LMGP_D uint64_t block_min(uint64_t v, uint64_t* sred) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, WAVE);
    v = o < v ? o : v;
  }
  if (lane_id() == 0) sred[threadIdx.x / WAVE] = v;
  __syncthreads();
  uint64_t r = sred[0];
  for (int i = 1; i < NW; ++i) r = sred[i] < r ? sred[i] : r;
  __syncthreads();
  return r;
}

template <int NW = NWAVE>
LMGP_D uint64_t block_max(uint64_t v, uint64_t* sred) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, WAVE);
    v = o > v ? o : v;
  }
  if (lane_id() == 0) sred[threadIdx.x / WAVE] = v;
  __syncthreads();
  uint64_t r = sred[0];
  for (int i = 1; i < NW; ++i) r = sred[i] > r ? sred[i] : r;
  __syncthreads();
  return r;
}

// Segments of more than 64 candidates: one block each.  Instead of sorting,
// a weighted MSB-first radix select finds the first key (in admission order)
// at which the summed node weight exceeds the room; every smaller key is
// admitted, which is exactly the longest fitting prefix (keys are unique).
// Each digit pass admits the candidates whose digit is below the threshold's,
// drops those above and carries only the ones that share it to the next pass
// (compacted into the segment's scratch, ping-pong with cpos), so the passes
// after the first touch few candidates.
constexpr int SEG_NT = 512;

__global__ __launch_bounds__(SEG_NT) void k_adm_seg(AdmitArgs a) {
  constexpr int NW = SEG_NT / WAVE;
  __shared__ unsigned long long whist[256];
  __shared__ uint64_t sred[NW];
  __shared__ int s_digit;
  __shared__ int64_t s_rem;
  __shared__ uint32_t s_cnt;
  // segments of at most 64 candidates: one wave each
  seg_waves(a, blockIdx.x * NW + threadIdx.x / WAVE, gridDim.x * NW);
  // larger segments: one block each
  const uint32_t nt = *a.ovcount;
  for (uint32_t j = blockIdx.x; j < nt; j += gridDim.x) {
    const uint32_t t = a.ovtgts[j];
    const uint32_t size = a.tally[t].ntgt;
    if (size <= WAVE) continue;
    const uint32_t base = a.segbase[t];
    // the segment's candidates as records (key, weight, slot) beside their
    // slots, written by the first pass; the digit passes read records, the
    // survivors as indices into them, ping-ponged between the segment's
    // slots (free once copied) and cpos (free once the segments are scattered)
    SegRec* rec = a.rec + base;
    uint32_t* in = a.seg + base;
    uint32_t* out = a.cpos + base;
    const uint32_t u0 = a.cands[in[0]].u;
    const int64_t room = a.gd[cand_graph(a, u0)].cap - a.W[t];
    // range of the keys: digits above the highest differing bit are shared
    uint64_t mnh = ~0ull, mxh = 0, mnl = ~0ull, mxl = 0;
    constexpr int U = 8;  // candidates per thread whose loads are issued together
    for (uint32_t i0 = threadIdx.x; i0 < size; i0 += U * SEG_NT) {
      uint32_t ci[U];
#pragma unroll
      for (int q = 0; q < U; ++q) ci[q] = i0 + q * SEG_NT < size ? in[i0 + q * SEG_NT] : ~0u;
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (ci[q] == ~0u) continue;
        const Cand c = a.cands[ci[q]];
        uint64_t h, l;
        cand_key(a, c, h, l);
        rec[i0 + q * SEG_NT] = SegRec{h, l, a.nw[c.u], ci[q], 0};
        mnh = h < mnh ? h : mnh;
        mxh = h > mxh ? h : mxh;
        mnl = l < mnl ? l : mnl;
        mxl = l > mxl ? l : mxl;
      }
    }
    mnh = block_min<NW>(mnh, sred);
    mxh = block_max<NW>(mxh, sred);
    mnl = block_min<NW>(mnl, sred);
    mxl = block_max<NW>(mxl, sred);
    // digit positions 15..0: 15..8 are the bytes of hi, 7..0 those of lo
    int top;
    if (mnh != mxh) top = 8 + (63 - __clzll(mnh ^ mxh)) / 8;
    else top = mnl != mxl ? (63 - __clzll(mnl ^ mxl)) / 8 : -1;
    int64_t rem = room;  // weight still admissible below the threshold
    uint32_t cur = size;  // candidates sharing the threshold's digits so far
    bool all = true;      // the survivors are every record (no index list yet)
    for (int pos = top; pos >= 0 && cur > 0; --pos) {
      for (int i = threadIdx.x; i < 256; i += SEG_NT) whist[i] = 0;
      if (threadIdx.x == 0) s_cnt = 0;
      __syncthreads();  // (also makes the first pass's records visible)
      const int sh = 8 * (pos & 7);
      for (uint32_t i0 = threadIdx.x; i0 < cur; i0 += U * SEG_NT) {
        uint32_t d[U];
        int64_t w[U];
        bool v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const uint32_t i = i0 + q * SEG_NT;
          v[q] = i < cur;
          if (!v[q]) continue;
          const SegRec r = rec[all ? i : in[i]];
          d[q] = (uint32_t)(((pos >= 8) ? r.hi : r.lo) >> sh) & 0xFF;
          w[q] = r.w;
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
          if (v[q]) atomicAdd(&whist[d[q]], (unsigned long long)w[q]);
      }
      __syncthreads();
      {
        // the threshold digit: the first one whose cumulative weight exceeds
        // rem (one block scan over the 256 bins; the survivors always weigh
        // more than rem, so exactly one digit qualifies)
        const uint64_t w = threadIdx.x < 256 ? whist[threadIdx.x] : 0;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t, NW>(w, sred, tot);
        if (threadIdx.x < 256 && (int64_t)ex <= rem && (int64_t)(ex + w) > rem) {
          s_digit = (int)threadIdx.x;
          s_rem = rem - (int64_t)ex;
        }
      }
      __syncthreads();
      const uint32_t dsel = (uint32_t)s_digit;
      for (uint32_t i0 = threadIdx.x; i0 < cur; i0 += U * SEG_NT) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const uint32_t i = i0 + q * SEG_NT;
          if (i >= cur) continue;
          const uint32_t j = all ? i : in[i];
          const SegRec r = rec[j];
          const uint32_t dg = (uint32_t)(((pos >= 8) ? r.hi : r.lo) >> sh) & 0xFF;
          if (dg < dsel) a.adm[r.ci] = 1;
          else if (dg == dsel) out[atomicAdd(&s_cnt, 1u)] = j;
        }
      }
      __syncthreads();
      rem = s_rem;
      cur = s_cnt;
      all = false;
      uint32_t* tmp = in;
      in = out;
      out = tmp;
      __syncthreads();
    }
    // what is left (one key: keys are unique) is the threshold: not admitted
  }
}

__global__ __launch_bounds__(256) void k_adm_apply(AdmitArgs a) {
  __shared__ int64_t sm[NWAVE];
  const uint32_t nc = a.plan ? a.plan->total : a.max_cands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t mv = 0;
  int64_t dn = 0;  // change of the non-empty cluster count by this move
  if (i < nc && a.adm[i]) {
    const Cand c = a.cands[i];
    const uint32_t t = c.tgt;
    const uint32_t own = a.label[c.u];
    const int64_t cu = a.nw[c.u];
    a.label[c.u] = t;
    if (a.label8) a.label8[c.u] = (uint8_t)t;
    if (a.ncl_part) {
      // weights are positive and only members leave, so a weight never drops
      // below zero: the target becomes non-empty iff it weighed 0 before this
      // add, the own cluster becomes empty iff it weighed exactly cu
      const int64_t ot =
          (int64_t)atomicAdd((unsigned long long*)&a.Wmut[t], (unsigned long long)cu);
      const int64_t oo =
          (int64_t)atomicAdd((unsigned long long*)&a.Wmut[own], (unsigned long long)(-cu));
      dn = (ot == 0 ? 1 : 0) - (oo == cu ? 1 : 0);
    } else {
      // a batch counts its clusters from W afterwards (k_count_clusters)
      atomicAdd((unsigned long long*)&a.Wmut[t], (unsigned long long)cu);
      atomicAdd((unsigned long long*)&a.Wmut[own], (unsigned long long)(-cu));
    }
    mv = 1;
    if (a.csize) {
      atomicAdd(&a.csize[t], 1u);
      atomicSub(&a.csize[own], 1u);
    }
    if (a.gid) mark_moved(a, a.gid[c.u]);
  }
  // clear the per-target scratch for the next sub-round (no kernel of this
  // admission reads it any more)
  if (i < nc && !a.few) {
    const uint32_t t = a.cands[i].tgt;
    if (t != EMPTY_KEY) {
      a.tally[t] = LabelTally{0, 0, 0};
    }
  }
  if (!a.gid && __ballot(mv != 0) && lane_id() == 0) mark_moved(a, 0);
  // every kernel of this admission that reads the overflow counters has run
  if (a.clear_ov && blockIdx.x == 0 && threadIdx.x == 0) a.ovtotal[0] = 0, a.ovcount[0] = 0;
  if (a.ncl_part) {
    const int64_t tot = block_reduce_sum(dn, sm);
    if (threadIdx.x == 0) a.ncl_part[blockIdx.x] = tot;
  }
}


// Non-empty clusters per graph after the moves.  Labels of one graph are
// contiguous, so a block's chunk spans few graphs: counts of the chunk's
// first graph stay in registers, the others go to LDS counters, and the
// block adds one total per graph (one counter per graph takes every block's
// add, so per-label or per-wave global atomics would serialise).
constexpr unsigned COUNT_BLOCKS = 1024;
constexpr uint32_t COUNT_SPAN = 256;

__global__ __launch_bounds__(256) void k_count_clusters(AdmitArgs a) {
  __shared__ uint32_t cnt[COUNT_SPAN];
  __shared__ uint32_t sm[NWAVE];
  const uint64_t n = a.nlabels;
  const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t k0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t k1 = k0 + chunk < n ? k0 + chunk : n;
  if (k0 >= k1) return;
  const uint32_t g0 = graph_of(a.gid, k0);
  const uint32_t span = graph_of(a.gid, k1 - 1) - g0 + 1;
  for (uint32_t i = threadIdx.x; i < COUNT_SPAN; i += 256) cnt[i] = 0;
  __syncthreads();
  uint32_t mine = 0;  // labels of graph g0
  for (uint64_t k = k0 + threadIdx.x; k < k1; k += 256) {
    if (a.Wmut[k] <= 0) continue;
    const uint32_t g = graph_of(a.gid, k);
    if (g == g0) ++mine;
    else if (span <= COUNT_SPAN) atomicAdd(&cnt[g - g0], 1u);
    else atomicAdd((unsigned long long*)&a.ncl_count[g], 1ull);
  }
  mine = block_reduce_sum(mine, sm);  // contains the barrier before cnt is read
  if (threadIdx.x == 0) cnt[0] += mine;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < span && i < COUNT_SPAN; i += 256)
    if (cnt[i]) atomicAdd((unsigned long long*)&a.ncl_count[g0 + i], (unsigned long long)cnt[i]);
}


}  // namespace

void launch_rate_hubs(int ew_kind, const RateArgs& a, Pool& pool, hipStream_t s) {
  if (a.count == 0) return;
  switch (ew_kind) {
    case EW_UNIT: launch_hubs_t<EW_UNIT>(a, pool, s); break;
    case EW_I32: launch_hubs_t<EW_I32>(a, pool, s); break;
    default: launch_hubs_t<EW_I64>(a, pool, s); break;
  }
}

void launch_rate_groups(int ew_kind, const RateArgs& a, const uint32_t* count,
                        const uint32_t* off, uint64_t degsum, hipStream_t s) {
  switch (ew_kind) {
    case EW_UNIT: launch_groups_t<EW_UNIT>(a, count, off, degsum, s); break;
    case EW_I32: launch_groups_t<EW_I32>(a, count, off, degsum, s); break;
    default: launch_groups_t<EW_I64>(a, count, off, degsum, s); break;
  }
}

void launch_rate(int cls, int ew_kind, const RateArgs& a, hipStream_t s) {
  switch (ew_kind) {
    case EW_UNIT: launch_rate_t<EW_UNIT>(cls, a, s); break;
    case EW_I32: launch_rate_t<EW_I32>(cls, a, s); break;
    default: launch_rate_t<EW_I64>(cls, a, s); break;
  }
}

void launch_bucket_count(const BucketArgs& a, hipStream_t s) {
  if (a.bkt && a.nbuckets > 255) throw InvalidArg("bucket ids do not fit a byte");
  if (a.nbuckets > MAX_BUCKETS) throw InvalidArg("too many sub-round buckets");
  unsigned g = grid_for(a.n, 256);
  if (g > 2048) g = 2048;
  k_bucket_count<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
}

void launch_bucket_offsets(const BucketArgs& a, hipStream_t s) {
  if (a.nbuckets > MAX_BUCKETS) throw InvalidArg("too many sub-round buckets");
  k_bucket_offsets<<<1, 64, 0, s>>>(a);
  LAUNCH_CHECK();
}

void launch_lp_plan(const unsigned long long* counts, const uint32_t* offs, uint32_t S, int dense,
                    SubPlan* plan, hipStream_t s) {
  if (S > 32 || S * NCLASS > MAX_BUCKETS) throw InvalidArg("too many sub-rounds for a plan");
  k_lp_plan<<<1, 64, 0, s>>>(counts, offs, S, dense, plan);
  LAUNCH_CHECK();
}

void launch_bucket_scatter(const BucketArgs& a, hipStream_t s) {
  if (a.nbuckets > MAX_BUCKETS) throw InvalidArg("too many sub-round buckets");
  unsigned g = grid_for(a.n, 256 * BK_ITEMS);
  if (a.ids && g > 1024) g = 1024;  // tiles strided over the list's length
  k_bucket_scatter<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
}

void launch_sub_list(const BucketArgs& a, const uint8_t* flag, uint32_t* block_cnt,
                     uint8_t* wsel, uint32_t* ids, unsigned long long* nids, hipStream_t s) {
  unsigned g = grid_for((a.n + 7) / 8, 256);
  if (g > SUB_BLOCKS) g = SUB_BLOCKS;
  k_sub_count<<<g, 256, 0, s>>>(a, flag, block_cnt, wsel);
  LAUNCH_CHECK();
  k_sub_write<<<g, 256, 0, s>>>(a, wsel, block_cnt, ids, nids);
  LAUNCH_CHECK();
}

void launch_admit(const AdmitArgs& a, hipStream_t s) {
  if (a.max_cands == 0) return;
  const unsigned g = grid_for(a.max_cands, 256);
  const bool few = a.few > 0 && a.few <= FEW_LABELS;
  const bool few_apply = few && !a.csize && !a.ncl_count;
  if (a.few > FEW_LABELS) throw InvalidArg("too many labels for the few-label admission");
  if (few) {
    const unsigned gi = grid_for(a.max_cands, 256 * ADM_ITEMS);
    k_adm_count_few<<<gi, 256, 0, s>>>(a);
    LAUNCH_CHECK();
    k_adm_classify_few<<<gi, 256, 0, s>>>(a);
  } else {
    k_adm_classify<<<g, 256, 0, s>>>(a);
  }
  LAUNCH_CHECK();
  k_adm_scatter<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
  // one wave per small segment, one block per segment above 64 candidates;
  // one block per CU at most (most launches find no segment at all, and
  // dispatching more blocks was most of their cost)
  unsigned gs = grid_for(a.max_cands, SEG_NT / WAVE);
  if (gs > 256) gs = 256;
  k_adm_seg<<<gs, SEG_NT, 0, s>>>(a);
  LAUNCH_CHECK();
  // apply (clearing the per-target scratch as it goes)
  if (few_apply) {
    k_adm_apply_few<<<grid_for(a.max_cands, 256 * ADM_ITEMS), 256, 0, s>>>(a);
  } else {
    k_adm_apply<<<g, 256, 0, s>>>(a);
    if (few) {
      LAUNCH_CHECK();
      k_adm_reset_few<<<grid_for(a.few, 256), 256, 0, s>>>(a);
    }
  }
  LAUNCH_CHECK();
  if (a.ncl_count && a.ncl_part) {
    // the caller's control kernel adds the apply blocks' changes
    if (few_apply) throw InvalidArg("cluster-count changes need the general apply");
  } else if (a.ncl_count && a.nlabels) {
    unsigned gc = grid_for(a.nlabels, 256 * 16);
    if (gc > COUNT_BLOCKS) gc = COUNT_BLOCKS;
    k_count_clusters<<<gc, 256, 0, s>>>(a);
    LAUNCH_CHECK();
  }
}

}  // namespace lmgp
