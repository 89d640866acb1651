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

LMGP_D void emit(const RateArgs& a, uint32_t u, const GraphDesc& gd, const Best& best,
                 int64_t r_own, int64_t cu) {
  if (a.mode == MODE_FAV) {
    a.fav[u] = best.r > 0 ? best.K : EMPTY_KEY;
    return;
  }
  if (best.r > r_own) {
    uint32_t i = atomicAdd(a.ncands, 1u);
    Cand c;
    c.u = u;
    c.tgt = best.K;
    c.hadm = (uint32_t)(hash_add(gd.pre_adm, (uint64_t)u - gd.node_base) >> 32);
    c.pad = 0;
    c.gain = best.r - r_own;
    a.cands[i] = c;
    atomicAdd((unsigned long long*)&a.demand[best.K], (unsigned long long)cu);
    atomicAdd(&a.ntgt[best.K], 1u);
  }
}

template <int T>
LMGP_D void lds_insert(uint32_t* key, unsigned long long* val, uint32_t K, uint64_t w) {
  constexpr int LOGT = __builtin_ctz(T);
  uint32_t s = (K * 0x9E3779B1u) >> (32 - LOGT);
  while (true) {
    uint32_t prev = atomicCAS(&key[s], EMPTY_KEY, K);
    if (prev == EMPTY_KEY || prev == K) {
      atomicAdd(&val[s], (unsigned long long)w);
      return;
    }
    s = (s + 1) & (T - 1);
  }
}

// Lane groups of G lanes (G <= 64) rate one node each; degree <= 2G, table 4G.
template <int G, int EWK>
__global__ __launch_bounds__(256) void k_rate_group(RateArgs a) {
  constexpr int T = 4 * G;
  constexpr int GPB = 256 / G;
  __shared__ uint32_t skey[GPB * T];
  __shared__ unsigned long long sval[GPB * T];
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  uint32_t* key = skey + grp * T;
  unsigned long long* val = sval + grp * T;
  const uint64_t idx = (uint64_t)blockIdx.x * GPB + grp;
  bool valid = idx < a.count;
  const uint32_t u = valid ? a.list[idx] : 0u;
  // graphs of a batch may stop in the middle of a round
  if (valid && a.gid && !a.gd[a.gid[u]].active) valid = false;
#pragma unroll
  for (int s = gl; s < T; s += G) {
    key[s] = EMPTY_KEY;
    val[s] = 0;
  }
  wave_sync();
  uint64_t beg = 0, end = 0;
  if (valid) {
    beg = a.xadj[u];
    end = a.xadj[u + 1];
  }
  for (uint64_t e = beg + gl; e < end; e += G) {
    uint32_t K = a.label[a.adj[e]];
    lds_insert<T>(key, val, K, (uint64_t)edge_w<EWK>(a.ew, e));
  }
  wave_sync();
  Best best{0, 0, 0};
  int64_t r_own = 0;
  GraphDesc gd{};
  uint32_t own = 0;
  int64_t cu = 0;
  if (valid) {
    gd = a.gd[graph_of(a.gid, u)];
    own = a.label[u];
    cu = a.nw[u];
    const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
#pragma unroll
    for (int s = gl; s < T; s += G) {
      uint32_t K = key[s];
      if (K != EMPTY_KEY)
        consider(a, K, (int64_t)val[s], own, cu, gd.cap, pre_u, gd.label_base, best, r_own);
    }
  }
  reduce_best<G>(best, r_own);
  if (valid && gl == 0) emit(a, u, gd, best, r_own, cu);
}

// One 256-thread block per node; degree <= 2048, LDS table of 4096 slots.
template <int EWK>
__global__ __launch_bounds__(256) void k_rate_block(RateArgs a) {
  constexpr int T = BLOCK_TABLE;
  __shared__ uint32_t key[T];
  __shared__ unsigned long long val[T];
  __shared__ Best sb[NWAVE];
  __shared__ int64_t so[NWAVE];
  const uint64_t idx = blockIdx.x;
  if (idx >= a.count) return;
  const uint32_t u = a.list[idx];
  if (a.gid && !a.gd[a.gid[u]].active) return;
  for (int s = threadIdx.x; s < T; s += 256) {
    key[s] = EMPTY_KEY;
    val[s] = 0;
  }
  __syncthreads();
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  for (uint64_t e = beg + threadIdx.x; e < end; e += 256)
    lds_insert<T>(key, val, a.label[a.adj[e]], (uint64_t)edge_w<EWK>(a.ew, e));
  __syncthreads();
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const uint32_t own = a.label[u];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (int s = threadIdx.x; s < T; s += 256) {
    uint32_t K = key[s];
    if (K != EMPTY_KEY)
      consider(a, K, (int64_t)val[s], own, cu, gd.cap, pre_u, gd.label_base, best, r_own);
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
    emit(a, u, gd, best, r_own, cu);
  }
}

// One block per node with a rating table in global memory (degree > 2048).
template <int EWK>
__global__ __launch_bounds__(256) void k_rate_global(RateArgs a) {
  __shared__ Best sb[NWAVE];
  __shared__ int64_t so[NWAVE];
  const uint64_t idx = blockIdx.x;
  if (idx >= a.count) return;
  const uint32_t u = a.list[idx];
  if (a.gid && !a.gd[a.gid[u]].active) return;
  const uint64_t beg = a.xadj[u], end = a.xadj[u + 1];
  uint64_t T = 1;
  while (T < 2 * (end - beg)) T <<= 1;
  uint32_t* key = a.gkeys + a.goff[idx];
  unsigned long long* val = (unsigned long long*)(a.gvals + a.goff[idx]);
  for (uint64_t s = threadIdx.x; s < T; s += 256) {
    key[s] = EMPTY_KEY;
    val[s] = 0;
  }
  __syncthreads();
  for (uint64_t e = beg + threadIdx.x; e < end; e += 256) {
    uint32_t K = a.label[a.adj[e]];
    uint64_t w = (uint64_t)edge_w<EWK>(a.ew, e);
    uint64_t s = ((uint64_t)K * 0x9E3779B97F4A7C15ull) & (T - 1);
    while (true) {
      uint32_t prev = atomicCAS(&key[s], EMPTY_KEY, K);
      if (prev == EMPTY_KEY || prev == K) {
        atomicAdd(&val[s], (unsigned long long)w);
        break;
      }
      s = (s + 1) & (T - 1);
    }
  }
  __syncthreads();
  const GraphDesc gd = a.gd[graph_of(a.gid, u)];
  const uint32_t own = a.label[u];
  const int64_t cu = a.nw[u];
  const uint64_t pre_u = hash_add(gd.pre_tie, (uint64_t)u - gd.node_base);
  Best best{0, 0, 0};
  int64_t r_own = 0;
  for (uint64_t s = threadIdx.x; s < T; s += 256) {
    uint32_t K = __hip_atomic_load(&key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (K == EMPTY_KEY) continue;
    int64_t r = (int64_t)__hip_atomic_load(&val[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    consider(a, K, r, own, cu, gd.cap, pre_u, gd.label_base, best, r_own);
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
    emit(a, u, gd, best, r_own, cu);
  }
}

const char* rate_name(int cls, int ewk) {
  static const char* names[3][NCLASS] = {
      {"lp_rate_g2_unit", "lp_rate_g4_unit", "lp_rate_g8_unit", "lp_rate_g16_unit",
       "lp_rate_g32_unit", "lp_rate_g64_unit", "lp_rate_block_unit", "lp_rate_global_unit"},
      {"lp_rate_g2_i32", "lp_rate_g4_i32", "lp_rate_g8_i32", "lp_rate_g16_i32",
       "lp_rate_g32_i32", "lp_rate_g64_i32", "lp_rate_block_i32", "lp_rate_global_i32"},
      {"lp_rate_g2_i64", "lp_rate_g4_i64", "lp_rate_g8_i64", "lp_rate_g16_i64",
       "lp_rate_g32_i64", "lp_rate_g64_i64", "lp_rate_block_i64", "lp_rate_global_i64"}};
  return names[ewk][cls];
}

// Algorithmic bytes of rating `count` nodes with `degsum` entries: per node the
// two offsets, its list slot, label and weight (32 B); per entry the neighbour
// id, its label and the edge weight (if stored).
uint64_t rate_bytes(int ewk, uint64_t count, uint64_t degsum) {
  const uint64_t bw = ewk == EW_UNIT ? 0 : ewk == EW_I32 ? 4 : 8;
  return 32 * count + (8 + bw) * degsum;
}

template <int EWK>
void launch_rate_t(int cls, const RateArgs& a, hipStream_t s) {
  if (a.count == 0) return;
  ProfScope prof(rate_name(cls, EWK), rate_bytes(EWK, a.count, a.degsum), s);
  if (cls < CLASS_BLOCK) {
    const int G = class_group(cls);
    const unsigned grid = grid_for(a.count, 256 / G);
    switch (G) {
      case 2: k_rate_group<2, EWK><<<grid, 256, 0, s>>>(a); break;
      case 4: k_rate_group<4, EWK><<<grid, 256, 0, s>>>(a); break;
      case 8: k_rate_group<8, EWK><<<grid, 256, 0, s>>>(a); break;
      case 16: k_rate_group<16, EWK><<<grid, 256, 0, s>>>(a); break;
      case 32: k_rate_group<32, EWK><<<grid, 256, 0, s>>>(a); break;
      default: k_rate_group<64, EWK><<<grid, 256, 0, s>>>(a); break;
    }
  } else if (cls == CLASS_BLOCK) {
    k_rate_block<EWK><<<a.count, 256, 0, s>>>(a);
  } else {
    k_rate_global<EWK><<<a.count, 256, 0, s>>>(a);
  }
  LAUNCH_CHECK();
}

// ------------------------------------------------------------- bucketing --
LMGP_D int bucket_of(const BucketArgs& a, uint64_t u) {
  const uint32_t g = graph_of(a.gid, u);
  const GraphDesc& gd = a.gd[g];
  if (!gd.active) return -1;
  const uint64_t d = a.xadj[u + 1] - a.xadj[u];
  if (d == 0) return -1;
  if (a.mode == 0) {
    uint32_t sr = subround_of(hash_add(gd.pre_sub, u - gd.node_base), gd.subrounds);
    return (int)(sr * NCLASS + degree_class(d));
  }
  // 2-hop: light singletons with neighbours
  if (a.csize[a.label[u]] != 1) return -1;
  if (2 * a.nw[u] > gd.cap) return -1;
  return degree_class(d);
}

__global__ __launch_bounds__(256) void k_bucket_count(BucketArgs a) {
  __shared__ uint32_t h[256];
  __shared__ unsigned long long hd[256];
  h[threadIdx.x] = 0;
  hd[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < a.n; u += stride) {
    int b = bucket_of(a, u);
    if (b >= 0) {
      atomicAdd(&h[b], 1u);
      atomicAdd(&hd[b], (unsigned long long)(a.xadj[u + 1] - a.xadj[u]));
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < a.nbuckets; i += 256)
    if (h[i]) {
      atomicAdd(&a.counts[i], h[i]);
      if (a.degs) atomicAdd(&a.degs[i], hd[i]);
    }
}

__global__ __launch_bounds__(256) void k_bucket_scatter(BucketArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t lt = lanemask_lt();
  // iterate whole waves so that the ballots below are convergent
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < a.n; base += stride) {
    const uint64_t u = base + threadIdx.x;
    int b = u < a.n ? bucket_of(a, u) : -1;
    uint64_t pending = __ballot(b >= 0);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int lb = __shfl(b, leader);
      const uint64_t peers = __ballot(b == lb) & pending;
      uint32_t basepos = 0;
      if (lane_id() == leader) basepos = atomicAdd(&a.fill[lb], (uint32_t)__popcll(peers));
      basepos = __shfl(basepos, leader);
      if ((peers >> lane_id()) & 1ull) {
        a.list[a.offs[lb] + basepos + (uint32_t)__popcll(peers & lt)] = (uint32_t)u;
      }
      pending &= ~peers;
    }
  }
}

// ------------------------------------------------------------- admission --
LMGP_D uint32_t cand_graph(const AdmitArgs& a, uint32_t u) { return graph_of(a.gid, u); }

__global__ __launch_bounds__(256) void k_adm_classify(AdmitArgs a) {
  const uint32_t nc = *a.ncands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const Cand c = a.cands[i];
  const int64_t cap = a.gd[cand_graph(a, c.u)].cap;
  const uint32_t t = c.tgt;
  if (a.W[t] + a.demand[t] <= cap) {
    a.adm[i] = 1;  // everything aimed at t fits
    return;
  }
  a.adm[i] = 0;
  const uint32_t p = atomicAdd(&a.fill[t], 1u);
  a.cpos[i] = p;
  if (p == 0) {
    a.segbase[t] = atomicAdd(a.ovtotal, a.ntgt[t]);
    a.ovtgts[atomicAdd(a.ovcount, 1u)] = t;
  }
}

__global__ __launch_bounds__(256) void k_adm_scatter(AdmitArgs a) {
  const uint32_t nc = *a.ncands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc || a.adm[i]) return;
  a.seg[a.segbase[a.cands[i].tgt] + a.cpos[i]] = i;
}

// Admission order key: (gain desc, hadm asc, u asc) as two uint64 words.
LMGP_D void cand_key(const Cand& c, uint64_t& hi, uint64_t& lo) {
  hi = (uint64_t)INT64_MAX - (uint64_t)c.gain;
  lo = ((uint64_t)c.hadm << 32) | c.u;
}
LMGP_D bool key_less(uint64_t ahi, uint64_t alo, uint64_t bhi, uint64_t blo) {
  return ahi < bhi || (ahi == bhi && alo < blo);
}

// Segments of at most 64 candidates: one wave, bitonic sort in registers.
__global__ __launch_bounds__(256) void k_adm_seg_wave(AdmitArgs a) {
  const uint32_t nt = *a.ovcount;
  const uint32_t waves = gridDim.x * (blockDim.x / WAVE);
  const int l = lane_id();
  for (uint32_t j = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; j < nt; j += waves) {
    const uint32_t t = a.ovtgts[j];
    const uint32_t size = a.ntgt[t];
    if (size > WAVE) continue;
    const uint32_t base = a.segbase[t];
    const bool valid = (uint32_t)l < size;
    uint32_t ci = valid ? a.seg[base + l] : 0u;
    uint64_t khi = ~0ull, klo = ~0ull;
    int64_t w = 0;
    if (valid) {
      Cand c = a.cands[ci];
      cand_key(c, khi, klo);
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

// Larger segments: one block each; LDS bitonic sort up to 1024 entries,
// in-place bitonic sort over global memory beyond that.
constexpr int SEG_LDS = 1024;

__global__ __launch_bounds__(256) void k_adm_seg_block(AdmitArgs a) {
  __shared__ uint64_t shi[SEG_LDS], slo[SEG_LDS];
  __shared__ uint32_t sci[SEG_LDS];
  __shared__ int64_t sm[NWAVE];
  __shared__ int64_t carry;
  const uint32_t nt = *a.ovcount;
  for (uint32_t j = blockIdx.x; j < nt; j += gridDim.x) {
    const uint32_t t = a.ovtgts[j];
    const uint32_t size = a.ntgt[t];
    if (size <= WAVE) continue;
    const uint32_t base = a.segbase[t];
    uint32_t N = 1;
    while (N < size) N <<= 1;
    const bool in_lds = size <= SEG_LDS;
    if (in_lds) {
      for (uint32_t i = threadIdx.x; i < N; i += 256) {
        if (i < size) {
          uint32_t ci = a.seg[base + i];
          cand_key(a.cands[ci], shi[i], slo[i]);
          sci[i] = ci;
        } else {
          shi[i] = ~0ull;
          slo[i] = ~0ull;
          sci[i] = 0;
        }
      }
      __syncthreads();
      for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j2 = k >> 1; j2 > 0; j2 >>= 1) {
          for (uint32_t i = threadIdx.x; i < N; i += 256) {
            const uint32_t p = (j2 == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j2);
            if (p > i && key_less(shi[p], slo[p], shi[i], slo[i])) {
              uint64_t th = shi[i], tl = slo[i];
              uint32_t tc = sci[i];
              shi[i] = shi[p], slo[i] = slo[p], sci[i] = sci[p];
              shi[p] = th, slo[p] = tl, sci[p] = tc;
            }
          }
          __syncthreads();
        }
      }
    } else {
      uint32_t* sg = a.seg + base;
      for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j2 = k >> 1; j2 > 0; j2 >>= 1) {
          for (uint32_t i = threadIdx.x; i < N; i += 256) {
            const uint32_t p = (j2 == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j2);
            if (p > i && p < size) {
              uint64_t ih, il, ph, pl;
              cand_key(a.cands[sg[i]], ih, il);
              cand_key(a.cands[sg[p]], ph, pl);
              if (key_less(ph, pl, ih, il)) {
                uint32_t tc = sg[i];
                sg[i] = sg[p];
                sg[p] = tc;
              }
            }
          }
          __threadfence_block();
          __syncthreads();
        }
      }
    }
    // prefix sums of node weights in sorted order, admit while within room
    const uint32_t u0 = a.cands[a.seg[base]].u;
    const int64_t room = a.gd[cand_graph(a, u0)].cap - a.W[t];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t off = 0; off < size; off += 256) {
      const uint32_t i = off + threadIdx.x;
      uint32_t ci = 0;
      int64_t w = 0;
      if (i < size) {
        ci = in_lds ? sci[i] : a.seg[base + i];
        w = a.nw[a.cands[ci].u];
      }
      int64_t tot;
      int64_t ex = block_exclusive_scan(w, sm, tot);
      const int64_t incl = carry + ex + w;
      if (i < size && incl <= room) a.adm[ci] = 1;
      __syncthreads();
      if (threadIdx.x == 0) carry += tot;
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_adm_apply(AdmitArgs a) {
  const uint32_t nc = *a.ncands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const Cand c = a.cands[i];
  const uint32_t t = c.tgt;
  if (a.adm[i]) {
    const uint32_t g = cand_graph(a, c.u);
    const uint32_t own = a.label[c.u];
    const int64_t cu = a.nw[c.u];
    a.label[c.u] = t;
    const int64_t old_t = (int64_t)atomicAdd((unsigned long long*)&a.Wmut[t], (unsigned long long)cu);
    const int64_t old_o =
        (int64_t)atomicAdd((unsigned long long*)&a.Wmut[own], (unsigned long long)(-cu));
    atomicAdd((unsigned long long*)&a.moves[g], 1ull);
    if (a.ncl_delta) {
      // clusters that become empty / non-empty; the sum over all moves is
      // order independent because W never goes negative
      int64_t d = (old_t == 0 ? 1 : 0) - (old_o == cu ? 1 : 0);
      if (d) atomicAdd((unsigned long long*)&a.ncl_delta[g], (unsigned long long)d);
    }
    if (a.csize) {
      atomicAdd(&a.csize[t], 1u);
      atomicSub(&a.csize[own], 1u);
    }
  }
}

// Reset the per-target scratch for the next sub-round (after every reader).
__global__ __launch_bounds__(256) void k_adm_reset(AdmitArgs a) {
  const uint32_t nc = *a.ncands;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const uint32_t t = a.cands[i].tgt;
  a.demand[t] = 0;
  a.ntgt[t] = 0;
  a.fill[t] = 0;
}

}  // namespace

void launch_rate(int cls, int ew_kind, const RateArgs& a, hipStream_t s) {
  switch (ew_kind) {
    case EW_UNIT: launch_rate_t<EW_UNIT>(cls, a, s); break;
    case EW_I32: launch_rate_t<EW_I32>(cls, a, s); break;
    default: launch_rate_t<EW_I64>(cls, a, s); break;
  }
}

void launch_bucket_count(const BucketArgs& a, hipStream_t s) {
  unsigned g = grid_for(a.n, 256);
  if (g > 2048) g = 2048;
  k_bucket_count<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
}

void launch_bucket_scatter(const BucketArgs& a, hipStream_t s) {
  unsigned g = grid_for(a.n, 256);
  if (g > 2048) g = 2048;
  k_bucket_scatter<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
}

void launch_admit(const AdmitArgs& a, hipStream_t s) {
  if (a.max_cands == 0) return;
  const unsigned g = grid_for(a.max_cands, 256);
  k_adm_classify<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
  k_adm_scatter<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
  unsigned gs = grid_for(a.max_cands, 4);
  if (gs > 1024) gs = 1024;
  k_adm_seg_wave<<<gs, 256, 0, s>>>(a);
  LAUNCH_CHECK();
  unsigned gb = a.max_cands < 1024 ? a.max_cands : 1024;
  k_adm_seg_block<<<gb, 256, 0, s>>>(a);
  LAUNCH_CHECK();
  k_adm_apply<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
  k_adm_reset<<<g, 256, 0, s>>>(a);
  LAUNCH_CHECK();
}

}  // namespace lmgp
