// Cluster contraction (Sec. 2): cluster C becomes a coarse node of weight
// c(C); clusters joined by edges get one coarse edge whose weight is the sum
// of the joining edge weights.  Coarse ids are the ranks of the non-empty
// labels in ascending label order; coarse rows are sorted and duplicate-free.
//
// Layout: the members of every coarse node are bucketed (counting sort);
// each coarse row gathers the mapped neighbours of its members and sums the
// weights of equal neighbour ids.  On the coarsening path the sums are formed
// in an LDS hash table and written in table order (no consumer depends on the
// order of a row); where order matters (the coarsest level handed to the
// initial partitioning, exported levels) rows are sorted: by neighbour id,
// then equal ids summed.  Rows of <= 64 fine entries are
// sorted in registers by one wavefront, rows of <= 2048 in LDS by one block,
// rows of <= 16384 (when every edge weight fits in 32 bits) as packed
// (neighbour << 32 | weight) words in LDS by one 1024-thread block, larger
// rows by the device-wide radix sort.  Rows are first written to a
// scratch area at offset prefix(sum of member degrees), then compacted.
#include <cstdlib>
#include <cstring>

#include <type_traits>

#include "contract.h"
#include "profiler.h"

namespace lmgp {

namespace {

constexpr int ROW_A = WAVE;   // <= 64 entries: wave
constexpr int ROW_B = 2048;   // <= 2048 entries: block, LDS
constexpr int ROW_C = 8192;   // <= 8192 entries: 1024-thread block, packed LDS words
constexpr int ROW_D = 16384;  // <= 16384 entries: the same with a 128 KiB LDS array
constexpr int NROWCLS = 13;
// Row classes.  Sorted: 0 wave, 1 block bitonic, 3/4 big bitonic (packed),
// 2 radix.  Hash aggregation: lane groups of 16, 32 and 64 lanes for <= 32,
// <= 64 and <= 128 entries (9, 10, 11), 12 a 128-thread block <= 256, 5 a
// 256-thread block <= 512 entries, 6 block <= 2048, 7 big <= 6144 and 8 big
// <= 12288 (packed), 2 radix.
LMGP_D int row_class(uint64_t d, int packed, int sorted) {
  if (!sorted && d <= 256) return d <= 32 ? 9 : d <= 64 ? 10 : d <= 128 ? 11 : 12;
  if (d <= ROW_A) return 0;
  if (sorted) {
    if (d <= ROW_B) return 1;
    if (packed && d <= ROW_C) return 3;
    if (packed && d <= ROW_D) return 4;
    return 2;
  }
  if (d <= 512) return 5;
  if (d <= ROW_B) return 6;
  if (packed && d <= 6144) return 7;
  if (packed && d <= 12288) return 8;
  return 2;
}

__global__ void k_gather_u32(const uint32_t* a, const uint64_t* idx, uint64_t n, uint32_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[idx[i]];
}

__global__ void k_map(const uint32_t* label, const uint32_t* cid, const uint32_t* gid,
                      const uint8_t* keep, uint64_t n, uint32_t* map) {
  uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  map[u] = keep[graph_of(gid, u)] ? cid[label[u]] : EMPTY_KEY;
}

// Members per label, counted from the labels of the kept graphs.
__global__ void k_label_count(const uint32_t* label, const uint32_t* gid, const uint8_t* keep,
                              uint64_t n, uint32_t* lcount) {
  uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  if (keep[graph_of(gid, u)]) atomicAdd(&lcount[label[u]], 1u);
}

// The same counts from the member counts the clustering kept (labels are node
// ids of their own graph, so K's graph is K's): a streaming pass, no atomics.
__global__ void k_label_count_sizes(const uint32_t* csize, const uint32_t* gid,
                                    const uint8_t* keep, uint64_t n, uint32_t* lcount) {
  const uint64_t K = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K < n) lcount[K] = keep[graph_of(gid, K)] ? csize[K] : 0u;
}

// For every used label K: coarse weight, member count, graph.
__global__ void k_coarse_nodes(const int64_t* W, const uint32_t* lcount, const uint32_t* cid,
                               const uint32_t* gid, uint64_t n, int64_t* cnw, uint32_t* ccount,
                               uint32_t* cgid) {
  uint64_t K = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n) return;
  if (lcount[K] > 0) {
    const uint32_t x = cid[K];
    cnw[x] = W[K];
    ccount[x] = lcount[K];
    if (cgid) cgid[x] = graph_of(gid, K);
  }
}

// Members of each coarse node (in any order: every consumer is order
// independent) and the summed degree of each.  Lanes holding consecutive
// nodes of one coarse node form a run; the run's last lane takes the slots
// and adds the degrees for the whole run (one pair of atomics per run).
__global__ __launch_bounds__(256) void k_members(const uint64_t* xadj, const uint32_t* map,
                                                 uint64_t n, const uint64_t* mstart, uint32_t* mfill,
                                                 uint32_t* members, unsigned long long* degsum) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = lane_id();
  const uint32_t x = u < n ? map[u] : EMPTY_KEY;
  const uint64_t d = u < n && x != EMPTY_KEY ? xadj[u + 1] - xadj[u] : 0;
  const uint32_t xp = __shfl_up(x, 1);
  const uint32_t xn = __shfl_down(x, 1);
  const uint64_t heads = __ballot(l == 0 || xp != x);
  const bool tail = l == WAVE - 1 || xn != x;
  // the run [h, t] holding this lane
  const uint64_t below = heads & ((2ull << l) - 1);  // heads at lanes <= l (l's own included)
  const int h = 63 - __clzll(below);
  const uint64_t above = heads & ~((2ull << l) - 1);
  const int t = above ? __ffsll((long long)above) - 2 : WAVE - 1;
  const uint64_t incl = wave_inclusive_scan(d);
  // every lane takes part in the shuffle (a lane left out of it would read 0
  // from a source lane that is)
  const uint64_t at_prev = __shfl(incl, h > 0 ? h - 1 : 0);
  const uint64_t before = h > 0 ? at_prev : 0;
  uint32_t base = 0;
  if (tail && x != EMPTY_KEY) {
    base = atomicAdd(&mfill[x], (uint32_t)(t - h + 1));
    const uint64_t run_deg = incl - before;
    if (run_deg) atomicAdd(&degsum[x], (unsigned long long)run_deg);
  }
  base = __shfl(base, t);
  if (x != EMPTY_KEY) members[mstart[x] + base + (uint32_t)(l - h)] = (uint32_t)u;
}

// Row size classes (see row_class), counted per block and listed.
__global__ __launch_bounds__(256) void k_row_classes(const unsigned long long* degsum, uint64_t nc,
                                                     int packed, int sorted, uint32_t* counts,
                                                     uint32_t* lists, uint64_t cap) {
  __shared__ uint32_t lc[NROWCLS], base[NROWCLS];
  if (threadIdx.x < NROWCLS) lc[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  uint32_t lp = 0;
  if (x < nc) {
    const uint64_t d = degsum[x];
    c = row_class(d, packed, sorted);
    lp = atomicAdd(&lc[c], 1u);
  }
  __syncthreads();
  if (threadIdx.x < NROWCLS && lc[threadIdx.x])
    base[threadIdx.x] = atomicAdd(&counts[threadIdx.x], lc[threadIdx.x]);
  __syncthreads();
  if (c >= 0) lists[(uint64_t)c * cap + base[c] + lp] = (uint32_t)x;
}

template <int EWK>
LMGP_D void load_entry(const ContractArgs& a, uint64_t e, uint32_t x, uint32_t& key, int64_t& w) {
  const uint32_t y = a.map[a.adj[e]];
  if (y == x) {
    key = EMPTY_KEY;
    w = 0;
  } else {
    key = y;
    w = edge_w<EWK>(a.ew, e);
  }
}

// Rows with <= 64 fine entries: one wave per row.
template <int EWK>
__global__ __launch_bounds__(256) void k_rows_wave(ContractArgs a, const uint32_t* rows,
                                                   uint32_t nrows) {
  const uint32_t r = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (r >= nrows) return;  // uniform per wave
  const int l = lane_id();
  const uint32_t x = rows[r];
  const uint64_t m0 = a.mstart[x], m1 = a.mstart[x + 1];
  uint32_t key = EMPTY_KEY;
  int64_t w = 0;
  uint64_t pos = 0;  // entries gathered so far (uniform)
  for (uint64_t mb = m0; mb < m1; mb += WAVE) {
    const uint64_t mi = mb + l;
    uint64_t beg = 0, d = 0;
    if (mi < m1) {
      const uint32_t u = a.members[mi];
      beg = a.xadj[u];
      d = a.xadj[u + 1] - beg;
    }
    const uint64_t incl = wave_inclusive_scan(d);
    const uint64_t excl = incl - d;
    const uint64_t tot = __shfl(incl, WAVE - 1);
    // lane l takes entry t = l - pos of this chunk, owned by the last member
    // whose exclusive offset is <= t
    const int64_t t = (int64_t)l - (int64_t)pos;
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int c = lo + step;
      const uint64_t ex = __shfl(excl, c < WAVE ? c : WAVE - 1);
      const bool ok_lane = c < WAVE && (mb + (uint64_t)c) < m1;
      if (ok_lane && t >= 0 && (uint64_t)t >= ex) lo = c;
    }
    const uint64_t mbeg = __shfl(beg, lo);
    const uint64_t mex = __shfl(excl, lo);
    if (t >= 0 && (uint64_t)t < tot) load_entry<EWK>(a, mbeg + ((uint64_t)t - mex), x, key, w);
    pos += tot;
  }
  // bitonic sort of (key, w) across the wave
  for (int k = 2; k <= WAVE; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int p = (j == (k >> 1)) ? (l ^ (k - 1)) : (l ^ j);
      const uint32_t ok = __shfl(key, p);
      const int64_t ow = __shfl(w, p);
      const bool take = (l < p) ? (ok < key) : (key < ok);
      if (take) key = ok, w = ow;
    }
  }
  // sum runs of equal keys
  const uint32_t prev = __shfl_up(key, 1);
  const bool valid = key != EMPTY_KEY;
  const bool head = valid && (l == 0 || prev != key);
  const uint64_t hmask = __ballot(head);
  const uint64_t le = lanemask_lt() | (1ull << l);
  const int runstart = valid ? 63 - __clzll(hmask & le) : l;
  int64_t s = w;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int64_t o = __shfl_up(s, d);
    if (l - d >= runstart) s += o;
  }
  const uint32_t next = __shfl_down(key, 1);
  const bool tail = valid && (l == WAVE - 1 || next != key);
  const uint64_t tmask = __ballot(tail);
  const uint64_t base = a.tmpoff[x];
  if (tail) {
    const uint64_t o = base + (uint64_t)__popcll(tmask & lanemask_lt());
    a.tkey[o] = key;
    a.tw[o] = s;
    if (a.tsrc) a.tsrc[o] = x;
  }
  const uint32_t nd = (uint32_t)__popcll(tmask);
  if (l == 0) a.ndist[x] = nd;
}

template <int G, class T>
LMGP_D T group_inclusive_scan(T v) {
  const int gl = lane_id() % G;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const T o = __shfl_up(v, d, G);
    if (gl >= d) v += o;
  }
  return v;
}

// Rows with at most 2G fine entries (unsorted output): a group of G lanes
// per row, 256 / G rows per block, an LDS hash table of 4G slots per row;
// the distinct entries are written in slot order.  Entry positions: every
// member with entries marks its first position in the group's bit mask and
// stores (row start - position) there, so the entry at position t belongs
// to the highest mark at or below t.
template <int EWK, int G>
__global__ __launch_bounds__(256) void k_rows_group(ContractArgs a, const uint32_t* rows,
                                                    uint32_t nrows) {
  constexpr int T = 4 * G, GPB = 256 / G, P = 2 * G, MW = (P + 63) / 64;
  __shared__ uint32_t skey[GPB * T];
  __shared__ unsigned long long sval[GPB * T];
  __shared__ uint64_t sbase[GPB * P];
  __shared__ unsigned long long smask[GPB * MW];
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  uint32_t* key = skey + grp * T;
  unsigned long long* val = sval + grp * T;
  uint64_t* mbase = sbase + grp * P;
  unsigned long long* mask = smask + grp * MW;
  const uint32_t r = blockIdx.x * GPB + grp;
  const bool valid = r < nrows;
#pragma unroll
  for (int i = gl; i < T; i += G) {
    key[i] = EMPTY_KEY;
    val[i] = 0;
  }
  uint32_t x = 0;
  uint64_t m0 = 0, m1 = 0;
  if (valid) {
    x = rows[r];
    m0 = a.mstart[x];
    m1 = a.mstart[x + 1];
  }
  // members in chunks of G (the row's entries, and so each chunk's, number
  // at most P = 2G): lane l takes positions l and l + G of the chunk
  for (uint64_t mb = m0; mb < m1; mb += G) {
    if (gl < MW) mask[gl] = 0;
    wave_sync();
    const uint64_t mi = mb + gl;
    uint64_t beg = 0;
    uint32_t d = 0;
    if (mi < m1) {
      const uint32_t u = a.members[mi];
      beg = a.xadj[u];
      d = (uint32_t)(a.xadj[u + 1] - beg);
    }
    const uint32_t incl = group_inclusive_scan<G>(d);
    const uint32_t excl = incl - d;
    const uint32_t tot = __shfl(incl, G - 1, G);
    if (d) {  // excl + d <= tot <= P, so excl < P
      mbase[excl] = beg - excl;
      atomicOr(&mask[excl >> 6], 1ull << (excl & 63));
    }
    wave_sync();
    unsigned long long mk[MW];
#pragma unroll
    for (int q = 0; q < MW; ++q) mk[q] = mask[q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t t = (uint32_t)gl + (uint32_t)h * G;
      uint32_t k = EMPTY_KEY;
      int64_t w = 0;
      if (t < tot) {
        // the first member with entries starts at 0, so a mark <= t exists
        uint32_t st;
        if (MW == 1 || t < 64) {
          const unsigned long long below = mk[0] & (~0ull >> (63 - (t & 63)));
          st = 63u - (uint32_t)__clzll(below);
        } else {
          const unsigned long long hi = mk[MW - 1] & (~0ull >> (63 - (t & 63)));
          st = hi ? 127u - (uint32_t)__clzll(hi) : 63u - (uint32_t)__clzll(mk[0]);
        }
        load_entry<EWK>(a, mbase[st] + t, x, k, w);
      }
      if (k != EMPTY_KEY) {
        uint32_t sl = (k * 0x9E3779B1u) >> (32 - __builtin_ctz(T));
        bool hit;
        do {
          const uint32_t prev = atomicCAS(&key[sl], EMPTY_KEY, k);
          hit = prev == EMPTY_KEY || prev == k;
          sl = hit ? sl : (sl + 1) & (T - 1);
        } while (!hit);
        atomicAdd(&val[sl], (unsigned long long)w);
      }
    }
    wave_sync();
  }
  wave_sync();
  if (!valid) return;
  // occupied slots -> consecutive outputs (each lane owns 4 slots)
  constexpr int SPL = T / G;
  uint32_t kk[SPL];
  int n = 0;
#pragma unroll
  for (int j = 0; j < SPL; ++j) {
    kk[j] = key[gl * SPL + j];
    n += kk[j] != EMPTY_KEY;
  }
  const int incl = group_inclusive_scan<G>(n);
  const int nd = __shfl(incl, G - 1, G);
  const uint64_t base = a.tmpoff[x];
  uint64_t o = base + (uint64_t)(incl - n);
#pragma unroll
  for (int j = 0; j < SPL; ++j)
    if (kk[j] != EMPTY_KEY) {
      a.tkey[o] = kk[j];
      a.tw[o] = (int64_t)val[gl * SPL + j];
      if (a.tsrc) a.tsrc[o] = x;
      ++o;
    }
  if (gl == 0) a.ndist[x] = (uint32_t)nd;
}

// Rows with 65..2048 fine entries: one block per row, sort in LDS.
template <int EWK>
__global__ __launch_bounds__(256) void k_rows_block(ContractArgs a, const uint32_t* rows,
                                                    uint32_t nrows) {
  __shared__ uint32_t sk[ROW_B];
  __shared__ int64_t sw[ROW_B];
  __shared__ uint64_t mex[256], mbeg[256];
  __shared__ uint64_t sm[NWAVE];
  __shared__ uint64_t s_pos;
  const uint32_t r = blockIdx.x;
  if (r >= nrows) return;
  const uint32_t x = rows[r];
  const uint64_t m0 = a.mstart[x], m1 = a.mstart[x + 1];
  const uint64_t deg = a.degsum[x];
  uint32_t N = 1;
  while (N < deg) N <<= 1;
  if (threadIdx.x == 0) s_pos = 0;
  __syncthreads();
  for (uint64_t mb = m0; mb < m1; mb += 256) {
    const uint64_t mi = mb + threadIdx.x;
    uint64_t beg = 0, d = 0;
    if (mi < m1) {
      const uint32_t u = a.members[mi];
      beg = a.xadj[u];
      d = a.xadj[u + 1] - beg;
    }
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan(d, sm, tot);
    mex[threadIdx.x] = (mi < m1) ? ex : ~0ull;
    mbeg[threadIdx.x] = beg;
    // members in this chunk: the owner search needs only log2 of that many
    // steps (mex is ~0 past them)
    const uint64_t nmem = m1 - mb < (uint64_t)blockDim.x ? m1 - mb : (uint64_t)blockDim.x;
    int top = 0;
    for (int q = 1; (uint64_t)q < nmem; q <<= 1) top = q;
    __syncthreads();
    const uint64_t pos = s_pos;
    for (uint64_t t = threadIdx.x; t < tot; t += 256) {
      int lo = 0;
      for (int step = top; step > 0; step >>= 1)
        if (mex[lo + step] <= t) lo += step;
      uint32_t k;
      int64_t w;
      load_entry<EWK>(a, mbeg[lo] + (t - mex[lo]), x, k, w);
      sk[pos + t] = k;
      sw[pos + t] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_pos = pos + tot;
    __syncthreads();
  }
  for (uint32_t i = (uint32_t)deg + threadIdx.x; i < N; i += 256) {
    sk[i] = EMPTY_KEY;
    sw[i] = 0;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < N; i += 256) {
        const uint32_t p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
        if (p > i && sk[p] < sk[i]) {
          uint32_t tk = sk[i];
          int64_t tw = sw[i];
          sk[i] = sk[p], sw[i] = sw[p];
          sk[p] = tk, sw[p] = tw;
        }
      }
      __syncthreads();
    }
  }
  // run heads, output positions by block scan
  const uint64_t base = a.tmpoff[x];
  uint64_t carry = 0;
  for (uint32_t off = 0; off < N; off += 256) {
    const uint32_t i = off + threadIdx.x;
    const bool head = i < N && sk[i] != EMPTY_KEY && (i == 0 || sk[i - 1] != sk[i]);
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan((uint64_t)head, sm, tot);
    if (head) {
      int64_t s = 0;
      for (uint32_t j = i; j < N && sk[j] == sk[i]; ++j) s += sw[j];
      const uint64_t o = base + carry + ex;
      a.tkey[o] = sk[i];
      a.tw[o] = s;
      if (a.tsrc) a.tsrc[o] = x;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)carry;
}

// Rows with 2049..CAP fine entries, every weight below 2^32: one 1024-thread
// block per row; entries are packed as (neighbour << 32 | weight), so one
// 64-bit LDS word moves per compare-exchange of the bitonic sort.  Self
// entries pack as (EMPTY_KEY << 32) and padding as all ones: both sort last.
template <int EWK, int CAP>
__global__ __launch_bounds__(1024) void k_rows_big(ContractArgs a, const uint32_t* rows,
                                                   uint32_t nrows) {
  constexpr int NT = 1024, NW = NT / WAVE;
  __shared__ unsigned long long sv[CAP];
  __shared__ uint64_t mex[NT], mbeg[NT];
  __shared__ uint64_t sm[NW];
  __shared__ uint64_t s_pos;
  const uint32_t r = blockIdx.x;
  if (r >= nrows) return;
  const uint32_t x = rows[r];
  const uint64_t m0 = a.mstart[x], m1 = a.mstart[x + 1];
  const uint64_t deg = a.degsum[x];
  uint32_t N = 1;
  while (N < deg) N <<= 1;
  if (threadIdx.x == 0) s_pos = 0;
  __syncthreads();
  for (uint64_t mb = m0; mb < m1; mb += NT) {
    const uint64_t mi = mb + threadIdx.x;
    uint64_t beg = 0, d = 0;
    if (mi < m1) {
      const uint32_t u = a.members[mi];
      beg = a.xadj[u];
      d = a.xadj[u + 1] - beg;
    }
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t, NW>(d, sm, tot);
    mex[threadIdx.x] = (mi < m1) ? ex : ~0ull;
    mbeg[threadIdx.x] = beg;
    // members in this chunk: the owner search needs only log2 of that many
    // steps (mex is ~0 past them)
    const uint64_t nmem = m1 - mb < (uint64_t)blockDim.x ? m1 - mb : (uint64_t)blockDim.x;
    int top = 0;
    for (int q = 1; (uint64_t)q < nmem; q <<= 1) top = q;
    __syncthreads();
    const uint64_t pos = s_pos;
    for (uint64_t t = threadIdx.x; t < tot; t += NT) {
      int lo = 0;
      for (int step = top; step > 0; step >>= 1)
        if (mex[lo + step] <= t) lo += step;
      uint32_t k;
      int64_t w;
      load_entry<EWK>(a, mbeg[lo] + (t - mex[lo]), x, k, w);
      sv[pos + t] = ((unsigned long long)k << 32) | (uint32_t)w;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_pos = pos + tot;
    __syncthreads();
  }
  for (uint32_t i = (uint32_t)deg + threadIdx.x; i < N; i += NT) sv[i] = ~0ull;
  __syncthreads();
  // bitonic sort, ascending: each thread owns compare-exchange pairs
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t q = threadIdx.x; q < N / 2; q += NT) {
        const uint32_t i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
        const uint32_t p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i | j);
        const unsigned long long vi = sv[i], vp = sv[p];
        if (vp < vi) {
          sv[i] = vp;
          sv[p] = vi;
        }
      }
      __syncthreads();
    }
  }
  const uint64_t base = a.tmpoff[x];
  uint64_t carry = 0;
  for (uint32_t off = 0; off < N; off += NT) {
    const uint32_t i = off + threadIdx.x;
    const uint32_t key = i < N ? (uint32_t)(sv[i] >> 32) : EMPTY_KEY;
    const bool head = key != EMPTY_KEY && (i == 0 || (uint32_t)(sv[i - 1] >> 32) != key);
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t, NW>((uint64_t)head, sm, tot);
    if (head) {
      int64_t sum = 0;
      for (uint32_t j = i; j < N && (uint32_t)(sv[j] >> 32) == key; ++j) sum += (uint32_t)sv[j];
      const uint64_t o = base + carry + ex;
      a.tkey[o] = key;
      a.tw[o] = sum;
      if (a.tsrc) a.tsrc[o] = x;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)carry;
}

// Linear probing with a single loop exit (the slot of K), the add after it:
// divergent probes of a wave then cost few scalar mask updates per step.
LMGP_D void row_insert(uint32_t* key, unsigned long long* val, uint32_t K, uint64_t w, int logt) {
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

// Packed slots: the compare-and-swap claims an empty slot with the first
// weight or returns the occupant; a found slot gets the add after the loop.
LMGP_D void row_insert_packed(unsigned long long* tab, uint32_t K, unsigned long long w, int logt) {
  const uint32_t mask = (1u << logt) - 1;
  const unsigned long long mine = ((unsigned long long)K << 32) | w;
  uint32_t s = (K * 0x9E3779B1u) >> (32 - logt);
  unsigned long long prev;
  bool hit;
  do {
    prev = atomicCAS(&tab[s], ~0ull, mine);
    hit = prev == ~0ull || (uint32_t)(prev >> 32) == K;
    s = hit ? s : (s + 1) & mask;
  } while (!hit);
  if (prev != ~0ull) atomicAdd(&tab[s], w);
}

// Hash-aggregated rows: one block of NT threads per coarse row, LDS table of
// 2^LOGT slots (load <= 1/2, 3/4 for the packed 1024-thread classes); packed
// slots hold (neighbour << 32 | summed weight).  The distinct neighbours are
// written in slot order.
template <int EWK, int NT, int LOGT, bool PACK>
__global__ __launch_bounds__(NT) void k_rows_hash(ContractArgs a, const uint32_t* rows,
                                                  uint32_t nrows) {
  constexpr int T = 1 << LOGT, NW = NT / WAVE;
  __shared__ unsigned long long tab[PACK ? T : 1];
  __shared__ uint32_t skey[PACK ? 1 : T];
  __shared__ unsigned long long sval[PACK ? 1 : T];
  __shared__ uint64_t mex[NT], mbeg[NT];
  __shared__ uint64_t sm[NW];
  __shared__ uint64_t s_pos;
  const uint32_t r = blockIdx.x;
  if (r >= nrows) return;
  const uint32_t x = rows[r];
  const uint64_t m0 = a.mstart[x], m1 = a.mstart[x + 1];
  for (int i = threadIdx.x; i < T; i += NT) {
    if (PACK) {
      tab[i] = ~0ull;
    } else {
      skey[i] = EMPTY_KEY;
      sval[i] = 0;
    }
  }
  if (threadIdx.x == 0) s_pos = 0;
  __syncthreads();
  for (uint64_t mb = m0; mb < m1; mb += NT) {
    const uint64_t mi = mb + threadIdx.x;
    uint64_t beg = 0, d = 0;
    if (mi < m1) {
      const uint32_t u = a.members[mi];
      beg = a.xadj[u];
      d = a.xadj[u + 1] - beg;
    }
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t, NW>(d, sm, tot);
    mex[threadIdx.x] = (mi < m1) ? ex : ~0ull;
    mbeg[threadIdx.x] = beg;
    // members in this chunk: the owner search needs only log2 of that many
    // steps (mex is ~0 past them)
    const uint64_t nmem = m1 - mb < (uint64_t)blockDim.x ? m1 - mb : (uint64_t)blockDim.x;
    int top = 0;
    for (int q = 1; (uint64_t)q < nmem; q <<= 1) top = q;
    __syncthreads();
    constexpr int U = 4;
    for (uint64_t t0 = threadIdx.x; t0 < tot; t0 += (uint64_t)U * NT) {
      uint32_t k[U];
      int64_t w[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const uint64_t t = t0 + (uint64_t)j * NT;
        k[j] = EMPTY_KEY;
        w[j] = 0;
        if (t < tot) {
          int lo = 0;
          for (int step = top; step > 0; step >>= 1)
            if (mex[lo + step] <= t) lo += step;
          load_entry<EWK>(a, mbeg[lo] + (t - mex[lo]), x, k[j], w[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        if (k[j] == EMPTY_KEY) continue;  // self entry or past the chunk
        if (PACK) row_insert_packed(tab, k[j], (unsigned long long)w[j], LOGT);
        else row_insert(skey, sval, k[j], (uint64_t)w[j], LOGT);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s_pos += tot;
    __syncthreads();
  }
  // occupied slots -> consecutive outputs; each thread owns T / NT slots
  constexpr int SPT = T / NT;
  const int s0 = threadIdx.x * SPT;
  uint64_t mine = 0;
#pragma unroll
  for (int j = 0; j < SPT; ++j)
    mine += PACK ? (tab[s0 + j] != ~0ull) : (skey[s0 + j] != EMPTY_KEY);
  uint64_t tot;
  uint64_t o = a.tmpoff[x] + block_exclusive_scan<uint64_t, NW>(mine, sm, tot);
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    uint32_t k;
    int64_t w;
    if (PACK) {
      const unsigned long long v = tab[s0 + j];
      k = (uint32_t)(v >> 32);
      w = (int64_t)(v & 0xFFFFFFFFull);
      if (v == ~0ull) continue;
    } else {
      k = skey[s0 + j];
      w = (int64_t)sval[s0 + j];
      if (k == EMPTY_KEY) continue;
    }
    a.tkey[o] = k;
    a.tw[o] = w;
    if (a.tsrc) a.tsrc[o] = x;
    ++o;
  }
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)tot;
}

// Rows with > 2048 entries: gather (rank << 32 | neighbour) keys for the
// radix sort; self entries get neighbour EMPTY_KEY and are dropped later.
template <int EWK>
__global__ __launch_bounds__(256) void k_rows_gather(ContractArgs a, const uint32_t* rows,
                                                     uint32_t nrows, const uint64_t* goff,
                                                     uint64_t* gkey, int64_t* gw) {
  __shared__ uint64_t mex[256], mbeg[256];
  __shared__ uint64_t sm[NWAVE];
  __shared__ uint64_t s_pos;
  const uint32_t r = blockIdx.x;
  if (r >= nrows) return;
  const uint32_t x = rows[r];
  const uint64_t m0 = a.mstart[x], m1 = a.mstart[x + 1];
  const uint64_t out0 = goff[r];
  if (threadIdx.x == 0) s_pos = 0;
  __syncthreads();
  for (uint64_t mb = m0; mb < m1; mb += 256) {
    const uint64_t mi = mb + threadIdx.x;
    uint64_t beg = 0, d = 0;
    if (mi < m1) {
      const uint32_t u = a.members[mi];
      beg = a.xadj[u];
      d = a.xadj[u + 1] - beg;
    }
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan(d, sm, tot);
    mex[threadIdx.x] = (mi < m1) ? ex : ~0ull;
    mbeg[threadIdx.x] = beg;
    // members in this chunk: the owner search needs only log2 of that many
    // steps (mex is ~0 past them)
    const uint64_t nmem = m1 - mb < (uint64_t)blockDim.x ? m1 - mb : (uint64_t)blockDim.x;
    int top = 0;
    for (int q = 1; (uint64_t)q < nmem; q <<= 1) top = q;
    __syncthreads();
    const uint64_t pos = s_pos;
    for (uint64_t t = threadIdx.x; t < tot; t += 256) {
      int lo = 0;
      for (int step = top; step > 0; step >>= 1)
        if (mex[lo + step] <= t) lo += step;
      uint32_t k;
      int64_t w;
      load_entry<EWK>(a, mbeg[lo] + (t - mex[lo]), x, k, w);
      gkey[out0 + pos + t] = ((uint64_t)r << 32) | k;
      gw[out0 + pos + t] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_pos = pos + tot;
    __syncthreads();
  }
}

// Rows of more than 12288 entries on the hash path (packed weights): the
// row's gathered entries are split into R = ceil(deg / 12288) hash ranges of
// their neighbour ids; block j of the row aggregates range j in a packed LDS
// table of 16384 slots (at most about 3/4 full: a range holds about 12288
// entries, fewer distinct ones) and appends its distinct entries to the row.
// Every block reads the whole row, so fewer, fuller ranges read less.
// Probing is bounded: a range that does not fit sets `overflow` and the
// caller rebuilds these rows with the radix sort.
constexpr int RANGE_ENTRIES = 12288;
constexpr int RANGE_LOGT = 14;

LMGP_D uint32_t key_range(uint32_t k, uint32_t R) {
  uint32_t h = k * 0x9E3779B1u;
  h ^= h >> 15;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  return (uint32_t)(((uint64_t)h * R) >> 32);
}

struct RangeCount {
  const unsigned long long* degsum;
  const uint32_t* rows;
  LMGP_D uint64_t operator()(uint64_t i) const { return ceil_div(degsum[rows[i]], RANGE_ENTRIES); }
};

__global__ __launch_bounds__(1024) void k_rows_range(ContractArgs a, const uint32_t* rows,
                                                     uint32_t nrows, const uint64_t* goff,
                                                     const uint64_t* gkey, const int64_t* gw,
                                                     const uint64_t* roff, uint32_t* rowfill,
                                                     uint32_t* overflow) {
  constexpr int T = 1 << RANGE_LOGT, NT = 1024, NW = NT / WAVE;
  __shared__ unsigned long long tab[T];
  __shared__ uint64_t sm[NW];
  __shared__ int s_full;
  __shared__ uint32_t s_base;
  const uint64_t b = blockIdx.x;
  uint32_t lo = 0, hi = nrows;  // roff[lo] <= b < roff[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (roff[mid] <= b) lo = mid;
    else hi = mid;
  }
  const uint32_t r = lo;
  const uint32_t x = rows[r];
  const uint32_t R = (uint32_t)(roff[r + 1] - roff[r]);
  const uint32_t j = (uint32_t)(b - roff[r]);
  for (int i = threadIdx.x; i < T; i += NT) tab[i] = ~0ull;
  if (threadIdx.x == 0) s_full = 0;
  __syncthreads();
  for (uint64_t e = goff[r] + threadIdx.x; e < goff[r + 1]; e += NT) {
    const uint32_t k = (uint32_t)gkey[e];
    if (k == EMPTY_KEY || key_range(k, R) != j) continue;
    const unsigned long long w = (unsigned long long)gw[e];
    const unsigned long long mine = ((unsigned long long)k << 32) | w;
    uint32_t sl = (k * 0x9E3779B1u) >> (32 - RANGE_LOGT);
    unsigned long long prev;
    bool hit;
    int probe = 0;
    do {  // bounded: a full table reports an overflow
      prev = atomicCAS(&tab[sl], ~0ull, mine);
      hit = prev == ~0ull || (uint32_t)(prev >> 32) == k;
      sl = hit ? sl : (sl + 1) & (T - 1);
    } while (!hit && ++probe < T);
    if (hit && prev != ~0ull) atomicAdd(&tab[sl], w);
    if (!hit) s_full = 1;
  }
  __syncthreads();
  if (s_full) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;  // uniform: s_full is read after the barrier
  }
  constexpr int SPT = T / NT;
  const int s0 = threadIdx.x * SPT;
  uint64_t mine = 0;
#pragma unroll
  for (int q = 0; q < SPT; ++q) mine += tab[s0 + q] != ~0ull;
  uint64_t tot;
  const uint64_t ex = block_exclusive_scan<uint64_t, NW>(mine, sm, tot);
  if (threadIdx.x == 0) s_base = atomicAdd(&rowfill[r], (uint32_t)tot);
  __syncthreads();
  uint64_t o = a.tmpoff[x] + s_base + ex;
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const unsigned long long v = tab[s0 + q];
    if (v == ~0ull) continue;
    a.tkey[o] = (uint32_t)(v >> 32);
    a.tw[o] = (int64_t)(v & 0xFFFFFFFFull);
    if (a.tsrc) a.tsrc[o] = x;
    ++o;
  }
}

__global__ void k_rows_range_finish(ContractArgs a, const uint32_t* rows, const uint32_t* rowfill) {
  const uint32_t r = blockIdx.x;
  const uint32_t x = rows[r];
  const uint64_t nd = rowfill[r];
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)nd;
}

struct HeadFlag {
  const uint64_t* k;
  LMGP_D uint64_t operator()(uint64_t i) const {
    const uint64_t v = k[i];
    return ((uint32_t)v != EMPTY_KEY) && (i == 0 || k[i - 1] != v);
  }
};

// Sorted gathered entries -> distinct (neighbour, summed weight) per row.
__global__ void k_rows_reduce(ContractArgs a, const uint32_t* rows, uint32_t nrows,
                              const uint64_t* goff, const uint64_t* gkey, const int64_t* gw,
                              const uint32_t* hpos, uint64_t total) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t k = gkey[i];
  if ((uint32_t)k == EMPTY_KEY) return;
  if (i > 0 && gkey[i - 1] == k) return;
  const uint32_t r = (uint32_t)(k >> 32);
  const uint32_t x = rows[r];
  int64_t s = 0;
  for (uint64_t j = i; j < total && gkey[j] == k; ++j) s += gw[j];
  const uint64_t o = a.tmpoff[x] + (hpos[i] - hpos[goff[r]]);
  a.tkey[o] = (uint32_t)k;
  a.tw[o] = s;
  if (a.tsrc) a.tsrc[o] = x;
}

__global__ void k_rows_finish(ContractArgs a, const uint32_t* rows, uint32_t nrows,
                              const uint64_t* goff, const uint32_t* hpos) {
  const uint32_t r = blockIdx.x;
  if (r >= nrows) return;
  const uint32_t x = rows[r];
  const uint64_t nd = hpos[goff[r + 1]] - hpos[goff[r]];
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)nd;
}

// Compact the scratch rows into the coarse CSR (weights stored as WT).
// Compact the scratch rows into the coarse CSR (weights stored as WT): row x's
// distinct entries sit at the front of its scratch range, ndist[x] of them.
// Balanced over the output: block b writes coarse entries [b C, (b + 1) C)
// (C = COPY_TILE); the rows they fall in are found by binary search over the
// coarse offsets, staged in LDS when the tile spans at most COPY_ROWS rows.
constexpr uint32_t COPY_TILE = 2048;
constexpr uint32_t COPY_ROWS = 2048;

// last row x in [lo, hi] with off[x] <= d (off ascending, off[lo] <= d)
template <class Off>
LMGP_D uint64_t row_of(const Off& off, uint64_t lo, uint64_t hi, uint64_t d) {
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (off(mid) <= d) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename WT>
__global__ __launch_bounds__(256) void k_rows_copy(ContractArgs a, uint64_t nc, uint64_t mc,
                                                   uint32_t* cadj, WT* cew, uint32_t* csrc,
                                                   const uint64_t* cxadj) {
  __shared__ uint64_t soff[COPY_ROWS + 1];
  __shared__ uint64_t s_x0, s_x1;
  const uint64_t d0 = (uint64_t)blockIdx.x * COPY_TILE;
  const uint64_t d1 = d0 + COPY_TILE < mc ? d0 + COPY_TILE : mc;
  auto goff = [&](uint64_t x) { return cxadj[x]; };
  if (threadIdx.x == 0) {
    // rows holding the tile's first and last entry (cxadj[nc] = mc > d)
    s_x0 = row_of(goff, 0, nc - 1, d0);
    s_x1 = row_of(goff, s_x0, nc - 1, d1 - 1);
  }
  __syncthreads();
  const uint64_t x0 = s_x0, x1 = s_x1;
  const bool staged = x1 - x0 < COPY_ROWS;
  if (staged)
    for (uint64_t j = threadIdx.x; j <= x1 - x0; j += 256) soff[j] = cxadj[x0 + j];
  __syncthreads();
  auto loff = [&](uint64_t x) { return soff[x - x0]; };
  for (uint64_t d = d0 + threadIdx.x; d < d1; d += 256) {
    const uint64_t x = staged ? row_of(loff, x0, x1, d) : row_of(goff, x0, x1, d);
    const uint64_t from = a.tmpoff[x] + (d - (staged ? loff(x) : goff(x)));
    cadj[d] = a.tkey[from];
    cew[d] = (WT)a.tw[from];
    csrc[d] = (uint32_t)x;
  }
}

struct FlagUsed {
  const uint32_t* lcount;
  LMGP_D uint64_t operator()(uint64_t K) const { return lcount[K] > 0; }
};
struct U32At {
  const uint32_t* a;
  LMGP_D uint64_t operator()(uint64_t i) const { return a[i]; }
};
struct U64AtList {
  const unsigned long long* a;
  const uint32_t* list;
  LMGP_D uint64_t operator()(uint64_t i) const { return a[list[i]]; }
};

// Rows of the coarse nodes 0..nc-1 described by a (members, degree sums,
// scratch offsets): one launch per row class.
void build_rows(const ContractArgs& a, uint64_t nc, int packed, bool sorted, int ew_kind,
                Pool& pool, hipStream_t s) {
  DBuf<uint32_t> rcount(&pool, s, NROWCLS), rlists(&pool, s, NROWCLS * (nc ? nc : 1));
  rcount.zero();
  if (nc) {
    k_row_classes<<<grid_for(nc, 256), 256, 0, s>>>(a.degsum, nc, packed, sorted ? 1 : 0,
                                                    rcount.get(), rlists.get(), nc);
    LAUNCH_CHECK();
  }
  uint32_t rc[NROWCLS] = {};
  read_now(rc, rcount.get(), sizeof(rc), s);
  const uint32_t* listA = rlists.get();
  const uint32_t* listB = rlists.get() + nc;
  const uint32_t* listC = rlists.get() + 2 * nc;
  const uint32_t* listD = rlists.get() + 3 * nc;
  const uint32_t* listE = rlists.get() + 4 * nc;
  auto list_of = [&](int c) { return (const uint32_t*)rlists.get() + (uint64_t)c * nc; };
  auto launch_rows = [&](auto ewk) {
    constexpr int EWK = decltype(ewk)::value;
    if (rc[0]) {
      k_rows_wave<EWK><<<grid_for(rc[0], 4), 256, 0, s>>>(a, listA, rc[0]);
      LAUNCH_CHECK();
    }
    if (rc[1]) {
      k_rows_block<EWK><<<rc[1], 256, 0, s>>>(a, listB, rc[1]);
      LAUNCH_CHECK();
    }
    if (rc[9]) {
      k_rows_group<EWK, 16><<<grid_for(rc[9], 16), 256, 0, s>>>(a, list_of(9), rc[9]);
      LAUNCH_CHECK();
    }
    if (rc[10]) {
      k_rows_group<EWK, 32><<<grid_for(rc[10], 8), 256, 0, s>>>(a, list_of(10), rc[10]);
      LAUNCH_CHECK();
    }
    if (rc[11]) {
      k_rows_group<EWK, 64><<<grid_for(rc[11], 4), 256, 0, s>>>(a, list_of(11), rc[11]);
      LAUNCH_CHECK();
    }
    if (rc[12]) {
      if (packed) k_rows_hash<EWK, 128, 9, true><<<rc[12], 128, 0, s>>>(a, list_of(12), rc[12]);
      else k_rows_hash<EWK, 128, 9, false><<<rc[12], 128, 0, s>>>(a, list_of(12), rc[12]);
      LAUNCH_CHECK();
    }
    if (rc[3]) {
      k_rows_big<EWK, ROW_C><<<rc[3], 1024, 0, s>>>(a, listD, rc[3]);
      LAUNCH_CHECK();
    }
    if (rc[4]) {
      k_rows_big<EWK, ROW_D><<<rc[4], 1024, 0, s>>>(a, listE, rc[4]);
      LAUNCH_CHECK();
    }
    if (rc[5]) {
      if (packed) k_rows_hash<EWK, 256, 10, true><<<rc[5], 256, 0, s>>>(a, list_of(5), rc[5]);
      else k_rows_hash<EWK, 256, 10, false><<<rc[5], 256, 0, s>>>(a, list_of(5), rc[5]);
      LAUNCH_CHECK();
    }
    if (rc[6]) {
      if (packed) k_rows_hash<EWK, 256, 12, true><<<rc[6], 256, 0, s>>>(a, list_of(6), rc[6]);
      else k_rows_hash<EWK, 256, 12, false><<<rc[6], 256, 0, s>>>(a, list_of(6), rc[6]);
      LAUNCH_CHECK();
    }
    if (rc[7]) {
      k_rows_hash<EWK, 1024, 13, true><<<rc[7], 1024, 0, s>>>(a, list_of(7), rc[7]);
      LAUNCH_CHECK();
    }
    if (rc[8]) {
      k_rows_hash<EWK, 1024, 14, true><<<rc[8], 1024, 0, s>>>(a, list_of(8), rc[8]);
      LAUNCH_CHECK();
    }
    if (rc[2]) {
      DBuf<uint64_t> goff(&pool, s, rc[2] + 1);
      exclusive_scan(U64AtList{a.degsum, listC}, rc[2], goff.get(), true, pool, s);
      uint64_t gt = 0;
      read_now(&gt, goff.get() + rc[2], sizeof(uint64_t), s);
      DBuf<uint64_t> gk(&pool, s, gt), gk2(&pool, s, gt);
      DBuf<int64_t> gwv(&pool, s, gt), gw2(&pool, s, gt);
      k_rows_gather<EWK><<<rc[2], 256, 0, s>>>(a, listC, rc[2], goff.get(), gk.get(), gwv.get());
      LAUNCH_CHECK();
      if (!sorted && packed) {
        DBuf<uint64_t> roff(&pool, s, rc[2] + 1);
        exclusive_scan(RangeCount{a.degsum, listC}, rc[2], roff.get(), true, pool, s);
        uint64_t nr = 0;
        read_now(&nr, roff.get() + rc[2], 8, s);
        DBuf<uint32_t> rowfill(&pool, s, rc[2]), ovf(&pool, s, 1);
        rowfill.zero();
        ovf.zero();
        k_rows_range<<<(unsigned)nr, 1024, 0, s>>>(a, listC, rc[2], goff.get(), gk.get(), gwv.get(),
                                                   roff.get(), rowfill.get(), ovf.get());
        LAUNCH_CHECK();
        uint32_t overflow = 0;
        read_now(&overflow, ovf.get(), 4, s);
        // LMGP_ROW_RANGES=overflow takes the fallback as if a range had not fit
        // (used by the tests: the radix rows must overwrite the range output)
        const char* force = std::getenv("LMGP_ROW_RANGES");
        if (force && std::strcmp(force, "overflow") == 0) overflow = 1;
        if (!overflow) {
          k_rows_range_finish<<<rc[2], 256, 0, s>>>(a, listC, rowfill.get());
          LAUNCH_CHECK();
          return;
        }
        // a range did not fit: sort these rows instead (overwrites them)
      }
      int rbits = 1;
      while ((1ull << rbits) < rc[2]) ++rbits;
      bool swapped = radix_sort_pairs<int64_t>(gk.get(), gwv.get(), gk2.get(), gw2.get(), gt, 0,
                                                32 + rbits, pool, s);
      const uint64_t* sk = swapped ? gk2.get() : gk.get();
      const int64_t* sw = swapped ? gw2.get() : gwv.get();
      DBuf<uint32_t> hpos(&pool, s, gt + 1);
      exclusive_scan(HeadFlag{sk}, gt, hpos.get(), true, pool, s);
      k_rows_reduce<<<grid_for(gt, 256), 256, 0, s>>>(a, listC, rc[2], goff.get(), sk, sw,
                                                      hpos.get(), gt);
      LAUNCH_CHECK();
      k_rows_finish<<<rc[2], 256, 0, s>>>(a, listC, rc[2], goff.get(), hpos.get());
      LAUNCH_CHECK();
    }
  };
  switch (ew_kind) {
    case EW_UNIT: launch_rows(std::integral_constant<int, EW_UNIT>()); break;
    case EW_I32: launch_rows(std::integral_constant<int, EW_I32>()); break;
    default: launch_rows(std::integral_constant<int, EW_I64>()); break;
  }
}

}  // namespace

void contract_level(const ContractIn& in, ContractOut& out, Pool& pool, hipStream_t s) {
  const uint64_t n = in.n;
  const unsigned gn = grid_for(n, 256);
  const uint64_t bw = in.ew_kind == EW_UNIT ? 0 : in.ew_kind == EW_I32 ? 4 : 8;
  // coarse ids: label read and counted, flags scanned, map written, cluster
  // weights gathered (per node 4 + 4 + 8 + 4 + 4 + 8 B)
  ProfScope prof_remap("ct:remap", 32 * n, s);
  DBuf<uint32_t> lcount(&pool, s, n ? n : 1);
  if (in.csize) {
    if (n) k_label_count_sizes<<<gn, 256, 0, s>>>(in.csize, in.gid, in.keep, n, lcount.get());
  } else {
    lcount.zero();
    k_label_count<<<gn, 256, 0, s>>>(in.label, in.gid, in.keep, n, lcount.get());
  }
  LAUNCH_CHECK();
  DBuf<uint32_t> cid(&pool, s, n + 1);
  exclusive_scan(FlagUsed{lcount.get()}, n, cid.get(), true, pool, s);
  uint32_t nc32 = 0;
  read_now(&nc32, cid.get() + n, sizeof(uint32_t), s);
  const uint64_t nc = nc32;
  out.nc = nc;
  out.map.reset(&pool, s, n);
  k_map<<<gn, 256, 0, s>>>(in.label, cid.get(), in.gid, in.keep, n, out.map.get());
  LAUNCH_CHECK();
  out.nw.reset(&pool, s, nc ? nc : 1);
  DBuf<uint32_t> ccount(&pool, s, nc + 1);
  if (in.gid) out.gid.reset(&pool, s, nc ? nc : 1);
  k_coarse_nodes<<<gn, 256, 0, s>>>(in.W, lcount.get(), cid.get(), in.gid, n, out.nw.get(),
                                    ccount.get(), in.gid ? out.gid.get() : nullptr);
  LAUNCH_CHECK();
  // graph boundaries of the coarse union
  const size_t nbnd = in.bounds.size();
  out.cid_at_bounds.resize(nbnd);
  // bounds at 0 and n map to 0 and nc (a single graph has no other)
  bool interior = false;
  for (size_t i = 0; i < nbnd; ++i) {
    interior |= in.bounds[i] != 0 && in.bounds[i] != n;
    out.cid_at_bounds[i] = in.bounds[i] == 0 ? 0u : (uint32_t)nc;
  }
  if (interior) {  // one gather and one read, whatever the number of graphs
    DBuf<uint64_t> dbnd(&pool, s, nbnd);
    DBuf<uint32_t> dval(&pool, s, nbnd);
    HIP_CHECK(hipMemcpyAsync(dbnd.get(), in.bounds.data(), nbnd * sizeof(uint64_t),
                             hipMemcpyHostToDevice, s));
    k_gather_u32<<<grid_for(nbnd, 256), 256, 0, s>>>(cid.get(), dbnd.get(), nbnd, dval.get());
    LAUNCH_CHECK();
    read_now(out.cid_at_bounds.data(), dval.get(), nbnd * sizeof(uint32_t), s);
  }
  cid.clear();
  lcount.clear();
  prof_remap.add_bytes(24 * nc);  // coarse weights, counts, graph ids
  prof_remap.end();
  // members and degree sums: per node its map entry and two offsets read, its
  // member slot written; per coarse node offsets and sums
  ProfScope prof_members("ct:members", 24 * n + 24 * nc, s);
  DBuf<uint64_t> mstart(&pool, s, nc + 1);
  exclusive_scan(U32At{ccount.get()}, nc, mstart.get(), true, pool, s);
  ccount.clear();
  DBuf<uint32_t> mfill(&pool, s, nc ? nc : 1), members(&pool, s, n ? n : 1);
  DBuf<unsigned long long> degsum(&pool, s, nc ? nc : 1);
  mfill.zero();
  degsum.zero();
  k_members<<<gn, 256, 0, s>>>(in.xadj, out.map.get(), n, mstart.get(), mfill.get(), members.get(),
                               degsum.get());
  LAUNCH_CHECK();
  mfill.clear();
  DBuf<uint64_t> tmpoff(&pool, s, nc + 1);
  exclusive_scan(ArrayU64{(const uint64_t*)degsum.get()}, nc, tmpoff.get(), true, pool, s);
  uint64_t mt = in.entries;
  if (!in.all_kept) read_now(&mt, tmpoff.get() + nc, sizeof(uint64_t), s);
  DBuf<uint32_t> tkey(&pool, s, mt ? mt : 1), ndist(&pool, s, nc + 1);
  DBuf<int64_t> tw(&pool, s, mt ? mt : 1);
  ContractArgs a{};
  a.xadj = in.xadj;
  a.adj = in.adj;
  a.ew = in.ew;
  a.map = out.map.get();
  a.mstart = mstart.get();
  a.members = members.get();
  a.degsum = degsum.get();
  a.tmpoff = tmpoff.get();
  a.tkey = tkey.get();
  a.tw = tw.get();
  a.tsrc = nullptr;  // the copy writes each entry's row
  a.ndist = ndist.get();
  prof_members.end();
  // rows: every member entry's neighbour, its map entry and weight read; the
  // distinct neighbours written to scratch (id, weight) and counted
  const uint64_t fine_entries = mt;
  ProfScope prof_rows("ct:rows", (8 + bw) * fine_entries + 8 * n + 16 * nc, s);
  build_rows(a, nc, in.packed, in.sorted, in.ew_kind, pool, s);
  // coarse CSR
  out.xadj.reset(&pool, s, nc + 1);
  exclusive_scan(U32At{ndist.get()}, nc, out.xadj.get(), true, pool, s);
  uint64_t mc = 0;
  read_now(&mc, out.xadj.get() + nc, sizeof(uint64_t), s);
  out.nnz = mc;
  prof_rows.add_bytes(12 * mc);
  prof_rows.end();
  // copy: scratch entries read (id, weight) with their row's two offsets,
  // coarse adjacency, weight and row written; the coarse offsets staged
  ProfScope prof_copy("ct:copy", (12 + 8 + 8 + (in.narrow ? 4 : 8)) * mc + 8 * nc, s);
  out.adj.reset(&pool, s, mc ? mc : 1);
  out.src.reset(&pool, s, mc ? mc : 1);
  out.ew_kind = in.narrow ? EW_I32 : EW_I64;
  if (in.narrow) out.ew32.reset(&pool, s, mc ? mc : 1);
  else out.ew.reset(&pool, s, mc ? mc : 1);
  if (mc) {
    const unsigned gc = (unsigned)((mc + COPY_TILE - 1) / COPY_TILE);
    if (in.narrow)
      k_rows_copy<int32_t><<<gc, 256, 0, s>>>(a, nc, mc, out.adj.get(), out.ew32.get(),
                                              out.src.get(), out.xadj.get());
    else
      k_rows_copy<int64_t><<<gc, 256, 0, s>>>(a, nc, mc, out.adj.get(), out.ew.get(),
                                              out.src.get(), out.xadj.get());
    LAUNCH_CHECK();
  }
  // no wait here: scratch freed on return goes back to a stream-ordered pool
  // (reused only by later work on this stream)
}

namespace {
__global__ void k_identity_rows(const uint64_t* xadj, uint64_t n, uint32_t* id, uint64_t* mstart,
                                unsigned long long* deg) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  mstart[i] = i;
  if (i < n) {
    id[i] = (uint32_t)i;
    deg[i] = xadj[i + 1] - xadj[i];
  }
}
}  // namespace

// Row sorting as a contraction with the identity map: every node is its own
// single member, no entry is a self entry and no two entries merge, so every
// row keeps its length and lands at its own offset.
void sort_rows(uint64_t n, uint64_t nnz, const uint64_t* xadj, const uint32_t* adj,
               const void* ew, int ew_kind, int packed, DBuf<uint32_t>& out_adj,
               DBuf<int64_t>& out_ew, DBuf<uint32_t>& out_src, Pool& pool, hipStream_t s) {
  out_adj.reset(&pool, s, nnz ? nnz : 1);
  out_ew.reset(&pool, s, nnz ? nnz : 1);
  out_src.reset(&pool, s, nnz ? nnz : 1);
  if (n == 0) return;
  DBuf<uint32_t> id(&pool, s, n), ndist(&pool, s, n);
  DBuf<uint64_t> mstart(&pool, s, n + 1);
  DBuf<unsigned long long> deg(&pool, s, n);
  k_identity_rows<<<grid_for(n + 1, 256), 256, 0, s>>>(xadj, n, id.get(), mstart.get(), deg.get());
  LAUNCH_CHECK();
  ContractArgs a{};
  a.xadj = xadj;
  a.adj = adj;
  a.ew = ew;
  a.map = id.get();
  a.mstart = mstart.get();
  a.members = id.get();
  a.degsum = deg.get();
  a.tmpoff = xadj;
  a.tkey = out_adj.get();
  a.tw = out_ew.get();
  a.tsrc = out_src.get();
  a.ndist = ndist.get();
  build_rows(a, n, packed, true, ew_kind, pool, s);
}

}  // namespace lmgp
