// Cluster contraction (Sec. 2): cluster C becomes a coarse node of weight
// c(C); clusters joined by edges get one coarse edge whose weight is the sum
// of the joining edge weights.  Coarse ids are the ranks of the non-empty
// labels in ascending label order; coarse rows are sorted and duplicate-free.
//
// Layout: the members of every coarse node are bucketed (counting sort);
// each coarse row gathers the mapped neighbours of its members, sorts them by
// neighbour id and sums runs of equal ids.  Rows of <= 64 fine entries are
// sorted in registers by one wavefront, rows of <= 2048 in LDS by one block,
// rows of <= 16384 (when every edge weight fits in 32 bits) as packed
// (neighbour << 32 | weight) words in LDS by one 1024-thread block, larger
// rows by the device-wide radix sort.  Rows are first written to a
// scratch area at offset prefix(sum of member degrees), then compacted.
#include "contract.h"

namespace lmgp {

namespace {

constexpr int ROW_A = WAVE;   // <= 64 entries: wave
constexpr int ROW_B = 2048;   // <= 2048 entries: block, LDS
constexpr int ROW_C = 8192;   // <= 8192 entries: 1024-thread block, packed LDS words
constexpr int ROW_D = 16384;  // <= 16384 entries: the same with a 128 KiB LDS array
constexpr int NROWCLS = 5;

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

__global__ void k_members(const uint64_t* xadj, const uint32_t* map, uint64_t n,
                          const uint64_t* mstart, uint32_t* mfill, uint32_t* members,
                          unsigned long long* degsum) {
  uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const uint32_t x = map[u];
  if (x == EMPTY_KEY) return;
  members[mstart[x] + atomicAdd(&mfill[x], 1u)] = (uint32_t)u;
  const uint64_t d = xadj[u + 1] - xadj[u];
  if (d) atomicAdd(&degsum[x], (unsigned long long)d);
}

// Row size classes: 0 = wave, 1 = block, 2 = radix sort, 3 and 4 = big block
// with 8192 / 16384 LDS words (only when `packed`).
__global__ __launch_bounds__(256) void k_row_classes(const unsigned long long* degsum, uint64_t nc,
                                                     int packed, uint32_t* counts, uint32_t* lists,
                                                     uint64_t cap) {
  __shared__ uint32_t lc[NROWCLS], base[NROWCLS];
  if (threadIdx.x < NROWCLS) lc[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  uint32_t lp = 0;
  if (x < nc) {
    const uint64_t d = degsum[x];
    c = d <= ROW_A ? 0 : d <= ROW_B ? 1 : (packed && d <= ROW_C) ? 3 : (packed && d <= ROW_D) ? 4 : 2;
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
  const uint64_t deg = a.degsum[x];
  if (tail) {
    const uint64_t o = base + (uint64_t)__popcll(tmask & lanemask_lt());
    a.tkey[o] = key;
    a.tw[o] = s;
    a.tsrc[o] = x;
  }
  const uint32_t nd = (uint32_t)__popcll(tmask);
  for (uint64_t i = nd + l; i < deg; i += WAVE) a.tkey[base + i] = EMPTY_KEY;
  if (l == 0) a.ndist[x] = nd;
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
    __syncthreads();
    const uint64_t pos = s_pos;
    for (uint64_t t = threadIdx.x; t < tot; t += 256) {
      int lo = 0;
      for (int step = 128; step > 0; step >>= 1)
        if (lo + step < 256 && mex[lo + step] <= t) lo += step;
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
      a.tsrc[o] = x;
    }
    carry += tot;
  }
  for (uint64_t i = carry + threadIdx.x; i < deg; i += 256) a.tkey[base + i] = EMPTY_KEY;
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
    __syncthreads();
    const uint64_t pos = s_pos;
    for (uint64_t t = threadIdx.x; t < tot; t += NT) {
      int lo = 0;
      for (int step = NT / 2; step > 0; step >>= 1)
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
      a.tsrc[o] = x;
    }
    carry += tot;
  }
  for (uint64_t i = carry + threadIdx.x; i < deg; i += NT) a.tkey[base + i] = EMPTY_KEY;
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)carry;
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
    __syncthreads();
    const uint64_t pos = s_pos;
    for (uint64_t t = threadIdx.x; t < tot; t += 256) {
      int lo = 0;
      for (int step = 128; step > 0; step >>= 1)
        if (lo + step < 256 && mex[lo + step] <= t) lo += step;
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
  a.tsrc[o] = x;
}

__global__ void k_rows_finish(ContractArgs a, const uint32_t* rows, uint32_t nrows,
                              const uint64_t* goff, const uint32_t* hpos) {
  const uint32_t r = blockIdx.x;
  if (r >= nrows) return;
  const uint32_t x = rows[r];
  const uint64_t nd = hpos[goff[r + 1]] - hpos[goff[r]];
  const uint64_t deg = a.degsum[x];
  for (uint64_t i = nd + threadIdx.x; i < deg; i += blockDim.x) a.tkey[a.tmpoff[x] + i] = EMPTY_KEY;
  if (threadIdx.x == 0) a.ndist[x] = (uint32_t)nd;
}

// Compact the scratch rows into the coarse CSR.
__global__ void k_rows_copy(ContractArgs a, uint64_t total, uint32_t* cadj, int64_t* cew,
                            uint32_t* csrc, const uint64_t* cxadj) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const uint32_t k = a.tkey[e];
  if (k == EMPTY_KEY) return;
  const uint32_t x = a.tsrc[e];
  const uint64_t d = cxadj[x] + (e - a.tmpoff[x]);
  cadj[d] = k;
  cew[d] = a.tw[e];
  csrc[d] = x;
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

}  // namespace

void contract_level(const ContractIn& in, ContractOut& out, Pool& pool, hipStream_t s) {
  const uint64_t n = in.n;
  const unsigned gn = grid_for(n, 256);
  // coarse ids
  DBuf<uint32_t> lcount(&pool, s, n ? n : 1);
  lcount.zero();
  k_label_count<<<gn, 256, 0, s>>>(in.label, in.gid, in.keep, n, lcount.get());
  LAUNCH_CHECK();
  DBuf<uint32_t> cid(&pool, s, n + 1);
  exclusive_scan(FlagUsed{lcount.get()}, n, cid.get(), true, pool, s);
  uint32_t nc32 = 0;
  HIP_CHECK(hipMemcpyAsync(&nc32, cid.get() + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
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
  out.cid_at_bounds.resize(in.bounds.size());
  for (size_t i = 0; i < in.bounds.size(); ++i)
    HIP_CHECK(hipMemcpyAsync(&out.cid_at_bounds[i], cid.get() + in.bounds[i], sizeof(uint32_t),
                             hipMemcpyDeviceToHost, s));
  cid.clear();
  lcount.clear();
  // members and degree sums
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
  uint64_t mt = 0;
  HIP_CHECK(hipMemcpyAsync(&mt, tmpoff.get() + nc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  // row classes
  DBuf<uint32_t> rcount(&pool, s, NROWCLS), rlists(&pool, s, NROWCLS * (nc ? nc : 1));
  rcount.zero();
  if (nc) {
    k_row_classes<<<grid_for(nc, 256), 256, 0, s>>>(degsum.get(), nc, in.packed, rcount.get(),
                                                    rlists.get(), nc);
    LAUNCH_CHECK();
  }
  uint32_t rc[NROWCLS] = {0, 0, 0, 0, 0};
  HIP_CHECK(hipMemcpyAsync(rc, rcount.get(), sizeof(rc), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  DBuf<uint32_t> tkey(&pool, s, mt ? mt : 1), tsrc(&pool, s, mt ? mt : 1), ndist(&pool, s, nc + 1);
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
  a.tsrc = tsrc.get();
  a.ndist = ndist.get();
  const uint32_t* listA = rlists.get();
  const uint32_t* listB = rlists.get() + nc;
  const uint32_t* listC = rlists.get() + 2 * nc;
  const uint32_t* listD = rlists.get() + 3 * nc;
  const uint32_t* listE = rlists.get() + 4 * nc;
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
    if (rc[3]) {
      k_rows_big<EWK, ROW_C><<<rc[3], 1024, 0, s>>>(a, listD, rc[3]);
      LAUNCH_CHECK();
    }
    if (rc[4]) {
      k_rows_big<EWK, ROW_D><<<rc[4], 1024, 0, s>>>(a, listE, rc[4]);
      LAUNCH_CHECK();
    }
    if (rc[2]) {
      DBuf<uint64_t> goff(&pool, s, rc[2] + 1);
      exclusive_scan(U64AtList{degsum.get(), listC}, rc[2], goff.get(), true, pool, s);
      uint64_t gt = 0;
      HIP_CHECK(hipMemcpyAsync(&gt, goff.get() + rc[2], sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      DBuf<uint64_t> gk(&pool, s, gt), gk2(&pool, s, gt);
      DBuf<int64_t> gwv(&pool, s, gt), gw2(&pool, s, gt);
      k_rows_gather<EWK><<<rc[2], 256, 0, s>>>(a, listC, rc[2], goff.get(), gk.get(), gwv.get());
      LAUNCH_CHECK();
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
      HIP_CHECK(hipStreamSynchronize(s));  // keep scratch alive until done
    }
  };
  switch (in.ew_kind) {
    case EW_UNIT: launch_rows(std::integral_constant<int, EW_UNIT>()); break;
    case EW_I32: launch_rows(std::integral_constant<int, EW_I32>()); break;
    default: launch_rows(std::integral_constant<int, EW_I64>()); break;
  }
  // coarse CSR
  out.xadj.reset(&pool, s, nc + 1);
  exclusive_scan(U32At{ndist.get()}, nc, out.xadj.get(), true, pool, s);
  uint64_t mc = 0;
  HIP_CHECK(hipMemcpyAsync(&mc, out.xadj.get() + nc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  out.nnz = mc;
  out.adj.reset(&pool, s, mc ? mc : 1);
  out.ew.reset(&pool, s, mc ? mc : 1);
  out.src.reset(&pool, s, mc ? mc : 1);
  if (mt) {
    k_rows_copy<<<grid_for(mt, 256), 256, 0, s>>>(a, mt, out.adj.get(), out.ew.get(),
                                                   out.src.get(), out.xadj.get());
    LAUNCH_CHECK();
  }
  HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace lmgp
