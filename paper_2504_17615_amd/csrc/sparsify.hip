// Weighted threshold sampling (Sec. 4.2), on the edge weights or on
// (Weighted) Forest Fire scores.  omega_t is the weight (score) of the
// m_hat-th heaviest coarse edge; heavier edges are kept, lighter ones
// dropped, and among the edges of weight omega_t exactly r = m_hat - |E^>|
// are kept: those with the smallest (H(seed, SPARS, level, a, b), a, b),
// a < b, so that the coarse graph has exactly m_hat edges.  The hash is
// symmetric in the edge, so both CSR entries of an edge get the same decision.
//
// omega_t: MSB-first radix select with 8-bit digits over the weights of the
// directed entries (every edge counted twice, so the (2 m_hat)-th largest
// entry).  The r-th smallest hash among E^=: one 12-bit histogram pass, then
// the entries of the selected bucket are gathered and ranked exactly, all on
// the device (the host learns omega_t, |E^>| and |E^=| from the weight
// passes; the rank decides only which of the E^= edges are kept).
#include <algorithm>
#include <cstdlib>

#include "contract.h"
#include "profiler.h"

namespace lmgp {

namespace {

template <typename KT>
__global__ __launch_bounds__(256) void k_wmax(const KT* key, uint64_t e0, uint64_t e1,
                                              unsigned long long* out) {
  __shared__ int64_t sm[NWAVE];
  int64_t m = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += stride)
    m = (int64_t)key[e] > m ? (int64_t)key[e] : m;
  m = wave_reduce_max(m);
  if (lane_id() == 0) sm[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NWAVE; ++i) m = sm[i] > m ? sm[i] : m;
    atomicMax(out, (unsigned long long)m);
  }
}

template <typename KT>
__global__ __launch_bounds__(256) void k_whist(const KT* key, uint64_t e0, uint64_t e1,
                                               int shift, uint64_t prefix,
                                               unsigned long long* hist) {
  // a block counts fewer than 2^32 entries; the device-wide bins are 64-bit
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const int hs = shift + 8;
  for (uint64_t e = e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += stride) {
    const uint64_t w = (uint64_t)(int64_t)key[e];
    const bool match = hs >= 64 || (w >> hs) == (prefix >> hs);
    if (match) atomicAdd(&h[(w >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

LMGP_D uint64_t edge_key(uint64_t pre, uint64_t a, uint64_t b) {
  return hash_add(hash_add(pre, a), b);
}

// 12-bit histogram of the top bits of the keys of E^= (a < b entries only).
template <typename KT>
__global__ __launch_bounds__(256) void k_khist(const uint32_t* src, const uint32_t* adj,
                                               const KT* key, uint64_t e0, uint64_t e1,
                                               int64_t w_t, uint64_t base, uint64_t pre,
                                               unsigned long long* hist) {
  __shared__ uint32_t h[4096];
  for (int i = threadIdx.x; i < 4096; i += 256) h[i] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += stride) {
    const uint32_t a = src[e], b = adj[e];
    if (a < b && (int64_t)key[e] == w_t)
      atomicAdd(&h[edge_key(pre, a - base, b - base) >> 52], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4096; i += 256)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

struct EqEntry {
  uint64_t key;
  uint32_t a, b;  // local ids
};

// The rank of the wanted entry, found on the device: sel[0] the 12-bit bucket
// holding the r-th smallest key, sel[1] its rank inside the bucket (1-based),
// sel[2] the bucket's size.  One 1024-thread block, four bins per thread.
constexpr int PICK_NT = 1024;
__global__ __launch_bounds__(PICK_NT) void k_eq_pick(const unsigned long long* hist, uint64_t r,
                                                      unsigned long long* sel) {
  __shared__ unsigned long long sm[PICK_NT / WAVE];
  const int t = threadIdx.x;
  unsigned long long h[4], loc = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) loc += (h[i] = hist[4 * t + i]);
  unsigned long long tot;
  unsigned long long cum = block_exclusive_scan<unsigned long long, PICK_NT / WAVE>(loc, sm, tot);
  // 1 <= r <= the number of keys, so exactly one bin qualifies
  if (cum < r && r <= cum + loc) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (cum + h[i] >= r) {
        sel[0] = (unsigned long long)(4 * t + i);
        sel[1] = r - cum;
        sel[2] = h[i];
        break;
      }
      cum += h[i];
    }
  }
}

template <typename KT>
__global__ __launch_bounds__(256) void k_kgather(const uint32_t* src, const uint32_t* adj,
                                                 const KT* key, uint64_t e0, uint64_t e1,
                                                 int64_t w_t, uint64_t base, uint64_t pre,
                                                 const unsigned long long* sel, EqEntry* out,
                                                 unsigned long long* cnt, uint64_t cap) {
  const uint64_t bucket = sel[0];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += stride) {
    const uint32_t a = src[e], b = adj[e];
    if (a < b && (int64_t)key[e] == w_t) {
      const uint64_t k = edge_key(pre, a - base, b - base);
      if ((k >> 52) == bucket) {
        const uint64_t p = atomicAdd(cnt, 1ull);
        if (p < cap) out[p] = EqEntry{k, a - (uint32_t)base, b - (uint32_t)base};
      }
    }
  }
}

struct SparsDesc {
  uint64_t node_base;
  uint64_t pre;
  int64_t w_t;
  uint64_t tkey;
  uint32_t ta, tb;
  // 0 keep all, 1 keep w >= w_t, 2 keep w > w_t and E^= up to (tkey, ta, tb),
  // 3 keep iff coin < coin_r (uniform sampling), 4 keep w > w_t and E^= edges
  // whose coin < coin_r; coin = floor(H(SPARS, level, a, b) * coin_n / 2^64)
  uint32_t mode;
  uint32_t pad;
  uint64_t coin_n, coin_r;
};

// The rin-th smallest (key, a, b) of the selected bucket, written into the
// graph's descriptor.  One block, MSB-first radix select over the 128-bit
// composite (key, a, b) in 8-bit digits: each pass counts the digit of every
// candidate that matches the digits chosen so far and picks the digit holding
// the wanted rank; once one candidate is left it is found by one more pass.
// Candidates: the gathered entries, or, if the gather overflowed its buffer,
// the E^= entries of the edge range whose key lies in the bucket.
constexpr int RANK_NT = 1024;

LMGP_D uint32_t eq_digit(uint64_t key, uint32_t a, uint32_t b, int pos) {
  // digit 15 is the top byte of key, digit 0 the low byte of b
  const uint64_t w = pos >= 8 ? key : ((uint64_t)a << 32 | b);
  return (uint32_t)(w >> (8 * (pos & 7))) & 0xFF;
}

template <typename KT>
struct EqSource {
  const EqEntry* buf;  // gathered entries, or NULL: scan the edge range
  uint64_t cnt;
  const uint32_t* src;
  const uint32_t* adj;
  const KT* key;
  uint64_t e0, e1, base, pre, bucket;
  int64_t w_t;
  // f(key, a, b) for every candidate, the block's threads striding over them
  template <class F>
  LMGP_D void each(F&& f) const {
    if (buf) {
      for (uint64_t i = threadIdx.x; i < cnt; i += RANK_NT) f(buf[i].key, buf[i].a, buf[i].b);
      return;
    }
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += RANK_NT) {
      const uint32_t a = src[e], b = adj[e];
      if (a < b && (int64_t)key[e] == w_t) {
        const uint64_t k = edge_key(pre, a - base, b - base);
        if ((k >> 52) == bucket) f(k, a - (uint32_t)base, b - (uint32_t)base);
      }
    }
  }
};

template <typename KT>
__global__ __launch_bounds__(RANK_NT) void k_eq_rank(EqSource<KT> in, const unsigned long long* cnt,
                                                     uint64_t cap, const unsigned long long* sel,
                                                     SparsDesc* d) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t s_digit, s_left;
  __shared__ uint64_t s_rank;
  __shared__ EqEntry s_out;
  in.bucket = sel[0];
  in.cnt = *cnt;
  if (in.cnt > cap) in.buf = nullptr;
  uint64_t rank = sel[1];
  // chosen digits so far: composite bits above `pos` (hi: key, lo: a << 32 | b)
  uint64_t phi = 0, plo = 0, mhi = 0, mlo = 0;
  auto matches = [&](uint64_t k, uint32_t a, uint32_t b) {
    return (k & mhi) == phi && (((uint64_t)a << 32 | b) & mlo) == plo;
  };
  int pos = 15;
  for (; pos >= 0; --pos) {
    for (int i = threadIdx.x; i < 256; i += RANK_NT) h[i] = 0;
    __syncthreads();
    in.each([&](uint64_t k, uint32_t a, uint32_t b) {
      if (matches(k, a, b)) atomicAdd(&h[eq_digit(k, a, b, pos)], 1u);
    });
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t cum = 0;
      int dg = 0;
      for (; dg < 255 && cum + h[dg] < rank; ++dg) cum += h[dg];
      s_digit = (uint32_t)dg;
      s_left = h[dg];
      s_rank = rank - cum;
    }
    __syncthreads();
    const uint64_t dm = 0xFFull << (8 * (pos & 7)), dv = (uint64_t)s_digit << (8 * (pos & 7));
    if (pos >= 8) mhi |= dm, phi |= dv;
    else mlo |= dm, plo |= dv;
    rank = s_rank;
    const uint32_t left = s_left;
    __syncthreads();
    if (left == 1) break;  // (keys are distinct: at the last digit one is left)
  }
  // the one candidate matching every chosen digit
  in.each([&](uint64_t k, uint32_t a, uint32_t b) {
    if (matches(k, a, b)) s_out = EqEntry{k, a, b};
  });
  __syncthreads();
  if (threadIdx.x == 0) {
    d->tkey = s_out.key;
    d->ta = s_out.a;
    d->tb = s_out.b;
  }
}

template <typename KT>
__global__ void k_keep(const uint32_t* src, const uint32_t* adj, const KT* keyv,
                       const uint32_t* gid, const SparsDesc* sd, uint64_t nnz, uint8_t* keep) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t u = src[e], v = adj[e];
  const SparsDesc d = sd[graph_of(gid, u)];
  const uint32_t a = (u < v ? u : v) - (uint32_t)d.node_base;
  const uint32_t b = (u < v ? v : u) - (uint32_t)d.node_base;
  uint8_t k = 1;
  if (d.mode == 3) {
    k = __umul64hi(edge_key(d.pre, a, b), d.coin_n) < d.coin_r;
  } else if (d.mode != 0) {
    const int64_t w = (int64_t)keyv[e];
    if (w > d.w_t) k = 1;
    else if (w < d.w_t) k = 0;
    else if (d.mode == 1) k = 1;
    else if (d.mode == 4) k = __umul64hi(edge_key(d.pre, a, b), d.coin_n) < d.coin_r;
    else {
      const uint64_t key = edge_key(d.pre, a, b);
      k = key < d.tkey || (key == d.tkey && (a < d.ta || (a == d.ta && b <= d.tb)));
    }
  }
  keep[e] = k;
}

struct U8At {
  const uint8_t* a;
  LMGP_D uint64_t operator()(uint64_t i) const { return a[i]; }
};

template <typename WT>
__global__ void k_scatter_kept(const uint32_t* src, const uint32_t* adj, const WT* ew,
                               const uint8_t* keep, const uint64_t* pos, uint64_t nnz,
                               uint32_t* osrc, uint32_t* oadj, WT* oew) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz || !keep[e]) return;
  const uint64_t p = pos[e];
  osrc[p] = src[e];
  oadj[p] = adj[e];
  oew[p] = ew[e];
}

__global__ void k_row_starts(const uint64_t* xadj, const uint64_t* pos, uint64_t n,
                             uint64_t* oxadj) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x > n) return;
  oxadj[x] = pos[xadj[x]];
}

unsigned sweep_grid(uint64_t cnt) {
  unsigned g = grid_for(cnt, 256);
  return g > 4096 ? 4096 : g;
}

}  // namespace

namespace {

// Selection on `key` (the weights, or the fire scores), output weights `ew`.
template <typename WT, typename KT>
void sparsify_t(uint64_t n, uint64_t nnz, const uint64_t* xadj, const uint32_t* adj,
                const WT* ew, const KT* key, const uint32_t* src, const uint32_t* gid,
                std::vector<SparsGraph>& graphs, SparsOut& out, WT* (*alloc_w)(SparsOut&, uint64_t, Pool&, hipStream_t),
                Pool& pool, hipStream_t s) {
  const size_t B = graphs.size();
  std::vector<SparsDesc> desc(B);
  struct EqRank {
    size_t g;       // graph
    uint64_t r;     // rank of the last kept edge of weight w_t (1-based)
    uint64_t n_eq;  // edges of weight w_t
  };
  std::vector<EqRank> eq_rank;
  DBuf<unsigned long long> dmax(&pool, s, 1);
  DBuf<unsigned long long> hist(&pool, s, 4096), cnt(&pool, s, 1);
  for (size_t g = 0; g < B; ++g) {
    SparsGraph& sg = graphs[g];
    SparsDesc& d = desc[g];
    d = SparsDesc{sg.node_base, sg.pre, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!sg.triggered) continue;
    if (sg.sampler == 1) {  // uniform: every edge keeps with probability m_hat / |E'|
      d.mode = 3;
      d.coin_n = (sg.e1 - sg.e0) / 2;
      d.coin_r = sg.m_hat;
      sg.w_t = 0;
      sg.n_gt = sg.n_eq = 0;
      continue;
    }
    if (sg.m_hat == 0) {  // keep nothing: threshold above every weight
      d.mode = 1;
      d.w_t = INT64_MAX;
      sg.w_t = 0;
      continue;
    }
    const uint64_t e0 = sg.e0, e1 = sg.e1;
    dmax.zero();
    k_wmax<KT><<<sweep_grid(e1 - e0), 256, 0, s>>>(key, e0, e1, dmax.get());
    LAUNCH_CHECK();
    unsigned long long wmax = 0;
    read_now(&wmax, dmax.get(), sizeof(wmax), s);
    int top = 0;
    while (top < 64 && (wmax >> top) != 0) top += 8;
    // the weight of every entry per 8-bit digit pass, with the host's digit
    // choice between passes
    ProfScope prof_sel("sp:select", sizeof(KT) * (e1 - e0) * (top / 8), s);
    // (2 m_hat)-th largest directed weight
    uint64_t R = 2 * sg.m_hat, gt = 0, eq = 0, prefix = 0;
    std::vector<unsigned long long> h(256);
    for (int shift = top - 8; shift >= 0; shift -= 8) {
      hist.zero();
      k_whist<KT><<<sweep_grid(e1 - e0), 256, 0, s>>>(key, e0, e1, shift, prefix, hist.get());
      LAUNCH_CHECK();
      read_now(h.data(), hist.get(), 256 * sizeof(unsigned long long), s);
      uint64_t cum = 0;
      int sel = 0;
      for (int dgt = 255; dgt >= 0; --dgt) {
        if (cum + h[dgt] >= R) {
          sel = dgt;
          break;
        }
        cum += h[dgt];
      }
      gt += cum;
      R -= cum;
      prefix |= (uint64_t)sel << shift;
      eq = h[sel];
    }
    prof_sel.end();
    sg.w_t = (int64_t)prefix;
    sg.n_gt = gt / 2;
    sg.n_eq = eq / 2;
    d.w_t = sg.w_t;
    const uint64_t r = sg.m_hat - sg.n_gt;
    if (r == sg.n_eq) {
      d.mode = 1;
      continue;
    }
    if (sg.sampler == 3) {  // independent coins for the edges of weight w_t
      d.mode = 4;
      d.coin_n = sg.n_eq;
      d.coin_r = r;
      continue;
    }
    // r-th smallest (key, a, b) among the n_eq undirected edges of weight w_t
    // (1 <= r < n_eq: fewer than 2 m_hat entries are heavier than w_t and at
    // least 2 m_hat weigh at least w_t): ranked on the device below
    d.mode = 2;
    eq_rank.push_back(EqRank{g, r, sg.n_eq});
  }
  DBuf<SparsDesc> dd(&pool, s, B);
  HIP_CHECK(hipMemcpyAsync(dd.get(), desc.data(), B * sizeof(SparsDesc), hipMemcpyHostToDevice, s));
  if (!eq_rank.empty()) {
    // the bucket of the r-th key from a 12-bit histogram, its entries
    // gathered, the rank inside it by radix select, all on the device.  The
    // gather buffer holds 4x a bucket's mean size plus 4096 entries (a bucket
    // larger than that has vanishing probability under a 64-bit hash; the
    // rank kernel then scans the edge range itself).  LMGP_EQ_GATHER_CAP
    // lowers the capacity (tests use it to take the scanning path).
    const char* cap_env = std::getenv("LMGP_EQ_GATHER_CAP");
    const uint64_t cap_max = cap_env ? std::strtoull(cap_env, nullptr, 10) : ~0ull;
    auto cap_of = [&](const EqRank& q) {
      const uint64_t c = std::min<uint64_t>(q.n_eq, 4 * ((q.n_eq + 4095) / 4096) + 4096);
      return std::max<uint64_t>(1, std::min(c, cap_max));
    };
    uint64_t buf_cap = 1;
    for (const EqRank& q : eq_rank) buf_cap = std::max(buf_cap, cap_of(q));
    DBuf<EqEntry> buf(&pool, s, buf_cap);
    DBuf<unsigned long long> sel(&pool, s, 3);
    for (const EqRank& q : eq_rank) {
      const SparsGraph& sg = graphs[q.g];
      const uint64_t e0 = sg.e0, e1 = sg.e1;
      // row, neighbour and weight of every entry in two passes
      ProfScope prof_hs("sp:hash_select", 2 * (8 + sizeof(KT)) * (e1 - e0), s);
      hist.zero();
      k_khist<KT><<<sweep_grid(e1 - e0), 256, 0, s>>>(src, adj, key, e0, e1, sg.w_t,
                                                   sg.node_base, sg.pre, hist.get());
      LAUNCH_CHECK();
      k_eq_pick<<<1, PICK_NT, 0, s>>>(hist.get(), q.r, sel.get());
      LAUNCH_CHECK();
      cnt.zero();
      const uint64_t cap = cap_of(q);
      k_kgather<KT><<<sweep_grid(e1 - e0), 256, 0, s>>>(src, adj, key, e0, e1, sg.w_t,
                                                     sg.node_base, sg.pre, sel.get(), buf.get(),
                                                     cnt.get(), cap);
      LAUNCH_CHECK();
      EqSource<KT> in{buf.get(), 0, src, adj, key, e0, e1, sg.node_base, sg.pre, 0, sg.w_t};
      k_eq_rank<KT><<<1, RANK_NT, 0, s>>>(in, cnt.get(), cap, sel.get(), dd.get() + q.g);
      LAUNCH_CHECK();
    }
  }
  // keep flags, positions, compaction: every entry read (row, neighbour,
  // weight) and flagged, positions scanned, the kept ones written
  uint64_t kept_est = 0;
  for (const SparsGraph& sg : graphs) kept_est += sg.triggered ? 2 * sg.m_hat : sg.e1 - sg.e0;
  ProfScope prof_cp("sp:compact", (8 + sizeof(KT) + 1 + 8) * nnz + (8 + sizeof(WT)) * kept_est +
                                      16 * (n + 1), s);
  DBuf<uint8_t> keep(&pool, s, nnz ? nnz : 1);
  if (nnz) {
    k_keep<KT><<<grid_for(nnz, 256), 256, 0, s>>>(src, adj, key, gid, dd.get(), nnz, keep.get());
    LAUNCH_CHECK();
  }
  DBuf<uint64_t> pos(&pool, s, nnz + 1);
  exclusive_scan(U8At{keep.get()}, nnz, pos.get(), true, pool, s);
  uint64_t total = 0;
  read_now(&total, pos.get() + nnz, sizeof(uint64_t), s);
  out.nnz = total;
  out.xadj.reset(&pool, s, n + 1);
  out.adj.reset(&pool, s, total ? total : 1);
  WT* oew = alloc_w(out, total ? total : 1, pool, s);
  out.src.reset(&pool, s, total ? total : 1);
  if (nnz) {
    k_scatter_kept<WT><<<grid_for(nnz, 256), 256, 0, s>>>(src, adj, ew, keep.get(), pos.get(), nnz,
                                                           out.src.get(), out.adj.get(), oew);
    LAUNCH_CHECK();
  }
  k_row_starts<<<grid_for(n + 1, 256), 256, 0, s>>>(xadj, pos.get(), n, out.xadj.get());
  LAUNCH_CHECK();
  HIP_CHECK(hipStreamSynchronize(s));
}

int64_t* alloc_w64(SparsOut& o, uint64_t n, Pool& pool, hipStream_t s) {
  o.ew.reset(&pool, s, n);
  o.ew_kind = EW_I64;
  return o.ew.get();
}
int32_t* alloc_w32(SparsOut& o, uint64_t n, Pool& pool, hipStream_t s) {
  o.ew32.reset(&pool, s, n);
  o.ew_kind = EW_I32;
  return o.ew32.get();
}

}  // namespace

void sparsify_level(uint64_t n, uint64_t nnz, const uint64_t* xadj, const uint32_t* adj,
                    const void* ew, int ew_kind, const uint32_t* src, const uint32_t* gid,
                    const uint32_t* score, std::vector<SparsGraph>& graphs, SparsOut& out,
                    Pool& pool, hipStream_t s) {
  if (ew_kind == EW_I32) {
    const int32_t* w = (const int32_t*)ew;
    if (score)
      sparsify_t<int32_t, uint32_t>(n, nnz, xadj, adj, w, score, src, gid, graphs, out, alloc_w32,
                                    pool, s);
    else
      sparsify_t<int32_t, int32_t>(n, nnz, xadj, adj, w, w, src, gid, graphs, out, alloc_w32, pool,
                                   s);
  } else if (ew_kind == EW_I64) {
    const int64_t* w = (const int64_t*)ew;
    if (score)
      sparsify_t<int64_t, uint32_t>(n, nnz, xadj, adj, w, score, src, gid, graphs, out, alloc_w64,
                                    pool, s);
    else
      sparsify_t<int64_t, int64_t>(n, nnz, xadj, adj, w, w, src, gid, graphs, out, alloc_w64, pool,
                                   s);
  } else {
    throw InvalidArg("sparsification needs stored edge weights");
  }
}

}  // namespace lmgp
