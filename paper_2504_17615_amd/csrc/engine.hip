// Host orchestration of the multilevel partitioner on one GPU.
//
// Algorithm 1 (coarsening with sparsification) runs over a union of graphs:
// every kernel launch covers all graphs still coarsening, and each graph
// keeps its own parameters (U, seed, budget, stop decisions).  A single
// graph is the union of one.  Level decisions need a few scalars per level
// on the host (cluster counts, coarse sizes, edge counts).
#include <algorithm>
#include <functional>
#include <atomic>
#include <cmath>
#include <thread>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "engine.h"
#include "initial.h"
#include "profiler.h"
#include "tuner.h"

namespace lmgp {

typedef unsigned __int128 u128;

namespace {

uint64_t chain(uint64_t seed, uint64_t tag, std::initializer_list<uint64_t> xs) {
  uint64_t s = hash_prefix(seed, tag);
  for (uint64_t x : xs) s = hash_add(s, x);
  return s;
}

// Small copies go through the thread's page-locked staging arena: an upload
// is copied into it first, a download lands in it and reaches its
// destination at the next sync(), which also gives the arena back (the
// stream has then passed every staged copy).  Every read of a download in
// this file follows a sync().
struct PendingRead {
  void* dst;
  const void* src;
  size_t bytes;
};
std::vector<PendingRead>& pending_reads() {
  static thread_local std::vector<PendingRead> v;
  return v;
}

template <class T>
void h2d(T* dst, const T* src, size_t n, hipStream_t s) {
  if (!n) return;
  const size_t bytes = n * sizeof(T);
  void* p = stage_take(bytes);
  if (p) std::memcpy(p, src, bytes);
  HIP_CHECK(hipMemcpyAsync(dst, p ? p : src, bytes, hipMemcpyHostToDevice, s));
}
template <class T>
void d2h(T* dst, const T* src, size_t n, hipStream_t s) {
  if (!n) return;
  const size_t bytes = n * sizeof(T);
  void* p = stage_take(bytes);
  HIP_CHECK(hipMemcpyAsync(p ? p : (void*)dst, src, bytes, hipMemcpyDeviceToHost, s));
  if (p) pending_reads().push_back(PendingRead{dst, p, bytes});
}
void sync(hipStream_t s) {
  Profiler::get().count("host:stream_syncs");
  HIP_CHECK(hipStreamSynchronize(s));
  for (const PendingRead& r : pending_reads()) std::memcpy(r.dst, r.src, r.bytes);
  pending_reads().clear();
  stage_reset(0);
}

// ------------------------------------------------------------ small kernels --
__global__ void k_iota(uint32_t* a, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (uint32_t)i;
}
__global__ void k_copy_i64(int64_t* d, const int64_t* s, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// LP control on the device, one thread per graph.  The stop decisions of a
// sub-round are taken where the counts are, so that the host reads them once
// per round (with the next round's bucket counts) instead of after every
// sub-round.
struct LpCtl {
  GraphDesc* gd;
  uint32_t B;
  unsigned long long* moves;        // 1 if the current sub-round moved a node (admission output)
  unsigned long long* delta;        // non-empty clusters after the sub-round (counted from W)
  unsigned long long* round_moves;  // sub-rounds of the current round that moved a node
  unsigned long long* ncl;          // cluster count (clustering) or NULL
  uint32_t* rounds_run;             // rounds in which the graph was active
  unsigned long long* rstate;       // [2 nb] bucket counters, then [B] active flags,
                                    // then [B] the next round's flags (k_lp_peek)
  uint32_t nb;                      // buckets (sub-rounds x degree classes)
  uint32_t* ovtotal;                // admission overflow counters [2], cleared here
  const uint64_t* pre;              // [round][graph][3]: SUB, TIE, ADM hash prefixes
  uint32_t shrink_num, shrink_den;
};

// After a sub-round: count its moves; in clustering apply the cluster-count
// change and stop a graph once shrink_num * |C| <= shrink_den * n.
// One graph (parts != NULL): the count is its count before the sub-round plus
// the admission apply blocks' changes, summed here first.
__global__ __launch_bounds__(256) void k_lp_after_sub(LpCtl c, const int64_t* parts,
                                                      uint32_t nparts) {
  if (parts) {
    __shared__ int64_t sm[NWAVE];
    int64_t v = 0;
    for (uint32_t j = threadIdx.x; j < nparts; j += 256) v += parts[j];
    const int64_t tot = block_reduce_sum(v, sm);
    if (threadIdx.x == 0) c.delta[0] = (unsigned long long)((int64_t)c.ncl[0] + tot);
    __syncthreads();
  }
  for (uint32_t b = threadIdx.x; b < c.B; b += blockDim.x) {
    GraphDesc& g = c.gd[b];
    if (g.active) {
      c.round_moves[b] += c.moves[b];
      if (c.ncl) {
        c.ncl[b] = c.delta[b];  // counted from the cluster weights
        if ((u128)c.shrink_num * c.ncl[b] <= (u128)c.shrink_den * g.nodes) g.active = 0;
      }
    }
    c.moves[b] = 0;
    c.delta[b] = 0;
  }
  if (threadIdx.x < 2) c.ovtotal[threadIdx.x] = 0;
}

// Start of round r: a graph that made no move in round r - 1 stops; the
// others take round r's hash prefixes.  A replayed round takes r from the
// device counter rdev and advances it.
__global__ void k_lp_round(LpCtl c, uint32_t r_arg, uint32_t* rdev) {
  const uint32_t r = rdev ? *rdev : r_arg;
  for (uint32_t b = threadIdx.x; b < c.B; b += blockDim.x) {
    GraphDesc& g = c.gd[b];
    if (r > 0 && g.active && c.round_moves[b] == 0) g.active = 0;
    c.round_moves[b] = 0;
    const uint64_t* p = c.pre + ((uint64_t)r * c.B + b) * 3;
    g.pre_sub = p[0];
    g.pre_tie = p[1];
    g.pre_adm = p[2];
    if (g.active) c.rounds_run[b] = r + 1;
    c.rstate[2 * c.nb + b] = g.active;
  }
  for (uint32_t i = threadIdx.x; i < 2 * c.nb; i += blockDim.x) c.rstate[i] = 0;
  __syncthreads();
  if (rdev && threadIdx.x == 0) *rdev = r + 1;
}

// The flags the next round's k_lp_round will compute (without changing any
// state), for the host to decide whether to run it.
__global__ void k_lp_peek(LpCtl c) {
  for (uint32_t b = threadIdx.x; b < c.B; b += blockDim.x)
    c.rstate[2 * c.nb + c.B + b] = c.gd[b].active && c.round_moves[b] != 0;
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

// Member count of every label (csize zeroed before): a block counts a
// contiguous chunk of nodes, and a run of equal labels within a wave adds
// once, from its last lane.
__global__ __launch_bounds__(256) void k_label_sizes(const uint32_t* label, uint64_t n,
                                                     uint32_t* csize) {
  const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t u0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t u1 = u0 + chunk < n ? u0 + chunk : n;
  const int lane = lane_id();
  for (uint64_t b = u0; b < u1; b += 256) {
    const uint64_t u = b + threadIdx.x;
    const bool valid = u < u1;  // the valid lanes of a wave are a prefix
    const uint32_t l = valid ? label[u] : 0u;
    const uint32_t prev = __shfl_up(l, 1);
    const bool head = valid && (lane == 0 || prev != l);
    const uint64_t heads = __ballot(head), vmask = __ballot(valid);
    const bool next_head = lane < WAVE - 1 && ((heads >> (lane + 1)) & 1);
    const bool next_valid = lane < WAVE - 1 && ((vmask >> (lane + 1)) & 1);
    if (valid && (next_head || !next_valid)) {
      const uint64_t upto = heads & ((2ull << lane) - 1);  // heads at lanes <= lane
      const int start = 63 - __builtin_clzll(upto);
      atomicAdd(&csize[l], (uint32_t)(lane - start + 1));
    }
  }
}

// Refinement: a node whose neighbours all share its block has no other block
// with a positive rating, so it can produce no move.  flag[u] = 1 for the
// other nodes (flag zeroed before), from the entries; `count` gets the number
// of flagged nodes.
__global__ void k_boundary(const uint32_t* src, const uint32_t* adj, uint64_t nnz,
                           const uint32_t* block, const uint8_t* block8, uint8_t* flag) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t u = src[e], v = adj[e];
  const uint32_t bu = block8 ? block8[u] : block[u], bv = block8 ? block8[v] : block[v];
  if (bu != bv) flag[u] = 1;
}

__global__ __launch_bounds__(256) void k_count_flags(const uint8_t* flag, uint64_t n,
                                                     unsigned long long* count) {
  __shared__ uint64_t sm[NWAVE];
  uint64_t c = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    c += flag[i] != 0;
  c = block_reduce_sum(c, sm);  // one add per block: a single counter serialises adds
  if (threadIdx.x == 0 && c) atomicAdd(count, (unsigned long long)c);
}

// After a sub-round: every neighbour of a node that moved may have become a
// boundary node; flag it (flags only grow within a level).
__global__ void k_mark_moved(const Cand* cands, const uint8_t* adm, uint32_t nc,
                             const uint64_t* xadj, const uint32_t* adj, uint8_t* flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc || !adm[i]) return;
  const uint32_t u = cands[i].u;
  for (uint64_t e = xadj[u]; e < xadj[u + 1]; ++e) flag[adj[e]] = 1;
}

// Pinned host memory for the per-round state copy (copies into pageable
// memory are staged by the runtime).  One buffer per thread, grown on demand
// and kept for the thread's life (a few KiB).
unsigned long long* pinned_state(size_t n) {
  static thread_local unsigned long long* p = nullptr;
  static thread_local size_t cap = 0;
  if (no_alloc_mode()) {  // pageable: no page-locked allocation
    static thread_local std::vector<unsigned long long> v;
    if (v.size() < n) v.resize(n);
    return v.data();
  }
  if (n > cap) {
    if (p) HIP_CHECK(hipHostFree(p));
    p = nullptr;
    cap = 0;
    HIP_CHECK(hipHostMalloc((void**)&p, n * sizeof(unsigned long long), hipHostMallocDefault));
    cap = n;
  }
  return p;
}

__global__ void k_gather_u64(const uint64_t* a, const uint64_t* idx, uint64_t n, uint64_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[idx[i]];
}

__global__ void k_remap_u32(uint32_t* g, uint64_t n, const uint32_t* map) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = map[g[i]];
}

// Every graph's blocks to its own output array, as graph-local ids.
__global__ void k_blocks_out(const uint32_t* block, const uint32_t* gid, uint64_t n,
                             const uint64_t* nbase, const uint64_t* kbase, uint32_t* const* out) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t b = graph_of(gid, v);
  uint32_t* o = out[b];
  if (o) o[v - nbase[b]] = block[v] - (uint32_t)kbase[b];
}

__global__ void k_to_u8(const uint32_t* a, uint64_t n, uint8_t* b) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (uint8_t)a[i];
}

// Refinement levels from this size rate only their boundary nodes (when at
// most half of the nodes are on the boundary).  Below it, one bucketing pass
// and one host wait per round cost less than a pass and a wait per sub-round.
constexpr uint64_t BOUNDARY_MIN_NODES = 1ull << 21;

// Levels (unions) up to this many nodes replay their LP rounds from a graph
// when asked: above it the rounds are long enough to hide their launches.
constexpr uint64_t REPLAY_MAX_NODES = 1ull << 18;

// Levels from this size gather refinement labels from a byte copy (with 4
// bytes per label the array no longer fits the 4 MiB L2 of an XCD).
constexpr uint64_t LABEL8_MIN_NODES = 1ull << 20;

// Graphs sharing a coarsest level from which the automatic choice bisects
// them on the device.
constexpr uint32_t IP_DEVICE_MIN_GRAPHS = 16;

// Stream on which replayed rounds are captured (capture needs a stream other
// than the null stream; nothing is executed on it), one per thread and device.
hipStream_t capture_stream() {
  static thread_local std::vector<hipStream_t> streams;
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
  if (!streams[dev]) HIP_CHECK(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}


// 2-hop: singletons lighter than their graph's cap (a node of weight >= cap
// fits with no other node), their sort keys and next-fit groups.
struct SingletonFlag {
  const uint32_t* label;
  const uint32_t* csize;
  const int64_t* nw;
  const uint32_t* gid;
  const GraphDesc* gd;
  LMGP_D uint64_t operator()(uint64_t v) const {
    const GraphDesc& d = gd[graph_of(gid, v)];
    return d.active && csize[label[v]] == 1 && nw[v] < d.cap;
  }
};

// Segment key of a singleton: 2 * favourite, or for an isolated node
// 2 * (last node of its graph) + 1, which orders ISO after every label of the
// graph and before the next graph's labels.
LMGP_D uint64_t favkey_of(const SingletonFlag& f, const uint64_t* xadj, const uint32_t* fav,
                          uint64_t v) {
  const GraphDesc& d = f.gd[graph_of(f.gid, v)];
  const uint32_t fv = xadj[v + 1] > xadj[v] ? fav[v] : EMPTY_KEY;
  return fv != EMPTY_KEY ? 2ull * fv : 2ull * (d.node_base + d.nodes - 1) + 1;
}

// key = favkey << fshift | c(v) << 32 | hi32 H(TWOHOP, level, v); fshift = 0
// leaves the favourite for a second (stable) sort.  vals in ascending v order,
// so equal keys stay ordered by id.
__global__ void k_twohop_keys(SingletonFlag f, const uint64_t* xadj, const uint32_t* fav,
                              const uint32_t* pos, uint64_t n, int fshift, uint64_t* keys,
                              uint32_t* vals) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !f(v)) return;
  const GraphDesc& d = f.gd[graph_of(f.gid, v)];
  const uint64_t h = hash_add(d.pre_two, v - d.node_base) >> 32;
  uint64_t key = ((uint64_t)f.nw[v] << 32) | h;
  if (fshift) key |= favkey_of(f, xadj, fav, v) << fshift;
  keys[pos[v]] = key;
  vals[pos[v]] = (uint32_t)v;
}

__global__ void k_twohop_favkeys(SingletonFlag f, const uint64_t* xadj, const uint32_t* fav,
                                 const uint32_t* vals, uint64_t ns, uint64_t* keys) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < ns) keys[p] = favkey_of(f, xadj, fav, vals[p]);
}

// One past the last position of every favourite segment, by segment key.
__global__ void k_seg_last(const uint64_t* keys, int sshift, uint64_t ns, uint32_t* last) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const uint64_t fk = keys[p] >> sshift;
  if (p + 1 == ns || (keys[p + 1] >> sshift) != fk) last[fk] = (uint32_t)(p + 1);
}

struct SortedWeight {
  const uint32_t* vals;
  const int64_t* nw;
  LMGP_D uint64_t operator()(uint64_t p) const { return (uint64_t)nw[vals[p]]; }
};

constexpr uint32_t NO_NEXT = 0xFFFFFFFFu;

// nxt[p]: where the next group starts if a next-fit group opens at p, i.e. the
// first q > p of p's segment with c(p..q) > cap (E = exclusive prefix sums of
// the sorted weights); NO_NEXT if the rest of the segment fits.  Every weight
// is >= 1, so q <= p + cap.
__global__ void k_nextfit(const uint64_t* keys, int sshift, const uint32_t* last, const uint64_t* E,
                          const uint32_t* vals, const uint32_t* gid, const GraphDesc* gd,
                          uint64_t ns, uint32_t* nxt) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const uint64_t end = last[keys[p] >> sshift];
  const uint64_t cap = (uint64_t)gd[graph_of(gid, vals[p])].cap;
  const uint64_t hi = cap < end - p ? p + 1 + cap : end;
  const uint64_t base = E[p];
  uint64_t a = p + 1, b = hi;
  while (a < b) {
    const uint64_t mid = (a + b) >> 1;
    if (E[mid + 1] - base > cap) b = mid;
    else a = mid + 1;
  }
  nxt[p] = a < hi ? (uint32_t)a : NO_NEXT;
}

// Pointer doubling: J2 = J o J.
__global__ void k_jump(const uint32_t* J, uint64_t ns, uint32_t* J2) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const uint32_t q = J[p];
  J2[p] = q == NO_NEXT ? NO_NEXT : J[q];
}

__global__ void k_mark_seg_first(const uint64_t* keys, int sshift, uint64_t ns, uint8_t top,
                                 uint8_t* mark) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  mark[p] = (p == 0 || (keys[p - 1] >> sshift) != (keys[p] >> sshift)) ? top : 0;
}

// Group starts are the positions J^t(segment first), t < 2^K.  Expansion from
// the top table down: positions marked before this pass (mark >= k + 2) also
// mark their 2^k-th successor with k + 1, which this pass does not expand.
__global__ void k_expand(const uint32_t* Jk, uint64_t ns, uint32_t k, uint8_t* mark) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns || mark[p] < k + 2) return;
  const uint32_t q = Jk[p];
  if (q != NO_NEXT && mark[q] == 0) mark[q] = (uint8_t)(k + 1);
}

// Scan value: a group start counts in the low half, a joiner in the high half.
struct StartJoin {
  const uint8_t* mark;
  LMGP_D uint64_t operator()(uint64_t p) const { return mark[p] ? 1ull : (1ull << 32); }
};

__global__ __launch_bounds__(256) void k_group_heads(const uint8_t* mark, const uint64_t* sj,
                                                     uint64_t ns, const uint32_t* vals,
                                                     const uint32_t* gid, uint32_t* head,
                                                     unsigned long long* joins) {
  __shared__ uint64_t sm[NWAVE];
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool join = false;
  if (p < ns) {
    if (mark[p]) head[(uint32_t)sj[p]] = (uint32_t)p;
    join = !mark[p];
    if (join && gid) atomicAdd(&joins[gid[vals[p]]], 1ull);
  }
  if (!gid) {  // one graph: one add per block (a single counter serialises adds)
    const uint64_t c = block_reduce_sum((uint64_t)(join ? 1 : 0), sm);
    if (threadIdx.x == 0 && c) atomicAdd(&joins[0], (unsigned long long)c);
  }
}

// A joiner takes its group head's label while its rank among its graph's
// joiners is below the graph's cap (joins in sorted order).
__global__ void k_group_merge(const uint32_t* vals, const uint8_t* mark, const uint64_t* sj,
                              const uint32_t* head, uint64_t ns, const uint32_t* gid,
                              const uint64_t* base, const uint64_t* cap, uint32_t* label,
                              int64_t* W, const int64_t* nw, uint32_t* csize) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns || mark[p]) return;
  const uint32_t b = vals[p];
  const uint32_t g = graph_of(gid, b);
  if ((sj[p] >> 32) - base[g] >= cap[g]) return;
  const uint32_t a = vals[head[(uint32_t)sj[p] - 1]];
  const uint32_t la = label[a], lb = label[b];
  label[b] = la;
  atomicAdd((unsigned long long*)&W[la], (unsigned long long)nw[b]);
  W[lb] -= nw[b];
  atomicAdd(&csize[la], 1u);
  csize[lb] -= 1;
}

// Coarse edge weights known to be below 2^31, stored as int32.
__global__ void k_narrow_i32(const int64_t* w, uint64_t n, int32_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)w[i];
}

// Union construction for batches: concatenate graphs with rebased ids.
struct UnionPart {
  const uint64_t* xadj;
  const uint32_t* adj;
  const void* ew;
  int ew_kind;
  const int64_t* nw;
  uint64_t nbase, ebase, n, nnz;
};

__device__ uint32_t find_part(const uint64_t* bounds, uint32_t B, uint64_t i) {
  uint32_t lo = 0, hi = B;  // bounds[lo] <= i < bounds[hi]
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (bounds[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void k_union_nodes(const UnionPart* parts, const uint64_t* nb, uint32_t B, uint64_t n,
                              uint64_t* xadj, int64_t* nw, uint32_t* gid) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t g = find_part(nb, B, i);
  const UnionPart pt = parts[g];
  const uint64_t li = i - pt.nbase;
  xadj[i] = pt.ebase + pt.xadj[li];
  nw[i] = pt.nw[li];
  gid[i] = g;
  if (i == n - 1) xadj[n] = pt.ebase + pt.xadj[li + 1];
}

__global__ void k_union_entries(const UnionPart* parts, const uint64_t* eb, uint32_t B,
                                uint64_t nnz, uint32_t* adj, int64_t* ew, uint32_t* src,
                                const uint32_t* psrc_dummy) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t g = find_part(eb, B, e);
  const UnionPart pt = parts[g];
  const uint64_t le = e - pt.ebase;
  adj[e] = (uint32_t)(pt.nbase + pt.adj[le]);
  if (ew) {
    int64_t w = 1;
    if (pt.ew_kind == EW_I32) w = ((const int32_t*)pt.ew)[le];
    else if (pt.ew_kind == EW_I64) w = ((const int64_t*)pt.ew)[le];
    ew[e] = w;
  }
  (void)psrc_dummy;
}

__global__ void k_union_src(const UnionPart* parts, const uint32_t* const* srcs, const uint64_t* eb,
                            uint32_t B, uint64_t nnz, uint32_t* src) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t g = find_part(eb, B, e);
  src[e] = (uint32_t)(parts[g].nbase + srcs[g][e - parts[g].ebase]);
}

// Extension of a union level by graphs that join a run in flight: part 0 is
// the level itself (its graph ids kept), parts 1.. are input graphs (graph id
// B0 + part - 1); entry weights converted to the level's stored type WT.
__global__ void k_extend_nodes(const UnionPart* parts, const uint64_t* nb, uint32_t P, uint64_t n,
                               const uint32_t* gid0, uint32_t B0, uint64_t* xadj, int64_t* nw,
                               uint32_t* gid) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = find_part(nb, P, i);
  const UnionPart pt = parts[p];
  const uint64_t li = i - pt.nbase;
  xadj[i] = pt.ebase + pt.xadj[li];
  nw[i] = pt.nw[li];
  gid[i] = p == 0 ? (gid0 ? gid0[li] : 0u) : B0 + p - 1;
  if (i == n - 1) xadj[n] = pt.ebase + pt.xadj[li + 1];
}

template <typename WT>
__global__ void k_extend_entries(const UnionPart* parts, const uint32_t* const* srcs,
                                 const uint64_t* eb, uint32_t P, uint64_t nnz, uint32_t* adj,
                                 WT* ew, uint32_t* src) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t p = find_part(eb, P, e);
  const UnionPart pt = parts[p];
  const uint64_t le = e - pt.ebase;
  adj[e] = (uint32_t)(pt.nbase + pt.adj[le]);
  src[e] = (uint32_t)(pt.nbase + srcs[p][le]);
  int64_t w = 1;
  if (pt.ew_kind == EW_I32) w = ((const int32_t*)pt.ew)[le];
  else if (pt.ew_kind == EW_I64) w = ((const int64_t*)pt.ew)[le];
  ew[e] = (WT)w;
}

class Timer {
 public:
  explicit Timer(hipStream_t s) : s_(s) {
    HIP_CHECK(hipEventCreate(&a_));
    HIP_CHECK(hipEventCreate(&b_));
  }
  ~Timer() {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
  }
  void start() { HIP_CHECK(hipEventRecord(a_, s_)); }
  int64_t stop_ns() {
    HIP_CHECK(hipEventRecord(b_, s_));
    HIP_CHECK(hipEventSynchronize(b_));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, a_, b_));
    return (int64_t)((double)ms * 1e6);
  }

 private:
  hipStream_t s_;
  hipEvent_t a_, b_;
};

}  // namespace

// A call that ends by an exception may leave staged copies in flight: wait
// for them before the staging arena is reused.
Engine::~Engine() {
  if (!pending_reads().empty() || stage_mark() != 0) {
    (void)hipStreamSynchronize(s_);
    pending_reads().clear();
    stage_reset(0);
  }
}

lmgp_params default_params() {
  lmgp_params p;
  p.tau_e_num = 1, p.tau_e_den = 2;
  p.tau_d_num = 1, p.tau_d_den = 2;
  p.rho_num = 4, p.rho_den = 1;
  p.sampler = 0;
  p.clim = 160;
  p.shrink_num = 5, p.shrink_den = 2;
  p.lp_rounds = 5, p.ref_rounds = 5, p.subrounds = 4;
  p.max_levels = 64;
  p.stop_num = 19, p.stop_den = 20;
  p.tune = LMGP_TUNE_OFF;
  p.graph_rounds = 0;
  p.ip_device = LMGP_IP_AUTO;
  p.ff_p_num = 3, p.ff_p_den = 5;
  p.ff_nu_num = 1, p.ff_nu_den = 2;
  return p;
}

void check_params(const lmgp_params& p) {
  if (!p.tau_e_den || !p.tau_d_den || !p.rho_den) throw InvalidArg("zero denominator in params");
  if (p.sampler > 5)
    throw InvalidArg("sampler must be 0 (threshold), 1 (uniform), 2 (off), 3 (threshold, coins), "
                     "4 (threshold on Forest Fire scores) or 5 (on Weighted Forest Fire scores)");
  if (!p.ff_p_den || !p.ff_nu_den) throw InvalidArg("zero denominator in the fire parameters");
  if (!p.clim) throw InvalidArg("clim must be positive");
  if (!p.shrink_num) throw InvalidArg("shrink_num must be positive");
  if (!p.subrounds || p.subrounds > 32) throw InvalidArg("subrounds must be in [1, 32]");
  if (!p.max_levels) throw InvalidArg("max_levels must be positive");
  if (!p.stop_den) throw InvalidArg("stop_den must be positive");
  if (p.tune > LMGP_TUNE_AUTO && p.tune < LMGP_TUNE_FORCE)
    throw InvalidArg("tune must be 0 (default classes), 1 (autotune) or 16 + preset");
  if (p.graph_rounds > 1) throw InvalidArg("graph_rounds must be 0 or 1");
  if (p.ip_device > LMGP_IP_AUTO) throw InvalidArg("ip_device must be 0, 1 or 2");
}

// ----------------------------------------------------------------- union --
void Engine::build_union(std::vector<Job>& jobs) {
  levels_.clear();
  auto L = std::make_unique<Level>();
  const uint32_t B = (uint32_t)jobs.size();
  L->sorted = true;
  for (auto& jb : jobs) L->sorted &= jb.g->rows_sorted;
  L->graphs.resize(B);
  L->nbase.assign(B + 1, 0);
  L->ebase.assign(B + 1, 0);
  for (uint32_t b = 0; b < B; ++b) {
    L->graphs[b] = b;
    L->nbase[b + 1] = L->nbase[b] + jobs[b].g->n;
    L->ebase[b + 1] = L->ebase[b] + jobs[b].g->nnz;
  }
  L->n = L->nbase[B];
  L->nnz = L->ebase[B];
  if (B == 1) {
    const InputGraph& g = *jobs[0].g;
    L->xadj = g.xadj.get();
    L->adj = g.adj.get();
    L->ew = g.ew();
    L->ew_kind = g.ew_kind;
    L->nw = g.nw.get();
    L->src = g.src.get();
    L->gid = nullptr;
  } else {
    bool all_unit = true, all_i32 = true;
    for (auto& j : jobs) {
      all_unit &= j.g->ew_kind == EW_UNIT;
      all_i32 &= j.g->ew_kind == EW_I32;
    }
    std::vector<UnionPart> parts(B);
    std::vector<const uint32_t*> srcs(B);
    for (uint32_t b = 0; b < B; ++b) {
      const InputGraph& g = *jobs[b].g;
      parts[b] = UnionPart{g.xadj.get(), g.adj.get(), g.ew(), g.ew_kind, g.nw.get(),
                           L->nbase[b], L->ebase[b], g.n, g.nnz};
      srcs[b] = g.src.get();
    }
    DBuf<UnionPart> dparts(&pool_, s_, B);
    DBuf<const uint32_t*> dsrcs(&pool_, s_, B);
    DBuf<uint64_t> dnb(&pool_, s_, B + 1), deb(&pool_, s_, B + 1);
    h2d(dparts.get(), parts.data(), B, s_);
    h2d(dsrcs.get(), srcs.data(), B, s_);
    h2d(dnb.get(), L->nbase.data(), B + 1, s_);
    h2d(deb.get(), L->ebase.data(), B + 1, s_);
    L->o_xadj.reset(&pool_, s_, L->n + 1);
    L->o_nw.reset(&pool_, s_, L->n ? L->n : 1);
    L->o_gid.reset(&pool_, s_, L->n ? L->n : 1);
    L->o_adj.reset(&pool_, s_, L->nnz ? L->nnz : 1);
    L->o_src.reset(&pool_, s_, L->nnz ? L->nnz : 1);
    if (!all_unit) L->o_ew.reset(&pool_, s_, L->nnz ? L->nnz : 1);
    if (L->n) {
      k_union_nodes<<<grid_for(L->n, 256), 256, 0, s_>>>(dparts.get(), dnb.get(), B, L->n,
                                                         L->o_xadj.get(), L->o_nw.get(),
                                                         L->o_gid.get());
      LAUNCH_CHECK();
    } else {
      device_zero(L->o_xadj.get(), sizeof(uint64_t), s_);
    }
    if (L->nnz) {
      k_union_entries<<<grid_for(L->nnz, 256), 256, 0, s_>>>(
          dparts.get(), deb.get(), B, L->nnz, L->o_adj.get(), all_unit ? nullptr : L->o_ew.get(),
          L->o_src.get(), nullptr);
      LAUNCH_CHECK();
      k_union_src<<<grid_for(L->nnz, 256), 256, 0, s_>>>(dparts.get(), dsrcs.get(), deb.get(), B,
                                                         L->nnz, L->o_src.get());
      LAUNCH_CHECK();
    }
    (void)all_i32;
    L->xadj = L->o_xadj.get();
    L->adj = L->o_adj.get();
    L->ew = all_unit ? nullptr : (const void*)L->o_ew.get();
    L->ew_kind = all_unit ? EW_UNIT : EW_I64;
    L->nw = L->o_nw.get();
    L->src = L->o_src.get();
    L->gid = L->o_gid.get();
    sync(s_);
  }
  levels_.push_back(std::move(L));
}

bool Engine::can_join(const InputGraph& g) const {
  if (!g.rows_sorted || g.n == 0) return false;
  if (packed_ && !(g.wtot < (1ull << 32) && g.nnz < (1ull << 32))) return false;
  if (narrow_ && !(g.wtot < (1ull << 31))) return false;
  return true;
}

// The jobs [first, jobs.size()) join at the current top union level: a new
// level made of the current one (ids unchanged, so the finer level's map
// stays valid) followed by their input graphs replaces it.
void Engine::extend_union(std::vector<Job>& jobs, size_t first) {
  Level& L = *levels_.back();
  const uint32_t B0 = (uint32_t)L.graphs.size();
  const uint32_t Bn = (uint32_t)(jobs.size() - first);
  const uint32_t P = 1 + Bn;
  const uint32_t d = (uint32_t)levels_.size() - 1;
  auto N = std::make_unique<Level>();
  N->sorted = L.sorted;  // joined inputs have sorted rows (can_join)
  N->graphs = L.graphs;
  N->nbase = L.nbase;
  N->ebase = L.ebase;
  std::vector<UnionPart> parts(P);
  std::vector<const uint32_t*> srcs(P);
  std::vector<uint64_t> pnb(P + 1, 0), peb(P + 1, 0);
  parts[0] = UnionPart{L.xadj, L.adj, L.ew, L.ew_kind, L.nw, 0, 0, L.n, L.nnz};
  srcs[0] = L.src;
  pnb[1] = L.n;
  peb[1] = L.nnz;
  for (uint32_t q = 0; q < Bn; ++q) {
    Job& jb = jobs[first + q];
    const InputGraph& g = *jb.g;
    jb.d0 = d;
    jb.nlevels = 1;
    jb.info.clear();
    lmgp_level_info i0{};
    i0.n = g.n;
    i0.m = g.nnz / 2;
    i0.m_prime = i0.m;
    jb.info.push_back(i0);
    parts[1 + q] = UnionPart{g.xadj.get(), g.adj.get(), g.ew(), g.ew_kind, g.nw.get(),
                             pnb[1 + q], peb[1 + q], g.n, g.nnz};
    srcs[1 + q] = g.src.get();
    pnb[2 + q] = pnb[1 + q] + g.n;
    peb[2 + q] = peb[1 + q] + g.nnz;
    N->graphs.push_back((uint32_t)(first + q));
    N->nbase.push_back(pnb[2 + q]);
    N->ebase.push_back(peb[2 + q]);
  }
  N->n = pnb[P];
  N->nnz = peb[P];
  DBuf<UnionPart> dparts(&pool_, s_, P);
  DBuf<const uint32_t*> dsrcs(&pool_, s_, P);
  DBuf<uint64_t> dnb(&pool_, s_, P + 1), deb(&pool_, s_, P + 1);
  h2d(dparts.get(), parts.data(), P, s_);
  h2d(dsrcs.get(), srcs.data(), P, s_);
  h2d(dnb.get(), pnb.data(), P + 1, s_);
  h2d(deb.get(), peb.data(), P + 1, s_);
  N->o_xadj.reset(&pool_, s_, N->n + 1);
  N->o_nw.reset(&pool_, s_, N->n ? N->n : 1);
  N->o_gid.reset(&pool_, s_, N->n ? N->n : 1);
  N->o_adj.reset(&pool_, s_, N->nnz ? N->nnz : 1);
  N->o_src.reset(&pool_, s_, N->nnz ? N->nnz : 1);
  if (narrow_) N->o_ew32.reset(&pool_, s_, N->nnz ? N->nnz : 1);
  else N->o_ew.reset(&pool_, s_, N->nnz ? N->nnz : 1);
  k_extend_nodes<<<grid_for(N->n, 256), 256, 0, s_>>>(dparts.get(), dnb.get(), P, N->n, L.gid, B0,
                                                      N->o_xadj.get(), N->o_nw.get(),
                                                      N->o_gid.get());
  LAUNCH_CHECK();
  if (N->nnz) {
    if (narrow_)
      k_extend_entries<int32_t><<<grid_for(N->nnz, 256), 256, 0, s_>>>(
          dparts.get(), dsrcs.get(), deb.get(), P, N->nnz, N->o_adj.get(), N->o_ew32.get(),
          N->o_src.get());
    else
      k_extend_entries<int64_t><<<grid_for(N->nnz, 256), 256, 0, s_>>>(
          dparts.get(), dsrcs.get(), deb.get(), P, N->nnz, N->o_adj.get(), N->o_ew.get(),
          N->o_src.get());
    LAUNCH_CHECK();
  }
  N->xadj = N->o_xadj.get();
  N->adj = N->o_adj.get();
  N->ew_kind = narrow_ ? EW_I32 : EW_I64;
  N->ew = narrow_ ? (const void*)N->o_ew32.get() : (const void*)N->o_ew.get();
  N->nw = N->o_nw.get();
  N->src = N->o_src.get();
  N->gid = N->o_gid.get();
  sync(s_);  // the host tables above are freed on return
  levels_.back() = std::move(N);
}

// -------------------------------------------------------------- LP driver --
// Rates the nodes of one sub-round: ra.list (and ra.cands) point at the
// first degree class; cnt/offs/degs per class, offs absolute in the list.
void Engine::rate_classes(RateArgs ra, const uint32_t* cnt, const uint32_t* offs,
                          const unsigned long long* degs, int ew_kind) {
  const uint32_t* list0 = ra.list;
  Cand* cands0 = ra.cands;
  auto span = [&](int c0, int c1) {
    RateArgs r = ra;
    r.list = list0 + (offs[c0] - offs[0]);
    if (cands0) r.cands = cands0 + (offs[c0] - offs[0]);
    r.count = 0;
    r.degsum = 0;
    for (int c = c0; c <= c1; ++c) {
      r.count += cnt[c];
      r.degsum += degs ? degs[c] : 0;
    }
    return r;
  };
  const bool dense = ra.few && ra.few <= FEW_LABELS && ra.mode == MODE_LP;
  // dense refinement rates every block class with one launch: only the lane
  // groups go through the merged small-class launch then
  const int nsmall = dense ? CLASS_BLOCK : GROUP_CLASSES;
  uint32_t gcnt[GROUP_CLASSES] = {}, goff[GROUP_CLASSES] = {};
  uint64_t gdeg = 0;
  for (int c = 0; c < nsmall; ++c) {
    gcnt[c] = cnt[c];
    goff[c] = offs[c] - offs[0];
    gdeg += degs ? degs[c] : 0;
  }
  launch_rate_groups(ew_kind, ra, gcnt, goff, gdeg, s_);
  if (dense) {  // refinement, few blocks: dense LDS rows, one launch per row width
    launch_rate(CLASS_BLOCK, ew_kind, span(CLASS_BLOCK, CLASS_BLOCK + 1), s_);
    launch_rate(CLASS_BLOCK + 2, ew_kind, span(CLASS_BLOCK + 2, CLASS_BIG - 1), s_);
    launch_rate(CLASS_BIG, ew_kind, span(CLASS_BIG, CLASS_GLOBAL - 1), s_);
  } else {
    for (int c = GROUP_CLASSES; c < CLASS_BIG; ++c) launch_rate(c, ew_kind, span(c, c), s_);
    for (int c = CLASS_BIG; c < CLASS_GLOBAL; ++c) {
      if (packed_) launch_rate(c, ew_kind, span(c, c), s_);
      else launch_rate_hubs(ew_kind, span(c, c), pool_, s_);
    }
  }
  launch_rate_hubs(ew_kind, span(CLASS_GLOBAL, CLASS_GLOBAL), pool_, s_);
}

void Engine::run_lp(Level& L, std::vector<Job>& jobs, const LpSpec& spec,
                    std::vector<uint8_t>& active, uint32_t* label, int64_t* W, size_t nlabels,
                    uint32_t* csize, const std::vector<uint64_t>& label_base,
                    std::vector<uint64_t>* ncl, std::vector<uint32_t>& rounds_run) {
  const uint32_t B = (uint32_t)L.graphs.size();
  const uint64_t n = L.n;
  const uint32_t S = p_.subrounds;
  const uint32_t NB = S * NCLASS;
  rounds_run.assign(B, 0);
  if (n == 0) return;
  std::vector<GraphDesc> gd(B);
  for (uint32_t b = 0; b < B; ++b) {
    const Job& jb = jobs[L.graphs[b]];
    gd[b] = GraphDesc{};
    gd[b].node_base = L.nbase[b];
    gd[b].nodes = L.nbase[b + 1] - L.nbase[b];
    gd[b].label_base = label_base[b];
    gd[b].cap = spec.refine ? jb.lmax : jb.U;
    gd[b].subrounds = S;
    gd[b].active = active[b];
  }
  DBuf<Cand> cands(&pool_, s_, n);
  DBuf<uint32_t> list(&pool_, s_, n);
  DBuf<LabelTally> tally(&pool_, s_, nlabels);
  DBuf<uint32_t> segbase(&pool_, s_, nlabels);
  DBuf<uint32_t> ovtgts(&pool_, s_, n), cpos(&pool_, s_, n), seg(&pool_, s_, n);
  DBuf<SegRec> segrec(&pool_, s_, n);
  DBuf<uint8_t> adm(&pool_, s_, n);
  // each node's bucket from the count pass for the scatter (ids fit a byte)
  DBuf<uint8_t> bkt;
  if (NB <= 255) bkt.reset(&pool_, s_, n);
  DBuf<uint32_t> boffs(&pool_, s_, NB), bfill(&pool_, s_, NB);
  // per-round state read by the host in one copy: bucket counts, bucket
  // degree sums, active flags
  DBuf<unsigned long long> rstate(&pool_, s_, 2 * NB + 2 * B);
  const size_t nstate = 2 * NB + B;
  unsigned long long* hstate = pinned_state(nstate);
  std::memset(hstate, 0, nstate * sizeof(unsigned long long));
  tally.zero();
  std::vector<uint32_t> cnt(NB), offs(NB);
  std::vector<unsigned long long> degs(NB);
  // refinement with few labels: demand and segment slots from block-privatised
  // histograms in the admission instead of contended atomics
  const uint32_t few = spec.refine && nlabels <= FEW_LABELS ? (uint32_t)nlabels : 0u;
  // the rating kernels' class cut-offs: dense per-block rows when few
  const bool dense = few != 0;
  // at most 256 labels on a level whose 4-byte labels outgrow an XCD's L2:
  // the neighbours' labels are gathered from a byte copy
  DBuf<uint8_t> label8;
  if (few && nlabels <= 256 && n >= LABEL8_MIN_NODES) {
    label8.reset(&pool_, s_, n);
    k_to_u8<<<grid_for(n, 256), 256, 0, s_>>>(label, n, label8.get());
    LAUNCH_CHECK();
  }
  // refinement of a large level: only nodes with a neighbour in another block
  // can move, so only those (and the neighbours of nodes that moved since)
  // are bucketed and rated, one sub-round at a time.  Exact: every node left
  // out has all its neighbours in its own block.  Used when at most half of
  // the nodes are on the boundary.
  DBuf<uint8_t> bflag;
  bool bmode = false;
  // LMGP_BOUNDARY_MIN_NODES overrides the size threshold (tests use it to run
  // the mode on small levels)
  const char* bmin_env = std::getenv("LMGP_BOUNDARY_MIN_NODES");
  const uint64_t bmin = bmin_env ? std::strtoull(bmin_env, nullptr, 10) : BOUNDARY_MIN_NODES;
  if (spec.refine && n >= bmin && L.nnz && !(p_.graph_rounds && n <= REPLAY_MAX_NODES)) {
    ProfScope prof("rf:boundary", (8 + (label8.get() ? 2 : 8)) * L.nnz + 2 * n, s_);
    bflag.reset(&pool_, s_, (n + 7) / 8 * 8);  // zero-padded to whole 8-byte words
    bflag.zero();
    k_boundary<<<grid_for(L.nnz, 256), 256, 0, s_>>>(L.src, L.adj, L.nnz, label, label8.get(),
                                                      bflag.get());
    LAUNCH_CHECK();
    DBuf<unsigned long long> bcount(&pool_, s_, 1);
    bcount.zero();
    unsigned g = grid_for(n, 256);
    k_count_flags<<<g > 1024 ? 1024 : g, 256, 0, s_>>>(bflag.get(), n, bcount.get());
    LAUNCH_CHECK();
    unsigned long long nb = 0;
    read_now(&nb, bcount.get(), sizeof(nb), s_);
    bmode = 2 * nb <= n;
    if (!bmode) bflag.clear();
  }
  // boundary mode: each sub-round's flagged nodes, listed before bucketing
  DBuf<uint32_t> subids, subcnt;
  DBuf<unsigned long long> nsub;
  DBuf<uint8_t> subsel;  // each flag word's selection of the sub-round
  if (bmode) {
    subids.reset(&pool_, s_, n);
    subcnt.reset(&pool_, s_, SUB_LIST_BLOCKS);
    nsub.reset(&pool_, s_, 1);
    subsel.reset(&pool_, s_, (n + 7) / 8);
  }
  const std::vector<CutPreset>& presets = cut_presets(dense);
  int preset = p_.tune >= LMGP_TUNE_FORCE ? (int)((p_.tune - LMGP_TUNE_FORCE) % presets.size()) : 0;
  const uint64_t tsub = spec.refine ? TAG_RSUB : TAG_SUB;
  const uint64_t ttie = spec.refine ? TAG_RTIE : TAG_TIE;
  const uint64_t tadm = spec.refine ? TAG_RADM : TAG_ADM;
  // hash prefixes of every round, uploaded once
  const uint32_t R = spec.rounds;
  std::vector<uint64_t> pre((size_t)R * B * 3);
  for (uint32_t r = 0; r < R; ++r)
    for (uint32_t b = 0; b < B; ++b) {
      const Job& jb = jobs[L.graphs[b]];
      uint64_t* q = &pre[((size_t)r * B + b) * 3];
      const uint64_t lv = spec.level - jb.d0;  // the graph's own level index
      q[0] = chain(jb.seed, tsub, {lv, r});
      q[1] = chain(jb.seed, ttie, {lv, r});
      q[2] = chain(jb.seed, tadm, {lv, r});
    }
  // the graphs' control state (zero: moves, cluster-count changes, round
  // moves, rounds run, admission overflow counters), their cluster counts,
  // graph table and the hash prefixes of every round: one block, one upload
  const size_t o_delta = 8 * (size_t)B, o_round = 16 * (size_t)B, o_rounds = 24 * (size_t)B;
  const size_t o_ov = o_rounds + 8 * (((size_t)B + 1) / 2), o_ncl = o_ov + 8;
  const size_t o_gd = o_ncl + 8 * (size_t)B, o_pre = o_gd + sizeof(GraphDesc) * B;
  const size_t ctl_bytes = o_pre + 8 * pre.size();
  std::vector<uint8_t> hctl(ctl_bytes, 0);
  if (ncl) std::memcpy(&hctl[o_ncl], ncl->data(), 8 * (size_t)B);
  std::memcpy(&hctl[o_gd], gd.data(), sizeof(GraphDesc) * B);
  if (!pre.empty()) std::memcpy(&hctl[o_pre], pre.data(), 8 * pre.size());
  DBuf<uint8_t> dctl(&pool_, s_, ctl_bytes);
  h2d(dctl.get(), hctl.data(), ctl_bytes, s_);
  unsigned long long* const dmoves = (unsigned long long*)dctl.get();
  unsigned long long* const ddelta = (unsigned long long*)(dctl.get() + o_delta);
  unsigned long long* const dround = (unsigned long long*)(dctl.get() + o_round);
  uint32_t* const drounds = (uint32_t*)(dctl.get() + o_rounds);
  uint32_t* const ovtotal = (uint32_t*)(dctl.get() + o_ov);
  unsigned long long* const dncl = (unsigned long long*)(dctl.get() + o_ncl);
  GraphDesc* const dgd = (GraphDesc*)(dctl.get() + o_gd);
  const uint64_t* const dpre = (const uint64_t*)(dctl.get() + o_pre);
  // one graph's cluster-count changes, one per admission apply block
  DBuf<int64_t> nclpart;
  if (ncl && B == 1 && !L.gid) nclpart.reset(&pool_, s_, grid_for(n ? n : 1, 256));
  LpCtl ctl{dgd, B, dmoves, ddelta, dround, ncl ? dncl : nullptr, drounds, rstate.get(), NB,
            ovtotal, dpre, p_.shrink_num, p_.shrink_den};
  BucketArgs ba{};
  ba.xadj = L.xadj;
  ba.gid = L.gid;
  ba.gd = dgd;
  ba.n = n;
  ba.nw = L.nw;
  ba.mode = 0;
  ba.nbuckets = NB;
  ba.counts = rstate.get();
  ba.degs = rstate.get() + NB;
  ba.degs_all = Profiler::get().on() || p_.tune || p_.graph_rounds;
  ba.offs = boffs.get();
  ba.fill = bfill.get();
  ba.list = list.get();
  ba.bkt = NB <= 255 ? bkt.get() : nullptr;
  ba.cuts = presets[preset].cuts;
  ba.only = bmode ? bflag.get() : nullptr;
  ba.only_sub = 0;
  // the three bucket passes: over all nodes, or (boundary mode) over the list
  // of the flagged nodes of sub-round ba.only_sub
  auto bucket_passes = [&](hipStream_t st) {
    if (!bmode) {
      launch_bucket_count(ba, st);
      launch_bucket_offsets(ba, st);
      launch_bucket_scatter(ba, st);
      return;
    }
    launch_sub_list(ba, bflag.get(), subcnt.get(), subsel.get(), subids.get(), nsub.get(), st);
    BucketArgs bl = ba;
    bl.only = nullptr;
    bl.ids = subids.get();
    bl.nids = nsub.get();
    launch_bucket_count(bl, st);
    launch_bucket_offsets(bl, st);
    launch_bucket_scatter(bl, st);
  };
  // Stop decisions (node-reduction cap after a sub-round, no moves in a
  // round) are taken on the device; the host reads the active flags together
  // with the next round's bucket counts, in one copy per round.
  auto begin_round = [&](uint32_t r) {
    {
      // every node's offsets and weight read twice (count, scatter), its
      // list slot written
      ProfScope prof(spec.refine ? "rf:bucket" : "cl:bucket", 52 * n, s_);
      k_lp_round<<<1, 256, 0, s_>>>(ctl, r, nullptr);  // also clears the bucket counters
      LAUNCH_CHECK();
      // the lists too, before the host waits: the scatter needs only the
      // device's offsets, and the first rating launch then follows the wait
      bucket_passes(s_);
    }
    d2h(hstate, rstate.get(), nstate, s_);
    sync(s_);
    for (uint32_t i = 0; i < NB; ++i) {
      cnt[i] = (uint32_t)hstate[i];
      degs[i] = hstate[NB + i];
    }
  };
  // boundary mode: the lists of sub-round sr (> 0) are built after the
  // moves of the sub-rounds before it (flags have grown since)
  auto begin_sub = [&](uint32_t sr) {
    {
      // the flags (8 per word) and, per listed node, its list slot written
      // and read and its bucket pass bytes (an eighth of the nodes, say)
      ProfScope prof("rf:bucket", n + 60 * (n / 8), s_);
      device_zero(rstate.get(), 2 * NB * sizeof(unsigned long long), s_);
      ba.only_sub = sr;
      bucket_passes(s_);
    }
    d2h(hstate, rstate.get(), 2 * NB, s_);
    sync(s_);
    for (uint32_t i = 0; i < NB; ++i) {
      cnt[i] = (uint32_t)hstate[i];
      degs[i] = hstate[NB + i];
    }
  };
  auto bucket_offsets = [&]() {
    uint32_t run = 0;
    for (uint32_t i = 0; i < NB; ++i) {
      offs[i] = run;  // the same prefix the device computed into boffs
      run += cnt[i];
    }
  };
  auto rating_args = [&](uint32_t sr) {
    RateArgs ra{};
    ra.xadj = L.xadj;
    ra.adj = L.adj;
    ra.ew = L.ew;
    ra.nw = L.nw;
    ra.label = label;
    ra.W = W;
    ra.gid = L.gid;
    ra.gd = dgd;
    ra.mode = MODE_LP;
    ra.phase = spec.refine ? 1 : 0;
    ra.packed = packed_ ? 1 : 0;
    ra.few = few;
    ra.tally = tally.get();
    ra.list = list.get() + offs[sr * NCLASS];
    ra.cands = cands.get();
    ra.label8 = label8.get();
    return ra;
  };
  // Autotuning: the first round's buckets under the default table give the
  // level's degree histogram; an unseen one is timed under every table on
  // the first sub-round (rating only, no tallies) and the fastest is cached.
  auto autotune = [&]() {
    uint64_t hist[NCLASS] = {};
    uint64_t entries = 0;
    for (uint32_t i = 0; i < NB; ++i) {
      hist[i % NCLASS] += cnt[i];
      entries += degs[i];
    }
    const std::string key = tune_key(spec.refine ? 1 : 0, dense, L.ew_kind, packed_, hist);
    Tuner& tuner = Tuner::get();
    int best = tuner.lookup(key);
    if (best < 0) {
      best = 0;
      if (entries >= TUNE_MIN_ENTRIES) {
        hipEvent_t e0, e1;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        float best_ms = 0.f;
        for (int p = 0; p < (int)presets.size(); ++p) {
          ba.cuts = presets[p].cuts;
          begin_round(0);
          bucket_offsets();
          RateArgs ra = rating_args(0);
          ra.trial = 1;
          float ms = 0.f;
          for (int rep = 0; rep < 2; ++rep) {  // the first one also warms the caches
            HIP_CHECK(hipEventRecord(e0, s_));
            rate_classes(ra, &cnt[0], &offs[0], &degs[0], L.ew_kind);
            HIP_CHECK(hipEventRecord(e1, s_));
            HIP_CHECK(hipEventSynchronize(e1));
            HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
          }
          tuner.note_trial();
          if (p == 0 || ms < best_ms) {
            best_ms = ms;
            best = p;
          }
        }
        HIP_CHECK(hipEventDestroy(e0));
        HIP_CHECK(hipEventDestroy(e1));
      }
      tuner.store(key, best);
    }
    preset = best;
    ba.cuts = presets[preset].cuts;
    begin_round(0);
  };
  auto admit_args = [&]() {
    AdmitArgs aa{};
    aa.cands = cands.get();
    aa.W = W;
    aa.Wmut = W;
    aa.nw = L.nw;
    aa.label = label;
    aa.gid = L.gid;
    aa.gd = dgd;
    aa.tally = tally.get();
    aa.segbase = segbase.get();
    aa.ovtotal = ovtotal;
    aa.ovcount = ovtotal + 1;
    aa.ovtgts = ovtgts.get();
    aa.adm = adm.get();
    aa.cpos = cpos.get();
    aa.seg = seg.get();
    aa.rec = segrec.get();
    aa.csize = csize;
    // refinement: no control kernel after a sub-round (its graphs change only
    // at round starts), the moves mark the round directly
    aa.moves = (uint64_t*)(ncl ? dmoves : dround);
    aa.clear_ov = ncl ? 0 : 1;
    aa.ncl_count = ncl ? (int64_t*)ddelta : nullptr;
    aa.nlabels = nlabels;
    aa.ncl_part = ncl && B == 1 && !L.gid ? nclpart.get() : nullptr;
    aa.few = few;
    aa.label8 = label8.get();
    return aa;
  };
  // Replayed rounds: on a small level the rounds after the first are launch
  // bound, so one round is captured into a HIP graph and replayed.  Its
  // launches cannot depend on host-read counts: grids are upper bounds (a
  // class never holds more nodes than in the first round, as graphs only
  // stop and node weights are fixed), and the kernels take their counts and
  // list ranges from the plan k_lp_plan writes on the device.  Hub nodes
  // (global tables, sized on the host) keep a level on the unplanned path.
  uint64_t ub[NCLASS] = {};
  auto plannable = [&]() {
    for (int c = 0; c < NCLASS; ++c) ub[c] = 0;
    for (uint32_t i = 0; i < NB; ++i) ub[i % NCLASS] += cnt[i];
    if (ub[CLASS_GLOBAL]) return false;
    if (!dense && !packed_ && ub[CLASS_BIG] + ub[CLASS_BIG + 1]) return false;
    return true;
  };
  DBuf<SubPlan> dplan;
  DBuf<uint32_t> drctr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  auto capture_round = [&]() {
    dplan.reset(&pool_, s_, S);
    drctr.reset(&pool_, s_, 1);
    const hipStream_t cs = capture_stream();
    const hipStream_t saved = s_;
    ProfSuspend quiet;
    uint64_t umax = 0;
    for (int c = 0; c < NCLASS; ++c) umax += ub[c];
    HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    s_ = cs;
    try {
      k_lp_round<<<1, 256, 0, cs>>>(ctl, 0, drctr.get());
      LAUNCH_CHECK();
      launch_bucket_count(ba, cs);
      launch_bucket_offsets(ba, cs);
      launch_lp_plan(rstate.get(), boffs.get(), S, dense ? 1 : 0, dplan.get(), cs);
      launch_bucket_scatter(ba, cs);
      for (uint32_t sr = 0; sr < S; ++sr) {
        RateArgs ra = rating_args(0);
        ra.list = list.get();
        ra.plan = dplan.get() + sr;
        const int nsmall = dense ? CLASS_BLOCK : GROUP_CLASSES;
        uint32_t gcnt[GROUP_CLASSES] = {}, goff[GROUP_CLASSES] = {};
        for (int c = 0; c < nsmall; ++c) gcnt[c] = (uint32_t)ub[c];
        launch_rate_groups(L.ew_kind, ra, gcnt, goff, 0, cs);
        auto span = [&](int c0, int c1) {
          RateArgs r = ra;
          r.plan_c0 = c0;
          r.plan_c1 = c1;
          uint64_t u = 0;
          for (int c = c0; c <= c1; ++c) u += ub[c];
          r.count = (uint32_t)u;
          return r;
        };
        if (dense) {
          launch_rate(CLASS_BLOCK, L.ew_kind, span(CLASS_BLOCK, CLASS_BLOCK + 1), cs);
          launch_rate(CLASS_BLOCK + 2, L.ew_kind, span(CLASS_BLOCK + 2, CLASS_BIG - 1), cs);
          launch_rate(CLASS_BIG, L.ew_kind, span(CLASS_BIG, CLASS_GLOBAL - 1), cs);
        } else {
          for (int c = GROUP_CLASSES; c < CLASS_GLOBAL; ++c)
            launch_rate(c, L.ew_kind, span(c, c), cs);
        }
        AdmitArgs aa = admit_args();
        aa.plan = dplan.get() + sr;
        aa.max_cands = (uint32_t)umax;
        launch_admit(aa, cs);
        if (ncl)
          k_lp_after_sub<<<1, 256, 0, cs>>>(ctl, aa.ncl_part, grid_for(aa.max_cands, 256));
        LAUNCH_CHECK();
      }
    } catch (...) {
      s_ = saved;
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    s_ = saved;
    HIP_CHECK(hipStreamEndCapture(cs, &graph));
    HIP_CHECK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    k_set_u32<<<1, 1, 0, s_>>>(drctr.get(), 1);  // the first replayed round
    LAUNCH_CHECK();
  };
  const bool want_replay = p_.graph_rounds && R > 1 && n <= REPLAY_MAX_NODES;
  bool replay = false;
  // the active flags the caller gets: those of the last round started (all
  // clear when the loop stops because no graph is left)
  std::vector<unsigned long long> hflags(2 * B);
  bool flags_from_peek = false;
  try {
    for (uint32_t r = 0; r < R; ++r) {
      if (!replay) {
        ba.only_sub = 0;
        begin_round(r);
        if (r == 0 && p_.tune == LMGP_TUNE_AUTO) autotune();
        bool any = false;
        for (uint32_t b = 0; b < B; ++b) any |= hstate[2 * NB + b] != 0;
        if (!any) break;
        bucket_offsets();
        for (uint32_t sr = 0; sr < S; ++sr) {
          if (bmode && sr > 0) {
            begin_sub(sr);
            bucket_offsets();
          }
          uint32_t total = 0;
          for (int c = 0; c < NCLASS; ++c) total += cnt[sr * NCLASS + c];
          if (total == 0) continue;
          RateArgs ra = rating_args(sr);
          rate_classes(ra, &cnt[sr * NCLASS], &offs[sr * NCLASS], &degs[sr * NCLASS], L.ew_kind);
          AdmitArgs aa = admit_args();
          aa.max_cands = total;
          {
            // per candidate slot: the slot (16 B) read by classification,
            // scatter and apply, its target's demand and weight (16 B)
            ProfScope prof(spec.refine ? "rf:admission" : "cl:admission", 64ull * total, s_);
            launch_admit(aa, s_);  // ovtotal was cleared by the control kernel or the apply
            if (ncl)
              k_lp_after_sub<<<1, 256, 0, s_>>>(ctl, aa.ncl_part, grid_for(total, 256));
            LAUNCH_CHECK();
          }
          if (bmode) {  // the next sub-round (or round) buckets from the grown flags
            k_mark_moved<<<grid_for(total, 256), 256, 0, s_>>>(cands.get(), adm.get(), total,
                                                              L.xadj, L.adj, bflag.get());
            LAUNCH_CHECK();
          }
        }
        // switch to replay after the first round; the capture waits until a
        // round is known to follow (a level that stops here pays nothing)
        if (r == 0 && want_replay && plannable()) replay = true;
      } else {
        if (!gexec) capture_round();
        HIP_CHECK(hipGraphLaunch(gexec, s_));
      }
      if (replay && r + 1 < R) {
        // one copy per round, as on the unplanned path: whether any graph
        // takes part in the next round
        k_lp_peek<<<1, 256, 0, s_>>>(ctl);
        LAUNCH_CHECK();
        d2h(hflags.data(), rstate.get() + 2 * NB, 2 * B, s_);
        sync(s_);
        bool any = false;
        for (uint32_t b = 0; b < B; ++b) any |= hflags[B + b] != 0;
        if (!any) {
          flags_from_peek = true;
          break;
        }
      }
    }
  } catch (...) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  std::vector<unsigned long long> hncl(B);
  d2h(rounds_run.data(), drounds, B, s_);
  if (ncl) d2h(hncl.data(), dncl, B, s_);
  if (replay && !flags_from_peek) d2h(hflags.data(), rstate.get() + 2 * NB, B, s_);
  sync(s_);
  if (gexec) HIP_CHECK(hipGraphExecDestroy(gexec));
  if (graph) HIP_CHECK(hipGraphDestroy(graph));
  if (ncl)
    for (uint32_t b = 0; b < B; ++b) (*ncl)[b] = hncl[b];
  for (uint32_t b = 0; b < B; ++b)
    active[b] = (!replay ? hstate[2 * NB + b] : flags_from_peek ? hflags[B + b] : hflags[b]) != 0;
}

// ------------------------------------------------------------ clustering --
void Engine::two_hop(Level& L, std::vector<Job>& jobs, const std::vector<uint8_t>& which,
                     uint32_t level, uint32_t* label, int64_t* W, uint32_t* csize,
                     std::vector<uint64_t>& ncl) {
  const uint32_t B = (uint32_t)L.graphs.size();
  const uint64_t n = L.n;
  std::vector<GraphDesc> gd(B);
  for (uint32_t b = 0; b < B; ++b) {
    const Job& jb = jobs[L.graphs[b]];
    gd[b] = GraphDesc{};
    gd[b].node_base = L.nbase[b];
    gd[b].nodes = L.nbase[b + 1] - L.nbase[b];
    gd[b].label_base = L.nbase[b];
    gd[b].cap = jb.U;
    gd[b].pre_tie = chain(jb.seed, TAG_FAV, {(uint64_t)(level - jb.d0)});
    gd[b].pre_two = chain(jb.seed, TAG_TWOHOP, {(uint64_t)(level - jb.d0)});
    gd[b].active = which[b];
    gd[b].subrounds = 1;
  }
  DBuf<GraphDesc> dgd(&pool_, s_, B);
  h2d(dgd.get(), gd.data(), B, s_);
  // favourites of the singletons with neighbours
  DBuf<unsigned long long> bcount(&pool_, s_, 2 * NCLASS);  // counts, then degree sums
  DBuf<uint32_t> boffs(&pool_, s_, NCLASS), bfill(&pool_, s_, NCLASS);
  DBuf<uint32_t> list(&pool_, s_, n), fav(&pool_, s_, n);
  BucketArgs ba{};
  ba.xadj = L.xadj;
  ba.gid = L.gid;
  ba.gd = dgd.get();
  ba.n = n;
  ba.mode = 1;
  ba.label = label;
  ba.csize = csize;
  ba.nw = L.nw;
  ba.nbuckets = NCLASS;
  ba.counts = bcount.get();
  ba.degs = bcount.get() + NCLASS;
  ba.degs_all = Profiler::get().on() || p_.tune;
  ba.offs = boffs.get();
  ba.fill = bfill.get();
  ba.list = list.get();
  ba.cuts = default_cuts();
  bcount.zero();
  launch_bucket_count(ba, s_);
  launch_bucket_offsets(ba, s_);
  launch_bucket_scatter(ba, s_);  // before the wait, as in run_lp
  std::vector<unsigned long long> hcnt(2 * NCLASS);
  std::vector<uint32_t> cnt(NCLASS), offs(NCLASS);
  d2h(hcnt.data(), bcount.get(), 2 * NCLASS, s_);
  sync(s_);
  uint32_t run = 0;
  for (int c = 0; c < NCLASS; ++c) {
    cnt[c] = (uint32_t)hcnt[c];
    offs[c] = run;
    run += cnt[c];
  }
  RateArgs ra{};
  ra.xadj = L.xadj;
  ra.adj = L.adj;
  ra.ew = L.ew;
  ra.nw = L.nw;
  ra.label = label;
  ra.W = W;
  ra.gid = L.gid;
  ra.gd = dgd.get();
  ra.mode = MODE_FAV;
  ra.phase = 2;
  ra.packed = packed_ ? 1 : 0;
  ra.fav = fav.get();
  ra.list = list.get();
  rate_classes(ra, cnt.data(), offs.data(), hcnt.data() + NCLASS, L.ew_kind);
  // order the singletons by (favourite, weight, hash, id)
  SingletonFlag sf{label, csize, L.nw, L.gid, dgd.get()};
  DBuf<uint32_t> pos(&pool_, s_, n + 1);
  exclusive_scan(sf, n, pos.get(), true, pool_, s_);
  uint32_t ns32 = 0;
  d2h(&ns32, pos.get() + n, 1, s_);
  sync(s_);
  const uint64_t ns = ns32;
  if (ns < 2) return;
  int kb = 1;  // bits of a segment key (< 2n + 2)
  while ((1ull << kb) <= 2 * n + 1) ++kb;
  int64_t maxcap = 1;
  uint64_t groups = 1;  // next-fit groups per segment: fewer than 2 c(V) / U + 1
  for (uint32_t b = 0; b < B; ++b) {
    if (!which[b]) continue;
    const Job& jb = jobs[L.graphs[b]];
    maxcap = std::max(maxcap, jb.U);
    groups = std::max<uint64_t>(groups, (uint64_t)(2 * (u128)jb.g->cV / (u128)jb.U) + 2);
  }
  int wb = 1;  // bits of a weight below the cap
  while (wb < 62 && (1ll << wb) <= maxcap - 1) ++wb;
  const bool one_key = kb + wb + 32 <= 64;
  const int sshift = one_key ? 32 + wb : 0;
  // per singleton: key and id written, read and written per 8-bit sort pass,
  // weight, prefix sum, successor, K jump tables, marks, scan and merge
  const int passes = one_key ? (kb + wb + 39) / 8 : (wb + 39) / 8 + (kb + 7) / 8;
  ProfScope prof_pack("fv:twohop_pack", (uint64_t)ns * (24ull * passes + 64), s_);
  DBuf<uint64_t> keys(&pool_, s_, ns), keys2(&pool_, s_, ns);
  DBuf<uint32_t> vals(&pool_, s_, ns), vals2(&pool_, s_, ns);
  const unsigned gs = grid_for(ns, 256);
  k_twohop_keys<<<grid_for(n, 256), 256, 0, s_>>>(sf, L.xadj, fav.get(), pos.get(), n, sshift,
                                                  keys.get(), vals.get());
  LAUNCH_CHECK();
  bool sw = radix_sort_pairs<uint32_t>(keys.get(), vals.get(), keys2.get(), vals2.get(), ns, 0,
                                       one_key ? kb + wb + 32 : wb + 32, pool_, s_);
  uint64_t* sk = sw ? keys2.get() : keys.get();
  uint32_t* sv = sw ? vals2.get() : vals.get();
  if (!one_key) {  // then stably by favourite
    uint64_t* ok = sw ? keys.get() : keys2.get();
    uint32_t* ov = sw ? vals.get() : vals2.get();
    k_twohop_favkeys<<<gs, 256, 0, s_>>>(sf, L.xadj, fav.get(), sv, ns, sk);
    LAUNCH_CHECK();
    if (radix_sort_pairs<uint32_t>(sk, sv, ok, ov, ns, 0, kb, pool_, s_)) sk = ok, sv = ov;
  }
  // next-fit groups of each favourite segment
  DBuf<uint32_t> last(&pool_, s_, 2 * n + 2);
  DBuf<uint64_t> E(&pool_, s_, ns + 1);
  k_seg_last<<<gs, 256, 0, s_>>>(sk, sshift, ns, last.get());
  LAUNCH_CHECK();
  exclusive_scan(SortedWeight{sv, L.nw}, ns, E.get(), true, pool_, s_);
  uint32_t K = 0;  // doubling levels: 2^K > groups - 1
  while (K < 32 && (1ull << K) < std::min<uint64_t>(ns, groups)) ++K;
  prof_pack.add_bytes((uint64_t)ns * 17 * K);
  DBuf<uint32_t> J(&pool_, s_, (size_t)std::max<uint32_t>(K, 1) * ns);
  k_nextfit<<<gs, 256, 0, s_>>>(sk, sshift, last.get(), E.get(), sv, L.gid, dgd.get(), ns, J.get());
  LAUNCH_CHECK();
  for (uint32_t k = 1; k < K; ++k) {
    k_jump<<<gs, 256, 0, s_>>>(J.get() + (size_t)(k - 1) * ns, ns, J.get() + (size_t)k * ns);
    LAUNCH_CHECK();
  }
  DBuf<uint8_t> mark(&pool_, s_, ns);
  k_mark_seg_first<<<gs, 256, 0, s_>>>(sk, sshift, ns, (uint8_t)(K + 1), mark.get());
  LAUNCH_CHECK();
  for (uint32_t k = K; k-- > 0;) {
    k_expand<<<gs, 256, 0, s_>>>(J.get() + (size_t)k * ns, ns, k, mark.get());
    LAUNCH_CHECK();
  }
  DBuf<uint64_t> sj(&pool_, s_, ns + 1);
  exclusive_scan(StartJoin{mark.get()}, ns, sj.get(), true, pool_, s_);
  DBuf<uint32_t> head(&pool_, s_, ns);
  DBuf<unsigned long long> joins(&pool_, s_, B);
  joins.zero();
  k_group_heads<<<gs, 256, 0, s_>>>(mark.get(), sj.get(), ns, sv, L.gid, head.get(), joins.get());
  LAUNCH_CHECK();
  std::vector<unsigned long long> hj(B);
  d2h(hj.data(), joins.get(), B, s_);
  sync(s_);
  std::vector<uint64_t> base(B), cap(B);
  uint64_t acc = 0;
  for (uint32_t b = 0; b < B; ++b) {
    base[b] = acc;
    acc += hj[b];
    const uint64_t nb = L.nbase[b + 1] - L.nbase[b];
    const uint64_t floor_cl = (uint64_t)(((u128)p_.shrink_den * nb + p_.shrink_num - 1) / p_.shrink_num);
    cap[b] = ncl[b] > floor_cl ? ncl[b] - floor_cl : 0;
    if (!which[b]) cap[b] = 0;
  }
  DBuf<uint64_t> dbase(&pool_, s_, B), dcap(&pool_, s_, B);
  h2d(dbase.get(), base.data(), B, s_);
  h2d(dcap.get(), cap.data(), B, s_);
  k_group_merge<<<gs, 256, 0, s_>>>(sv, mark.get(), sj.get(), head.get(), ns, L.gid, dbase.get(),
                                    dcap.get(), label, W, L.nw, csize);
  LAUNCH_CHECK();
  for (uint32_t b = 0; b < B; ++b) ncl[b] -= std::min<uint64_t>(hj[b], cap[b]);
  sync(s_);
}

void Engine::cluster(Level& L, std::vector<Job>& jobs, std::vector<uint8_t>& active,
                     DBuf<uint32_t>& label, DBuf<int64_t>& W, DBuf<uint32_t>& csize,
                     std::vector<uint64_t>& ncl, std::vector<lmgp_level_info>& stats) {
  const uint32_t B = (uint32_t)L.graphs.size();
  const uint64_t n = L.n;
  const uint32_t level = (uint32_t)levels_.size();  // 1-based index of L
  label.reset(&pool_, s_, n ? n : 1);
  W.reset(&pool_, s_, n ? n : 1);
  csize.reset(&pool_, s_, n ? n : 1);
  if (n) {
    k_iota<<<grid_for(n, 256), 256, 0, s_>>>(label.get(), n);
    LAUNCH_CHECK();
    k_copy_i64<<<grid_for(n, 256), 256, 0, s_>>>(W.get(), L.nw, n);
    LAUNCH_CHECK();
  }
  ncl.resize(B);
  for (uint32_t b = 0; b < B; ++b) ncl[b] = L.nbase[b + 1] - L.nbase[b];
  std::vector<uint8_t> act = active;
  std::vector<uint32_t> rounds;
  LpSpec spec{false, level, p_.lp_rounds};
  // member counts are read only after LP (2-hop, contraction): counted once
  // from the labels instead of two atomics per move
  run_lp(L, jobs, spec, act, label.get(), W.get(), n, nullptr, L.nbase, &ncl, rounds);
  if (n) {
    device_zero(csize.get(), n * sizeof(uint32_t), s_);
    unsigned g = grid_for(n, 256 * 16);
    k_label_sizes<<<g > 2048 ? 2048 : g, 256, 0, s_>>>(label.get(), n, csize.get());
    LAUNCH_CHECK();
  }
  stats.assign(B, lmgp_level_info{});
  std::vector<uint8_t> which(B, 0);
  bool any = false;
  for (uint32_t b = 0; b < B; ++b) {
    stats[b].lp_rounds = rounds[b];
    stats[b].nclusters_lp = ncl[b];
    const uint64_t nb = L.nbase[b + 1] - L.nbase[b];
    which[b] = active[b] && 2 * ncl[b] > nb;
    stats[b].twohop = which[b];
    any |= which[b] != 0;
  }
  if (any) two_hop(L, jobs, which, level, label.get(), W.get(), csize.get(), ncl);
}

void Engine::ensure_sorted(size_t i) {
  Level& L = *levels_.at(i);
  // the input level keeps the caller's row order (the oracle's order too)
  if (L.sorted || i == 0) return;
  DBuf<uint32_t> adj, src;
  DBuf<int64_t> ew;
  sort_rows(L.n, L.nnz, L.xadj, L.adj, L.ew, L.ew_kind, packed_ ? 1 : 0, adj, ew, src, pool_, s_);
  L.o_adj = std::move(adj);
  L.o_ew = std::move(ew);
  L.o_src = std::move(src);
  L.adj = L.o_adj.get();
  L.ew = L.o_ew.get();
  L.ew_kind = EW_I64;
  L.src = L.o_src.get();
  L.sorted = true;
  narrow_weights(L);
}

// A coarse level's int64 weights (o_ew) stored as int32 when narrow_.
void Engine::narrow_weights(Level& L) {
  L.o_ew32.clear();
  if (!narrow_ || !L.nnz || L.ew_kind != EW_I64) return;
  L.o_ew32.reset(&pool_, s_, L.nnz);
  k_narrow_i32<<<grid_for(L.nnz, 256), 256, 0, s_>>>(L.o_ew.get(), L.nnz, L.o_ew32.get());
  LAUNCH_CHECK();
  L.o_ew.clear();
  L.ew = L.o_ew32.get();
  L.ew_kind = EW_I32;
}

// -------------------------------------------------------------- coarsening --
void Engine::coarsen(std::vector<Job>& jobs) {
  Timer tm(s_);
  tm.start();
  build_union(jobs);
  // a rating never exceeds the total entry weight of its graph (contraction
  // only merges weight, sparsification only drops it)
  packed_ = true;
  for (auto& jb : jobs) packed_ &= jb.g->wtot < (1ull << 32) && jb.g->nnz < (1ull << 32);
  // the same bound on every coarse edge weight: int32 storage holds them
  // (a third fewer bytes per entry for every pass over a coarse level)
  narrow_ = true;
  for (auto& jb : jobs) narrow_ &= jb.g->wtot < (1ull << 31);
  for (auto& jb : jobs) {
    jb.nlevels = 1;
    jb.info.clear();
    lmgp_level_info i0{};
    i0.n = jb.g->n;
    i0.m = jb.g->nnz / 2;
    i0.m_prime = i0.m;
    jb.info.push_back(i0);
  }
  while (true) {
    if (admit && levels_.size() >= 2) {  // graphs joining the run in flight
      std::vector<Job> more = admit();
      if (!more.empty()) {
        const size_t first = jobs.size();
        for (Job& jb : more) jobs.push_back(std::move(jb));
        extend_union(jobs, first);
      }
    }
    Level& L = *levels_.back();
    const uint32_t B = (uint32_t)L.graphs.size();
    const uint32_t depth = (uint32_t)levels_.size();
    std::vector<uint8_t> active(B, 0);
    bool any = false;
    for (uint32_t b = 0; b < B; ++b) {
      const Job& jb = jobs[L.graphs[b]];
      const uint64_t nb = L.nbase[b + 1] - L.nbase[b];
      active[b] = ((u128)nb > (u128)p_.clim * jb.k) && depth - jb.d0 < p_.max_levels;
      any |= active[b] != 0;
    }
    if (!any) break;
    DBuf<uint32_t> label, csize;
    DBuf<int64_t> W;
    std::vector<uint64_t> ncl;
    std::vector<lmgp_level_info> stats;
    cluster(L, jobs, active, label, W, csize, ncl, stats);
    // shrink test before contraction: the coarse node count is the cluster count
    std::vector<uint8_t> keep(B, 0);
    std::vector<uint32_t> newpos(B, 0);
    uint32_t nkeep = 0;
    for (uint32_t b = 0; b < B; ++b) {
      const uint64_t nb = L.nbase[b + 1] - L.nbase[b];
      keep[b] = active[b] && (u128)p_.stop_den * ncl[b] <= (u128)p_.stop_num * nb;
      if (keep[b]) newpos[b] = nkeep++;
    }
    if (!nkeep) break;
    DBuf<uint8_t> dkeep(&pool_, s_, B);
    h2d(dkeep.get(), keep.data(), B, s_);
    ContractIn ci;
    ci.n = L.n;
    ci.xadj = L.xadj;
    ci.adj = L.adj;
    ci.ew = L.ew;
    ci.ew_kind = L.ew_kind;
    ci.narrow = narrow_;
    ci.label = label.get();
    ci.W = W.get();
    ci.csize = csize.get();
    ci.gid = L.gid;
    ci.keep = dkeep.get();
    ci.bounds = L.nbase;
    ci.all_kept = nkeep == B;
    ci.entries = L.nnz;
    ci.packed = packed_;
    ci.sorted = false;
    ContractOut co;
    contract_level(ci, co, pool_, s_);
    label.clear();
    csize.clear();
    W.clear();
    // the coarse union: kept graphs in order
    auto C = std::make_unique<Level>();
    C->n = co.nc;
    C->nnz = co.nnz;
    for (uint32_t b = 0; b < B; ++b)
      if (keep[b]) {
        C->graphs.push_back(L.graphs[b]);
        C->nbase.push_back(co.cid_at_bounds[b]);
      }
    C->nbase.push_back(co.nc);
    const uint32_t BC = nkeep;
    C->ebase.resize(BC + 1);
    // entry offsets of the graphs: one gather and one read (a single graph's
    // are 0 and the level's entry count)
    auto read_ebase = [&](const uint64_t* xadj, uint64_t total) {
      if (BC == 1) {
        C->ebase[0] = 0;
        C->ebase[1] = total;
        return;
      }
      DBuf<uint64_t> didx(&pool_, s_, BC + 1), dval(&pool_, s_, BC + 1);
      h2d(didx.get(), C->nbase.data(), BC + 1, s_);
      k_gather_u64<<<grid_for(BC + 1, 256), 256, 0, s_>>>(xadj, didx.get(), BC + 1, dval.get());
      LAUNCH_CHECK();
      d2h(C->ebase.data(), dval.get(), BC + 1, s_);
      sync(s_);
    };
    read_ebase(co.xadj.get(), co.nnz);
    // remap coarse graph ids to positions in the coarse union
    if (BC > 1) {
      std::vector<uint32_t> remap(B);
      for (uint32_t b = 0; b < B; ++b) remap[b] = newpos[b];
      DBuf<uint32_t> drm(&pool_, s_, B);
      h2d(drm.get(), remap.data(), B, s_);
      // gid values were written as old positions; translate in place
      if (co.nc) {
        k_remap_u32<<<grid_for(co.nc, 256), 256, 0, s_>>>(co.gid.get(), co.nc, drm.get());
        LAUNCH_CHECK();
      }
      sync(s_);  // drm is freed on return
    }
    // budget and sparsification per kept graph
    std::vector<SparsGraph> sgs(BC);
    std::vector<lmgp_level_info> infos(BC);
    bool any_trig = false;
    for (uint32_t c = 0, b = 0; b < B; ++b) {
      if (!keep[b]) continue;
      const Job& jb = jobs[L.graphs[b]];
      const uint64_t m_i = (L.ebase[b + 1] - L.ebase[b]) / 2;
      const uint64_t n_i = L.nbase[b + 1] - L.nbase[b];
      const uint64_t n_c = C->nbase[c + 1] - C->nbase[c];
      const uint64_t m_c = (C->ebase[c + 1] - C->ebase[c]) / 2;
      const u128 a1 = (u128)p_.tau_e_num * m_i / p_.tau_e_den;
      const u128 a2 = (u128)p_.tau_d_num * m_i * n_c / ((u128)p_.tau_d_den * n_i);
      const uint64_t m_hat = (uint64_t)(a1 < a2 ? a1 : a2);
      const bool trig = p_.sampler != 2 && (u128)m_c * p_.rho_den > (u128)p_.rho_num * m_hat;
      lmgp_level_info& li = infos[c];
      li = stats[b];
      li.n = n_c;
      li.m_prime = m_c;
      li.m_hat = m_hat;
      li.triggered = trig;
      SparsGraph& sg = sgs[c];
      sg.node_base = C->nbase[c];
      sg.e0 = C->ebase[c];
      sg.e1 = C->ebase[c + 1];
      sg.m_hat = m_hat;
      sg.triggered = trig;
      sg.sampler = p_.sampler;
      sg.pre = chain(jb.seed, TAG_SPARS, {(uint64_t)(depth + 1 - jb.d0)});
      any_trig |= trig;
      ++c;
    }
    // fire samplers: the draws scan rows in ascending order, so the coarse
    // rows are sorted first (and the level keeps them sorted)
    const bool fire = any_trig && (p_.sampler == 4 || p_.sampler == 5);
    if (any_trig) {
      const uint32_t* sadj = co.adj.get();
      const void* sew = co.weights();
      int sewk = co.ew_kind;
      const uint32_t* ssrc = co.src.get();
      DBuf<uint32_t> f_adj, f_src, score;
      DBuf<int64_t> f_ew;
      if (fire) {
        sort_rows(co.nc, co.nnz, co.xadj.get(), co.adj.get(), co.weights(), co.ew_kind,
                  packed_ ? 1 : 0, f_adj, f_ew, f_src, pool_, s_);
        sadj = f_adj.get();
        sew = f_ew.get();
        sewk = EW_I64;
        ssrc = f_src.get();
        FireLevel fl;
        fl.n = co.nc;
        fl.nnz = co.nnz;
        fl.xadj = co.xadj.get();
        fl.adj = sadj;
        fl.ew = sew;
        fl.ew_kind = sewk;
        fl.src = ssrc;
        fl.weighted = p_.sampler == 5;
        fl.p_num = p_.ff_p_num, fl.p_den = p_.ff_p_den;
        fl.nu_num = p_.ff_nu_num, fl.nu_den = p_.ff_nu_den;
        std::vector<FireGraph> fg(BC);
        for (uint32_t c = 0, b = 0; b < B; ++b) {
          if (!keep[b]) continue;
          const Job& jb = jobs[L.graphs[b]];
          const uint64_t lv = depth + 1 - jb.d0;  // the level being created
          FireGraph& g = fg[c];
          g.node_base = C->nbase[c];
          g.n = C->nbase[c + 1] - C->nbase[c];
          g.e0 = C->ebase[c];
          g.e1 = C->ebase[c + 1];
          g.pre_start = chain(jb.seed, TAG_FFSTART, {lv});
          g.pre_draw = chain(jb.seed, TAG_FFDRAW, {lv});
          g.pre_break = chain(jb.seed, TAG_FFBREAK, {lv});
          g.pre_claim = chain(jb.seed, TAG_FFCLAIM, {lv});
          g.active = sgs[c].triggered;
          ++c;
        }
        score.reset(&pool_, s_, co.nnz ? co.nnz : 1);
        fire_scores(fl, fg, score.get(), pool_, s_);
      }
      SparsOut so;
      sparsify_level(co.nc, co.nnz, co.xadj.get(), sadj, sew, sewk, ssrc,
                     BC > 1 ? co.gid.get() : nullptr, fire ? score.get() : nullptr, sgs, so,
                     pool_, s_);
      C->nnz = so.nnz;
      C->o_xadj = std::move(so.xadj);
      C->o_adj = std::move(so.adj);
      C->o_ew = std::move(so.ew);
      C->o_ew32 = std::move(so.ew32);
      C->ew_kind = so.ew_kind;
      C->o_src = std::move(so.src);
      read_ebase(C->o_xadj.get(), C->nnz);
    } else {
      C->o_xadj = std::move(co.xadj);
      C->o_adj = std::move(co.adj);
      C->o_ew = std::move(co.ew);
      C->o_ew32 = std::move(co.ew32);
      C->ew_kind = co.ew_kind;
      C->o_src = std::move(co.src);
    }
    C->o_nw = std::move(co.nw);
    if (BC > 1) C->o_gid = std::move(co.gid);
    C->sorted = fire;
    C->xadj = C->o_xadj.get();
    C->adj = C->o_adj.get();
    C->ew = C->ew_kind == EW_I32 ? (const void*)C->o_ew32.get() : (const void*)C->o_ew.get();
    C->nw = C->o_nw.get();
    C->src = C->o_src.get();
    C->gid = BC > 1 ? C->o_gid.get() : nullptr;
    L.map = std::move(co.map);
    for (uint32_t c = 0; c < BC; ++c) {
      Job& jb = jobs[C->graphs[c]];
      lmgp_level_info li = infos[c];
      li.m = (C->ebase[c + 1] - C->ebase[c]) / 2;
      li.w_t = sgs[c].triggered ? sgs[c].w_t : 0;
      li.n_gt = sgs[c].n_gt;
      li.n_eq = sgs[c].n_eq;
      jb.info.push_back(li);
      jb.nlevels++;
    }
    levels_.push_back(std::move(C));
  }
  // The initial partitioning visits neighbours in ascending order; coarse
  // rows are built in hash order.  The device search expands rows in stored
  // order, so a coarsest level bisected there is sorted here.  The host search
  // can order what each row scan finds itself; it does so on dense coarsest
  // levels (average degree >= 64), whose sort would cost the device far more
  // than the host's few short sorts, and gets sparse ones sorted.
  for (size_t j = 1; j < levels_.size(); ++j) {
    bool coarsest = false;
    for (uint32_t g : levels_[j]->graphs) coarsest |= jobs[g].top() == j;
    if (coarsest && (ip_on_device(jobs, j) || levels_[j]->nnz < 64 * levels_[j]->n))
      ensure_sorted(j);
  }
  t_coarsen_ns = tm.stop_ns();
}

bool Engine::ip_on_device(const std::vector<Job>& jobs, size_t j) const {
  if (!p_.ip_device || j >= levels_.size()) return false;
  const Level& L = *levels_[j];
  uint64_t Ktot = 0;
  for (const Job& jb : jobs) Ktot += jb.k;
  uint32_t taking = 0;
  for (uint32_t g : L.graphs) taking += jobs[g].top() == j;
  // block ids, node ids and frontier ranks are 32-bit in the device search
  if (!taking || L.nnz >= (1ull << 32) || L.n >= (1ull << 31) || Ktot >= IP_NONE) return false;
  // automatic choice: the device search gives each subproblem one workgroup,
  // which pays when many graphs are bisected side by side; a few large
  // coarsest levels are faster on the host's cores
  return p_.ip_device != LMGP_IP_AUTO || taking >= IP_DEVICE_MIN_GRAPHS;
}

// ------------------------------------------------------------ partitioning --
namespace {
// Page-locked host copies of a coarsest level for the host bisection: the
// device writes them directly (a pageable destination is staged through a
// bounce buffer and copied again by the CPU).  Buffer sets are pooled across
// calls and threads, grown on demand and kept until the process ends.
struct IpHostBuffers {
  uint64_t* xadj = nullptr;
  uint32_t* adj = nullptr;
  uint16_t* adj16 = nullptr;
  int64_t* nw = nullptr;
  size_t cx = 0, ca = 0, ca16 = 0, cn = 0;
  bool pageable = false;  // plain host memory (allocation-free calls), not pooled
};

// Neighbour ids of a graph's entries as 16-bit local ids (graphs of at most
// 2^16 nodes): half the bytes to copy to the host.
__global__ void k_local_u16(const uint32_t* adj, uint64_t m, uint32_t n0, uint16_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = (uint16_t)(adj[i] - n0);
}
template <typename T>
T* pinned_grow(T*& p, size_t& cap, size_t n, bool pageable) {
  if (n > cap) {
    if (p) {
      if (pageable) std::free(p);
      else HIP_CHECK(hipHostFree(p));
    }
    p = nullptr;
    cap = 0;
    if (pageable) {
      p = (T*)std::malloc((n ? n : 1) * sizeof(T));
      if (!p) throw OutOfMemory("host buffer of " + std::to_string(n * sizeof(T)) + " bytes");
    } else {
      HIP_CHECK(hipHostMalloc((void**)&p, (n ? n : 1) * sizeof(T), hipHostMallocDefault));
    }
    cap = n;
  }
  return p;
}
std::mutex ip_pool_mu;
std::vector<IpHostBuffers*> ip_pool;
struct IpBuffersLease {
  IpHostBuffers* b;
  IpBuffersLease() {
    if (no_alloc_mode()) {
      b = new IpHostBuffers;
      b->pageable = true;
      return;
    }
    std::lock_guard<std::mutex> g(ip_pool_mu);
    if (ip_pool.empty()) {
      b = new IpHostBuffers;
    } else {
      b = ip_pool.back();
      ip_pool.pop_back();
    }
  }
  ~IpBuffersLease() {
    if (b->pageable) {
      std::free(b->xadj);
      std::free(b->adj);
      std::free(b->adj16);
      std::free(b->nw);
      delete b;
      return;
    }
    std::lock_guard<std::mutex> g(ip_pool_mu);
    ip_pool.push_back(b);
  }
};
}  // namespace

void Engine::partition(std::vector<Job>& jobs, uint32_t* const* block_out, bool on_device) {
  const uint32_t NJ = (uint32_t)jobs.size();
  std::vector<uint64_t> kbase(NJ + 1, 0);
  for (uint32_t g = 0; g < NJ; ++g) kbase[g + 1] = kbase[g] + jobs[g].k;
  const uint64_t Ktot = kbase[NJ];
  Timer tm(s_);
  // initial partitioning of every graph's coarsest level: on the device, all
  // graphs whose coarsest level is level j at once, or on the host
  tm.start();
  std::vector<std::vector<uint32_t>> ip(NJ);
  std::vector<DBuf<uint32_t>> ipdev(levels_.size());
  std::vector<uint8_t> on_dev_ip(NJ, 0);
  if (p_.ip_device) {
    for (size_t j = 0; j < levels_.size(); ++j) {
      Level& L = *levels_[j];
      const uint32_t B = (uint32_t)L.graphs.size();
      std::vector<uint32_t> gbase(B, IP_NONE);
      bool any = false;
      for (uint32_t b = 0; b < B; ++b) {
        const uint32_t g = L.graphs[b];
        if (jobs[g].top() == j) {
          gbase[b] = (uint32_t)kbase[g];
          any = true;
        }
      }
      if (!any || !ip_on_device(jobs, j)) continue;
      ensure_sorted(j);  // (done by coarsen; the input level keeps its order)
      ipdev[j].reset(&pool_, s_, L.n ? L.n : 1);
      DBuf<uint32_t> dgb(&pool_, s_, B);
      h2d(dgb.get(), gbase.data(), B, s_);
      ip_device_init(L.gid, dgb.get(), L.n, ipdev[j].get(), s_);
      IpDevice ipd(IpLevel{L.xadj, L.adj, L.nw, L.gid, L.n}, ipdev[j].get(), Ktot, pool_, s_);
      struct Part {
        uint32_t b, off, kS;
      };
      std::vector<Part> cur;
      for (uint32_t b = 0; b < B; ++b)
        if (gbase[b] != IP_NONE) {
          cur.push_back(Part{b, 0, jobs[L.graphs[b]].k});
          on_dev_ip[L.graphs[b]] = 1;
        }
      while (true) {
        std::vector<IpSub> subs;
        std::vector<uint32_t> sob(Ktot, IP_NONE);
        std::vector<Part> next;
        for (const Part& q : cur) {
          if (q.kS <= 1) continue;
          const Job& jb = jobs[L.graphs[q.b]];
          const uint32_t k1 = (q.kS + 1) / 2;
          sob[kbase[L.graphs[q.b]] + q.off] = (uint32_t)subs.size();
          subs.push_back(IpSub{chain(jb.seed, TAG_IP, {(uint64_t)(j + 1 - jb.d0), (uint64_t)q.off,
                                                       (uint64_t)q.kS}),
                               L.nbase[q.b], q.kS, k1});
          next.push_back(Part{q.b, q.off, k1});
          next.push_back(Part{q.b, q.off + k1, q.kS - k1});
        }
        if (subs.empty()) break;
        ipd.depth(subs, sob);
        cur.swap(next);
      }
      ipd.finish();
    }
  }
  for (uint32_t g = 0; g < NJ; ++g) {
    if (on_dev_ip[g]) continue;
    const uint32_t top = jobs[g].top();
    Level& L = *levels_[top];
    uint32_t b = 0;
    while (L.graphs[b] != g) ++b;
    const uint64_t n0 = L.nbase[b], n1 = L.nbase[b + 1], e0 = L.ebase[b], e1 = L.ebase[b + 1];
    // host copies in buffers kept by the calling thread (no page faults after
    // the first call); ids and offsets stay global, the bisection subtracts
    IpBuffersLease lease;
    IpHostBuffers& hb = *lease.b;
    uint64_t* hx = pinned_grow(hb.xadj, hb.cx, n1 - n0 + 1, hb.pageable);
    int64_t* hn = pinned_grow(hb.nw, hb.cn, n1 - n0, hb.pageable);
    d2h(hx, L.xadj + n0, n1 - n0 + 1, s_);
    d2h(hn, L.nw + n0, n1 - n0, s_);
    // coarse levels: neighbours in ascending order (the oracle's coarse rows
    // are sorted); the input level: in the caller's order
    const bool asc = top > jobs[g].d0 || L.sorted;
    if (n1 - n0 <= (1u << 16)) {
      DBuf<uint16_t> a16(&pool_, s_, e1 > e0 ? e1 - e0 : 1);
      if (e1 > e0) {
        k_local_u16<<<grid_for(e1 - e0, 256), 256, 0, s_>>>(L.adj + e0, e1 - e0, (uint32_t)n0,
                                                            a16.get());
        LAUNCH_CHECK();
      }
      uint16_t* ha = pinned_grow(hb.adj16, hb.ca16, e1 - e0, hb.pageable);
      d2h(ha, a16.get(), e1 - e0, s_);
      sync(s_);
      initial_partition_host<uint16_t>(n1 - n0, hx, ha, hn, e0, 0, L.sorted, asc, jobs[g].k,
                                       jobs[g].seed, jobs[g].nlevels, ip[g]);
    } else {
      uint32_t* ha = pinned_grow(hb.adj, hb.ca, e1 - e0, hb.pageable);
      d2h(ha, L.adj + e0, e1 - e0, s_);
      sync(s_);
      initial_partition_host<uint32_t>(n1 - n0, hx, ha, hn, e0, n0, L.sorted, asc, jobs[g].k,
                                       jobs[g].seed, jobs[g].nlevels, ip[g]);
    }
    for (auto& x : ip[g]) x += (uint32_t)kbase[g];
  }
  t_initial_ns = tm.stop_ns();
  tm.start();
  DBuf<int64_t> BW(&pool_, s_, Ktot ? Ktot : 1);
  DBuf<uint32_t> upper;  // blocks of level j+1
  for (int j = (int)levels_.size() - 1; j >= 0; --j) {
    Level& L = *levels_[j];
    const uint32_t B = (uint32_t)L.graphs.size();
    DBuf<uint32_t> block;
    if (ipdev[j].get()) block = std::move(ipdev[j]);  // graphs initially partitioned here
    else block.reset(&pool_, s_, L.n ? L.n : 1);
    for (uint32_t b = 0; b < B; ++b) {
      const uint32_t g = L.graphs[b];
      if (jobs[g].top() == (uint32_t)j && !on_dev_ip[g])
        h2d(block.get() + L.nbase[b], ip[g].data(), ip[g].size(), s_);
    }
    if ((size_t)j + 1 < levels_.size()) project_blocks(L.map.get(), upper.get(), L.n, block.get(), s_);
    BW.zero();
    block_weights(block.get(), L.nw, L.n, BW.get(), Ktot, s_);
    std::vector<uint8_t> active(B, 1);
    std::vector<uint64_t> lb(B);
    for (uint32_t b = 0; b < B; ++b) lb[b] = kbase[L.graphs[b]];
    std::vector<uint32_t> rounds;
    LpSpec spec{true, (uint32_t)j + 1, p_.ref_rounds};
    run_lp(L, jobs, spec, active, block.get(), BW.get(), Ktot, nullptr, lb, nullptr, rounds);
    // graphs whose input graph is this level: cut, balance, output
    bool inputs_here = false;
    for (uint32_t g : L.graphs) inputs_here |= jobs[g].d0 == (uint32_t)j;
    if (inputs_here) finish_level(jobs, (size_t)j, block.get(), kbase, block_out, on_device);
    upper = std::move(block);
  }
  t_refine_ns = tm.stop_ns();
}

// Cut, block weights and output blocks of the graphs whose input graph is
// union level j (d0 == j), from that level's blocks.
void Engine::finish_level(std::vector<Job>& jobs, size_t j, const uint32_t* block,
                          const std::vector<uint64_t>& kbase, uint32_t* const* block_out,
                          bool on_device) {
  Level& L0 = *levels_[j];
  const uint32_t B0 = (uint32_t)L0.graphs.size();
  const uint64_t Ktot = kbase.back();
  DBuf<int64_t> cut(&pool_, s_, B0), BW(&pool_, s_, Ktot ? Ktot : 1);
  cut.zero();
  edge_cut(L0.src, L0.adj, L0.ew, L0.ew_kind, block, L0.gid, L0.nnz, cut.get(), s_);
  BW.zero();
  block_weights(block, L0.nw, L0.n, BW.get(), Ktot, s_);
  std::vector<int64_t> hcut(B0), hbw(Ktot);
  d2h(hcut.data(), cut.get(), B0, s_);
  d2h(hbw.data(), BW.get(), Ktot, s_);
  // device outputs: one launch for all graphs; host outputs: one copy each
  DBuf<uint32_t*> douts;
  DBuf<uint64_t> dnb0, dkb0;
  if (on_device && block_out && L0.n) {
    std::vector<uint32_t*> outs(B0, nullptr);
    std::vector<uint64_t> kb(B0, 0);
    for (uint32_t b = 0; b < B0; ++b)
      if (jobs[L0.graphs[b]].d0 == j) {
        outs[b] = block_out[L0.graphs[b]];
        kb[b] = kbase[L0.graphs[b]];
      }
    douts.reset(&pool_, s_, B0);
    dnb0.reset(&pool_, s_, B0 + 1);
    dkb0.reset(&pool_, s_, B0);
    h2d(douts.get(), outs.data(), B0, s_);
    h2d(dnb0.get(), L0.nbase.data(), B0 + 1, s_);
    h2d(dkb0.get(), kb.data(), B0, s_);
    k_blocks_out<<<grid_for(L0.n, 256), 256, 0, s_>>>(block, L0.gid, L0.n, dnb0.get(),
                                                      dkb0.get(), douts.get());
    LAUNCH_CHECK();
  } else if (!on_device && block_out) {
    for (uint32_t b = 0; b < B0; ++b) {
      const uint32_t g = L0.graphs[b];
      const uint64_t n0 = L0.nbase[b], nn = L0.nbase[b + 1] - n0;
      if (jobs[g].d0 == j && block_out[g]) d2h(block_out[g], block + n0, nn, s_);
    }
  }
  sync(s_);
  for (uint32_t b = 0; b < B0; ++b) {
    const uint32_t g = L0.graphs[b];
    Job& jb = jobs[g];
    if (jb.d0 != j) continue;
    if (!on_device && block_out && block_out[g]) {
      const uint64_t nn = L0.nbase[b + 1] - L0.nbase[b];
      for (uint64_t i = 0; i < nn; ++i) block_out[g][i] -= (uint32_t)kbase[g];
    }
    int64_t mx = 0;
    for (uint64_t i = kbase[g]; i < kbase[g + 1]; ++i) mx = std::max(mx, hbw[i]);
    jb.res.cut = hcut[b];
    jb.res.max_block_weight = mx;
    jb.res.lmax = jb.lmax;
    jb.res.levels = jb.nlevels;
  }
}

// ------------------------------------------------ initial partitioning --
// Recursive bipartitioning by greedy graph growing (Sec. 4.3's recursive
// bipartitioning; the growing rule is this library's reading).  For a node
// set S receiving blocks [off, off + kS): k1 = ceil(kS/2),
// T1 = ceil(c(S) k1 / kS).  A breadth-first search over G[S] starts at the
// unvisited node with the smallest (H(seed, IP, level, off, kS, u), u); a
// dequeued node joins part 1 iff it still fits T1, and only joined nodes
// enqueue their unvisited neighbours of S (in adjacency order).  When the
// queue runs dry the next start is taken, until part 1 weighs T1 or S is
// exhausted.
namespace {

template <typename A>
struct IpState {
  uint64_t n;
  const uint64_t* xadj;  // entry offsets, relative to e0
  const A* adj;          // neighbour ids, relative to n0
  const int64_t* nw;
  uint64_t e0, n0;
  bool sorted;           // rows stored in ascending order
  bool asc;              // a row's neighbours are enqueued in ascending order (coarse
                         // levels: the oracle's rows are sorted); else in stored order
  uint64_t seed, level;
  std::vector<uint32_t>* block;
  // stamps: sibling subproblems own disjoint node sets, so they may run on
  // different threads; a stamp read for a node of another set only tells
  // "not mine"
  std::unique_ptr<std::atomic<uint32_t>[]> inset, visited;
  std::vector<uint8_t> part1;
  std::atomic<uint32_t> stamp{0};
};

constexpr int IP_PAR_DEPTH = 4;  // up to 16 concurrent subproblems

template <typename A>
void grow_bisect(IpState<A>& st, std::vector<uint32_t>& S, uint32_t kS, uint32_t off, int depth) {
  if (S.empty()) return;
  if (kS == 1) {
    for (uint32_t v : S) (*st.block)[v] = off;
    return;
  }
  const auto rl = std::memory_order_relaxed;
  const uint32_t k1 = (kS + 1) / 2;
  int64_t cS = 0;
  for (uint32_t v : S) cS += st.nw[v];
  const int64_t T1 = (int64_t)(((u128)cS * k1 + kS - 1) / kS);
  const uint32_t my = st.stamp.fetch_add(1) + 1;
  const uint64_t pre = chain(st.seed, TAG_IP, {st.level, (uint64_t)off, (uint64_t)kS});
  std::vector<std::pair<uint64_t, uint32_t>> order(S.size());
  for (size_t i = 0; i < S.size(); ++i) {
    st.inset[S[i]].store(my, rl);
    order[i] = {hash_add(pre, S[i]), S[i]};
  }
  // start order: a min-heap, popped lazily (a search usually needs few
  // starts, so sorting all of S would cost more than the search)
  std::make_heap(order.begin(), order.end(), std::greater<>());
  for (uint32_t v : S) st.part1[v] = 0;
  // Unvisited members of S that a row scan can still find: those with
  // neighbours (a node with an empty row is in no row of a symmetric graph).
  // Once none is left, a joined node's row is not scanned at all.  When S is
  // not much smaller than the level they are also kept as a bitset over node
  // ids, which a row scan tests instead of the stamps.  With ascending enqueue
  // order, walking the bitset in ascending order and keeping the nodes y
  // adjacent to v enqueues exactly what a scan of v's row would; adjacency is
  // a binary search of the shorter of the two rows when rows are stored
  // sorted, else a scan of y's row.  The walk is taken when it costs less
  // than the scan: v's row is long and the nodes left are few or have short
  // rows (dense coarse graphs, where some nodes of small degree stay
  // unvisited for long).
  auto deg_of = [&](uint32_t x) { return st.xadj[x + 1] - st.xadj[x]; };
  auto bitlen = [](uint64_t d) { return (uint64_t)(64 - __builtin_clzll(d | 1)); };
  const bool use_bits = (uint64_t)S.size() * 64 >= st.n;
  const uint64_t nwords = use_bits ? (st.n + 63) / 64 : 0;
  std::vector<uint64_t> unv(nwords, 0);
  // nodes left, sums of their rows' bit lengths and lengths
  uint64_t nunv = 0, sumlen = 0, sumdeg = 0;
  for (uint32_t v : S)
    if (deg_of(v)) {
      ++nunv;
      sumlen += bitlen(deg_of(v));
      sumdeg += deg_of(v);
      if (use_bits) unv[v >> 6] |= 1ull << (v & 63);
    }
  auto visit = [&](uint32_t x) {
    st.visited[x].store(my, rl);
    const uint64_t d = deg_of(x);
    if (!d) return;
    if (use_bits) unv[x >> 6] &= ~(1ull << (x & 63));
    --nunv;
    sumlen -= bitlen(d);
    sumdeg -= d;
  };
  // a scan of an unsorted row enqueues what it finds in ascending order
  const bool sort_found = st.asc && !st.sorted;
  std::vector<uint32_t> found;
  // Once the rows of the nodes left hold no more entries than the row about
  // to be scanned, they are indexed by neighbour: (x, y) for every entry x of
  // the row of a left node y, sorted.  A joined node v then enqueues the
  // unvisited y of its pairs, in ascending order: exactly the left nodes in
  // v's row, as a scan would find them.  No row is scanned after that.
  std::vector<std::pair<uint32_t, uint32_t>> watch;
  bool watching = false;
  std::vector<uint32_t> queue;
  queue.reserve(S.size());
  int64_t w1 = 0;
  // Members of S not dequeued yet (unvisited or waiting in the queue) by
  // weight, weights below LIGHT one by one: once the capacity left is below
  // LIGHT and none of them fits it, no node can join part 1 any more and the
  // search ends (going on would only visit nodes that do not fit).
  constexpr int64_t LIGHT = 64;
  uint32_t light[LIGHT] = {};
  // (weights <= 0, which always fit, are counted as 0)
  auto light_of = [&](uint32_t v) { return st.nw[v] > 0 ? st.nw[v] : 0; };
  for (uint32_t v : S)
    if (st.nw[v] < LIGHT) ++light[light_of(v)];
  auto nothing_fits = [&]() {
    const int64_t R = T1 - w1;
    if (R >= LIGHT) return false;
    for (int64_t w = 0; w <= R; ++w)
      if (light[w]) return false;
    return true;
  };
  bool done = false;
  while (w1 < T1 && !done && !nothing_fits()) {
    while (!order.empty() && st.visited[order.front().second].load(rl) == my) {
      std::pop_heap(order.begin(), order.end(), std::greater<>());
      order.pop_back();
    }
    if (order.empty()) break;
    queue.clear();
    size_t head = 0;
    visit(order.front().second);
    queue.push_back(order.front().second);
    while (head < queue.size() && w1 < T1) {
      const uint32_t v = queue[head++];
      if (st.nw[v] < LIGHT) --light[light_of(v)];
      if (w1 + st.nw[v] > T1) continue;
      st.part1[v] = 1;
      w1 += st.nw[v];
      if (nothing_fits()) {
        done = true;
        break;
      }
      if (nunv == 0) continue;  // nothing left to enqueue
      const A* rb = st.adj + (st.xadj[v] - st.e0);
      const A* re = st.adj + (st.xadj[v + 1] - st.e0);
      const uint64_t deg = (uint64_t)(re - rb);
      if (!watching && use_bits && st.asc && sumdeg <= deg) {
        watch.clear();
        watch.reserve(sumdeg);
        for (uint64_t w = 0; w < nwords; ++w)
          for (uint64_t bits = unv[w]; bits; bits &= bits - 1) {
            const uint32_t y = (uint32_t)(w * 64 + __builtin_ctzll(bits));
            const A* yb = st.adj + (st.xadj[y] - st.e0);
            const A* ye = st.adj + (st.xadj[y + 1] - st.e0);
            for (const A* p = yb; p < ye; ++p) watch.emplace_back((uint32_t)*p - (uint32_t)st.n0, y);
          }
        std::sort(watch.begin(), watch.end());
        watching = true;
      }
      if (watching) {
        auto it = std::lower_bound(watch.begin(), watch.end(), std::make_pair(v, 0u));
        for (; it != watch.end() && it->first == v; ++it) {
          const uint32_t y = it->second;
          if ((unv[y >> 6] >> (y & 63)) & 1) {
            visit(y);
            queue.push_back(y);
          }
        }
        continue;
      }
      const uint64_t walk_cost =
          st.sorted ? 2 * std::min(sumlen, nunv * bitlen(deg)) : 2 * sumdeg;
      if (use_bits && st.asc && nwords + walk_cost < deg) {
        const uint32_t vg = (uint32_t)(v + st.n0);
        for (uint64_t w = 0; w < nwords; ++w) {
          uint64_t bits = unv[w];
          while (bits) {
            const uint32_t x = (uint32_t)(w * 64 + __builtin_ctzll(bits));
            bits &= bits - 1;
            const uint64_t dx = deg_of(x);
            const A* xb = st.adj + (st.xadj[x] - st.e0);
            bool adj;
            if (!st.sorted) adj = std::find(xb, xb + dx, vg) != xb + dx;
            else if (dx < deg) adj = std::binary_search(xb, xb + dx, vg);
            else adj = std::binary_search(rb, re, (uint32_t)(x + st.n0));
            if (adj) {
              visit(x);
              queue.push_back(x);
            }
          }
        }
      } else {
        found.clear();
        auto take = [&](uint32_t x) {
          visit(x);
          if (sort_found) found.push_back(x);
          else queue.push_back(x);
        };
        if (use_bits) {
          for (const A* p = rb; p < re; ++p) {
            const uint32_t x = (uint32_t)*p - (uint32_t)st.n0;
            if ((unv[x >> 6] >> (x & 63)) & 1) take(x);
          }
        } else {
          for (const A* p = rb; p < re; ++p) {
            const uint32_t x = (uint32_t)*p - (uint32_t)st.n0;
            if (st.inset[x].load(rl) == my && st.visited[x].load(rl) != my) take(x);
          }
        }
        if (sort_found) {
          if (found.size() > 1) std::sort(found.begin(), found.end());
          queue.insert(queue.end(), found.begin(), found.end());
        }
      }
    }
  }
  std::vector<uint32_t> S1, S2;
  for (uint32_t v : S) (st.part1[v] ? S1 : S2).push_back(v);
  S.clear();
  S.shrink_to_fit();
  if (depth < IP_PAR_DEPTH && !S1.empty() && !S2.empty()) {
    std::thread t([&] { grow_bisect(st, S1, k1, off, depth + 1); });
    grow_bisect(st, S2, kS - k1, off + k1, depth + 1);
    t.join();
  } else {
    grow_bisect(st, S1, k1, off, depth + 1);
    grow_bisect(st, S2, kS - k1, off + k1, depth + 1);
  }
}

}  // namespace

template <typename A>
void initial_partition_host(uint64_t n, const uint64_t* xadj, const A* adj, const int64_t* nw,
                            uint64_t e0, uint64_t n0, bool sorted, bool asc, uint32_t k,
                            uint64_t seed, uint64_t level, std::vector<uint32_t>& block) {
  IpState<A> st;
  st.n = n;
  st.xadj = xadj;
  st.adj = adj;
  st.nw = nw;
  st.e0 = e0;
  st.n0 = n0;
  st.sorted = sorted;
  st.asc = asc;
  st.seed = seed;
  st.level = level;
  block.assign(n, 0);
  st.block = &block;
  st.inset.reset(new std::atomic<uint32_t>[n]);
  st.visited.reset(new std::atomic<uint32_t>[n]);
  for (uint64_t v = 0; v < n; ++v) {
    st.inset[v].store(0, std::memory_order_relaxed);
    st.visited[v].store(0, std::memory_order_relaxed);
  }
  st.part1.assign(n, 0);
  std::vector<uint32_t> S(n);
  for (uint64_t v = 0; v < n; ++v) S[v] = (uint32_t)v;
  grow_bisect(st, S, k, 0, 0);
}

template void initial_partition_host<uint32_t>(uint64_t, const uint64_t*, const uint32_t*,
                                               const int64_t*, uint64_t, uint64_t, bool, bool,
                                               uint32_t, uint64_t, uint64_t,
                                               std::vector<uint32_t>&);
template void initial_partition_host<uint16_t>(uint64_t, const uint64_t*, const uint16_t*,
                                               const int64_t*, uint64_t, uint64_t, bool, bool,
                                               uint32_t, uint64_t, uint64_t,
                                               std::vector<uint32_t>&);

}  // namespace lmgp
