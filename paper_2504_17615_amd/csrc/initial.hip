// Initial partitioning on the device (recursive bisection by greedy graph
// growing, Sec. 4.3's recursive bipartitioning with this library's growing
// rule).  For a node set S receiving kS blocks: k1 = ceil(kS / 2),
// T1 = ceil(c(S) k1 / kS); a breadth-first search over G[S] starts at the
// unvisited node with the smallest (H(seed, IP, level, off, kS, u), u); a
// dequeued node joins part 1 iff it still fits T1 and only joined nodes
// enqueue their unvisited neighbours of S, in adjacency order; when the queue
// runs dry the next start is taken, until part 1 weighs T1 or S is exhausted.
//
// The subproblems of one recursion depth run concurrently, one 1024-thread
// workgroup each.  A workgroup dequeues the whole queue at once (the queue
// holds one BFS frontier): the join decisions of the dequeued nodes do not
// depend on what they enqueue, so they are taken in queue order first (a
// block scan while everything fits, then one by one on one wave), and the
// joined nodes' rows are expanded after.  The expansion keeps the sequential
// order exactly: every candidate entry (joined node i of the frontier, row
// position j) has the rank t of (i, j) in frontier-then-row order, each
// neighbour keeps its smallest t (an atomic max on an iteration-tagged key)
// and is enqueued at the prefix count of the winners before it.
#include "initial.h"

#include "kernels.h"
#include "primitives.h"

namespace lmgp {

namespace {

typedef unsigned __int128 u128;
// Subproblems of at most this many nodes on average take 256-thread groups.
constexpr uint64_t IP_SMALL_SUB = 4096;
// Node weights below this are counted one by one for the end-of-search test.
constexpr int IP_LIGHT = 64;

struct IpArgs {
  const uint64_t* xadj;
  const uint32_t* adj;
  const int64_t* nw;
  uint64_t n;
  const IpSub* subs;
  const uint32_t* sub_of_block;  // block id -> subproblem (IP_NONE: finished)
  uint32_t nsub;
  const uint32_t* segoff;        // [nsub + 1] start of each subproblem in `order`
  uint32_t* cnt;                 // [nsub] nodes
  unsigned long long* cS;        // [nsub] node weight
  const uint32_t* order;         // nodes by (subproblem, start hash, id)
  uint32_t* sub;                 // subproblem of each node
  uint32_t* boff;                // block id of each node
  uint32_t* queue;               // per subproblem: its BFS queue (each node once)
  uint32_t* jl;                  // per subproblem: joined frontier nodes with neighbours
  uint64_t* dpre;                // per subproblem (+1 slot each): their degree prefix
  uint8_t* visited;
  uint8_t* part1;
  unsigned long long* first;     // per node: best (iteration, -rank) key of an expansion
  uint32_t* err;
  uint64_t* keys;
  uint32_t* vals;
};

__global__ void k_ip_init(const uint32_t* gid, const uint32_t* gbase, uint64_t n, uint32_t* boff) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) boff[v] = gbase[graph_of(gid, v)];
}

// Subproblem of every node (from its current block), node count and weight
// per subproblem, and the start-order key of the node.
__global__ void k_ip_assign(IpArgs a) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  const uint32_t b = a.boff[v];
  const uint32_t s = b == IP_NONE ? IP_NONE : a.sub_of_block[b];
  a.sub[v] = s;
  uint64_t key = 0;
  if (s != IP_NONE) {
    atomicAdd(&a.cnt[s], 1u);
    atomicAdd(&a.cS[s], (unsigned long long)a.nw[v]);
    key = hash_add(a.subs[s].pre, v - a.subs[s].n0);
  }
  a.keys[v] = key;
  a.vals[v] = (uint32_t)v;
}

// Second sort key: the subproblem (finished nodes last).
__global__ void k_ip_subkeys(const uint32_t* sub, const uint32_t* vals, uint64_t n, uint32_t nsub,
                             uint64_t* keys) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = sub[vals[i]];
  keys[i] = s == IP_NONE ? nsub : s;
}

// A subproblem's nodes are touched by its own workgroup only: workgroup-scope
// atomics and fences suffice (agent scope would make every fence write the
// XCD's L2 back to memory).
LMGP_D unsigned long long load_first(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
LMGP_D void wg_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// NT threads per subproblem: 256 when subproblems are small (more of them
// in flight per CU), 1024 for large ones.
template <int IP_NT>
__global__ __launch_bounds__(IP_NT) void k_ip_grow(IpArgs a) {
  constexpr int IP_NW = IP_NT / WAVE;
  __shared__ int64_t sm[IP_NW];
  __shared__ uint64_t smu[IP_NW];
  __shared__ uint64_t sdp[IP_NT + 1];
  __shared__ long long sh_w1;
  __shared__ uint32_t sh_head, sh_tail, sh_ptr, sh_done, sh_r0;
  // nodes not dequeued yet (unvisited or queued) by weight, below IP_LIGHT
  __shared__ uint32_t sh_light[IP_LIGHT];
  const uint32_t s = blockIdx.x;
  const uint32_t seg = a.segoff[s];
  const uint32_t m = a.segoff[s + 1] - seg;
  if (m == 0) return;
  const IpSub sp = a.subs[s];
  const uint64_t cS = a.cS[s];
  const int64_t T1 = (int64_t)(((u128)cS * sp.k1 + sp.kS - 1) / sp.kS);
  const uint32_t* order = a.order + seg;
  uint32_t* queue = a.queue + seg;
  uint32_t* jl = a.jl + seg;
  uint64_t* dpre = a.dpre + seg + s;
  const int tid = threadIdx.x, lane = lane_id();
  for (int w = tid; w < IP_LIGHT; w += IP_NT) sh_light[w] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < m; i += IP_NT) {
    const uint32_t v = order[i];
    a.visited[v] = 0;
    a.part1[v] = 0;
    __hip_atomic_store(&a.first[v], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const int64_t c = a.nw[v];
    if (c < IP_LIGHT) atomicAdd(&sh_light[c > 0 ? c : 0], 1u);  // weights <= 0 always fit
  }
  wg_fence();
  if (tid == 0) {
    sh_w1 = 0;
    sh_head = sh_tail = sh_ptr = sh_done = 0;
  }
  __syncthreads();
  uint32_t iter = 0;
  // every pass of the loop starts a search or dequeues at least one node
  const uint64_t guard_max = 4ull * m + 8;
  for (uint64_t guard = 0;; ++guard) {
    if (guard > guard_max) {
      if (tid == 0) atomicOr(a.err, 1u);
      break;
    }
    // (1) queue empty: the next unvisited node of the start order starts a
    // search; nodes without neighbours are settled on the way (their search
    // would enqueue nothing)
    if (tid < WAVE && sh_head == sh_tail) {
      uint32_t ptr = sh_ptr, tail = sh_tail;
      int64_t w1 = sh_w1;
      bool stop = false, started = false;
      while (!stop && !started) {
        if (ptr >= m) {
          stop = true;
          break;
        }
        const uint32_t base = ptr;
        const uint32_t i = base + lane;
        const bool in = i < m;
        const uint32_t v = in ? order[i] : 0u;
        const int vis = in ? (a.visited[v] != 0) : 1;
        const int iso = in && !vis && a.xadj[v + 1] == a.xadj[v];
        const int64_t c = in && !vis ? a.nw[v] : 0;
        for (int l = 0; l < WAVE; ++l) {
          if (base + l >= m) {
            ptr = m;
            stop = true;
            break;
          }
          ptr = base + l + 1;
          if (__shfl(vis, l)) continue;
          const uint32_t vv = __shfl(v, l);
          if (__shfl(iso, l)) {
            const int64_t cl = __shfl(c, l);
            const bool join = w1 + cl <= T1;
            if (lane == 0) {
              a.visited[vv] = 1;
              if (join) a.part1[vv] = 1;
              if (cl < IP_LIGHT) --sh_light[cl > 0 ? cl : 0];
            }
            if (join) w1 += cl;
            if (w1 >= T1) {
              stop = true;
              break;
            }
            continue;
          }
          if (lane == 0) {
            a.visited[vv] = 1;
            queue[tail] = vv;
          }
          ++tail;
          started = true;
          break;
        }
      }
      if (lane == 0) {
        sh_ptr = ptr;
        sh_tail = tail;
        sh_w1 = w1;
        if (stop) sh_done = 1;
      }
    }
    __syncthreads();
    if (sh_done) break;
    // (2) join decisions of the dequeued frontier [h0, t0), in queue order
    const uint32_t h0 = sh_head, t0 = sh_tail;
    int64_t w1 = sh_w1;
    __syncthreads();
    bool settled = false;
    for (uint32_t b0 = h0; b0 < t0 && !settled; b0 += IP_NT) {
      const uint32_t i = b0 + tid;
      const bool in = i < t0;
      const uint32_t v = in ? queue[i] : 0u;
      const int64_t c = in ? a.nw[v] : 0;
      int64_t tot;
      const int64_t ex = block_exclusive_scan<int64_t, IP_NW>(c, sm, tot);
      if (w1 + tot <= T1) {
        if (in) a.part1[v] = 1;
        w1 += tot;
        if (w1 >= T1) settled = true;
        continue;
      }
      // the nodes that fit form a prefix (weights are positive) ...
      const bool fit = in && w1 + ex + c <= T1;
      if (fit) a.part1[v] = 1;
      int64_t got, nfit;
      (void)block_exclusive_scan<int64_t, IP_NW>(fit ? c : 0, sm, got);
      (void)block_exclusive_scan<int64_t, IP_NW>(fit ? 1 : 0, sm, nfit);
      // ... and the rest of the frontier is decided one node at a time
      if (tid < WAVE) {
        int64_t w = w1 + got;
        for (uint32_t q0 = b0 + (uint32_t)nfit; q0 < t0 && w < T1; q0 += WAVE) {
          const uint32_t q = q0 + lane;
          const uint32_t vq = q < t0 ? queue[q] : 0u;
          const int64_t cq = q < t0 ? a.nw[vq] : 0;
          for (int l = 0; l < WAVE && q0 + l < t0; ++l) {
            const int64_t cl = __shfl(cq, l);
            if (w + cl <= T1) {
              w += cl;
              if (lane == l) a.part1[vq] = 1;
              if (w >= T1) break;
            }
          }
        }
        if (lane == 0) sh_w1 = w;
      }
      __syncthreads();
      w1 = sh_w1;
      settled = true;
    }
    for (uint32_t i = h0 + tid; i < t0; i += IP_NT) {  // the frontier is decided
      const int64_t c = a.nw[queue[i]];
      if (c < IP_LIGHT) atomicSub(&sh_light[c > 0 ? c : 0], 1u);
    }
    if (tid == 0) {
      sh_w1 = w1;
      sh_head = t0;
    }
    __syncthreads();
    if (w1 >= T1) break;
    // capacity left below IP_LIGHT and no undecided node that light: no node
    // can join part 1 any more (the rest of the search would only visit)
    if (T1 - w1 < IP_LIGHT) {
      bool any = false;
      for (int64_t w = 0; w <= T1 - w1; ++w) any |= sh_light[w] != 0;
      if (!any) break;
    }
    // (3) joined frontier nodes that have neighbours, with their degree prefix
    uint32_t J = 0;
    uint64_t D = 0;
    for (uint32_t b0 = h0; b0 < t0; b0 += IP_NT) {
      const uint32_t i = b0 + tid;
      const bool in = i < t0;
      const uint32_t v = in ? queue[i] : 0u;
      const uint64_t d = in && a.part1[v] ? a.xadj[v + 1] - a.xadj[v] : 0;
      uint64_t nf, dsum;
      const uint64_t pf = block_exclusive_scan<uint64_t, IP_NW>(d > 0 ? 1 : 0, smu, nf);
      const uint64_t pd = block_exclusive_scan<uint64_t, IP_NW>(d, smu, dsum);
      if (d > 0) {
        jl[J + pf] = v;
        dpre[J + pf] = D + pd;
      }
      J += (uint32_t)nf;
      D += dsum;
    }
    if (tid == 0) dpre[J] = D;
    __syncthreads();
    if (D == 0) continue;
    ++iter;
    // (4) expansion: pass 0 marks each new neighbour with its smallest rank,
    // pass 1 enqueues the winners in rank order
    uint32_t pushed = 0;
    for (int pass = 0; pass < 2; ++pass) {
      for (uint64_t T0 = 0; T0 < D; T0 += IP_NT) {
        if (tid == 0) {
          uint32_t lo = 0, hi = J;  // dpre[lo] <= T0 < dpre[hi]
          while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (dpre[mid] <= T0) lo = mid;
            else hi = mid;
          }
          sh_r0 = lo;
        }
        __syncthreads();
        const uint32_t r0 = sh_r0;
        // every row has an entry, so the tile ends within IP_NT rows
        const uint32_t nr = J - r0 < (uint32_t)IP_NT ? J - r0 : (uint32_t)IP_NT;
        for (uint32_t q = tid; q <= nr; q += IP_NT) sdp[q] = dpre[r0 + q];
        __syncthreads();
        const uint64_t t = T0 + tid;
        bool win = false;
        uint32_t x = 0;
        if (t < D) {
          uint32_t lo = 0, hi = nr;  // sdp[lo] <= t < sdp[hi]
          while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (sdp[mid] <= t) lo = mid;
            else hi = mid;
          }
          const uint32_t v = jl[r0 + lo];
          x = a.adj[a.xadj[v] + (t - sdp[lo])];
          const unsigned long long key =
              ((unsigned long long)iter << 32) | (0xFFFFFFFFull - (uint32_t)t);
          if (a.sub[x] == s) {
            if (pass == 0) {
              if (!a.visited[x])
                __hip_atomic_fetch_max(&a.first[x], key, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
              win = load_first(&a.first[x]) == key;
            }
          }
        }
        if (pass == 1) {
          uint64_t nwin;
          const uint64_t pw = block_exclusive_scan<uint64_t, IP_NW>(win ? 1 : 0, smu, nwin);
          if (win) {
            queue[t0 + pushed + pw] = x;
            a.visited[x] = 1;
          }
          pushed += (uint32_t)nwin;
        } else {
          __syncthreads();  // sdp is refilled for the next tile
        }
      }
      wg_fence();  // the pass's atomics and stores are visible to the workgroup
      __syncthreads();
    }
    if (tid == 0) sh_tail = t0 + pushed;
    __syncthreads();
  }
  __syncthreads();
  for (uint32_t i = tid; i < m; i += IP_NT) {
    const uint32_t v = order[i];
    if (!a.part1[v]) a.boff[v] += sp.k1;
  }
}

}  // namespace

IpDevice::IpDevice(const IpLevel& L, uint32_t* boff, uint64_t nblocks, Pool& pool, hipStream_t s)
    : L_(L), boff_(boff), nblocks_(nblocks), pool_(pool), s_(s) {
  const uint64_t n = L.n ? L.n : 1;
  sub_.reset(&pool, s, n);
  queue_.reset(&pool, s, n);
  jl_.reset(&pool, s, n);
  err_.reset(&pool, s, 1);
  err_.zero();
  dpre_.reset(&pool, s, n + nblocks + 1);
  keys_.reset(&pool, s, n);
  keys2_.reset(&pool, s, n);
  vals_.reset(&pool, s, n);
  vals2_.reset(&pool, s, n);
  visited_.reset(&pool, s, n);
  part1_.reset(&pool, s, n);
  first_.reset(&pool, s, n);
}

void IpDevice::depth(const std::vector<IpSub>& subs, const std::vector<uint32_t>& sub_of_block) {
  const uint32_t nsub = (uint32_t)subs.size();
  if (!nsub || !L_.n) return;
  if (sub_of_block.size() != nblocks_) throw InvalidArg("block table size");
  hold_subs_.push_back(subs);
  hold_sob_.push_back(sub_of_block);
  DBuf<IpSub> dsubs(&pool_, s_, nsub);
  DBuf<uint32_t> dsob(&pool_, s_, nblocks_ ? nblocks_ : 1);
  DBuf<uint32_t> cnt(&pool_, s_, nsub), segoff(&pool_, s_, nsub + 1);
  DBuf<unsigned long long> cS(&pool_, s_, nsub);
  HIP_CHECK(hipMemcpyAsync(dsubs.get(), hold_subs_.back().data(), nsub * sizeof(IpSub),
                           hipMemcpyHostToDevice, s_));
  HIP_CHECK(hipMemcpyAsync(dsob.get(), hold_sob_.back().data(), nblocks_ * sizeof(uint32_t),
                           hipMemcpyHostToDevice, s_));
  cnt.zero();
  cS.zero();
  const uint64_t n = L_.n;
  IpArgs a{};
  a.xadj = L_.xadj;
  a.adj = L_.adj;
  a.nw = L_.nw;
  a.n = n;
  a.subs = dsubs.get();
  a.sub_of_block = dsob.get();
  a.nsub = nsub;
  a.segoff = segoff.get();
  a.cnt = cnt.get();
  a.cS = cS.get();
  a.sub = sub_.get();
  a.boff = boff_;
  a.queue = queue_.get();
  a.jl = jl_.get();
  a.dpre = dpre_.get();
  a.visited = visited_.get();
  a.part1 = part1_.get();
  a.first = first_.get();
  a.err = err_.get();
  a.keys = keys_.get();
  a.vals = vals_.get();
  k_ip_assign<<<grid_for(n, 256), 256, 0, s_>>>(a);
  LAUNCH_CHECK();
  exclusive_scan(ArrayU32{cnt.get()}, nsub, segoff.get(), true, pool_, s_);
  // start order: by hash (ids ascending among equal hashes: the sort is
  // stable), then grouped by subproblem
  const bool sw1 = radix_sort_pairs<uint32_t>(keys_.get(), vals_.get(), keys2_.get(), vals2_.get(),
                                              n, 0, 64, pool_, s_);
  uint64_t* k1 = sw1 ? keys2_.get() : keys_.get();
  uint32_t* v1 = sw1 ? vals2_.get() : vals_.get();
  uint64_t* k2 = sw1 ? keys_.get() : keys2_.get();
  uint32_t* v2 = sw1 ? vals_.get() : vals2_.get();
  k_ip_subkeys<<<grid_for(n, 256), 256, 0, s_>>>(sub_.get(), v1, n, nsub, k1);
  LAUNCH_CHECK();
  int bits = 1;
  while ((1ull << bits) <= nsub) ++bits;
  const bool sw2 = radix_sort_pairs<uint32_t>(k1, v1, k2, v2, n, 0, bits, pool_, s_);
  a.order = sw2 ? v2 : v1;
  if (n <= (uint64_t)nsub * IP_SMALL_SUB) k_ip_grow<256><<<nsub, 256, 0, s_>>>(a);
  else k_ip_grow<1024><<<nsub, 1024, 0, s_>>>(a);
  LAUNCH_CHECK();
}

void IpDevice::finish() {
  uint32_t err = 0;
  HIP_CHECK(hipMemcpyAsync(&err, err_.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s_));
  HIP_CHECK(hipStreamSynchronize(s_));
  hold_subs_.clear();
  hold_sob_.clear();
  if (err) throw std::runtime_error("device initial partitioning exceeded its iteration bound");
}

void ip_device_init(const uint32_t* gid, const uint32_t* gbase_dev, uint64_t n, uint32_t* boff,
                    hipStream_t s) {
  if (!n) return;
  k_ip_init<<<grid_for(n, 256), 256, 0, s>>>(gid, gbase_dev, n, boff);
  LAUNCH_CHECK();
}

}  // namespace lmgp
