// C ABI of the library (declared in include/lmgp.h).  No exception crosses
// this boundary; failures become an lmgp_status plus a thread-local message.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "engine.h"
#include "tuner.h"


struct lmgp_hierarchy {
  std::shared_ptr<lmgp::Pool> pool;
  hipStream_t stream = nullptr;
  std::unique_ptr<lmgp::Engine> engine;
  std::vector<lmgp::Job> jobs;
};

namespace lmgp {

namespace {

thread_local std::string g_err;

template <class F>
lmgp_status guard(F&& f) {
  try {
    g_err.clear();
    f();
    return LMGP_OK;
  } catch (const InvalidArg& e) {
    g_err = e.what();
    return LMGP_EINVAL;
  } catch (const OutOfMemory& e) {
    g_err = e.what();
    return LMGP_ENOMEM;
  } catch (const HipError& e) {
    g_err = e.what();
    return LMGP_EDEVICE;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return LMGP_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return LMGP_EDEVICE;
  }
}

// ------------------------------------------------------------ validation --
enum : uint32_t {
  BAD_XADJ = 1, BAD_ID = 2, BAD_LOOP = 4, BAD_WEIGHT = 8, BAD_ORDER = 16, BAD_SYM = 32,
  BAD_VWEIGHT = 64
};

__global__ void k_check_xadj(const uint64_t* xadj, uint64_t n, uint64_t nnz, uint32_t* err) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > n) return;
  if (u == 0 && xadj[0] != 0) atomicOr(err, (uint32_t)BAD_XADJ);
  if (u == n && xadj[n] != nnz) atomicOr(err, (uint32_t)BAD_XADJ);
  if (u < n && xadj[u + 1] < xadj[u]) atomicOr(err, (uint32_t)BAD_XADJ);
}

__global__ void k_src(const uint64_t* xadj, uint64_t n, uint64_t nnz, uint32_t* src) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  uint64_t lo = 0, hi = n;  // xadj[lo] <= e < xadj[hi]
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) / 2;
    if (xadj[mid] <= e) lo = mid;
    else hi = mid;
  }
  src[e] = (uint32_t)lo;
}

template <int EWK>
__global__ void k_check_entries(const uint64_t* xadj, const uint32_t* adj, const void* ew,
                                const uint32_t* src, uint64_t n, uint64_t nnz, int full,
                                uint32_t* err) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t u = src[e], v = adj[e];
  uint32_t bad = 0;
  if (v >= n) bad |= BAD_ID;
  else if (v == u) bad |= BAD_LOOP;
  const int64_t w = edge_w<EWK>(ew, e);
  if (w <= 0) bad |= BAD_WEIGHT;
  if (!(bad & BAD_ID) && e > xadj[u] && adj[e - 1] >= v) {
    // an error in full validation; otherwise only recorded (the initial
    // bisection may walk ascending rows faster)
    if (full) bad |= BAD_ORDER;
    else atomicOr(&err[1], 1u);
  }
  if (full && !(bad & BAD_ID)) {
    // reverse entry (v, u) with the same weight
    uint64_t lo = xadj[v], hi = xadj[v + 1];
    bool found = false;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      const uint32_t x = adj[mid];
      if (x == u) {
        found = edge_w<EWK>(ew, mid) == w;
        break;
      }
      if (x < u) lo = mid + 1;
      else hi = mid;
    }
    if (!found) bad |= BAD_SYM;
  }
  if (bad) atomicOr(err, bad);
}

__global__ void k_nw_from(const void* vw, int bits, uint64_t n, int64_t* nw, uint32_t* err) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int64_t c = 1;
  if (vw) c = bits == 32 ? (int64_t)((const int32_t*)vw)[u] : ((const int64_t*)vw)[u];
  if (c <= 0) atomicOr(err, (uint32_t)BAD_VWEIGHT);
  nw[u] = c;
}

__global__ __launch_bounds__(256) void k_sum_i64(const int64_t* a, uint64_t n, int64_t* out) {
  __shared__ int64_t sm[NWAVE];
  int64_t s = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) s += a[i];
  const int64_t t = block_reduce_sum(s, sm);
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)out, (unsigned long long)t);
}

// Sum of the weights of all entries (weights are validated positive).
template <int EWK>
__global__ __launch_bounds__(256) void k_sum_w(const void* ew, uint64_t nnz, int64_t* out) {
  __shared__ int64_t sm[NWAVE];
  int64_t s = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int64_t w = edge_w<EWK>(ew, e);
    s += w > 0 ? w : 0;
    if (s > (1ll << 40)) s = 1ll << 40;  // saturate: only "below 2^32" matters
  }
  const int64_t t = block_reduce_sum(s, sm);
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)out, (unsigned long long)t);
}

std::string describe(uint32_t bad) {
  std::string m = "invalid graph:";
  if (bad & BAD_XADJ) m += " xadj not monotone from 0 to nnz;";
  if (bad & BAD_ID) m += " neighbour id >= n;";
  if (bad & BAD_LOOP) m += " self-loop;";
  if (bad & BAD_WEIGHT) m += " edge weight <= 0;";
  if (bad & BAD_VWEIGHT) m += " node weight <= 0;";
  if (bad & BAD_ORDER) m += " row not strictly ascending (unsorted or duplicate);";
  if (bad & BAD_SYM) m += " not symmetric (missing reverse entry or different weight);";
  return m;
}

int64_t cluster_limit(int64_t cV, uint32_t k, const lmgp_params& p) {
  const int64_t U = (int64_t)((unsigned __int128)cV / ((unsigned __int128)p.clim * k));
  return U < 1 ? 1 : U;
}

int64_t balance_limit(int64_t cV, uint32_t k, double eps) {
  const int64_t avg = (cV + (int64_t)k - 1) / (int64_t)k;
  return (int64_t)std::floor((1.0 + eps) * (double)avg);
}

Job make_job(const InputGraph* g, uint32_t k, double eps, uint64_t seed, const lmgp_params& p) {
  if (k == 0) throw InvalidArg("k must be >= 1");
  if ((uint64_t)k > g->n) throw InvalidArg("k must not exceed the number of nodes");
  if (!(eps > 0.0) || !std::isfinite(eps)) throw InvalidArg("eps must be a positive finite number");
  Job j;
  j.g = g;
  j.k = k;
  j.eps = eps;
  j.seed = seed;
  j.U = cluster_limit(g->cV, k, p);
  j.lmax = balance_limit(g->cV, k, eps);
  return j;
}

}  // namespace

// The host-side checks of a view (before any device work).
void check_view(const lmgp_csr_view& v) {
  if (v.n == 0) throw InvalidArg("graph must have at least one node");
  if (v.n >= (1ull << 31)) throw InvalidArg("n must be < 2^31");
  if (v.nnz >= (1ull << 40)) throw InvalidArg("nnz must be < 2^40");
  if (v.nnz % 2) throw InvalidArg("nnz must be even (symmetric CSR)");
  if (!v.xadj) throw InvalidArg("xadj is NULL");
  if (v.nnz && !v.adjncy) throw InvalidArg("adjncy is NULL");
  if (v.vwgt && v.vwgt_bits != 32 && v.vwgt_bits != 64) throw InvalidArg("vwgt_bits must be 32 or 64");
  if (v.adjwgt && v.adjwgt_bits != 32 && v.adjwgt_bits != 64)
    throw InvalidArg("adjwgt_bits must be 32 or 64");
}

void create_input_graph(const lmgp_csr_view& v, InputGraph& g, hipStream_t s) {
  check_view(v);
  g.stream = s;
  g.n = v.n;
  g.nnz = v.nnz;
  // One device allocation holds every array of the graph (offsets,
  // neighbours, weights, node weights, entry rows and the checks' words): a
  // process holds a bounded number of device mappings, and a server keeping
  // thousands of graphs resident would otherwise use six per graph.
  {
    auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
    const uint64_t e1 = v.nnz ? v.nnz : 1;
    uint64_t need = al(8 * (v.n + 1)) + 2 * al(4 * e1) + al(8 * v.n) + 2 * al(16);
    if (v.adjwgt) need += al((uint64_t)(v.adjwgt_bits / 8) * e1);
    if (v.vwgt && !v.on_device) need += al((uint64_t)(v.vwgt_bits / 8) * v.n);
    g.storage.reset(g.pool, s, need);
    g.arena = std::make_shared<Pool>(g.storage.get(), need);
  }
  Pool& pool = *g.arena;
  const hipMemcpyKind kind = v.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  g.xadj.reset(&pool, s, v.n + 1);
  HIP_CHECK(hipMemcpyAsync(g.xadj.get(), v.xadj, (v.n + 1) * sizeof(uint64_t), kind, s));
  g.adj.reset(&pool, s, v.nnz ? v.nnz : 1);
  if (v.nnz) HIP_CHECK(hipMemcpyAsync(g.adj.get(), v.adjncy, v.nnz * sizeof(uint32_t), kind, s));
  g.ew_kind = EW_UNIT;
  if (v.adjwgt) {
    if (v.adjwgt_bits == 32) {
      g.ew_kind = EW_I32;
      g.ew32.reset(&pool, s, v.nnz ? v.nnz : 1);
      if (v.nnz) HIP_CHECK(hipMemcpyAsync(g.ew32.get(), v.adjwgt, v.nnz * 4, kind, s));
    } else {
      g.ew_kind = EW_I64;
      g.ew64.reset(&pool, s, v.nnz ? v.nnz : 1);
      if (v.nnz) HIP_CHECK(hipMemcpyAsync(g.ew64.get(), v.adjwgt, v.nnz * 8, kind, s));
    }
  }
  DBuf<uint32_t> err(&pool, s, 2);  // [0] error bits, [1] some row not ascending
  err.zero();
  // node weights (always materialised as int64)
  DBuf<uint8_t> vtmp;
  const void* vw = nullptr;
  if (v.vwgt) {
    const size_t bytes = v.n * (v.vwgt_bits / 8);
    if (v.on_device) {
      vw = v.vwgt;
    } else {
      vtmp.reset(&pool, s, bytes);
      HIP_CHECK(hipMemcpyAsync(vtmp.get(), v.vwgt, bytes, hipMemcpyHostToDevice, s));
      vw = vtmp.get();
    }
  }
  g.nw.reset(&pool, s, v.n);
  k_nw_from<<<grid_for(v.n, 256), 256, 0, s>>>(vw, (int)v.vwgt_bits, v.n, g.nw.get(), err.get());
  LAUNCH_CHECK();
  k_check_xadj<<<grid_for(v.n + 1, 256), 256, 0, s>>>(g.xadj.get(), v.n, v.nnz, err.get());
  LAUNCH_CHECK();
  uint32_t bad = 0;
  HIP_CHECK(hipMemcpyAsync(&bad, err.get(), 4, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (bad) throw InvalidArg(describe(bad));
  g.src.reset(&pool, s, v.nnz ? v.nnz : 1);
  if (v.nnz) {
    k_src<<<grid_for(v.nnz, 256), 256, 0, s>>>(g.xadj.get(), v.n, v.nnz, g.src.get());
    LAUNCH_CHECK();
    const int full = v.validate ? 1 : 0;
    const unsigned gr = grid_for(v.nnz, 256);
    switch (g.ew_kind) {
      case EW_UNIT:
        k_check_entries<EW_UNIT><<<gr, 256, 0, s>>>(g.xadj.get(), g.adj.get(), nullptr, g.src.get(),
                                                    v.n, v.nnz, full, err.get());
        break;
      case EW_I32:
        k_check_entries<EW_I32><<<gr, 256, 0, s>>>(g.xadj.get(), g.adj.get(), g.ew32.get(),
                                                   g.src.get(), v.n, v.nnz, full, err.get());
        break;
      default:
        k_check_entries<EW_I64><<<gr, 256, 0, s>>>(g.xadj.get(), g.adj.get(), g.ew64.get(),
                                                   g.src.get(), v.n, v.nnz, full, err.get());
        break;
    }
    LAUNCH_CHECK();
  }
  DBuf<int64_t> tot(&pool, s, 2);
  tot.zero();
  unsigned gs = grid_for(v.n, 256);
  k_sum_i64<<<gs > 1024 ? 1024 : gs, 256, 0, s>>>(g.nw.get(), v.n, tot.get());
  LAUNCH_CHECK();
  if (v.nnz && g.ew_kind != EW_UNIT) {
    unsigned ge = grid_for(v.nnz, 256);
    if (g.ew_kind == EW_I32)
      k_sum_w<EW_I32><<<ge > 1024 ? 1024 : ge, 256, 0, s>>>(g.ew32.get(), v.nnz, tot.get() + 1);
    else
      k_sum_w<EW_I64><<<ge > 1024 ? 1024 : ge, 256, 0, s>>>(g.ew64.get(), v.nnz, tot.get() + 1);
    LAUNCH_CHECK();
  }
  int64_t hw = 0;
  uint32_t unsorted = 0;
  HIP_CHECK(hipMemcpyAsync(&bad, err.get(), 4, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&unsorted, err.get() + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&g.cV, tot.get(), 8, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&hw, tot.get() + 1, 8, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (bad) throw InvalidArg(describe(bad));
  g.wtot = g.ew_kind == EW_UNIT ? v.nnz : (uint64_t)hw;
  g.rows_sorted = unsorted == 0;
}

// ------------------------------------------------- allocation-free calls --
// Device scratch of lmgp_partition_noalloc: each GPU the library runs on holds
// its own copy from the library's load until the process ends.  Host code
// never passes the symbol itself (a host-side stand-in): it uses the address
// that hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[LMGP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

struct ScratchSlot {
  void* ptr = nullptr;  // device address of `scratch` on this device
  std::mutex call_mu;   // calls on one device share its array: one at a time
};

// The calling device's slot; the first call on a device (that device current)
// looks up the array's address.
ScratchSlot& scratch_slot() {
  static std::mutex mu;
  static ScratchSlot slots[MAX_DEVICES];
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw InvalidArg("device index out of range");
  std::lock_guard<std::mutex> g(mu);
  ScratchSlot& slot = slots[dev];
  if (!slot.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw HipError(e, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    slot.ptr = p;
  }
  return slot;
}

// Waits for the stream before the call gives the scratch array back (also
// when the call ends by an exception with work in flight).
struct StreamDrain {
  hipStream_t s;
  ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

}  // namespace

}  // namespace lmgp

using namespace lmgp;

extern "C" {

lmgp_status lmgp_partition_noalloc(lmgp_graph* g, uint32_t k, double eps, uint64_t seed,
                                   const lmgp_params* params, void* stream, uint32_t* block_out,
                                   uint32_t block_on_device, lmgp_result* res) {
  return guard([&] {
    if (!g) throw InvalidArg("NULL graph");
    if (!block_out) throw InvalidArg("block_out is NULL");
    if (g->g.n > LMGP_NOALLOC_MAX_NODES || g->g.nnz > LMGP_NOALLOC_MAX_ENTRIES)
      throw InvalidArg("graph too large for lmgp_partition_noalloc: n = " +
                       std::to_string(g->g.n) + " (max " + std::to_string(LMGP_NOALLOC_MAX_NODES) +
                       "), nnz = " + std::to_string(g->g.nnz) + " (max " +
                       std::to_string(LMGP_NOALLOC_MAX_ENTRIES) + ")");
    lmgp_params p = params ? *params : default_params();
    check_params(p);
    p.tune = LMGP_TUNE_OFF;  // no timing trials
    p.graph_rounds = 0;      // no stream capture
    std::vector<Job> jobs;
    jobs.push_back(make_job(&g->g, k, eps, seed, p));
    ScratchSlot& slot = scratch_slot();
    std::lock_guard<std::mutex> lock(slot.call_mu);
    StreamDrain drain{(hipStream_t)stream};
    NoAllocScope no_alloc;
    Pool arena(slot.ptr, LMGP_NOALLOC_SCRATCH_BYTES);
    Engine e(arena, (hipStream_t)stream, p);
    e.coarsen(jobs);
    uint32_t* outs[1] = {block_out};
    e.partition(jobs, outs, block_on_device != 0);
    if (res) {
      *res = jobs[0].res;
      res->t_coarsen_ns = e.t_coarsen_ns;
      res->t_initial_ns = e.t_initial_ns;
      res->t_refine_ns = e.t_refine_ns;
      res->t_total_ns = e.t_coarsen_ns + e.t_initial_ns + e.t_refine_ns;
    }
  });
}

void lmgp_default_params(lmgp_params* out) {
  if (out) *out = default_params();
}

const char* lmgp_last_error(void) { return g_err.c_str(); }

lmgp_status lmgp_tuner_info(uint64_t* entries, uint64_t* trials) {
  return guard([&] {
    if (entries) *entries = Tuner::get().entries();
    if (trials) *trials = Tuner::get().trials();
  });
}

void lmgp_tuner_clear(void) { Tuner::get().clear(); }

lmgp_status lmgp_graph_create(const lmgp_csr_view* view, const lmgp_allocator* alloc, void* stream,
                              lmgp_graph** out) {
  return guard([&] {
    if (!view || !out) throw InvalidArg("NULL argument");
    check_view(*view);
    auto h = std::make_unique<lmgp_graph>();
    h->g.own_pool = alloc ? std::make_shared<Pool>(alloc) : device_pool();
    h->g.pool = h->g.own_pool.get();
    create_input_graph(*view, h->g, (hipStream_t)stream);
    *out = h.release();
  });
}

void lmgp_graph_destroy(lmgp_graph* g) {
  if (!g) return;
  try {
    (void)hipStreamSynchronize(g->g.stream);
    auto pool = g->g.own_pool;
    delete g;
  } catch (...) {
  }
}

lmgp_status lmgp_graph_info(const lmgp_graph* g, uint64_t* n, uint64_t* nnz, int64_t* total_weight) {
  return guard([&] {
    if (!g) throw InvalidArg("NULL graph");
    if (n) *n = g->g.n;
    if (nnz) *nnz = g->g.nnz;
    if (total_weight) *total_weight = g->g.cV;
  });
}

lmgp_status lmgp_coarsen(lmgp_graph* g, uint32_t k, uint64_t seed, const lmgp_params* params,
                         void* stream, lmgp_hierarchy** out) {
  return guard([&] {
    if (!g || !out) throw InvalidArg("NULL argument");
    const lmgp_params p = params ? *params : default_params();
    check_params(p);
    auto h = std::make_unique<lmgp_hierarchy>();
    h->pool = g->g.own_pool;
    h->stream = (hipStream_t)stream;
    h->jobs.push_back(make_job(&g->g, k, 0.03, seed, p));
    h->engine = std::make_unique<Engine>(*h->pool, h->stream, p);
    h->engine->coarsen(h->jobs);
    *out = h.release();
  });
}

lmgp_status lmgp_hierarchy_levels(const lmgp_hierarchy* h, uint32_t* num_levels) {
  return guard([&] {
    if (!h || !num_levels) throw InvalidArg("NULL argument");
    *num_levels = h->jobs[0].nlevels;
  });
}

lmgp_status lmgp_hierarchy_level_info(const lmgp_hierarchy* h, uint32_t level, lmgp_level_info* out) {
  return guard([&] {
    if (!h || !out) throw InvalidArg("NULL argument");
    if (level >= h->jobs[0].nlevels) throw InvalidArg("level out of range");
    *out = h->jobs[0].info[level];
  });
}

lmgp_status lmgp_hierarchy_copy_level(const lmgp_hierarchy* h, uint32_t level, uint64_t* xadj,
                                      uint32_t* adjncy, int64_t* vwgt, int64_t* adjwgt,
                                      uint32_t* map) {
  return guard([&] {
    if (!h) throw InvalidArg("NULL hierarchy");
    if (level >= h->jobs[0].nlevels) throw InvalidArg("level out of range");
    h->engine->ensure_sorted(level);  // exported rows are sorted by neighbour id
    auto& levels = h->engine->levels();
    const Level& L = *levels[level];
    hipStream_t s = h->stream;
    if (xadj) HIP_CHECK(hipMemcpyAsync(xadj, L.xadj, (L.n + 1) * 8, hipMemcpyDeviceToHost, s));
    if (adjncy && L.nnz) HIP_CHECK(hipMemcpyAsync(adjncy, L.adj, L.nnz * 4, hipMemcpyDeviceToHost, s));
    if (vwgt) HIP_CHECK(hipMemcpyAsync(vwgt, L.nw, L.n * 8, hipMemcpyDeviceToHost, s));
    std::vector<int32_t> w32;
    if (adjwgt && L.nnz) {
      if (L.ew_kind == EW_I64) {
        HIP_CHECK(hipMemcpyAsync(adjwgt, L.ew, L.nnz * 8, hipMemcpyDeviceToHost, s));
      } else if (L.ew_kind == EW_I32) {
        w32.resize(L.nnz);
        HIP_CHECK(hipMemcpyAsync(w32.data(), L.ew, L.nnz * 4, hipMemcpyDeviceToHost, s));
      }
    }
    if (map && level + 1 < h->jobs[0].nlevels)
      HIP_CHECK(hipMemcpyAsync(map, L.map.get(), L.n * 4, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (adjwgt && L.nnz && L.ew_kind == EW_UNIT)
      for (uint64_t e = 0; e < L.nnz; ++e) adjwgt[e] = 1;
    if (adjwgt && L.nnz && L.ew_kind == EW_I32)
      for (uint64_t e = 0; e < L.nnz; ++e) adjwgt[e] = w32[e];
  });
}

void lmgp_hierarchy_destroy(lmgp_hierarchy* h) {
  if (!h) return;
  try {
    (void)hipStreamSynchronize(h->stream);
    auto pool = h->pool;
    delete h;
  } catch (...) {
  }
}

lmgp_status lmgp_partition(lmgp_graph* g, uint32_t k, double eps, uint64_t seed,
                           const lmgp_params* params, void* stream, uint32_t* block_out,
                           uint32_t block_on_device, lmgp_result* res) {
  return guard([&] {
    if (!g) throw InvalidArg("NULL graph");
    if (!block_out) throw InvalidArg("block_out is NULL");
    const lmgp_params p = params ? *params : default_params();
    check_params(p);
    std::vector<Job> jobs;
    jobs.push_back(make_job(&g->g, k, eps, seed, p));
    Engine e(*g->g.pool, (hipStream_t)stream, p);
    e.coarsen(jobs);
    uint32_t* outs[1] = {block_out};
    e.partition(jobs, outs, block_on_device != 0);
    if (res) {
      *res = jobs[0].res;
      res->t_coarsen_ns = e.t_coarsen_ns;
      res->t_initial_ns = e.t_initial_ns;
      res->t_refine_ns = e.t_refine_ns;
      res->t_total_ns = e.t_coarsen_ns + e.t_initial_ns + e.t_refine_ns;
    }
  });
}

lmgp_status lmgp_fire_scores(const lmgp_graph* g, uint64_t seed, uint64_t level, uint32_t weighted,
                             const lmgp_params* params, void* stream, uint32_t* score_out,
                             uint32_t out_on_device, uint64_t* stats_out) {
  return guard([&] {
    if (!g) throw InvalidArg("NULL graph");
    if (!score_out && g->g.nnz) throw InvalidArg("score_out is NULL");
    if (!g->g.rows_sorted) throw InvalidArg("fire scores need a graph with sorted rows");
    const lmgp_params p = params ? *params : default_params();
    check_params(p);
    const InputGraph& ig = g->g;
    const hipStream_t s = (hipStream_t)stream;
    Pool& pool = *ig.pool;
    FireLevel fl;
    fl.n = ig.n;
    fl.nnz = ig.nnz;
    fl.xadj = ig.xadj.get();
    fl.adj = ig.adj.get();
    fl.ew = ig.ew();
    fl.ew_kind = ig.ew_kind;
    fl.src = ig.src.get();
    fl.weighted = weighted != 0;
    fl.p_num = p.ff_p_num, fl.p_den = p.ff_p_den;
    fl.nu_num = p.ff_nu_num, fl.nu_den = p.ff_nu_den;
    std::vector<FireGraph> fg(1);
    fg[0].node_base = 0;
    fg[0].n = ig.n;
    fg[0].e0 = 0;
    fg[0].e1 = ig.nnz;
    auto pre = [&](uint64_t tag) { return hash_add(hash_prefix(seed, tag), level); };
    fg[0].pre_start = pre(TAG_FFSTART);
    fg[0].pre_draw = pre(TAG_FFDRAW);
    fg[0].pre_break = pre(TAG_FFBREAK);
    fg[0].pre_claim = pre(TAG_FFCLAIM);
    DBuf<uint32_t> tmp;
    uint32_t* dst = score_out;
    if (!out_on_device) {
      tmp.reset(&pool, s, ig.nnz ? ig.nnz : 1);
      dst = tmp.get();
    }
    fire_scores(fl, fg, dst, pool, s);
    if (!out_on_device && ig.nnz)
      HIP_CHECK(hipMemcpyAsync(score_out, dst, ig.nnz * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (stats_out) {
      stats_out[0] = fg[0].fires;
      stats_out[1] = fg[0].burns;
      stats_out[2] = fg[0].steps;
    }
  });
}

lmgp_status lmgp_partition_batch(lmgp_graph* const* graphs, const uint32_t* k, const double* eps,
                                 const uint64_t* seed, uint32_t count, const lmgp_params* params,
                                 void* stream, uint32_t* const* block_out, uint32_t block_on_device,
                                 lmgp_result* res) {
  return guard([&] {
    if (!graphs || !k || !eps || !seed || !block_out) throw InvalidArg("NULL argument");
    if (count == 0) return;
    const lmgp_params p = params ? *params : default_params();
    check_params(p);
    std::vector<Job> jobs;
    for (uint32_t i = 0; i < count; ++i) {
      if (!graphs[i]) throw InvalidArg("NULL graph in batch");
      if (!block_out[i]) throw InvalidArg("NULL block_out in batch");
      jobs.push_back(make_job(&graphs[i]->g, k[i], eps[i], seed[i], p));
    }
    Engine e(*graphs[0]->g.pool, (hipStream_t)stream, p);
    e.coarsen(jobs);
    e.partition(jobs, block_out, block_on_device != 0);
    if (res)
      for (uint32_t i = 0; i < count; ++i) {
        res[i] = jobs[i].res;
        res[i].t_coarsen_ns = e.t_coarsen_ns;
        res[i].t_initial_ns = e.t_initial_ns;
        res[i].t_refine_ns = e.t_refine_ns;
        res[i].t_total_ns = e.t_coarsen_ns + e.t_initial_ns + e.t_refine_ns;
      }
  });
}

}  // extern "C"
