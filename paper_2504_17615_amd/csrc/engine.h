// Host orchestration of the multilevel pipeline on one GPU.
#pragma once
#include <functional>
#include <memory>
#include <vector>

#include "contract.h"
#include "lmgp.h"

namespace lmgp {

// A validated input graph in device memory (what lmgp_graph owns).
struct InputGraph {
  Pool* pool = nullptr;  // the graph's work memory (caching pool)
  std::shared_ptr<Pool> own_pool;
  // the block holding the arrays below and the arena handing them out
  // (declared before the arrays: released after them)
  DBuf<uint8_t> storage;
  std::shared_ptr<Pool> arena;
  hipStream_t stream = nullptr;
  uint64_t n = 0, nnz = 0;
  int ew_kind = EW_UNIT;
  int64_t cV = 0;
  uint64_t wtot = 0;  // sum of the weights of all entries (bounds every rating)
  bool rows_sorted = false;  // every row strictly ascending (checked at creation)
  DBuf<uint64_t> xadj;
  DBuf<uint32_t> adj;
  DBuf<int32_t> ew32;
  DBuf<int64_t> ew64;
  DBuf<int64_t> nw;
  DBuf<uint32_t> src;
  const void* ew() const {
    return ew_kind == EW_I32 ? (const void*)ew32.get()
         : ew_kind == EW_I64 ? (const void*)ew64.get() : nullptr;
  }
};

void create_input_graph(const lmgp_csr_view& v, InputGraph& g, hipStream_t s);

// One level of the union hierarchy.
struct Level {
  uint64_t n = 0, nnz = 0;
  const uint64_t* xadj = nullptr;
  const uint32_t* adj = nullptr;
  const void* ew = nullptr;
  int ew_kind = EW_UNIT;
  const int64_t* nw = nullptr;
  const uint32_t* src = nullptr;
  const uint32_t* gid = nullptr;  // NULL when a single graph is present
  // storage when owned
  DBuf<uint64_t> o_xadj;
  DBuf<uint32_t> o_adj;
  DBuf<int64_t> o_ew;
  DBuf<int32_t> o_ew32;  // coarse edge weights stored narrow (ew_kind EW_I32)
  DBuf<int64_t> o_nw;
  DBuf<uint32_t> o_src;
  DBuf<uint32_t> o_gid;
  DBuf<uint32_t> map;              // node of the next level (EMPTY_KEY if the graph stops)
  bool sorted = true;              // rows sorted by neighbour id (else in hash-table order)
  std::vector<uint32_t> graphs;    // batch indices of the graphs present, in union order
  std::vector<uint64_t> nbase;     // node boundaries (graphs.size() + 1)
  std::vector<uint64_t> ebase;     // entry boundaries (graphs.size() + 1)
};

// Per-graph state of a run.
struct Job {
  const InputGraph* g = nullptr;
  uint32_t k = 1;
  double eps = 0.03;
  uint64_t seed = 0;
  int64_t U = 1;
  int64_t lmax = 0;
  uint32_t nlevels = 1;  // levels of this graph's hierarchy
  // Union level holding this graph's input: 0, or the depth at which the
  // graph joined a run already in flight.  Its own level i (1-based, the
  // index every hash uses) is union level d0 + i - 1.
  uint32_t d0 = 0;
  uint32_t top() const { return d0 + nlevels - 1; }  // union level of its coarsest graph
  std::vector<lmgp_level_info> info;
  std::vector<uint32_t> block;  // host copy of the final blocks (when requested)
  lmgp_result res{};
};

class Engine {
 public:
  Engine(Pool& pool, hipStream_t s, const lmgp_params& p) : pool_(pool), s_(s), p_(p) {}
  ~Engine();
  // Builds the hierarchy for all jobs (one union).
  void coarsen(std::vector<Job>& jobs);
  // Optional: asked before every level after the first; the jobs it returns
  // join the run, their input graphs appended to the union level about to be
  // clustered (each must pass can_join).  coarsen appends them to `jobs`.
  std::function<std::vector<Job>()> admit;
  // Whether a graph may join this run in flight: rows sorted (its input level
  // then needs no order of its own) and edge weights within the widths the run
  // stores (packed ratings, narrow coarse weights).
  bool can_join(const InputGraph& g) const;
  // Initial partitioning, refinement and evaluation; writes blocks.
  void partition(std::vector<Job>& jobs, uint32_t* const* block_out, bool on_device);
  std::vector<std::unique_ptr<Level>>& levels() { return levels_; }
  // Sorts the rows of coarse level i (i >= 1) in place if they are not
  // sorted yet; the input level keeps its given order.
  void ensure_sorted(size_t i);

  int64_t t_coarsen_ns = 0, t_initial_ns = 0, t_refine_ns = 0;

 private:
  struct LpSpec {
    bool refine;
    uint32_t level;  // 1-based level index used in hashes
    uint32_t rounds;
  };
  void cluster(Level& L, std::vector<Job>& jobs, std::vector<uint8_t>& active,
               DBuf<uint32_t>& label, DBuf<int64_t>& W, DBuf<uint32_t>& csize,
               std::vector<uint64_t>& ncl, std::vector<lmgp_level_info>& stats);
  void run_lp(Level& L, std::vector<Job>& jobs, const LpSpec& spec, std::vector<uint8_t>& active,
              uint32_t* label, int64_t* W, size_t nlabels, uint32_t* csize,
              const std::vector<uint64_t>& label_base, std::vector<uint64_t>* ncl,
              std::vector<uint32_t>& rounds_run);
  void finish_level(std::vector<Job>& jobs, size_t j, const uint32_t* block,
                    const std::vector<uint64_t>& kbase, uint32_t* const* block_out,
                    bool on_device);
  void two_hop(Level& L, std::vector<Job>& jobs, const std::vector<uint8_t>& which,
               uint32_t level, uint32_t* label, int64_t* W, uint32_t* csize,
               std::vector<uint64_t>& ncl);
  void build_union(std::vector<Job>& jobs);
  void extend_union(std::vector<Job>& jobs, size_t first);
  void narrow_weights(Level& L);
  void rate_classes(RateArgs ra, const uint32_t* cnt, const uint32_t* offs,
                    const unsigned long long* degs, int ew_kind);

  Pool& pool_;
  hipStream_t s_;
  lmgp_params p_;
  bool packed_ = false;  // all ratings < 2^32: packed hub tables
  bool narrow_ = false;  // all entry weights < 2^31: coarse weights stored as int32
  // Whether the graphs whose coarsest level is level j are bisected on the
  // device (which needs sorted rows) rather than on the host.
  bool ip_on_device(const std::vector<Job>& jobs, size_t j) const;
  std::vector<std::unique_ptr<Level>> levels_;
};

// Recursive bipartitioning of a small host graph (coarsest level).
// xadj holds n + 1 global entry offsets (first = e0), adj global neighbour
// ids (minus n0 = local); `sorted`: every row is stored ascending; `asc`: the
// neighbours a row scan finds are enqueued in ascending order (as if sorted)
// rather than in stored order.
// A: uint32_t, or uint16_t for graphs of at most 2^16 nodes.
template <typename A>
void initial_partition_host(uint64_t n, const uint64_t* xadj, const A* adj, const int64_t* nw,
                            uint64_t e0, uint64_t n0, bool sorted, bool asc, uint32_t k,
                            uint64_t seed, uint64_t level, std::vector<uint32_t>& block);

lmgp_params default_params();
void check_params(const lmgp_params& p);

}  // namespace lmgp

// The opaque graph handle of the C ABI.
struct lmgp_graph {
  lmgp::InputGraph g;
};
