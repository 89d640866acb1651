// Contraction, sparsification and uncoarsening helpers (host interfaces).
#pragma once
#include <vector>

#include "kernels.h"

namespace lmgp {

struct ContractIn {
  uint64_t n = 0;
  const uint64_t* xadj = nullptr;
  const uint32_t* adj = nullptr;
  const void* ew = nullptr;
  int ew_kind = EW_UNIT;
  const uint32_t* label = nullptr;
  const int64_t* W = nullptr;       // cluster weights indexed by label
  const uint32_t* csize = nullptr;  // cluster member counts indexed by label
  const uint32_t* gid = nullptr;
  const uint8_t* keep = nullptr;    // device, per graph: contract this graph
  int packed = 0;                   // every edge weight and row sum is below 2^32
  // false: coarse rows are aggregated in LDS hash tables and left in table
  // order (every consumer on the device is order independent); true: rows
  // sorted by neighbour id
  bool sorted = true;
  // every coarse edge weight is below 2^31: the coarse weights are stored as
  // int32 (ew32, ew_kind EW_I32) instead of int64
  bool narrow = false;
  std::vector<uint64_t> bounds;     // node boundaries of the graphs (B + 1 values)
  // every graph is kept: every node is mapped, so the summed member degree
  // is the level's entry count, entries (no read back)
  bool all_kept = false;
  uint64_t entries = 0;
};

struct ContractOut {
  uint64_t nc = 0, nnz = 0;
  DBuf<uint32_t> map;  // fine node -> coarse node (EMPTY_KEY for graphs not kept)
  DBuf<int64_t> nw;
  DBuf<uint32_t> gid;
  DBuf<uint64_t> xadj;
  DBuf<uint32_t> adj;
  DBuf<int64_t> ew;
  DBuf<int32_t> ew32;
  int ew_kind = EW_I64;  // which of ew / ew32 holds the coarse weights
  DBuf<uint32_t> src;
  std::vector<uint32_t> cid_at_bounds;  // coarse node boundaries of the graphs
  const void* weights() const { return ew_kind == EW_I32 ? (const void*)ew32.get() : ew.get(); }
};

struct ContractArgs {
  const uint64_t* xadj;
  const uint32_t* adj;
  const void* ew;
  const uint32_t* map;
  const uint64_t* mstart;
  const uint32_t* members;
  const unsigned long long* degsum;
  const uint64_t* tmpoff;
  uint32_t* tkey;   // scratch rows: row x's distinct neighbours at tmpoff[x] ..
  int64_t* tw;      //   tmpoff[x] + ndist[x] - 1, their summed weights
  uint32_t* tsrc;   //   and their row (written only when not NULL)
  uint32_t* ndist;
};

void contract_level(const ContractIn& in, ContractOut& out, Pool& pool, hipStream_t s);

// Sorts every row of a duplicate-free CSR by neighbour id (the row lengths do
// not change, so xadj stays valid); the weights come out as int64.
void sort_rows(uint64_t n, uint64_t nnz, const uint64_t* xadj, const uint32_t* adj,
               const void* ew, int ew_kind, int packed, DBuf<uint32_t>& out_adj,
               DBuf<int64_t>& out_ew, DBuf<uint32_t>& out_src, Pool& pool, hipStream_t s);

// ---------------------------------------------------------- sparsification --
struct SparsGraph {
  uint64_t node_base = 0;
  uint64_t e0 = 0, e1 = 0;   // entry range of the graph
  uint64_t m_hat = 0;
  bool triggered = false;
  uint32_t sampler = 0;      // 0 exact-size threshold, 1 uniform, 3 threshold with
                             // coins, 4 / 5 exact-size threshold on fire scores
  uint64_t pre = 0;          // H(seed, SPARS, level) prefix
  // outputs
  int64_t w_t = 0;
  uint64_t n_gt = 0, n_eq = 0;
};

struct SparsOut {
  uint64_t nnz = 0;
  DBuf<uint64_t> xadj;
  DBuf<uint32_t> adj;
  DBuf<int64_t> ew;
  DBuf<int32_t> ew32;
  int ew_kind = EW_I64;  // the input's: EW_I64 (ew) or EW_I32 (ew32)
  DBuf<uint32_t> src;
};

// Sparsify the triggered graphs of a union level in place of a new CSR.  The
// weights are int64 (ew_kind EW_I64) or int32 (EW_I32) and keep their width.
// Threshold sampling selects on the weights, or on `score` (one per entry,
// symmetric) when it is given.
void sparsify_level(uint64_t n, uint64_t nnz, const uint64_t* xadj, const uint32_t* adj,
                    const void* ew, int ew_kind, const uint32_t* src, const uint32_t* gid,
                    const uint32_t* score, std::vector<SparsGraph>& graphs, SparsOut& out,
                    Pool& pool, hipStream_t s);

// ------------------------------------------------ (Weighted) Forest Fire --
// A union level with sorted rows, and the fire parameters: break probability
// p = p_num / p_den, burn ratio nu = nu_num / nu_den.
struct FireLevel {
  uint64_t n = 0, nnz = 0;
  const uint64_t* xadj = nullptr;
  const uint32_t* adj = nullptr;
  const void* ew = nullptr;
  int ew_kind = EW_UNIT;
  const uint32_t* src = nullptr;
  bool weighted = true;  // Weighted Forest Fire (draws by edge weight), else Forest Fire
  uint32_t p_num = 3, p_den = 5, nu_num = 1, nu_den = 2;
};
struct FireGraph {
  uint64_t node_base = 0, n = 0;
  uint64_t e0 = 0, e1 = 0;  // entry range of the graph
  // H(seed, tag, level) prefixes of the four fire hashes
  uint64_t pre_start = 0, pre_draw = 0, pre_break = 0, pre_claim = 0;
  bool active = true;
  // outputs
  uint64_t fires = 0, burns = 0, steps = 0;
};
// Burn scores of every entry of the active graphs (score[e] = burns of e's
// undirected edge; entries of inactive graphs are zero).
void fire_scores(const FireLevel& lv, std::vector<FireGraph>& graphs, uint32_t* score, Pool& pool,
                 hipStream_t s);

// --------------------------------------------------------------- refinement --
void project_blocks(const uint32_t* map, const uint32_t* cblock, uint64_t n, uint32_t* block,
                    hipStream_t s);
void block_weights(const uint32_t* block, const int64_t* nw, uint64_t n, int64_t* BW, uint64_t K,
                   hipStream_t s);
// cut per graph over entries with src < adj (int64 atomics into cut[g])
void edge_cut(const uint32_t* src, const uint32_t* adj, const void* ew, int ew_kind,
              const uint32_t* block, const uint32_t* gid, uint64_t nnz, int64_t* cut,
              hipStream_t s);

}  // namespace lmgp
