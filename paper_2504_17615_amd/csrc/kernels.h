// Kernel interfaces of the coarsening / refinement pipeline.  Every kernel
// works on a union of one or more graphs laid out back to back (graph g owns
// nodes [node_base, node_base + nodes) and their CSR entries); `gid` maps a
// node to its graph and may be NULL when the union holds a single graph.
#pragma once
#include "common.h"
#include "memory.h"
#include "primitives.h"

namespace lmgp {

// Per-graph parameters, device resident, indexed by graph id.
struct GraphDesc {
  uint64_t node_base;   // first node of the graph in the union
  uint64_t nodes;       // its node count
  uint64_t label_base;  // subtracted from labels before hashing (clusters: node_base,
                        // refinement: first global block id of the graph)
  int64_t cap;          // U (clustering) or L_max (refinement)
  uint64_t pre_sub;     // hash prefixes: H(seed, SUB|RSUB, level, round)
  uint64_t pre_tie;     //               H(seed, TIE|RTIE, level, round) or H(seed, FAV, level)
  uint64_t pre_adm;     //               H(seed, ADM|RADM, level, round)
  uint64_t pre_two;     //               H(seed, TWOHOP, level)
  uint32_t active;      // graph takes part in the current phase
  uint32_t subrounds;
};

LMGP_D uint32_t graph_of(const uint32_t* gid, uint64_t u) { return gid ? gid[u] : 0u; }

// An LP move candidate (its admission-order hash is computed from u where a
// segment of an overfull target needs it).
struct Cand {
  uint32_t u;     // node
  uint32_t tgt;   // target cluster / block (global label)
  int64_t gain;   // r(target) - r(own)
};

// Degree classes of the rating kernel: lane groups of 2..64 lanes take nodes
// of degree <= 2*G (classes 0..5); a 256-thread block takes degree <= 256,
// 512, 1024 or 2048 with an LDS table of twice that many slots (classes
// 6..9, so that small tables keep occupancy high); a 1024-thread block with a
// packed LDS table of 8192 slots (load <= 3/4) takes degree <= 6144 and one
// of 16384 slots (128 KiB of the 160 KiB LDS) degree <= 8192 (classes 10,
// 11); larger degrees use tables in global memory (class 12).
constexpr int NCLASS = 13;
constexpr int CLASS_BLOCK = 6;   // first block class
constexpr int CLASS_BIG = 10;    // first big-block class
constexpr int CLASS_GLOBAL = 12;
constexpr int BLOCK_TABLE = 4096;  // largest LDS table of the block classes
constexpr int BIG_TABLE = 16384;   // largest packed LDS table of the big-block classes
LMGP_HD int degree_class(uint64_t d) {
  return d <= 4 ? 0 : d <= 8 ? 1 : d <= 16 ? 2 : d <= 32 ? 3 : d <= 64 ? 4 : d <= 128 ? 5
       : d <= 256 ? 6 : d <= 512 ? 7 : d <= 1024 ? 8 : d <= 2048 ? 9
       : d <= 6144 ? 10 : d <= 8192 ? 11 : 12;
}
// A class cut-off table: class c takes the degrees in (ub[c-1], ub[c]], the
// last class every degree above ub[NCLASS-2].  The default table is the one of
// degree_class; other tables (chosen by the autotuner) move degrees between
// kernels that can all hold them, which changes the speed and never a result.
struct ClassCuts {
  uint32_t ub[NCLASS - 1];
};
LMGP_HD int class_of(uint64_t d, const ClassCuts& c) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < NCLASS - 1; ++i) k += d > c.ub[i];
  return k;
}
LMGP_HD int class_group(int c) { return c < 6 ? (2 << c) : 256; }
// log2 of the LDS table of a block / big-block class
LMGP_HD int class_table_log(int c) { return c < CLASS_BIG ? c + 3 : c == CLASS_BIG ? 13 : 14; }
LMGP_HD bool is_big_class(int c) { return c == CLASS_BIG || c == CLASS_BIG + 1; }
// Sub-round bucket histograms hold at most this many (sub-round, class) pairs.
constexpr uint32_t MAX_BUCKETS = 512;

enum RateMode : int { MODE_LP = 0, MODE_FAV = 1 };

// Per-label tallies of one LP sub-round, one 16-byte record per label so that
// a target's tallies share a cache line (and are cleared by one store):
// summed weight of the candidates targeting the label, their number, and
// the admission's slot counter of an overfull target.
struct alignas(16) LabelTally {
  int64_t demand;
  uint32_t ntgt;
  uint32_t fill;
};

struct RateArgs {
  const uint64_t* xadj;
  const uint32_t* adj;
  const void* ew;
  const int64_t* nw;
  const uint32_t* label;
  const int64_t* W;        // weight of each label (cluster / block)
  const uint32_t* gid;
  const GraphDesc* gd;
  const uint32_t* list;    // nodes to rate
  uint32_t count;
  uint64_t degsum;         // summed degree of the listed nodes (for measurement)
  int phase;               // 0 clustering, 1 refinement, 2 favourites (for measurement)
  int mode;
  // MODE_LP outputs
  Cand* cands;             // slot i belongs to list[i]; tgt = EMPTY_KEY: no move
  LabelTally* tally;       // per label: demand and ntgt of the candidates targeting it
  // MODE_FAV output
  uint32_t* fav;
  // global-table class
  uint32_t* gkeys;
  int64_t* gvals;
  const uint64_t* goff;    // table offset of each listed node (class 7 only)
  unsigned long long* gtab;  // packed (label << 32 | rating) slots
  int packed;              // every rating fits in 32 bits: use gtab
  uint32_t few;            // labels < few <= FEW_LABELS: the tallies are counted
                           // by the admission (block-privatised), not here
  uint32_t trial;          // timing trial: candidates are written, the tallies
                           // are not counted
  // Planned launch (rounds replayed from a HIP graph): the grid is an upper
  // bound and the kernel takes its node count and list range from the
  // device-side plan of its sub-round, for the classes plan_c0..plan_c1 (list
  // and cands then point at the start of the whole bucket list and of the
  // sub-round's candidate slots).
  const struct SubPlan* plan;
  int plan_c0, plan_c1;
  // Refinement with at most 256 labels: the labels as bytes, gathered for the
  // neighbours instead of `label` (a quarter of the footprint: the array of a
  // large level stays in an XCD's L2).  NULL otherwise.
  const uint8_t* label8;
};

// Label counts up to this use block-privatised LDS histograms in admission
// (refinement: labels are the k blocks of each graph).
constexpr uint32_t FEW_LABELS = 1024;
// Waves (one node each) per block of the smallest dense-row classes.
constexpr int RW_WAVES = 4;

// Split of one launch over the classes 0..GROUP_CLASSES-1 (lane groups and
// the two smallest block classes).
constexpr int GROUP_CLASSES = 8;
struct GroupSplit {
  uint32_t bstart[GROUP_CLASSES + 1];  // first block of each class (and the total)
  uint32_t off[GROUP_CLASSES];         // list (and candidate slot) offset of each class
  uint32_t count[GROUP_CLASSES];       // nodes of each class
};

// Launch plan of one LP sub-round, written on the device from the bucket
// counts and offsets (what the host computes from them otherwise).
struct SubPlan {
  GroupSplit gs;              // the merged lane-group launch
  uint32_t lbase;             // list offset of the sub-round's first bucket
  uint32_t total;             // nodes listed in the sub-round (candidate slots)
  uint32_t cnt[NCLASS];       // nodes per class
  uint32_t off[NCLASS];       // list offset of each class, from lbase
};
// Plan of every sub-round: counts/offs are the bucket histogram and its
// exclusive prefix (S * NCLASS entries); dense: refinement with dense rows
// (only the lane-group classes go through the merged launch).
void launch_lp_plan(const unsigned long long* counts, const uint32_t* offs, uint32_t S, int dense,
                    SubPlan* plan, hipStream_t s);

// One rating launch for a degree class >= CLASS_BLOCK (a.count nodes of a.list).
void launch_rate(int cls, int ew_kind, const RateArgs& a, hipStream_t s);
// The classes 0..GROUP_CLASSES-1 in one launch; count/off per class, off
// relative to a.list (and a.cands).
void launch_rate_groups(int ew_kind, const RateArgs& a, const uint32_t* count,
                        const uint32_t* off, uint64_t degsum, hipStream_t s);
// Degree class CLASS_GLOBAL: tables in global memory, split over many blocks.
void launch_rate_hubs(int ew_kind, const RateArgs& a, Pool& pool, hipStream_t s);

// Sub-round bucketing of the nodes to rate: bucket = subround * NCLASS + class.
struct BucketArgs {
  const uint64_t* xadj;
  const uint32_t* gid;
  const GraphDesc* gd;
  uint64_t n;
  int mode;                // 0: LP sub-rounds (hash), 1: 2-hop singletons (filter arrays)
  const uint32_t* label;   // mode 1
  const uint32_t* csize;   // mode 1: member count per label
  const int64_t* nw;       // node weights
  uint32_t nbuckets;
  unsigned long long* counts;  // [nbuckets]
  unsigned long long* degs;  // [nbuckets] summed degrees (count pass): of every bucket
                             // when degs_all, else of the hub class only (its
                             // launches are sized by them; the others serve
                             // measurement and the autotuner)
  uint32_t degs_all;
  uint32_t* offs;          // [nbuckets] (offsets pass writes, scatter pass reads)
  uint32_t* fill;          // [nbuckets] (scatter pass)
  uint32_t* list;          // output
  uint8_t* bkt;            // per node: its bucket, written by the count pass and read
                           // by the scatter (0xFF: none), or NULL (recomputed)
  ClassCuts cuts;          // degree -> class (non-decreasing bounds)
  // mode 0, refinement of boundary nodes only: when `only` is set, a node is
  // bucketed only if only[u] != 0 and its sub-round is only_sub
  const uint8_t* only;
  uint32_t only_sub;
  // when set, the passes take the nodes ids[0 .. *nids) instead of 0 .. n-1
  const uint32_t* ids;
  const unsigned long long* nids;
};
void launch_bucket_count(const BucketArgs& a, hipStream_t s);
// The nodes u with flag[u] != 0 whose sub-round (mode 0 hash) is a.only_sub,
// written to ids in ascending order, *nids their count.  flag holds n bytes
// padded with zeros to a multiple of 8; block_cnt holds SUB_LIST_BLOCKS
// counters and wsel one byte per 8-byte flag word of scratch.
constexpr unsigned SUB_LIST_BLOCKS = 2048;
void launch_sub_list(const BucketArgs& a, const uint8_t* flag, uint32_t* block_cnt,
                     uint8_t* wsel, uint32_t* ids, unsigned long long* nids, hipStream_t s);
// offs = exclusive prefix of counts, fill = 0 (one small block on the device).
void launch_bucket_offsets(const BucketArgs& a, hipStream_t s);
void launch_bucket_scatter(const BucketArgs& a, hipStream_t s);

// A candidate of an overfull target's segment as the segment select reads it:
// its admission key (hi, lo), node weight and slot.
struct SegRec {
  uint64_t hi, lo;
  int64_t w;
  uint32_t ci, pad;
};

// Admission of LP candidates and application of moves.
struct AdmitArgs {
  Cand* cands;             // dense slots, tgt = EMPTY_KEY for no candidate
  uint32_t max_cands;      // number of slots
  const int64_t* W;
  int64_t* Wmut;
  const int64_t* nw;
  uint32_t* label;
  const uint32_t* gid;
  const GraphDesc* gd;
  LabelTally* tally;       // per label (cleared for the next sub-round by the apply)
  uint32_t* segbase;
  uint32_t* ovtotal;       // [1]
  uint32_t* ovcount;       // [1]
  uint32_t* ovtgts;
  uint8_t* adm;
  uint32_t* cpos;
  uint32_t* seg;
  SegRec* rec;             // [max_cands] records of the segments (beside seg)
  uint32_t* csize;         // member counts (clustering) or NULL
  uint64_t* moves;         // per graph: set to 1 when the sub-round moved a node
  uint32_t clear_ov;       // the apply clears ovtotal and ovcount (no control
                           // kernel runs after this admission)
  int64_t* ncl_count;      // per graph (clustering): non-empty clusters after the
                           // sub-round; a batch counts them from Wmut over nlabels
                           // labels (zero before), one graph through ncl_part;
                           // NULL in refinement
  uint64_t nlabels;
  // one graph: the apply kernel takes the count from the cluster weights'
  // transitions instead (returned by its atomics), one change per apply block
  // (grid_for(max_cands, 256) of them) into ncl_part, which the caller adds to
  // the count before the sub-round; NULL for a batch (counted from Wmut)
  int64_t* ncl_part;
  uint32_t few;            // labels < few <= FEW_LABELS (see RateArgs), else 0
  const SubPlan* plan;     // planned launch: max_cands is an upper bound, the
                           // slot count is plan->total
  uint8_t* label8;         // byte copy of the labels kept in step (or NULL)
};
void launch_admit(const AdmitArgs& a, hipStream_t s);

}  // namespace lmgp
