// (Weighted) Forest Fire edge scores (Sec. 4.2; the appendix's WFF
// algorithm), for threshold sampling on scores instead of edge weights.
//
// A fire starts at a random node and spreads frontier by frontier: every node
// of the frontier draws, one at a time and without replacement, neighbours
// that were not visited when the frontier began, each with probability
// proportional to its edge weight among the remaining ones (Weighted Forest
// Fire) or uniformly (Forest Fire), and stops after a draw with probability
// p.  A node drawn by several frontier nodes is burned by the draw with the
// smallest (upper 32 bits of H(FFCLAIM, level, f, l, v, u), u); the burned
// edge's score goes up by one and the node joins the visited set and the
// next frontier.  Fire f is started while the burns of fires 0..f-1 are at
// most nu |E|.  Every draw and break is a counter hash, so the scores do not
// depend on scheduling.
//
// Fires are independent apart from that schedule, so they run side by side,
// as the appendix's parallel loop over fires does: a batch of up to 64 fires
// advances in lock-step, one frontier step for all of them at a time.  A
// node's visited sets are the bits of one 64-bit word (bit s: the fire in
// slot s), claims are resolved per (slot, node), and burns go to a log.  When
// the batch is out, the burns per fire decide the prefix of its fires that
// the schedule runs, and only their logged burns reach the scores; a batch
// that overshoots the budget costs work, never a different result.  Fires
// whose start node is isolated burn nothing and leave the schedule's
// condition as it was: a batch takes the next fires with a non-isolated
// start and counts the others as run.
//
// A step is three launches: the draws (a wavefront per frontier entry, the
// rows of up to 256 entries held in registers across its draws, longer rows
// with their drawn positions in a register mask and an LDS list), each claim folded at once
// into its (slot, node) minimum claim word (64-bit atomicMin; no claim can
// target a node of the current frontier of its fire, whose words the same
// kernel clears); the winners (visited bits, log, next frontier); and a
// one-thread kernel that swaps the frontiers.  The host reads the control
// word once per 32 steps.  Rows must be sorted: draws scan them in ascending
// neighbour order and a burn finds the reverse entry by binary search.
#include <algorithm>

#include "contract.h"
#include "primitives.h"
#include "profiler.h"

namespace lmgp {

namespace {

struct FireCtl {
  uint32_t cur;       // frontier buffer being drawn from
  uint32_t out;       // the batch's fires are all out
  uint32_t overflow;  // a step's claims did not fit: the batch is redone
  uint32_t nslots;    // fires in this batch
  uint32_t long_overflow;  // a node drew past its list of long-row draws: the
                           // batch is redone one fire at a time with flags
  uint32_t pad;
  uint64_t l;         // current frontier step of the batch
  uint64_t nfront, nnext, nclaims, nlog;
  uint64_t scan_end;  // first fire id the batch did not examine
  uint64_t steps, scanned, claims_total;
};

struct FireArgs {
  const uint64_t* xadj;
  const uint32_t* adj;
  const void* ew;
  const uint32_t* src;
  uint64_t nb;  // first node of the graph (hashes, frontiers and bits use local ids)
  uint64_t n;   // nodes of the graph
  uint64_t* fid;             // fire id of each slot
  unsigned long long* vis;   // visited bits per local node
  uint32_t* taken;           // drawn entries of long rows when batches hold one fire
  uint64_t* claims;          // (slot << 58) | entry, this step
  uint64_t claim_cap;
  unsigned long long* cw;    // [slot][local node] smallest claim word (all ones when none)
  uint64_t* front0;          // (slot << 32) | local node
  uint64_t* front1;
  uint64_t* log;             // (slot << 58) | entry of every burn of the batch
  uint32_t* score;           // burns of each entry's edge
  FireCtl* ctl;
  uint64_t pre_start, pre_draw, pre_break, pre_claim;
  uint64_t pthr;             // break iff H < pthr, or always
  uint32_t always;
};

constexpr int FF_NT = 256;
constexpr int FF_WAVES = FF_NT / WAVE;
constexpr int FF_CACHE = 4;                            // rows of up to 4 x 64 entries in registers
constexpr uint64_t FF_MASK_ROW = (uint64_t)WAVE * 64;  // rows up to this: register masks
constexpr uint32_t FF_SLOTS = 64;
constexpr uint32_t FF_LONG = 256;  // a wave's listed draws beyond the masked part of a row
constexpr int ENTRY_BITS = 58;
constexpr uint64_t ENTRY_MASK = (1ull << ENTRY_BITS) - 1;

LMGP_D uint64_t* front_of(const FireArgs& a, uint32_t i) { return i ? a.front1 : a.front0; }

// floor(H * W / 2^64): a draw position in [0, W)
LMGP_D uint64_t scaled(uint64_t h, uint64_t w) { return __umul64hi(h, w); }

LMGP_D uint32_t start_of(const FireArgs& a, uint64_t f) {
  return (uint32_t)scaled(hash_add(a.pre_start, f), a.n);
}

// The batch's fires: the next (at most) `want` fires from f0 on whose start
// node has a neighbour, among at most `scan_max` fire ids; one block.
__global__ __launch_bounds__(1024) void k_ff_batch(FireArgs a, uint64_t f0, uint32_t want,
                                                   uint64_t scan_max) {
  __shared__ uint32_t sm[16];
  uint32_t found = 0;
  uint64_t end = f0;
  for (uint64_t base = f0; found < want && base - f0 < scan_max; base += 1024) {
    const uint64_t f = base + threadIdx.x;
    const uint32_t s = start_of(a, f);
    const uint64_t u = a.nb + s;
    const uint32_t live = a.xadj[u + 1] > a.xadj[u] ? 1u : 0u;
    uint32_t tot;
    const uint32_t pos = block_exclusive_scan<uint32_t, 16>(live, sm, tot);
    const uint32_t slot = found + pos;
    if (live && slot < want) {
      a.fid[slot] = f;
      a.front0[slot] = ((uint64_t)slot << 32) | s;
    }
    if (found + tot >= want) {
      // the batch ends after the want-th live fire of this chunk
      if (live && slot == want - 1) sm[0] = threadIdx.x;
      __syncthreads();
      end = base + sm[0] + 1;
      found = want;
      __syncthreads();
    } else {
      found += tot;
      end = base + 1024;
    }
  }
  if (threadIdx.x == 0) {
    FireCtl c{};
    c.nslots = found;
    c.nfront = found;
    c.out = found == 0 ? 1u : 0u;
    c.scan_end = end;
    *a.ctl = c;
  }
}

LMGP_D unsigned long long claim_word(const FireArgs& a, uint64_t hc, uint64_t e, uint32_t& ul,
                                     uint32_t& vl) {
  vl = (uint32_t)(a.adj[e] - a.nb);
  ul = (uint32_t)(a.src[e] - a.nb);
  const uint64_t key = hash_add(hash_add(hc, vl), ul) >> 32;
  return (key << 32) | ul;
}

// Stages a wave's claims in registers (lane i holds the i-th) and writes them
// out 64 at a time with one reservation; each claim's word goes into its
// (slot, node) minimum as it is made.
struct ClaimStage {
  uint64_t mine = 0;
  int cnt = 0;
  LMGP_D void push(const FireArgs& a, uint64_t slot, uint64_t e, uint64_t hc) {
    if (lane_id() == cnt) {
      mine = (slot << ENTRY_BITS) | e;
      uint32_t ul, vl;
      const unsigned long long w = claim_word(a, hc, e, ul, vl);
      atomicMin(&a.cw[slot * a.n + vl], w);
    }
    if (++cnt == WAVE) flush(a);
  }
  LMGP_D void flush(const FireArgs& a) {
    if (!cnt) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd((unsigned long long*)&a.ctl->nclaims, (unsigned long long)cnt);
    base = __shfl(base, 0);
    if (base + cnt > a.claim_cap) {
      if (lane_id() == 0) a.ctl->overflow = 1;  // the same value from every writer
    } else if (lane_id() < cnt) {
      a.claims[base + lane_id()] = mine;
    }
    cnt = 0;
  }
};

LMGP_D bool taken_at(const FireArgs& a, uint64_t e) {
  return __hip_atomic_load(&a.taken[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// The draws of the frontier: one wavefront per (fire, node) entry.
template <int EWK>
__global__ __launch_bounds__(FF_NT) void k_ff_draw(FireArgs a) {
  __shared__ uint32_t longpick[FF_WAVES][FF_LONG];
  const FireCtl* cp = a.ctl;
  if (cp->out || cp->overflow || cp->long_overflow) return;
  uint32_t* lp = longpick[threadIdx.x / WAVE];
  const uint64_t nfront = cp->nfront, l = cp->l;
  const uint64_t* front = front_of(a, cp->cur);
  const int lane = lane_id();
  const uint64_t nw = (uint64_t)gridDim.x * FF_WAVES;
  ClaimStage st;
  uint64_t scanned = 0;  // entries read (lane 0's count)
  for (uint64_t i = (uint64_t)blockIdx.x * FF_WAVES + threadIdx.x / WAVE; i < nfront; i += nw) {
    const uint64_t fe = front[i];
    const uint64_t slot = fe >> 32;
    const uint32_t ul = (uint32_t)fe;
    const uint64_t u = a.nb + ul;
    const uint64_t f = a.fid[slot];
    const uint64_t bit = 1ull << slot;
    const uint64_t hd = hash_add(hash_add(hash_add(a.pre_draw, f), l), ul);
    const uint64_t hb = hash_add(hash_add(hash_add(a.pre_break, f), l), ul);
    const uint64_t hc = hash_add(hash_add(a.pre_claim, f), l);
    if (lane == 0) a.cw[slot * a.n + ul] = ~0ull;  // cleared for this step's claims
    const uint64_t beg = a.xadj[u], deg = a.xadj[u + 1] - beg;
    if (deg <= (uint64_t)FF_CACHE * WAVE) {
      scanned += deg;
      // candidate weights in registers; a drawn entry's weight drops to 0
      int64_t wv[FF_CACHE];
#pragma unroll
      for (int c = 0; c < FF_CACHE; ++c) {
        const uint64_t k = (uint64_t)c * WAVE + lane;
        wv[c] = 0;
        if (k < deg && !(a.vis[a.adj[beg + k] - a.nb] & bit)) wv[c] = edge_w<EWK>(a.ew, beg + k);
      }
      // each draw removes a candidate, so at most deg draws
      for (uint64_t j = 0; j < deg; ++j) {
        int64_t t = 0;
#pragma unroll
        for (int c = 0; c < FF_CACHE; ++c) t += wv[c];
        const uint64_t W = (uint64_t)wave_reduce_sum(t);
        if (W == 0) break;
        const uint64_t R = scaled(hash_add(hd, j), W);
        uint64_t run = 0;
        int pick = -1;
#pragma unroll
        for (int c = 0; c < FF_CACHE; ++c) {
          if (pick < 0) {
            const int64_t inc = wave_inclusive_scan(wv[c]);
            const uint64_t mask = __ballot(run + (uint64_t)inc > R);
            if (mask) {
              const int ln = __builtin_ctzll(mask);
              pick = c * WAVE + ln;
              if (lane == ln) wv[c] = 0;
            } else {
              run += (uint64_t)__shfl(inc, WAVE - 1);
            }
          }
        }
        if (pick < 0) break;  // unreachable: R < W
        st.push(a, slot, beg + (uint64_t)pick, hc);
        if (a.always || hash_add(hb, j) < a.pthr) break;
      }
    } else {
      // longer rows: two passes per draw.  Each lane keeps its drawn
      // positions among the first 64 x 64 entries in a register mask (bit c:
      // entry c * 64 + lane); draws further along the row go to a list in
      // LDS (a node that outgrows it stops the batch, which is then run one
      // fire at a time).  With one fire per batch, `taken` flags replace the
      // list: read and written at device scope with a fence after each flag,
      // so that the wave's next pass sees its own flags whatever the L1 holds
      // (the fence writes back the L2, so only these rows pay it)
      const bool flags = a.taken != nullptr;
      uint64_t tk = 0;
      uint32_t nlong = 0;
      auto drawn = [&](uint64_t k, uint32_t c) -> bool {
        if (flags) return taken_at(a, beg + k);
        if (c < 64) return ((tk >> c) & 1) != 0;
        for (uint32_t q = 0; q < nlong; ++q)
          if (lp[q] == (uint32_t)k) return true;
        return false;
      };
      for (uint64_t j = 0; j < deg; ++j) {
        int64_t t = 0;
        scanned += deg;
        uint32_t c = 0;
        for (uint64_t k = lane; k < deg; k += WAVE, ++c) {
          const uint64_t e = beg + k;
          if (!drawn(k, c) && !(a.vis[a.adj[e] - a.nb] & bit)) t += edge_w<EWK>(a.ew, e);
        }
        const uint64_t W = (uint64_t)wave_reduce_sum(t);
        if (W == 0) break;
        const uint64_t R = scaled(hash_add(hd, j), W);
        uint64_t run = 0, pick = ~0ull;
        uint32_t pc = 0;
        c = 0;
        for (uint64_t k0 = 0; k0 < deg; k0 += WAVE, ++c) {
          const uint64_t k = k0 + lane, e = beg + k;
          int64_t w = 0;
          if (k < deg && !drawn(k, c) && !(a.vis[a.adj[e] - a.nb] & bit))
            w = edge_w<EWK>(a.ew, e);
          scanned += WAVE;
          const int64_t inc = wave_inclusive_scan(w);
          const uint64_t mask = __ballot(run + (uint64_t)inc > R);
          if (mask) {
            const int ln = __builtin_ctzll(mask);
            pick = k0 + (uint64_t)ln;
            pc = c;
            if (!flags && c < 64 && lane == ln) tk |= 1ull << c;
            break;
          }
          run += (uint64_t)__shfl(inc, WAVE - 1);
        }
        if (pick == ~0ull) break;  // unreachable: R < W
        if (flags) {
          if (lane == 0)
            __hip_atomic_store(&a.taken[beg + pick], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          __threadfence();  // performed before the next pass reads
        } else if (pc >= 64) {
          if (nlong == FF_LONG) {
            if (lane == 0) a.ctl->long_overflow = 1;
            break;
          }
          if (lane == 0) lp[nlong] = (uint32_t)pick;
          ++nlong;
          wave_sync();
        }
        st.push(a, slot, beg + pick, hc);
        if (a.always || hash_add(hb, j) < a.pthr) break;
      }
    }
  }
  st.flush(a);
  if (lane_id() == 0 && scanned)
    atomicAdd((unsigned long long*)&a.ctl->scanned, (unsigned long long)scanned);
}

// The winners: one per claimed (slot, node), the claim equal to its minimum.
__global__ __launch_bounds__(256) void k_ff_win(FireArgs a, uint32_t use_taken) {
  const FireCtl* cp = a.ctl;
  if (cp->out || cp->overflow || cp->long_overflow) return;
  const uint64_t nc = cp->nclaims, l = cp->l;
  uint64_t* next = front_of(a, cp->cur ^ 1u);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // whole waves run every iteration (the appends are wave-aggregated)
  const uint64_t span = (nc + WAVE - 1) / WAVE * WAVE;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += stride) {
    bool win = false;
    uint64_t cl = 0, slot = 0;
    uint32_t vl = 0;
    if (i < nc) {
      cl = a.claims[i];
      slot = cl >> ENTRY_BITS;
      const uint64_t e = cl & ENTRY_MASK;
      const uint64_t hc = hash_add(hash_add(a.pre_claim, a.fid[slot]), l);
      uint32_t ul;
      const unsigned long long w = claim_word(a, hc, e, ul, vl);
      if (use_taken) a.taken[e] = 0;
      if (a.cw[slot * a.n + vl] == w) {
        win = true;
        atomicOr(&a.vis[vl], 1ull << slot);
      }
    }
    const uint64_t mask = __ballot(win);
    if (mask) {
      unsigned long long fb = 0, lb = 0;
      const int leader = __builtin_ctzll(mask);
      const unsigned long long cnt = (unsigned long long)__popcll(mask);
      if (lane_id() == leader) {
        fb = atomicAdd((unsigned long long*)&a.ctl->nnext, cnt);
        lb = atomicAdd((unsigned long long*)&a.ctl->nlog, cnt);
      }
      fb = __shfl(fb, leader);
      lb = __shfl(lb, leader);
      const uint64_t r = __popcll(mask & lanemask_lt());
      if (win) {
        next[fb + r] = (slot << 32) | vl;
        a.log[lb + r] = cl;
      }
    }
  }
}

// One thread ends the step.  (A last-block-done ending inside k_ff_win
// would need a device-scope fence in every block, which writes back each
// XCD's L2 and costs more than this launch.)
__global__ void k_ff_control(FireArgs a) {
  FireCtl c = *a.ctl;
  if (c.out || c.overflow || c.long_overflow) return;
  c.claims_total += c.nclaims;
  c.nfront = c.nnext;
  c.nnext = 0;
  c.nclaims = 0;
  c.cur ^= 1u;
  c.l += 1;
  c.steps += 1;
  if (c.nfront == 0) c.out = 1;
  *a.ctl = c;
}

// Burns per slot from the log.
__global__ __launch_bounds__(256) void k_ff_burns(const uint64_t* log, const FireCtl* ctl,
                                                  unsigned long long* sburn) {
  __shared__ uint32_t h[FF_SLOTS];
  if (threadIdx.x < FF_SLOTS) h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t nl = ctl->nlog;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += stride)
    atomicAdd(&h[log[i] >> ENTRY_BITS], 1u);
  __syncthreads();
  if (threadIdx.x < FF_SLOTS && h[threadIdx.x])
    atomicAdd(&sburn[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// The burns of the fires the schedule runs (slots below `accepted`) reach
// the scores of both entries of their edges.
__global__ __launch_bounds__(256) void k_ff_apply(FireArgs a, uint32_t accepted) {
  const uint64_t nl = a.ctl->nlog;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += stride) {
    const uint64_t cl = a.log[i];
    if ((cl >> ENTRY_BITS) >= accepted) continue;
    const uint64_t e = cl & ENTRY_MASK;
    atomicAdd(&a.score[e], 1u);
    // the reverse entry: u in v's sorted row
    const uint32_t u = a.src[e], v = a.adj[e];
    uint64_t lo = a.xadj[v], hi = a.xadj[v + 1];
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (a.adj[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    if (lo < a.xadj[v + 1] && a.adj[lo] == u) atomicAdd(&a.score[lo], 1u);
  }
}

// Maximum degree and number of non-isolated nodes of a node range.
__global__ __launch_bounds__(256) void k_deg_stats(const uint64_t* xadj, uint64_t n0, uint64_t n1,
                                                   unsigned long long* out) {
  uint64_t m = 0, live = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t u = n0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n1; u += stride) {
    const uint64_t d = xadj[u + 1] - xadj[u];
    m = d > m ? d : m;
    live += d ? 1 : 0;
  }
  m = wave_reduce_max(m);
  live = wave_reduce_sum(live);
  if (lane_id() == 0) {
    if (m) atomicMax(&out[0], (unsigned long long)m);
    if (live) atomicAdd(&out[1], (unsigned long long)live);
  }
}

constexpr int FF_STEPS = 32;                  // steps enqueued between reads of the control word
constexpr uint64_t FF_SCAN_MAX = 1ull << 20;  // fire ids examined per batch

bool u128_le(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  return (unsigned __int128)a * b <= (unsigned __int128)c * d;
}

}  // namespace

void fire_scores(const FireLevel& lv, std::vector<FireGraph>& graphs, uint32_t* score, Pool& pool,
                 hipStream_t s) {
  if (lv.ew_kind != EW_UNIT && lv.ew_kind != EW_I32 && lv.ew_kind != EW_I64)
    throw InvalidArg("fire scores: unknown edge weight kind");
  if (lv.p_den == 0 || lv.nu_den == 0) throw InvalidArg("fire scores: zero denominator");
  if (lv.nnz) device_zero(score, lv.nnz * sizeof(uint32_t), s);
  for (FireGraph& g : graphs) g.fires = g.burns = g.steps = 0;
  if (lv.n == 0 || lv.nnz == 0) return;
  if (lv.n >= 0xFFFFFFFFull || lv.nnz > ENTRY_MASK)
    throw InvalidArg("fire scores: graph too large");
  const bool always = lv.p_num >= lv.p_den;
  const uint64_t pthr = always ? 0 : (uint64_t)(((unsigned __int128)lv.p_num << 64) / lv.p_den);
  const bool weighted = lv.weighted && lv.ew_kind != EW_UNIT;
  const int ewk = weighted ? lv.ew_kind : EW_UNIT;
  const uint64_t wb = weighted ? (lv.ew_kind == EW_I32 ? 4 : 8) : 0;
  DBuf<unsigned long long> dstat(&pool, s, 2);
  DBuf<FireCtl> ctl(&pool, s, 1);
  DBuf<unsigned long long> sburn(&pool, s, FF_SLOTS);
  DBuf<uint64_t> fid(&pool, s, FF_SLOTS);
  for (FireGraph& g : graphs) {
    if (!g.active || g.n == 0 || g.e1 == g.e0) continue;
    const uint64_t m = (g.e1 - g.e0) / 2, n = g.n, ne = g.e1 - g.e0;
    dstat.zero();
    k_deg_stats<<<std::min(grid_for(n, 256), 1024u), 256, 0, s>>>(lv.xadj, g.node_base,
                                                                  g.node_base + n, dstat.get());
    LAUNCH_CHECK();
    unsigned long long dst[2] = {0, 0};
    read_now(dst, dstat.get(), sizeof(dst), s);
    const uint64_t nlive = dst[1];  // dst[0]: the maximum degree
    // slots: 64, fewer when the per-slot arrays would outgrow 2^25 words
    uint64_t cap_slots =
        std::min<uint64_t>(FF_SLOTS, std::max<uint64_t>(1, (1ull << 25) / (n + 1)));
    DBuf<unsigned long long> vis(&pool, s, n);
    DBuf<unsigned long long> cw(&pool, s, cap_slots * n);
    DBuf<uint64_t> front0(&pool, s, cap_slots * (n + 1)), front1(&pool, s, cap_slots * (n + 1));
    DBuf<uint64_t> log(&pool, s, cap_slots * (n + 1));
    DBuf<uint32_t> taken;  // set when batches fall back to one fire
    uint64_t claim_cap = std::max<uint64_t>(4 * cap_slots * (n + 1), 1u << 16);
    claim_cap = std::min<uint64_t>(claim_cap, cap_slots * ne);
    DBuf<uint64_t> claims(&pool, s, claim_cap);
    device_fill_u32((uint32_t*)cw.get(), 0xFFFFFFFFu, 2 * cap_slots * n, s);
    FireArgs a{};
    a.xadj = lv.xadj;
    a.adj = lv.adj;
    a.ew = lv.ew;
    a.src = lv.src;
    a.nb = g.node_base;
    a.n = n;
    a.fid = fid.get();
    a.vis = vis.get();
    a.taken = taken.get();
    a.claims = claims.get();
    a.claim_cap = claim_cap;
    a.cw = cw.get();
    a.front0 = front0.get();
    a.front1 = front1.get();
    a.log = log.get();
    a.score = score;
    a.ctl = ctl.get();
    a.pre_start = g.pre_start;
    a.pre_draw = g.pre_draw;
    a.pre_break = g.pre_break;
    a.pre_claim = g.pre_claim;
    a.pthr = pthr;
    a.always = always ? 1u : 0u;
    const unsigned gd = std::min(grid_for(cap_slots * n, FF_WAVES), 4096u);
    unsigned gw = std::min(grid_for(claim_cap, 256), 4096u);
    // bytes from the device's counts: per frontier entry its offsets and
    // fire (24 B), per entry read by a draw its neighbour, the neighbour's
    // visited word and the weight, per claim its word (atomicMin), 8 B
    // written and read back with its row, neighbour, fire and claim word by
    // the winners, per burn the visited bits, frontier and log slots, the
    // log read twice and the two score updates with the reverse search
    ProfScope prof("sp:fire", 0, s);
    uint64_t bytes = 0;
    uint64_t f0 = 0, burns = 0, fires = 0, steps = 0, avg = 0, nbatch = 0;
    // the first batch: as many fires as the budget would take if each burned
    // every non-isolated node once, plus two
    const unsigned __int128 budget = (unsigned __int128)lv.nu_num * m / lv.nu_den;
    uint32_t want = (uint32_t)std::min<unsigned __int128>(cap_slots, budget / std::max<uint64_t>(1, nlive) + 2);
    bool done = false;
    while (!done) {
      vis.zero();
      k_ff_batch<<<1, 1024, 0, s>>>(a, f0, want, FF_SCAN_MAX);
      LAUNCH_CHECK();
      FireCtl hc{};
      for (;;) {
        for (int b = 0; b < FF_STEPS; ++b) {
          if (ewk == EW_UNIT) k_ff_draw<EW_UNIT><<<gd, FF_NT, 0, s>>>(a);
          else if (ewk == EW_I32) k_ff_draw<EW_I32><<<gd, FF_NT, 0, s>>>(a);
          else k_ff_draw<EW_I64><<<gd, FF_NT, 0, s>>>(a);
          LAUNCH_CHECK();
          k_ff_win<<<gw, 256, 0, s>>>(a, taken.get() ? 1u : 0u);
          LAUNCH_CHECK();
          k_ff_control<<<1, 1, 0, s>>>(a);
          LAUNCH_CHECK();
        }
        read_now(&hc, ctl.get(), sizeof(hc), s);
        if (hc.out || hc.overflow || hc.long_overflow) break;
        // every fire of the batch visits a new node each step
        if (hc.steps > n + 2) throw InvalidArg("fire scores: a batch does not end");
      }
      if (hc.overflow) {
        // a step drew more claims than the buffer holds: grow it and run the
        // batch again (nothing has reached the scores)
        claim_cap = std::min<uint64_t>(claim_cap * 4, cap_slots * ne);
        claims.reset(&pool, s, claim_cap);
        a.claims = claims.get();
        a.claim_cap = claim_cap;
        gw = std::min(grid_for(claim_cap, 256), 4096u);
        device_fill_u32((uint32_t*)cw.get(), 0xFFFFFFFFu, 2 * cap_slots * n, s);
        if (taken.get()) taken.zero();
        continue;
      }
      if (hc.long_overflow) {
        // a node drew more often than its list holds, beyond the masked part
        // of its row: from now on one fire per batch, with per-entry flags
        cap_slots = 1;
        want = 1;
        taken.reset(&pool, s, lv.nnz);
        taken.zero();
        a.taken = taken.get();
        device_fill_u32((uint32_t*)cw.get(), 0xFFFFFFFFu, 2 * n, s);
        continue;
      }
      ++nbatch;
      steps += hc.steps;
      const uint32_t ns = hc.nslots;
      std::vector<unsigned long long> sb(FF_SLOTS, 0);
      std::vector<uint64_t> fids(FF_SLOTS, 0);
      if (ns) {
        sburn.zero();
        k_ff_burns<<<std::min(grid_for(hc.nlog, 256), 1024u), 256, 0, s>>>(log.get(), ctl.get(),
                                                                            sburn.get());
        LAUNCH_CHECK();
        read_now(sb.data(), sburn.get(), ns * sizeof(unsigned long long), s);
        read_now(fids.data(), fid.get(), ns * sizeof(uint64_t), s);
      }
      // the schedule over this batch's fires, in order; the fires between
      // them start at isolated nodes, burn nothing and run
      uint32_t accepted = 0;
      for (uint32_t q = 0; q < ns; ++q) {
        accepted = q + 1;
        burns += sb[q];
        fires = fids[q] + 1;
        if (!u128_le(burns, lv.nu_den, lv.nu_num, m)) {
          done = true;
          break;
        }
      }
      if (!done) {
        fires = hc.scan_end;
        f0 = hc.scan_end;
      }
      if (accepted) {
        k_ff_apply<<<std::min(grid_for(hc.nlog, 256), 4096u), 256, 0, s>>>(a, accepted);
        LAUNCH_CHECK();
      }
      bytes += 24 * (hc.nslots + hc.nlog) + (8 + 8 + wb) * hc.scanned + 48 * hc.claims_total +
               56 * hc.nlog;
      // the next batch: about as many fires as the rest of the budget needs
      uint64_t live = 0;
      for (uint32_t q = 0; q < accepted; ++q) live += sb[q];
      if (accepted) avg = std::max<uint64_t>(1, live / accepted);
      if (!done && avg) {
        const uint64_t left = budget >= burns ? (uint64_t)(budget - burns) : 0;
        want = (uint32_t)std::min<uint64_t>(cap_slots, left / avg + 2);
      }
      if (nbatch > (1ull << 32)) throw InvalidArg("fire scores: the fire schedule does not end");
    }
    prof.add_bytes(bytes);
    g.fires = fires;
    g.burns = burns;
    g.steps = steps;
  }
}

}  // namespace lmgp
