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
// next frontier.  Fires are started while the burns so far are at most
// nu |E|.  Every draw and break is a counter hash, so the scores do not
// depend on scheduling.
//
// One step of a fire is four launches: the draws (a wavefront per frontier
// node, the rows of up to 256 entries held in registers across its draws),
// the claim minimum per drawn node (64-bit atomicMin on the packed claim
// word), the winners (scores, visited stamps, next frontier), and a one-thread
// control kernel that advances the frontier and starts the next fire on the
// device.  The host reads the control word once per batch of steps.  Rows
// must be sorted: draws scan them in ascending neighbour order and a burn
// finds the reverse entry by binary search.
#include "contract.h"
#include "primitives.h"
#include "profiler.h"

namespace lmgp {

namespace {

struct FireCtl {
  uint32_t cur;   // frontier buffer being drawn from
  uint32_t done;  // no further fire is scheduled
  uint64_t f;     // current fire
  uint64_t l;     // current frontier of the fire
  uint64_t nfront, nnext, nclaims;
  uint64_t burns, fires, steps;
  uint64_t scanned, claims_total;  // entries read by the draws, claims made
};

struct FireArgs {
  const uint64_t* xadj;
  const uint32_t* adj;
  const void* ew;
  const uint32_t* src;
  uint64_t nb;  // first node of the graph (hashes and frontiers use local ids)
  uint64_t n;   // nodes of the graph
  uint64_t m;   // undirected edges of the graph
  uint32_t* visited;         // fire stamp (f + 1) of each node's last visit
  uint32_t* taken;           // drawn entries of long rows, cleared by the winners
  uint64_t* claims;          // entries drawn in this step
  unsigned long long* cw;    // smallest claim word per node (all ones when none)
  uint32_t* front0;
  uint32_t* front1;
  uint32_t* score;           // burns of each entry's edge
  FireCtl* ctl;
  uint64_t pre_start, pre_draw, pre_break, pre_claim;
  uint64_t pthr;             // break iff H < pthr, or always
  uint32_t always;
  uint32_t nu_num, nu_den;
};

constexpr int FF_NT = 256;
constexpr int FF_WAVES = FF_NT / WAVE;
constexpr int FF_CACHE = 4;  // rows of up to 4 x 64 entries stay in registers

LMGP_D uint32_t* front_of(const FireArgs& a, uint32_t i) { return i ? a.front1 : a.front0; }

// floor(H * W / 2^64): a draw position in [0, W)
LMGP_D uint64_t scaled(uint64_t h, uint64_t w) { return __umul64hi(h, w); }

// a * b <= c * d for 64-bit operands (128-bit products)
LMGP_HD bool mul_le(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  const unsigned __int128 x = (unsigned __int128)a * b, y = (unsigned __int128)c * d;
  return x <= y;
}

__global__ void k_ff_init(FireArgs a) {
  FireCtl c{};
  c.done = a.m == 0 ? 1u : 0u;
  c.nfront = c.done ? 0 : 1;
  if (!c.done) a.front0[0] = (uint32_t)scaled(hash_add(a.pre_start, 0), a.n);
  *a.ctl = c;
}

// Stages a wave's claims in registers (lane i holds the i-th) and writes them
// out 64 at a time with one reservation.
struct ClaimStage {
  uint64_t mine = 0;
  int cnt = 0;
  LMGP_D void push(const FireArgs& a, uint64_t e) {
    if (lane_id() == cnt) mine = e;
    if (++cnt == WAVE) flush(a);
  }
  LMGP_D void flush(const FireArgs& a) {
    if (!cnt) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd((unsigned long long*)&a.ctl->nclaims, (unsigned long long)cnt);
    base = __shfl(base, 0);
    if (lane_id() < cnt) a.claims[base + lane_id()] = mine;
    cnt = 0;
  }
};

LMGP_D bool taken_at(const FireArgs& a, uint64_t e) {
  return __hip_atomic_load(&a.taken[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

template <int EWK>
LMGP_D int64_t fire_w(const FireArgs& a, uint64_t e) {
  return edge_w<EWK>(a.ew, e);
}

// The draws of the frontier: one wavefront per node, grid-strided.
template <int EWK>
__global__ __launch_bounds__(FF_NT) void k_ff_draw(FireArgs a) {
  const FireCtl* cp = a.ctl;
  if (cp->done) return;
  const uint64_t nfront = cp->nfront, f = cp->f, l = cp->l;
  const uint32_t stamp = (uint32_t)(f + 1);
  const uint32_t* front = front_of(a, cp->cur);
  const uint64_t hd = hash_add(hash_add(a.pre_draw, f), l);
  const uint64_t hb = hash_add(hash_add(a.pre_break, f), l);
  const int lane = lane_id();
  const uint64_t nw = (uint64_t)gridDim.x * FF_WAVES;
  ClaimStage st;
  uint64_t scanned = 0;  // entries read (lane 0's count)
  for (uint64_t i = (uint64_t)blockIdx.x * FF_WAVES + threadIdx.x / WAVE; i < nfront; i += nw) {
    const uint32_t ul = front[i];
    const uint64_t u = a.nb + ul;
    if (lane == 0) a.cw[u] = ~0ull;  // cleared for this step's claims
    const uint64_t beg = a.xadj[u], deg = a.xadj[u + 1] - beg;
    const uint64_t hdu = hash_add(hd, ul), hbu = hash_add(hb, ul);
    if (deg <= (uint64_t)FF_CACHE * WAVE) {
      scanned += deg;
      // candidate weights in registers; a drawn entry's weight drops to 0
      int64_t wv[FF_CACHE];
#pragma unroll
      for (int c = 0; c < FF_CACHE; ++c) {
        const uint64_t k = (uint64_t)c * WAVE + lane;
        wv[c] = 0;
        if (k < deg && a.visited[a.adj[beg + k]] != stamp) wv[c] = fire_w<EWK>(a, beg + k);
      }
      // each draw removes a candidate, so at most deg draws
      for (uint64_t j = 0; j < deg; ++j) {
        int64_t t = 0;
#pragma unroll
        for (int c = 0; c < FF_CACHE; ++c) t += wv[c];
        const uint64_t W = (uint64_t)wave_reduce_sum(t);
        if (W == 0) break;
        const uint64_t R = scaled(hash_add(hdu, j), W);
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
        st.push(a, beg + (uint64_t)pick);
        if (a.always || hash_add(hbu, j) < a.pthr) break;
      }
    } else {
      // long row: two passes per draw, drawn entries flagged in `taken`
      // (read and written at device scope, so that this wave's next pass
      // sees its own flags whatever the L1 holds)
      for (uint64_t j = 0; j < deg; ++j) {
        int64_t t = 0;
        scanned += deg;
        for (uint64_t k = lane; k < deg; k += WAVE) {
          const uint64_t e = beg + k;
          if (!taken_at(a, e) && a.visited[a.adj[e]] != stamp) t += fire_w<EWK>(a, e);
        }
        const uint64_t W = (uint64_t)wave_reduce_sum(t);
        if (W == 0) break;
        const uint64_t R = scaled(hash_add(hdu, j), W);
        uint64_t run = 0, pick = ~0ull;
        for (uint64_t k0 = 0; k0 < deg; k0 += WAVE) {
          const uint64_t k = k0 + lane, e = beg + k;
          int64_t w = 0;
          if (k < deg && !taken_at(a, e) && a.visited[a.adj[e]] != stamp) w = fire_w<EWK>(a, e);
          scanned += WAVE;
          const int64_t inc = wave_inclusive_scan(w);
          const uint64_t mask = __ballot(run + (uint64_t)inc > R);
          if (mask) {
            pick = k0 + (uint64_t)__builtin_ctzll(mask);
            break;
          }
          run += (uint64_t)__shfl(inc, WAVE - 1);
        }
        if (pick == ~0ull) break;  // unreachable: R < W
        if (lane == 0)
          __hip_atomic_store(&a.taken[beg + pick], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();  // performed before the next pass reads
        st.push(a, beg + pick);
        if (a.always || hash_add(hbu, j) < a.pthr) break;
      }
    }
  }
  st.flush(a);
  if (lane_id() == 0 && scanned)
    atomicAdd((unsigned long long*)&a.ctl->scanned, (unsigned long long)scanned);
}

LMGP_D unsigned long long claim_word(const FireArgs& a, uint64_t hc, uint64_t e, uint32_t& ul,
                                     uint32_t& v) {
  v = a.adj[e];
  ul = (uint32_t)(a.src[e] - a.nb);
  const uint64_t key = hash_add(hash_add(hc, (uint64_t)v - a.nb), ul) >> 32;
  return (key << 32) | ul;
}

__global__ __launch_bounds__(256) void k_ff_min(FireArgs a) {
  const FireCtl* cp = a.ctl;
  if (cp->done) return;
  const uint64_t nc = cp->nclaims;
  const uint64_t hc = hash_add(hash_add(a.pre_claim, cp->f), cp->l);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
    uint32_t ul, v;
    const unsigned long long w = claim_word(a, hc, a.claims[i], ul, v);
    atomicMin(&a.cw[v], w);
  }
}

__global__ __launch_bounds__(256) void k_ff_win(FireArgs a) {
  const FireCtl* cp = a.ctl;
  if (cp->done) return;
  const uint64_t nc = cp->nclaims;
  const uint64_t hc = hash_add(hash_add(a.pre_claim, cp->f), cp->l);
  const uint32_t stamp = (uint32_t)(cp->f + 1);
  uint32_t* next = front_of(a, cp->cur ^ 1u);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // whole waves run every iteration (the frontier append is wave-aggregated)
  const uint64_t span = (nc + WAVE - 1) / WAVE * WAVE;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += stride) {
    bool win = false;
    uint32_t v = 0;
    if (i < nc) {
      const uint64_t e = a.claims[i];
      uint32_t ul;
      const unsigned long long w = claim_word(a, hc, e, ul, v);
      a.taken[e] = 0;
      if (a.cw[v] == w) {
        win = true;
        a.visited[v] = stamp;
        atomicAdd(&a.score[e], 1u);
        // the reverse entry: u in v's sorted row
        const uint32_t u = a.src[e];
        uint64_t lo = a.xadj[v], hi = a.xadj[v + 1];
        while (lo < hi) {
          const uint64_t mid = (lo + hi) / 2;
          if (a.adj[mid] < u) lo = mid + 1;
          else hi = mid;
        }
        if (lo < a.xadj[v + 1] && a.adj[lo] == u) atomicAdd(&a.score[lo], 1u);
      }
    }
    const uint64_t mask = __ballot(win);
    if (mask) {
      unsigned long long base = 0;
      const int leader = __builtin_ctzll(mask);
      if (lane_id() == leader)
        base = atomicAdd((unsigned long long*)&a.ctl->nnext, (unsigned long long)__popcll(mask));
      base = __shfl(base, leader);
      if (win) next[base + __popcll(mask & lanemask_lt())] = (uint32_t)(v - a.nb);
    }
  }
}

__global__ void k_ff_control(FireArgs a) {
  FireCtl c = *a.ctl;
  if (c.done) return;
  c.burns += c.nnext;
  c.claims_total += c.nclaims;
  c.nfront = c.nnext;
  c.nnext = 0;
  c.nclaims = 0;
  c.cur ^= 1u;
  c.l += 1;
  c.steps += 1;
  if (c.nfront == 0) {  // fire f is out
    c.fires = c.f + 1;
    if (mul_le(c.burns, a.nu_den, a.nu_num, a.m)) {
      c.f += 1;
      c.l = 0;
      front_of(a, c.cur)[0] = (uint32_t)scaled(hash_add(a.pre_start, c.f), a.n);
      c.nfront = 1;
    } else {
      c.done = 1;
    }
  }
  *a.ctl = c;
}

constexpr int FF_BATCH = 16;  // steps enqueued between reads of the control word

}  // namespace

void fire_scores(const FireLevel& lv, std::vector<FireGraph>& graphs, uint32_t* score, Pool& pool,
                 hipStream_t s) {
  if (lv.ew_kind != EW_UNIT && lv.ew_kind != EW_I32 && lv.ew_kind != EW_I64)
    throw InvalidArg("fire scores: unknown edge weight kind");
  if (lv.p_den == 0 || lv.nu_den == 0) throw InvalidArg("fire scores: zero denominator");
  uint64_t maxn = 0, maxe = 0;
  for (const FireGraph& g : graphs) {
    maxn = std::max(maxn, g.n);
    maxe = std::max(maxe, g.e1 - g.e0);
  }
  if (lv.n == 0 || lv.nnz == 0 || maxe == 0) {
    if (lv.nnz) device_zero(score, lv.nnz * sizeof(uint32_t), s);
    for (FireGraph& g : graphs) g.fires = g.burns = 0;
    return;
  }
  if (lv.n >= 0xFFFFFFFFull) throw InvalidArg("fire scores: too many nodes");
  DBuf<uint32_t> visited(&pool, s, lv.n), front0(&pool, s, maxn + 1), front1(&pool, s, maxn + 1);
  DBuf<uint32_t> taken(&pool, s, lv.nnz);
  DBuf<uint64_t> claims(&pool, s, maxe);
  DBuf<unsigned long long> cw(&pool, s, lv.n);
  DBuf<FireCtl> ctl(&pool, s, 1);
  visited.zero();
  taken.zero();
  device_zero(score, lv.nnz * sizeof(uint32_t), s);
  device_fill_u32((uint32_t*)cw.get(), 0xFFFFFFFFu, 2 * lv.n, s);
  const bool always = lv.p_num >= lv.p_den;
  const uint64_t pthr = always ? 0 : (uint64_t)(((unsigned __int128)lv.p_num << 64) / lv.p_den);
  for (FireGraph& g : graphs) {
    g.fires = g.burns = 0;
    if (!g.active || g.n == 0) continue;
    FireArgs a{};
    a.xadj = lv.xadj;
    a.adj = lv.adj;
    a.ew = lv.ew;
    a.src = lv.src;
    a.nb = g.node_base;
    a.n = g.n;
    a.m = (g.e1 - g.e0) / 2;
    a.visited = visited.get();
    a.taken = taken.get();
    a.claims = claims.get();
    a.cw = cw.get();
    a.front0 = front0.get();
    a.front1 = front1.get();
    a.score = score;
    a.ctl = ctl.get();
    a.pre_start = g.pre_start;
    a.pre_draw = g.pre_draw;
    a.pre_break = g.pre_break;
    a.pre_claim = g.pre_claim;
    a.pthr = pthr;
    a.always = always ? 1u : 0u;
    a.nu_num = lv.nu_num;
    a.nu_den = lv.nu_den;
    // bytes from the device's counts: per frontier node its offsets (16 B),
    // per entry read by a draw its neighbour, the neighbour's stamp and the
    // weight, per claim 8 B written and (claim, row, neighbour, claim word)
    // read by both resolve passes plus the flag clear, per burn the stamp,
    // two score updates, the frontier slot and the reverse search
    ProfScope prof("sp:fire", 0, s);
    k_ff_init<<<1, 1, 0, s>>>(a);
    LAUNCH_CHECK();
    unsigned gd = grid_for(g.n, FF_WAVES);
    if (gd > 2048) gd = 2048;
    unsigned gc = grid_for(g.e1 - g.e0, 256);
    if (gc > 2048) gc = 2048;
    const bool weighted = lv.weighted && lv.ew_kind != EW_UNIT;
    FireCtl hc{};
    for (;;) {
      for (int b = 0; b < FF_BATCH; ++b) {
        if (!weighted) k_ff_draw<EW_UNIT><<<gd, FF_NT, 0, s>>>(a);
        else if (lv.ew_kind == EW_I32) k_ff_draw<EW_I32><<<gd, FF_NT, 0, s>>>(a);
        else k_ff_draw<EW_I64><<<gd, FF_NT, 0, s>>>(a);
        LAUNCH_CHECK();
        k_ff_min<<<gc, 256, 0, s>>>(a);
        LAUNCH_CHECK();
        k_ff_win<<<gc, 256, 0, s>>>(a);
        LAUNCH_CHECK();
        k_ff_control<<<1, 1, 0, s>>>(a);
        LAUNCH_CHECK();
      }
      read_now(&hc, ctl.get(), sizeof(hc), s);
      if (hc.done) break;
      // a fire visits a new node every step (its start node at most twice)
      if (hc.steps > (hc.f + 1) * (g.n + 2) || hc.f >= 0xFFFFFFF0ull)
        throw InvalidArg("fire scores: the fire schedule does not end");
    }
    const uint64_t wb = weighted ? (lv.ew_kind == EW_I32 ? 4 : 8) : 0;
    prof.add_bytes(16 * (hc.burns + hc.fires) + (8 + wb) * hc.scanned + 60 * hc.claims_total +
                   32 * hc.burns);
    g.fires = hc.fires;
    g.burns = hc.burns;
    g.steps = hc.steps;
  }
}

}  // namespace lmgp
