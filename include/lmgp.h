/*
 * lmgp.h -- C ABI of the MI355X (gfx950) multilevel graph partitioner with
 * edge sparsification (Linear-Time Multilevel Graph Partitioning via Edge
 * Sparsification, arXiv 2504.17615).
 *
 * The library computes, on one GPU:
 *   - the coarsening hierarchy of Algorithm 1: size-constrained label
 *     propagation clustering with 2-hop clustering (Sec. 3, Sec. 4.1),
 *     contraction (Sec. 2), the edge budget m_hat and weighted threshold
 *     sampling (Sec. 4.2), termination rules (Sec. 4.3);
 *   - a k-way partition: recursive bipartitioning of the coarsest graph
 *     (Sec. 4.3) and size-constrained label propagation refinement on every
 *     level on the way back up (Sec. 2, Sec. 3);
 * every step running in the library's own HIP kernels.
 *
 * Graphs (Sec. 2): undirected, node weights c > 0, edge weights omega > 0,
 * stored as a canonical symmetric CSR: xadj[n+1] (uint64, xadj[0] = 0,
 * non-decreasing), adjncy[nnz] (uint32 node ids < n), every undirected edge
 * {u,v} present as both entries (u,v) and (v,u) with equal weight, rows sorted
 * strictly ascending (no duplicates), no self-loops.  nnz = 2|E|.
 * Limits: n < 2^31, nnz < 2^40.
 *
 * Conventions for every call:
 *   - returns an lmgp_status; output parameters are written only on LMGP_OK;
 *   - no C++ exception crosses the ABI; lmgp_last_error() returns a message for
 *     the calling thread's most recent failure (valid until its next call);
 *   - `stream` is a hipStream_t (NULL = the default stream); all device work is
 *     ordered on it; calls return after the result is complete unless stated;
 *   - results are a pure function of (graph, k, eps, seed, params): bit-exact
 *     across runs, batch compositions and the serving loop.
 */
#ifndef LMGP_H
#define LMGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LMGP_OK = 0,
  LMGP_EINVAL = 1,      /* invalid argument or malformed graph                 */
  LMGP_ENOMEM = 2,      /* device allocation failed (or caller allocator NULL) */
  LMGP_EDEVICE = 3,     /* HIP runtime / kernel error                          */
  LMGP_ENOTREADY = 4,   /* serving: request not finished yet                   */
  LMGP_EBUSY = 5,       /* serving: request can never be admitted              */
  LMGP_ECANCELLED = 6   /* serving: server shut down before completion         */
} lmgp_status;

/* Optional device allocator.  alloc returns device memory of at least
 * `bytes` bytes usable in stream order on `stream` (NULL on failure); free
 * releases it in stream order.  When no allocator is given the library uses
 * a stream-ordered caching pool of hipMalloc'd memory, one per device, shared
 * by every graph created there without an allocator (and by the calls on
 * them); its cached blocks go back to the device when a hipMalloc fails. */
typedef struct {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*free)(void *ctx, void *ptr, void *stream);
} lmgp_allocator;

/* A CSR graph handed to lmgp_graph_create.  Pointers are host memory
 * (on_device = 0) or device memory (on_device = 1).  vwgt / adjwgt may be
 * NULL for unit weights; otherwise their element width is given by
 * vwgt_bits / adjwgt_bits (32 or 64, signed).  validate = 1 runs the full
 * canonical-form check (sorted rows, no duplicates, symmetry with equal
 * weights) in addition to the always-on checks. */
typedef struct {
  uint64_t n;
  uint64_t nnz;
  const uint64_t *xadj;
  const uint32_t *adjncy;
  const void *vwgt;
  const void *adjwgt;
  uint32_t vwgt_bits;
  uint32_t adjwgt_bits;
  uint32_t on_device;
  uint32_t validate;
} lmgp_csr_view;

/* Parameters (defaults from lmgp_default_params).  Rational thresholds make
 * every decision exact integer arithmetic. */
typedef struct {
  uint32_t tau_e_num, tau_e_den; /* edge threshold tau_e = 1/2 (Sec. 4.2, Sec. 5.1)  */
  uint32_t tau_d_num, tau_d_den; /* density threshold tau_d = 1/2                   */
  uint32_t rho_num, rho_den;     /* minimum reduction factor rho = 4               */
  uint32_t sampler;              /* Sec. 4.2 sparsifier: 0 = weighted threshold
                                  * sampling, the edges of weight omega_t sampled to
                                  * exactly m_hat; 1 = uniform random sampling, each
                                  * edge kept with probability m_hat/|E'|; 2 = off;
                                  * 3 = weighted threshold sampling with each edge of
                                  * weight omega_t kept with probability
                                  * (m_hat - |E'^>|)/|E'^=|.  Coins are
                                  * H(seed, SPARS, level, a, b) as 64-bit fractions.
                                  * 4 / 5 = threshold sampling (as 0) on Forest Fire
                                  * / Weighted Forest Fire burn scores instead of
                                  * weights (Sec. 4.2, the appendix's WFF algorithm;
                                  * see lmgp_fire_scores); the sampled levels are
                                  * stored with sorted rows.                          */
  uint32_t clim;                 /* C = 160: U = c(V)/(C k), stop at C k nodes     */
  uint32_t shrink_num, shrink_den; /* node reduction cap 5/2 = 2.5x (Sec. 4.3)     */
  uint32_t lp_rounds;            /* LP clustering rounds, 5                        */
  uint32_t ref_rounds;           /* LP refinement rounds per level, 5              */
  uint32_t subrounds;            /* synchronous sub-rounds per LP round, 4         */
  uint32_t max_levels;           /* hierarchy depth cap, 64                        */
  uint32_t stop_num, stop_den;   /* stop when stop_den*n' > stop_num*n (19/20)     */
  uint32_t tune;                 /* degree-class cut-offs of the rating kernels (no
                                  * effect on any result, only on speed):
                                  * LMGP_TUNE_OFF (0) = fixed default table;
                                  * LMGP_TUNE_AUTO (1) = per level, the table timed
                                  * fastest for the level's (phase, degree histogram),
                                  * cached for the process (and in the file named by
                                  * LMGP_TUNE_CACHE if set); LMGP_TUNE_FORCE + p =
                                  * table p (modulo the number of tables).          */
  uint32_t graph_rounds;         /* 1 = on levels of at most 2^18 nodes (over a batch)
                                  * with no node rated through global tables, the LP
                                  * rounds after the first are captured once into a
                                  * HIP graph and replayed (grids sized from the first
                                  * round, counts planned on the device); 0 = every
                                  * round launched kernel by kernel.  No effect on any
                                  * result, only on launch overhead.                 */
  uint32_t ip_device;            /* initial partitioning (Sec. 4.3's recursive
                                  * bipartitioning, greedy growing): LMGP_IP_HOST (0)
                                  * on the host; LMGP_IP_DEVICE (1) on the device, the
                                  * subproblems of one recursion depth concurrently, one
                                  * workgroup each; LMGP_IP_AUTO (2, default) on the
                                  * device when at least 16 graphs of a batch share their
                                  * coarsest level, else on the host.  Same result
                                  * either way.                                       */
  uint32_t ff_p_num, ff_p_den;   /* samplers 4, 5: a node reached by a fire stops
                                  * drawing after each draw with probability
                                  * p = 3/5                                          */
  uint32_t ff_nu_num, ff_nu_den; /* samplers 4, 5: burn ratio nu = 1/2; fires are
                                  * started while the burns so far are <= nu |E|     */
} lmgp_params;

#define LMGP_IP_HOST 0u
#define LMGP_IP_DEVICE 1u
#define LMGP_IP_AUTO 2u

#define LMGP_TUNE_OFF 0u
#define LMGP_TUNE_AUTO 1u
#define LMGP_TUNE_FORCE 16u

typedef struct lmgp_graph lmgp_graph;
typedef struct lmgp_hierarchy lmgp_hierarchy;
typedef struct lmgp_server lmgp_server;

/* Per-level statistics; level 0 is the input graph. */
typedef struct {
  uint64_t n, m;        /* nodes and undirected edges of this level           */
  uint64_t m_prime;     /* |E'| before sparsification (= m if not triggered)  */
  uint64_t m_hat;       /* edge budget of Algorithm 1                          */
  uint32_t triggered;   /* 1 if sparsification ran                             */
  uint32_t lp_rounds;   /* LP rounds run when clustering the previous level   */
  uint32_t twohop;      /* 1 if 2-hop clustering ran on the previous level    */
  uint32_t pad;
  int64_t w_t;          /* threshold weight omega_t (0 if not triggered)      */
  uint64_t n_gt, n_eq;  /* |E'^>| and |E'^=| (undirected)                     */
  uint64_t nclusters_lp;/* clusters after LP, before 2-hop                    */
} lmgp_level_info;

typedef struct {
  int64_t cut;               /* cut(Pi) on the input graph (Sec. 2)              */
  int64_t max_block_weight;  /* max_i c(V_i)                                     */
  int64_t lmax;              /* L_max = floor((1+eps) * ceil(c(V)/k))            */
  uint32_t levels;           /* hierarchy depth l                                */
  uint32_t pad;
  int64_t t_coarsen_ns;      /* phase times measured with events on the stream  */
  int64_t t_initial_ns;
  int64_t t_refine_ns;
  int64_t t_total_ns;
} lmgp_result;

/* Serving configuration. */
typedef struct {
  uint64_t hbm_budget_bytes;  /* admission limit on the summed estimated footprint */
  uint32_t max_slots;         /* requests resident at once                          */
  uint32_t max_batch;         /* requests fused into one batched run (a run also
                                 stops before 2^21 directed entries; a request
                                 above that runs alone)                             */
  uint32_t streams;           /* concurrent device streams (worker threads)         */
  uint32_t ip_device;         /* lmgp_params.ip_device of every batched run          */
  uint32_t join_runs;         /* 1: a request that finds every stream busy joins a
                                 run still coarsening at its next level (requests
                                 with sorted rows and the run's parameters).  A
                                 run ends with its last request, so under steady
                                 arrivals joined runs grow long and every request
                                 in them waits: 0 serves a steady stream better */
} lmgp_server_cfg;

void lmgp_default_params(lmgp_params *out);

/* The autotuner's process-wide cache (see lmgp_params.tune): number of cached
 * (phase, degree histogram) entries and of timed trials so far.  Either
 * pointer may be NULL. */
lmgp_status lmgp_tuner_info(uint64_t *entries, uint64_t *trials);
/* Forgets the process-wide cache (a cache file is left unchanged). */
void lmgp_tuner_clear(void);

/* Last error message of the calling thread ("" if none). */
const char *lmgp_last_error(void);

/* Copies and validates a graph into library-owned device memory (allocated
 * with `alloc` if given).  Always checked: n, nnz, xadj monotone with
 * xadj[0] = 0 and xadj[n] = nnz, adjncy < n, no self-loops, weights > 0.
 * EINVAL on any violation. The caller keeps ownership of the view's buffers.
 * Definitions: Sec. 2 (graph, weights). */
lmgp_status lmgp_graph_create(const lmgp_csr_view *view, const lmgp_allocator *alloc,
                              void *stream, lmgp_graph **out);
void lmgp_graph_destroy(lmgp_graph *g);
/* n, nnz and the total node weight c(V) of a created graph. */
lmgp_status lmgp_graph_info(const lmgp_graph *g, uint64_t *n, uint64_t *nnz, int64_t *total_weight);

/* Builds the coarsening hierarchy of Algorithm 1 for k blocks (k >= 1,
 * k <= n) and keeps it device-resident.  params NULL = defaults. */
lmgp_status lmgp_coarsen(lmgp_graph *g, uint32_t k, uint64_t seed, const lmgp_params *params,
                         void *stream, lmgp_hierarchy **out);
lmgp_status lmgp_hierarchy_levels(const lmgp_hierarchy *h, uint32_t *num_levels);
lmgp_status lmgp_hierarchy_level_info(const lmgp_hierarchy *h, uint32_t level,
                                      lmgp_level_info *out);
/* Copies level `level` (0 = input) into host buffers sized from its info:
 * xadj[n+1], adjncy[2m], vwgt[n] (int64), adjwgt[2m] (int64), map[n] (node
 * of level+1 for each node; not written for the last level).  Any pointer may
 * be NULL to skip that array. */
lmgp_status lmgp_hierarchy_copy_level(const lmgp_hierarchy *h, uint32_t level, uint64_t *xadj,
                                      uint32_t *adjncy, int64_t *vwgt, int64_t *adjwgt,
                                      uint32_t *map);
void lmgp_hierarchy_destroy(lmgp_hierarchy *h);

/* Full partition into k blocks with imbalance eps > 0 (Sec. 2: balance
 * constraint c(V_i) <= L_max).  block_out[n] receives block ids in [0, k);
 * it is device memory if block_on_device = 1, else host memory.  res may be
 * NULL. */
lmgp_status lmgp_partition(lmgp_graph *g, uint32_t k, double eps, uint64_t seed,
                           const lmgp_params *params, void *stream, uint32_t *block_out,
                           uint32_t block_on_device, lmgp_result *res);

/* Allocation-free variant of lmgp_partition, for callers that cannot
 * allocate device memory (code that must not call hipMalloc, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, result and
 * errors as lmgp_partition, with these differences:
 *   - every device buffer the call needs comes from a fixed scratch array of
 *     LMGP_NOALLOC_SCRATCH_BYTES that the library's code object holds on each
 *     GPU it runs on (resident until the process ends); the call makes no
 *     device or page-locked host allocation and no allocator callback; its
 *     host copies go through pageable memory;
 *   - graphs above LMGP_NOALLOC_MAX_NODES nodes or LMGP_NOALLOC_MAX_ENTRIES
 *     directed entries are rejected with LMGP_EINVAL before any work; a run
 *     whose buffers still do not fit the array fails with LMGP_ENOMEM;
 *   - params.tune and params.graph_rounds are ignored (taken as 0);
 *   - all calls on one GPU share its array, which keeps the last call's
 *     contents (every buffer is initialised by the call that uses it): calls
 *     on one device from several threads are serialised by the library, and
 *     each returns only after its stream has finished with the array.
 * The graph itself (lmgp_graph_create) and block_out are the caller's. */
#define LMGP_NOALLOC_SCRATCH_BYTES (256ull << 20)
#define LMGP_NOALLOC_MAX_NODES (1ull << 19)
#define LMGP_NOALLOC_MAX_ENTRIES (1ull << 22)
lmgp_status lmgp_partition_noalloc(lmgp_graph *g, uint32_t k, double eps, uint64_t seed,
                                   const lmgp_params *params, void *stream, uint32_t *block_out,
                                   uint32_t block_on_device, lmgp_result *res);

/* (Weighted) Forest Fire burn scores (Sec. 4.2; the appendix's WFF
 * algorithm), as samplers 4 (weighted = 0) and 5 (weighted = 1) compute them
 * on a coarse level whose hash index is `level`.  Fires start at node
 * floor(H(seed, FFSTART, level, f) n / 2^64) while the burns so far are at
 * most nu |E| (nu from params, NULL = defaults).  A fire spreads one frontier
 * at a time: each frontier node u draws, without replacement, among the
 * neighbours not visited when the frontier began, its j-th draw taking the
 * first entry of its row (ascending) at which the summed weight (1 per entry
 * when weighted = 0) of the remaining candidates exceeds
 * floor(H(seed, FFDRAW, level, f, l, u, j) W / 2^64), W their total; it stops
 * after a draw iff p >= 1 or H(seed, FFBREAK, level, f, l, u, j) <
 * floor(p 2^64).  A node drawn by several frontier nodes is burned by the
 * draw with the smallest (H(seed, FFCLAIM, level, f, l, v, u) >> 32, u); it
 * is then visited and in the next frontier.  score_out[e] (nnz entries,
 * device memory if out_on_device = 1, else host) receives the burns of entry
 * e's undirected edge; stats_out (3 entries, may be NULL) receives the
 * number of fires, burns and frontier steps.  The graph's rows must be
 * sorted (LMGP_EINVAL otherwise). */
lmgp_status lmgp_fire_scores(const lmgp_graph *g, uint64_t seed, uint64_t level, uint32_t weighted,
                             const lmgp_params *params, void *stream, uint32_t *score_out,
                             uint32_t out_on_device, uint64_t *stats_out);

/* Partitions `count` graphs as one batched run: every kernel launch covers
 * all graphs of the batch.  Outputs are identical to `count` separate
 * lmgp_partition calls.  k, eps, seed, block_out and res are arrays of
 * `count` entries (res may be NULL). */
lmgp_status lmgp_partition_batch(lmgp_graph *const *graphs, const uint32_t *k, const double *eps,
                                 const uint64_t *seed, uint32_t count, const lmgp_params *params,
                                 void *stream, uint32_t *const *block_out,
                                 uint32_t block_on_device, lmgp_result *res);

/* Serving loop: requests are admitted while their estimated device footprint
 * fits hbm_budget_bytes and a slot is free; admitted requests that wait
 * together are fused into batched runs on `streams` device streams. */
lmgp_status lmgp_server_create(const lmgp_server_cfg *cfg, const lmgp_allocator *alloc,
                               lmgp_server **out);
/* Submits a request; the graph must stay alive until the request finishes.
 * block_out is host memory of n entries.  EBUSY if the request's footprint
 * exceeds the whole budget. */
lmgp_status lmgp_server_submit(lmgp_server *s, lmgp_graph *g, uint32_t k, double eps,
                               uint64_t seed, uint32_t *block_out, uint64_t *ticket);
/* As lmgp_server_submit, with the request's own parameters (NULL =
 * defaults; params.ip_device is taken from the server configuration).  Only
 * requests with identical parameters share a batched run.  EINVAL for
 * invalid parameters. */
lmgp_status lmgp_server_submit_params(lmgp_server *s, lmgp_graph *g, uint32_t k, double eps,
                                      uint64_t seed, const lmgp_params *params,
                                      uint32_t *block_out, uint64_t *ticket);
/* ENOTREADY until the request is done; then fills res (latency fields:
 * t_total_ns = submit-to-completion). */
lmgp_status lmgp_server_poll(lmgp_server *s, uint64_t ticket, lmgp_result *res);
lmgp_status lmgp_server_wait(lmgp_server *s, uint64_t ticket, lmgp_result *res);
/* Counters of a server since its creation.  peak_pool_bytes is the largest
 * device memory in use by one worker's run (library pool; 0 with a caller
 * allocator), beside the largest summed footprint estimate of the resident
 * requests that admission used. */
typedef struct {
  uint64_t completed;              /* requests finished (including failed)        */
  uint64_t failed;                 /* requests finished with an error             */
  uint64_t runs;                   /* batched runs started                        */
  uint64_t max_run_requests;       /* largest number of requests in one run       */
  uint64_t retried_alone;          /* requests re-run alone after a run's ENOMEM  */
  uint64_t joined;                 /* requests that joined a run in flight        */
  uint64_t peak_resident_estimate; /* bytes, admission's summed estimate          */
  uint64_t peak_pool_bytes;        /* bytes, measured peak in use of one worker   */
} lmgp_server_stats;
lmgp_status lmgp_server_stats_read(lmgp_server *s, lmgp_server_stats *out);
void lmgp_server_destroy(lmgp_server *s);

/* Measurement support.  When enabled (process-wide), launches of the main
 * kernels are bracketed by events on their stream; each kernel family
 * accumulates its launch count, summed event time and the algorithmic bytes
 * the launches must move (input reads and output writes counted once).
 * Enabling adds two event records per launch. */
typedef struct {
  char name[48];
  uint64_t launches;
  uint64_t total_ns;
  uint64_t bytes;
} lmgp_kernel_stat;

lmgp_status lmgp_profile_enable(uint32_t on);
/* Times only the launches of one kernel (the part of a family name after its
 * phase prefix, e.g. "k_rate_big<2, 13>"); NULL or "" times every profiled
 * launch.  Event timing adds work to each launch it covers, so timing one
 * kernel keeps the rest of a timed run undisturbed. */
lmgp_status lmgp_profile_filter(const char *kernel);
/* Writes up to `max` entries to `out` (may be NULL), the number of families
 * to *count; reset = 1 clears the accumulated statistics afterwards. */
lmgp_status lmgp_profile_read(lmgp_kernel_stat *out, uint32_t max, uint32_t *count,
                              uint32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* LMGP_H */
