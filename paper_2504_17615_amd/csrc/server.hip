// Serving loop: continuous batching of partition requests on one GPU.
//
// Requests enter a FIFO queue.  Worker threads (one device stream each) admit
// requests from the head of the queue while a slot is free and the summed
// footprint estimate of resident requests stays within the HBM budget, up to
// max_batch per run and 2^21 directed entries per run (a larger request runs
// alone), and partition the admitted set as one batched run (all graphs of
// the run share every kernel launch).  A run holds requests with identical
// parameters only (it stops at the first request whose parameters differ).
// Requests arriving while runs are on the device are admitted by the next
// free worker as soon as slots and memory free up, so their work overlaps
// with the runs in flight.  With join_runs set, a request that finds every
// worker busy joins a run that is still coarsening, at the next level
// boundary: its input graph is appended to the union level about to be
// clustered and from then on shares every launch (the run's kernels advance
// all its graphs one level step at a time).  A batched run that runs out of
// memory gives its worker's cached blocks back and runs its requests one at a
// time.  Every result is identical to a plain lmgp_partition call (per-graph
// rules only).
#include <cstring>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "engine.h"


namespace lmgp {

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  lmgp_graph* graph = nullptr;
  uint32_t k = 0;
  double eps = 0;
  uint64_t seed = 0;
  uint32_t* out = nullptr;
  lmgp_params params{};
  uint64_t footprint = 0;
  clk::time_point t_submit;
  bool done = false;
  lmgp_status status = LMGP_OK;
  std::string error;
  lmgp_result res{};
};

}  // namespace

// Conservative device footprint of one request: hierarchy levels (each at most
// the input size), per-level scratch, and the batch union copy.
uint64_t request_footprint(uint64_t n, uint64_t nnz) {
  return 4096 + n * 160 + nnz * 64;
}

// Directed entries above which a run takes no further request.
constexpr uint64_t RUN_ENTRIES = 1ull << 21;

}  // namespace lmgp

struct lmgp_server {
  lmgp_server_cfg cfg{};
  bool have_alloc = false;
  lmgp_allocator alloc{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<lmgp::Request*> queue;
  std::map<uint64_t, std::unique_ptr<lmgp::Request>> all;
  uint64_t next_ticket = 1;
  uint64_t resident_bytes = 0;
  uint32_t resident = 0;
  uint32_t idle = 0;  // workers waiting for work
  lmgp_server_stats stats{};
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace lmgp {

namespace {

void worker_main(lmgp_server* sv) {
  (void)hipSetDevice(sv->device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
  Pool pool(sv->have_alloc ? &sv->alloc : nullptr);
  while (true) {
    std::vector<Request*> batch;
    uint64_t bytes = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->idle++;
      sv->cv_work.wait(lk, [&] {
        if (sv->stop) return true;
        if (sv->queue.empty()) return false;
        Request* r = sv->queue.front();
        return sv->resident < sv->cfg.max_slots &&
               sv->resident_bytes + r->footprint <= sv->cfg.hbm_budget_bytes;
      });
      sv->idle--;
      if (sv->stop) break;
      uint64_t entries = 0;
      while (!sv->queue.empty() && batch.size() < sv->cfg.max_batch) {
        Request* r = sv->queue.front();
        if (sv->resident >= sv->cfg.max_slots ||
            sv->resident_bytes + r->footprint > sv->cfg.hbm_budget_bytes)
          break;
        // a run ends where the next request would take it past RUN_ENTRIES
        // (a large request runs alone): every graph of a run waits for the
        // run's last one, so a small request should not wait for a large one
        const uint64_t e = r->graph->g.nnz;
        if (!batch.empty() && entries + e > RUN_ENTRIES) break;
        if (!batch.empty() &&
            std::memcmp(&r->params, &batch[0]->params, sizeof(lmgp_params)) != 0)
          break;
        entries += e;
        sv->queue.pop_front();
        sv->resident++;
        sv->resident_bytes += r->footprint;
        bytes += r->footprint;
        batch.push_back(r);
      }
      sv->stats.runs++;
      sv->stats.max_run_requests = std::max<uint64_t>(sv->stats.max_run_requests, batch.size());
      sv->stats.peak_resident_estimate =
          std::max<uint64_t>(sv->stats.peak_resident_estimate, sv->resident_bytes);
    }
    lmgp_params p = batch[0]->params;
    p.ip_device = sv->cfg.ip_device <= LMGP_IP_AUTO ? sv->cfg.ip_device : LMGP_IP_AUTO;
    auto make_job = [&](Request* r) {
      Job j;
      j.g = &r->graph->g;
      j.k = r->k;
      j.eps = r->eps;
      j.seed = r->seed;
      const int64_t cV = r->graph->g.cV;
      int64_t U = (int64_t)((unsigned __int128)cV / ((unsigned __int128)p.clim * r->k));
      j.U = U < 1 ? 1 : U;
      const int64_t avg = (cV + (int64_t)r->k - 1) / (int64_t)r->k;
      j.lmax = (int64_t)std::floor((1.0 + r->eps) * (double)avg);
      return j;
    };
    // one batched run of `reqs` (requests that join it in flight are appended
    // when `join`); per request: its status, message and result
    auto run = [&](std::vector<Request*>& reqs, bool join, std::vector<lmgp_status>& st,
                   std::vector<std::string>& err, std::vector<lmgp_result>& res) {
      try {
        std::vector<Job> jobs;
        for (Request* r : reqs) jobs.push_back(make_job(r));
        Engine e(pool, s, p);
        if (join)
          e.admit = [&]() {
            // requests that find every worker busy, with the run's
            // parameters, while slots and memory allow
            std::vector<Job> more;
            std::lock_guard<std::mutex> lk(sv->mu);
            while (!sv->queue.empty() && sv->idle == 0 && reqs.size() < sv->cfg.max_slots) {
              Request* r = sv->queue.front();
              if (sv->resident >= sv->cfg.max_slots ||
                  sv->resident_bytes + r->footprint > sv->cfg.hbm_budget_bytes ||
                  std::memcmp(&r->params, &batch[0]->params, sizeof(lmgp_params)) != 0 ||
                  !e.can_join(r->graph->g))
                break;
              sv->queue.pop_front();
              sv->resident++;
              sv->resident_bytes += r->footprint;
              bytes += r->footprint;
              sv->stats.joined++;
              reqs.push_back(r);
              more.push_back(make_job(r));
            }
            return more;
          };
        e.coarsen(jobs);
        std::vector<uint32_t*> outs;
        for (Request* r : reqs) outs.push_back(r->out);
        e.partition(jobs, outs.data(), false);
        st.assign(reqs.size(), LMGP_OK);
        err.assign(reqs.size(), "");
        res.assign(reqs.size(), lmgp_result{});
        for (size_t i = 0; i < reqs.size(); ++i) res[i] = jobs[i].res;
      } catch (const OutOfMemory& ex) {
        st.assign(reqs.size(), LMGP_ENOMEM);
        err.assign(reqs.size(), ex.what());
        res.assign(reqs.size(), lmgp_result{});
      } catch (const std::exception& ex) {
        st.assign(reqs.size(), LMGP_EDEVICE);
        err.assign(reqs.size(), ex.what());
        res.assign(reqs.size(), lmgp_result{});
      }
    };
    pool.reset_peak();
    std::vector<lmgp_status> st;
    std::vector<std::string> err;
    std::vector<lmgp_result> res;
    run(batch, sv->cfg.join_runs != 0, st, err, res);
    uint64_t retried = 0;
    if (batch.size() > 1 && st[0] == LMGP_ENOMEM) {
      // out of memory as a batch: cached blocks back to the device, then one
      // request at a time (a request fails only if it does not fit alone)
      (void)hipStreamSynchronize(s);
      pool.trim();
      for (size_t i = 0; i < batch.size(); ++i) {
        std::vector<lmgp_status> st1;
        std::vector<std::string> err1;
        std::vector<lmgp_result> res1;
        std::vector<Request*> one{batch[i]};
        run(one, false, st1, err1, res1);
        st[i] = st1[0], err[i] = err1[0], res[i] = res1[0];
        ++retried;
      }
    }
    const auto now = clk::now();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (size_t i = 0; i < batch.size(); ++i) {
        Request* r = batch[i];
        r->status = st[i];
        r->error = err[i];
        if (st[i] == LMGP_OK) r->res = res[i];
        r->res.t_total_ns =
            std::chrono::duration_cast<std::chrono::nanoseconds>(now - r->t_submit).count();
        r->done = true;
        sv->stats.completed++;
        if (st[i] != LMGP_OK) sv->stats.failed++;
      }
      sv->stats.retried_alone += retried;
      sv->stats.peak_pool_bytes =
          std::max<uint64_t>(sv->stats.peak_pool_bytes, pool.peak_in_use());
      sv->resident -= (uint32_t)batch.size();
      sv->resident_bytes -= bytes;
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
  (void)hipStreamSynchronize(s);
  pool.release();
  (void)hipStreamDestroy(s);
}

thread_local std::string s_err;

}  // namespace

}  // namespace lmgp

using namespace lmgp;

extern "C" {

const char* lmgp_last_error(void);

lmgp_status lmgp_server_create(const lmgp_server_cfg* cfg, const lmgp_allocator* alloc,
                               lmgp_server** out) {
  if (!cfg || !out) return LMGP_EINVAL;
  if (!cfg->max_slots || !cfg->max_batch || !cfg->streams || !cfg->hbm_budget_bytes)
    return LMGP_EINVAL;
  try {
    auto sv = std::make_unique<lmgp_server>();
    sv->cfg = *cfg;
    if (alloc) sv->alloc = *alloc, sv->have_alloc = true;
    if (hipGetDevice(&sv->device) != hipSuccess) return LMGP_EDEVICE;
    for (uint32_t i = 0; i < cfg->streams; ++i) sv->workers.emplace_back(worker_main, sv.get());
    *out = sv.release();
    return LMGP_OK;
  } catch (...) {
    return LMGP_ENOMEM;
  }
}

lmgp_status lmgp_server_submit(lmgp_server* sv, lmgp_graph* g, uint32_t k, double eps,
                               uint64_t seed, uint32_t* block_out, uint64_t* ticket) {
  return lmgp_server_submit_params(sv, g, k, eps, seed, nullptr, block_out, ticket);
}

lmgp_status lmgp_server_submit_params(lmgp_server* sv, lmgp_graph* g, uint32_t k, double eps,
                                      uint64_t seed, const lmgp_params* params,
                                      uint32_t* block_out, uint64_t* ticket) {
  if (!sv || !g || !block_out || !ticket) return LMGP_EINVAL;
  if (k == 0 || (uint64_t)k > g->g.n || !(eps > 0.0)) return LMGP_EINVAL;
  lmgp_params prm = params ? *params : default_params();
  try {
    check_params(prm);
  } catch (const std::exception&) {
    return LMGP_EINVAL;
  }
  prm.ip_device = 0;  // the server's configuration decides (no effect on results)
  auto r = std::make_unique<Request>();
  r->params = prm;
  r->graph = g;
  r->k = k;
  r->eps = eps;
  r->seed = seed;
  r->out = block_out;
  r->footprint = request_footprint(g->g.n, g->g.nnz);
  if (r->footprint > sv->cfg.hbm_budget_bytes) return LMGP_EBUSY;
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return LMGP_ECANCELLED;
    r->ticket = sv->next_ticket++;
    *ticket = r->ticket;
    sv->queue.push_back(r.get());
    sv->all[r->ticket] = std::move(r);
  }
  sv->cv_work.notify_one();
  return LMGP_OK;
}

static lmgp_status finish(lmgp_server* sv, uint64_t ticket, lmgp_result* res, bool block) {
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return LMGP_EINVAL;
  Request* r = it->second.get();
  if (block) sv->cv_done.wait(lk, [&] { return r->done || sv->stop; });
  if (!r->done) return sv->stop ? LMGP_ECANCELLED : LMGP_ENOTREADY;
  const lmgp_status st = r->status;
  if (res) *res = r->res;
  sv->all.erase(it);
  return st;
}

lmgp_status lmgp_server_poll(lmgp_server* sv, uint64_t ticket, lmgp_result* res) {
  if (!sv) return LMGP_EINVAL;
  return finish(sv, ticket, res, false);
}

lmgp_status lmgp_server_wait(lmgp_server* sv, uint64_t ticket, lmgp_result* res) {
  if (!sv) return LMGP_EINVAL;
  return finish(sv, ticket, res, true);
}

lmgp_status lmgp_server_stats_read(lmgp_server* sv, lmgp_server_stats* out) {
  if (!sv || !out) return LMGP_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  return LMGP_OK;
}

void lmgp_server_destroy(lmgp_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  for (auto& t : sv->workers) t.join();
  delete sv;
}

}  // extern "C"
