#include <cstring>

#include "profiler.h"
#include "lmgp.h"

namespace lmgp {

Profiler& Profiler::get() {
  static Profiler p;
  return p;
}

hipEvent_t Profiler::take_event() {
  if (!free_.empty()) {
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}

int Profiler::begin(const char* name, uint64_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> g(mu_);
  Rec r{name, bytes, take_event(), take_event()};
  HIP_CHECK(hipEventRecord(r.a, s));
  pending_.push_back(r);
  return (int)pending_.size() - 1;
}

void Profiler::begin_ext(const char* name, uint64_t bytes, hipEvent_t* a, hipEvent_t* b) {
  std::lock_guard<std::mutex> g(mu_);
  Rec r{name, bytes, take_event(), take_event()};
  pending_.push_back(r);
  *a = r.a;
  *b = r.b;
}

void Profiler::end(int slot, hipStream_t s) {
  std::lock_guard<std::mutex> g(mu_);
  if (slot < 0 || (size_t)slot >= pending_.size()) return;
  HIP_CHECK(hipEventRecord(pending_[slot].b, s));
}

void Profiler::add_bytes(int slot, uint64_t bytes) {
  std::lock_guard<std::mutex> g(mu_);
  if (slot >= 0 && (size_t)slot < pending_.size()) pending_[slot].bytes += bytes;
}

void Profiler::count(const char* name) {
  if (!on()) return;
  std::lock_guard<std::mutex> g(mu_);
  stats_[name].launches++;
}

void Profiler::collect() {
  std::lock_guard<std::mutex> g(mu_);
  for (Rec& r : pending_) {
    HIP_CHECK(hipEventSynchronize(r.b));
    float ms = 0;
    // a launch that failed before it ran left its events unrecorded: skip it
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      KernelStat& st = stats_[r.name];
      st.launches++;
      st.total_ns += (uint64_t)((double)ms * 1e6);
      st.bytes += r.bytes;
    } else {
      (void)hipGetLastError();
    }
    free_.push_back(r.a);
    free_.push_back(r.b);
  }
  pending_.clear();
}

std::map<std::string, KernelStat> Profiler::read(bool reset) {
  collect();
  std::lock_guard<std::mutex> g(mu_);
  auto out = stats_;
  const uint64_t nl = reset ? launches_.exchange(0) : launches_.load();
  if (nl) out["host:kernel_launches"].launches = nl;
  if (reset) stats_.clear();
  return out;
}

void Profiler::reset() {
  collect();
  std::lock_guard<std::mutex> g(mu_);
  stats_.clear();
  launches_.store(0);
}

void note_launch() { Profiler::get().count_launch(); }

void Profiler::set_filter(const std::string& kernel) {
  std::lock_guard<std::mutex> g(mu_);
  filter_ = kernel;
}

bool Profiler::wants(const char* family) {
  std::lock_guard<std::mutex> g(mu_);
  if (filter_.empty()) return true;
  const char* k = std::strchr(family, ':');
  return filter_ == (k ? k + 1 : family);
}

bool& Profiler::suspended() {
  static thread_local bool v = false;
  return v;
}

ProfSuspend::ProfSuspend() { Profiler::suspended() = true; }
ProfSuspend::~ProfSuspend() { Profiler::suspended() = false; }

}  // namespace lmgp

extern "C" {

lmgp_status lmgp_profile_enable(uint32_t on) {
  lmgp::Profiler::get().enable(on != 0);
  return LMGP_OK;
}

lmgp_status lmgp_profile_filter(const char* kernel) {
  lmgp::Profiler::get().set_filter(kernel ? kernel : "");
  return LMGP_OK;
}

lmgp_status lmgp_profile_read(lmgp_kernel_stat* out, uint32_t max, uint32_t* count,
                              uint32_t reset) {
  if (!count) return LMGP_EINVAL;
  try {
    auto st = lmgp::Profiler::get().read(reset != 0);
    uint32_t i = 0;
    for (auto& kv : st) {
      if (out && i < max) {
        std::memset(out[i].name, 0, sizeof(out[i].name));
        std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
        out[i].launches = kv.second.launches;
        out[i].total_ns = kv.second.total_ns;
        out[i].bytes = kv.second.bytes;
      }
      ++i;
    }
    *count = i;
    return LMGP_OK;
  } catch (...) {
    return LMGP_EDEVICE;
  }
}

}  // extern "C"
