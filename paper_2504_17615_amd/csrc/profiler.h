// Optional per-kernel timing: launches of the main kernels are timed with
// events (recorded by the launch itself where the launch is a single kernel,
// else bracketing the launches on their stream) and charged the algorithmic
// bytes they must move.
#pragma once
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace lmgp {

struct KernelStat {
  uint64_t launches = 0;
  uint64_t total_ns = 0;
  uint64_t bytes = 0;
};

class Profiler {
 public:
  static Profiler& get();
  bool on() const { return on_.load(std::memory_order_relaxed) && !suspended(); }
  // Time only the launches of one kernel: `kernel` is the part of a family
  // name after its phase prefix ("k_rate_big<2, 13>"); empty = every launch.
  void set_filter(const std::string& kernel);
  bool wants(const char* family);
  static bool& suspended();
  void enable(bool v) { on_.store(v); }
  // Record the start of a launch; returns a slot id (or -1 when disabled).
  int begin(const char* name, uint64_t bytes, hipStream_t s);
  // For a launch that records its own start and end (hipExtLaunchKernelGGL):
  // hands out the two events to pass to it.
  void begin_ext(const char* name, uint64_t bytes, hipEvent_t* a, hipEvent_t* b);
  void end(int slot, hipStream_t s);
  // Adds bytes to a started launch record (sizes known only later).
  void add_bytes(int slot, uint64_t bytes);
  // Counts an event of the host (e.g. a stream synchronisation) under `name`:
  // launches = count, no time or bytes.
  void count(const char* name);
  // Kernel launches while recording (reported as "host:kernel_launches").
  void count_launch() {
    if (on()) launches_.fetch_add(1, std::memory_order_relaxed);
  }
  // Resolve recorded events (synchronises them) and accumulate.
  void collect();
  std::map<std::string, KernelStat> read(bool reset);
  void reset();

 private:
  struct Rec {
    std::string name;
    uint64_t bytes;
    hipEvent_t a, b;
  };
  hipEvent_t take_event();
  std::atomic<bool> on_{false};
  std::atomic<uint64_t> launches_{0};
  std::mutex mu_;
  std::vector<Rec> pending_;
  std::vector<hipEvent_t> free_;
  std::map<std::string, KernelStat> stats_;
  std::string filter_;
};

// RAII bracket of one launch.
class ProfScope {
 public:
  ProfScope(const char* name, uint64_t bytes, hipStream_t s) : s_(s) {
    Profiler& p = Profiler::get();
    slot_ = p.on() && p.wants(name) ? p.begin(name, bytes, s) : -1;
  }
  ~ProfScope() { end(); }
  void add_bytes(uint64_t b) {
    if (slot_ >= 0) Profiler::get().add_bytes(slot_, b);
  }
  // Ends the bracket before the scope does.
  void end() {
    if (slot_ >= 0) Profiler::get().end(slot_, s_);
    slot_ = -1;
  }

 private:
  hipStream_t s_;
  int slot_;
};

// Events for one hipExtLaunchKernelGGL launch, which timestamps the kernel's
// own start and end (null when profiling is off: a plain launch).
class ProfLaunch {
 public:
  ProfLaunch(const char* name, uint64_t bytes) {
    Profiler& p = Profiler::get();
    if (p.on() && p.wants(name)) p.begin_ext(name, bytes, &a_, &b_);
  }
  hipEvent_t start() const { return a_; }
  hipEvent_t stop() const { return b_; }

 private:
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// Launch that timestamps itself when given events (profiling), else a plain
// launch (the form a stream capture records).
template <typename... Args>
void launch_k(void (*kernel)(Args...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0,
              hipEvent_t e1, Args... args) {
  if (e0) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
    return;
  }
  void* ptrs[] = {(void*)&args...};
  HIP_CHECK(hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, 0, s));
}

// As launch_k, with `lds` bytes of dynamic LDS per block.
template <typename... Args>
void launch_k_lds(void (*kernel)(Args...), dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                  hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0) {
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, e0, e1, 0, args...);
    return;
  }
  void* ptrs[] = {(void*)&args...};
  HIP_CHECK(hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, lds, s));
}

// Suspends profiling on the calling thread (launches recorded into a graph
// cannot carry event timestamps).
class ProfSuspend {
 public:
  ProfSuspend();
  ~ProfSuspend();
};

}  // namespace lmgp
