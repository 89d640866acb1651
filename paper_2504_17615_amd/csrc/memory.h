// Device memory for the library: either the caller's allocator (e.g. the
// PyTorch caching allocator, passed through the C ABI) or a stream-ordered
// caching pool of hipMalloc'd blocks.
#pragma once
#include <algorithm>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "common.h"
#include "lmgp.h"

namespace lmgp {

// Zero device memory with a kernel on stream s (graph-capture safe).
void device_zero(void* p, size_t bytes, hipStream_t s);

// True while the calling thread runs an allocation-free call: host copies
// then go through pageable memory (no page-locked buffers are allocated).
bool& no_alloc_mode();

struct NoAllocScope {
  bool prev;
  NoAllocScope() : prev(no_alloc_mode()) { no_alloc_mode() = true; }
  ~NoAllocScope() { no_alloc_mode() = prev; }
};

class Pool {
 public:
  explicit Pool(const lmgp_allocator* user) {
    if (user) user_ = *user, have_user_ = true;
  }
  // Arena over caller-provided device memory [base, base + bytes): first-fit
  // ranges of 256-byte granules, nothing is ever allocated or freed on the
  // device.  A range freed by the host is handed out again only to later
  // allocations; all work of one arena is ordered on one stream, so reuse
  // follows the stream order.
  Pool(void* base, size_t bytes) : arena_base_((char*)base), arena_bytes_(bytes & ~(size_t)255) {
    if (arena_bytes_) arena_free_[0] = arena_bytes_;
  }
  ~Pool() { release(); }
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;

  // Highest arena offset handed out so far (arena mode).
  size_t arena_high_water() const { return arena_high_; }

  // Bytes handed out and not yet freed (caching-pool mode), and their peak
  // since the last reset_peak().
  size_t in_use() const { return in_use_; }
  size_t peak_in_use() const { return peak_; }
  void reset_peak() {
    std::lock_guard<std::mutex> g(mu_);
    peak_ = in_use_;
  }

  void* alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 1;
    if (arena_base_) return arena_alloc(bytes);
    if (have_user_) {
      void* p = user_.alloc(user_.ctx, bytes, (void*)s);
      if (!p) throw OutOfMemory("caller allocator returned NULL for " + std::to_string(bytes) + " bytes");
      return p;
    }
    size_t sz = round_up(bytes);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto& fl = free_[Key{s, sz}];
      if (!fl.empty()) {
        void* p = fl.back();
        fl.pop_back();
        sizes_[p] = sz;
        note_alloc(sz);
        return p;
      }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, sz);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw OutOfMemory("hipMalloc failed for " + std::to_string(sz) + " bytes: " +
                          hipGetErrorString(e));
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    sizes_[p] = sz;
    owned_.push_back(p);
    note_alloc(sz);
    return p;
  }

  void free(void* p, hipStream_t s) {
    if (!p) return;
    if (arena_base_) {
      arena_release(p);
      return;
    }
    if (have_user_) {
      user_.free(user_.ctx, p, (void*)s);
      return;
    }
    std::lock_guard<std::mutex> g(mu_);
    auto it = sizes_.find(p);
    if (it == sizes_.end()) return;
    free_[Key{s, it->second}].push_back(p);
    in_use_ -= it->second;
    sizes_.erase(it);
  }

  // Return cached blocks to the device (blocks in use stay allocated).
  void trim() {
    std::lock_guard<std::mutex> g(mu_);
    std::vector<void*> keep;
    for (auto& kv : free_)
      for (void* p : kv.second) {
        (void)hipFree(p);
        for (auto& q : owned_)
          if (q == p) q = nullptr;
      }
    free_.clear();
    for (void* q : owned_)
      if (q) keep.push_back(q);
    owned_.swap(keep);
  }

  void release() {
    if (have_user_ || arena_base_) return;
    std::lock_guard<std::mutex> g(mu_);
    for (void* p : owned_)
      if (p) (void)hipFree(p);
    owned_.clear();
    free_.clear();
    sizes_.clear();
  }

 private:
  void note_alloc(size_t sz) {  // mu_ held
    in_use_ += sz;
    if (in_use_ > peak_) peak_ = in_use_;
  }
  void* arena_alloc(size_t bytes) {
    const size_t sz = (bytes + 255) & ~(size_t)255;
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = arena_free_.begin(); it != arena_free_.end(); ++it) {
      if (it->second < sz) continue;
      const size_t off = it->first, len = it->second;
      arena_free_.erase(it);
      if (len > sz) arena_free_[off + sz] = len - sz;
      arena_used_[off] = sz;
      arena_high_ = std::max(arena_high_, off + sz);
      return arena_base_ + off;
    }
    throw OutOfMemory("scratch arena of " + std::to_string(arena_bytes_) +
                      " bytes exhausted (a request of " + std::to_string(sz) + " bytes)");
  }
  void arena_release(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    auto u = arena_used_.find((size_t)((char*)p - arena_base_));
    if (u == arena_used_.end()) return;
    size_t off = u->first, len = u->second;
    arena_used_.erase(u);
    auto next = arena_free_.lower_bound(off);
    if (next != arena_free_.end() && next->first == off + len) {
      len += next->second;
      next = arena_free_.erase(next);
    }
    if (next != arena_free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    arena_free_[off] = len;
  }

  size_t in_use_ = 0, peak_ = 0;
  char* arena_base_ = nullptr;
  size_t arena_bytes_ = 0, arena_high_ = 0;
  std::map<size_t, size_t> arena_free_, arena_used_;  // offset -> length
  struct Key {
    hipStream_t s;
    size_t sz;
    bool operator<(const Key& o) const { return s != o.s ? s < o.s : sz < o.sz; }
  };
  // Size classes of the free lists: powers of two up to 1 MiB, then
  // sixteenths of the next power of two (at most 1/8 more than asked for a
  // large array, rather than up to twice as much).
  static size_t round_up(size_t b) {
    size_t r = 512;
    while (r < b) r <<= 1;
    if (r <= (1u << 20)) return r;
    const size_t step = r >> 4;
    return (b + step - 1) / step * step;
  }
  bool have_user_ = false;
  lmgp_allocator user_{};
  std::mutex mu_;
  std::map<Key, std::vector<void*>> free_;
  std::map<void*, size_t> sizes_;
  std::vector<void*> owned_;
};

// The caching pool of the current device that every graph created without a
// caller allocator works from, so that blocks one graph's call returns serve
// the next call on any graph (per-graph pools would each keep their own
// working set cached, and a process holding thousands of graphs would fill
// the device with them).  Created on first use, kept until the process ends.
std::shared_ptr<Pool> device_pool();

// Owning device buffer bound to a pool and a stream.
template <class T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(Pool* pool, hipStream_t s, size_t n) { reset(pool, s, n); }
  ~DBuf() { clear(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      clear();
      p_ = o.p_, n_ = o.n_, pool_ = o.pool_, s_ = o.s_;
      o.p_ = nullptr, o.n_ = 0;
    }
    return *this;
  }
  void reset(Pool* pool, hipStream_t s, size_t n) {
    clear();
    pool_ = pool, s_ = s, n_ = n;
    p_ = (T*)pool->alloc(n * sizeof(T), s);
  }
  void clear() {
    if (p_ && pool_) pool_->free(p_, s_);
    p_ = nullptr, n_ = 0;
  }
  void zero() {
    if (p_ && n_) device_zero(p_, n_ * sizeof(T), s_);
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  operator T*() const { return p_; }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
  Pool* pool_ = nullptr;
  hipStream_t s_ = nullptr;
};

// Page-locked staging for the small host <-> device copies of the calling
// thread (copies from or into pageable memory are staged by the runtime).
// stage_take returns room for `bytes` (16-byte aligned) or nullptr when the
// arena is full or the copy is large.  Room is given back by
// stage_reset(mark) to an earlier stage_mark(), which the caller makes only
// once the stream has passed every copy that used the room.
constexpr size_t STAGE_BYTES = 1u << 20;
constexpr size_t STAGE_MAX_COPY = 16u << 10;
void* stage_take(size_t bytes);
size_t stage_mark();
void stage_reset(size_t mark);

// Reads `bytes` from the device now: the stream is synchronised.
void read_now(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace lmgp
