// Primitive kernels: fills and the stable LSD radix sort.
#include "primitives.h"
#include "profiler.h"

#include <cstring>

namespace lmgp {

__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}
__global__ void k_zero_u8(uint8_t* p, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Zeroing by kernel (not hipMemsetAsync) so that captured graphs stay valid.
void device_zero(void* p, size_t bytes, hipStream_t s) {
  if (!p || bytes == 0) return;
  if ((bytes & 3) == 0 && ((uintptr_t)p & 3) == 0) {
    uint64_t n = bytes / 4;
    unsigned g = grid_for(n, BLK);
    if (g > 8192) g = 8192;
    k_zero_u32<<<g, BLK, 0, s>>>((uint32_t*)p, n);
  } else {
    unsigned g = grid_for(bytes, BLK);
    if (g > 8192) g = 8192;
    k_zero_u8<<<g, BLK, 0, s>>>((uint8_t*)p, bytes);
  }
  LAUNCH_CHECK();
}

void device_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (!p || n == 0) return;
  unsigned g = grid_for(n, BLK);
  if (g > 8192) g = 8192;
  k_fill_u32<<<g, BLK, 0, s>>>(p, v, n);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ radix sort --
constexpr int RS_ITEMS = 8;
constexpr int RS_WAVE_ITEMS = WAVE * RS_ITEMS;    // 512 keys per wave
constexpr int RS_TILE = BLK * RS_ITEMS;           // 2048 keys per block

__global__ __launch_bounds__(BLK) void k_radix_hist(const uint64_t* keys, uint64_t n, int shift,
                                                    uint32_t* hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    uint64_t i = base + (uint64_t)j * BLK + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Tile layout: wave w owns keys [tile + w*512, tile + (w+1)*512); item j of
// lane l is key tile + w*512 + j*64 + l.  Keys are ranked in that order, so
// equal digits keep their input order (stability).
template <class V>
__global__ __launch_bounds__(BLK) void k_radix_scatter(const uint64_t* kin, const V* vin,
                                                       uint64_t* kout, V* vout, uint64_t n,
                                                       int shift, const uint32_t* offs,
                                                       uint32_t ntiles) {
  __shared__ uint32_t cnt[NWAVE][256];
  __shared__ uint32_t woff[NWAVE][256];
  const int w = threadIdx.x / WAVE, l = lane_id();
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) cnt[i][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t wbase = (uint64_t)blockIdx.x * RS_TILE + (uint64_t)w * RS_WAVE_ITEMS;
  uint64_t k[RS_ITEMS];
  V v[RS_ITEMS];
  uint32_t d[RS_ITEMS], r[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    uint64_t i = wbase + (uint64_t)j * WAVE + l;
    bool valid = i < n;
    k[j] = valid ? kin[i] : 0;
    v[j] = valid ? vin[i] : V();
    d[j] = (uint32_t)((k[j] >> shift) & 0xFF);
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    uint64_t i = wbase + (uint64_t)j * WAVE + l;
    bool valid = i < n;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((d[j] >> b) & 1u);
      peers &= ((d[j] >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank_in = (uint32_t)__popcll(peers & lt);
    uint32_t cur = valid ? cnt[w][d[j]] : 0;
    wave_sync();
    if (valid && (peers & lt) == 0) cnt[w][d[j]] = cur + (uint32_t)__popcll(peers);
    wave_sync();
    r[j] = cur + rank_in;
  }
  __syncthreads();
  {
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) {
      woff[i][threadIdx.x] = run;
      run += cnt[i][threadIdx.x];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    uint64_t i = wbase + (uint64_t)j * WAVE + l;
    if (i < n) {
      uint64_t pos = (uint64_t)offs[(uint64_t)d[j] * ntiles + blockIdx.x] + woff[w][d[j]] + r[j];
      kout[pos] = k[j];
      vout[pos] = v[j];
    }
  }
}

template <class V>
bool radix_sort_pairs(uint64_t* keys, V* vals, uint64_t* tmp_keys, V* tmp_vals, uint64_t n,
                      int begin_bit, int end_bit, Pool& pool, hipStream_t s) {
  if (n <= 1 || end_bit <= begin_bit) return false;
  if (n >= (1ull << 32)) throw InvalidArg("radix sort limited to 2^32 elements");
  const uint32_t ntiles = (uint32_t)ceil_div(n, RS_TILE);
  DBuf<uint32_t> hist(&pool, s, (size_t)256 * ntiles), offs(&pool, s, (size_t)256 * ntiles);
  uint64_t *ka = keys, *kb = tmp_keys;
  V *va = vals, *vb = tmp_vals;
  bool in_tmp = false;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    k_radix_hist<<<ntiles, BLK, 0, s>>>(ka, n, shift, hist.get(), ntiles);
    LAUNCH_CHECK();
    exclusive_scan(ArrayU32{hist.get()}, (uint64_t)256 * ntiles, offs.get(), false, pool, s);
    k_radix_scatter<V><<<ntiles, BLK, 0, s>>>(ka, va, kb, vb, n, shift, offs.get(), ntiles);
    LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
    in_tmp = !in_tmp;
  }
  return in_tmp;
}

template bool radix_sort_pairs<uint32_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, uint64_t,
                                         int, int, Pool&, hipStream_t);
template bool radix_sort_pairs<uint64_t>(uint64_t*, uint64_t*, uint64_t*, uint64_t*, uint64_t,
                                         int, int, Pool&, hipStream_t);
template bool radix_sort_pairs<int64_t>(uint64_t*, int64_t*, uint64_t*, int64_t*, uint64_t, int,
                                        int, Pool&, hipStream_t);

namespace {
struct Stage {
  char* buf = nullptr;
  size_t used = 0;
};
Stage& stage() {
  static thread_local Stage st;  // kept for the thread's life (1 MiB)
  return st;
}
}  // namespace

std::shared_ptr<Pool> device_pool() {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  static std::mutex mu;
  // never destroyed: freeing device memory while the runtime shuts down at
  // process exit is not safe
  static auto* pools = new std::map<int, std::shared_ptr<Pool>>();
  std::lock_guard<std::mutex> g(mu);
  auto& p = (*pools)[dev];
  if (!p) p = std::make_shared<Pool>(nullptr);
  return p;
}

bool& no_alloc_mode() {
  static thread_local bool on = false;
  return on;
}

void* stage_take(size_t bytes) {
  if (bytes == 0 || bytes > STAGE_MAX_COPY || no_alloc_mode()) return nullptr;
  Stage& st = stage();
  if (!st.buf) HIP_CHECK(hipHostMalloc((void**)&st.buf, STAGE_BYTES, hipHostMallocDefault));
  const size_t off = (st.used + 15) & ~(size_t)15;
  if (off + bytes > STAGE_BYTES) return nullptr;
  st.used = off + bytes;
  return st.buf + off;
}

size_t stage_mark() { return stage().used; }
void stage_reset(size_t mark) { stage().used = mark; }

void read_now(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  Profiler::get().count("host:stream_syncs");
  const size_t mark = stage_mark();
  void* p = stage_take(bytes);
  HIP_CHECK(hipMemcpyAsync(p ? p : dst, src, bytes, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (p) std::memcpy(dst, p, bytes);
  stage_reset(mark);  // room taken after `mark` is this call's alone
}

}  // namespace lmgp
