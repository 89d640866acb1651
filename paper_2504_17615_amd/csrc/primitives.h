// Device-wide primitives written for 64-wide wavefronts: exclusive scan over
// a generated sequence, and a stable LSD radix sort of (uint64 key, value)
// pairs.  Both are three-phase (tile reduce / scan of tile totals / tile
// scan-or-scatter) so that results do not depend on scheduling.
#pragma once
#include "common.h"
#include "memory.h"

namespace lmgp {

void device_zero(void* p, size_t bytes, hipStream_t s);
void device_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);

// ------------------------------------------------------------ block scans --
constexpr int BLK = 256;
constexpr int NWAVE = BLK / WAVE;

template <class T>
LMGP_D T wave_inclusive_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T o = __shfl_up(v, d, WAVE);
    if (l >= d) v += o;
  }
  return v;
}

template <class T>
LMGP_D T wave_reduce_sum(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

template <class T>
LMGP_D T wave_reduce_max(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    T o = __shfl_xor(v, d, WAVE);
    v = o > v ? o : v;
  }
  return v;
}

// Exclusive scan across a block of NW waves (default: a 256-thread block);
// `total` receives the block sum.  smem must hold NW elements.  Contains
// __syncthreads.
template <class T, int NW = NWAVE>
LMGP_D T block_exclusive_scan(T v, T* smem, T& total) {
  const int w = threadIdx.x / WAVE, l = lane_id();
  T inc = wave_inclusive_scan(v);
  if (l == WAVE - 1) smem[w] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    T s = smem[i];
    if (i < w) before += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return before + inc - v;
}

template <class T>
LMGP_D T block_reduce_sum(T v, T* smem) {
  T tot;
  (void)block_exclusive_scan(v, smem, tot);
  return tot;
}

// --------------------------------------------------------- device scan --
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLK * SCAN_ITEMS;

template <class F>
__global__ __launch_bounds__(BLK) void k_scan_reduce(F f, uint64_t n, uint64_t* sums) {
  __shared__ uint64_t sm[NWAVE];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    uint64_t i = base + (uint64_t)j * BLK + threadIdx.x;
    if (i < n) s += (uint64_t)f(i);
  }
  uint64_t t = block_reduce_sum(s, sm);
  if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

// Tile scan: items of a tile are assigned blocked (thread t owns
// [t*ITEMS, (t+1)*ITEMS) of the tile) so every thread writes a contiguous run.
template <class F, class Out>
__global__ __launch_bounds__(BLK) void k_scan_down(F f, uint64_t n, const uint64_t* tile_off,
                                                   Out* out, int write_total) {
  __shared__ uint64_t sm[NWAVE];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint64_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    uint64_t i = base + j;
    v[j] = i < n ? (uint64_t)f(i) : 0;
    s += v[j];
  }
  uint64_t tot;
  uint64_t run = block_exclusive_scan(s, sm, tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    uint64_t i = base + j;
    if (i < n) out[i] = (Out)run;
    run += v[j];
  }
  if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == BLK - 1) out[n] = (Out)run;
}

struct ArrayU64 {
  const uint64_t* a;
  LMGP_D uint64_t operator()(uint64_t i) const { return a[i]; }
};
struct ArrayU32 {
  const uint32_t* a;
  LMGP_D uint64_t operator()(uint64_t i) const { return a[i]; }
};

// out[i] = sum_{j<i} f(j) for i < n; out[n] = total if write_total.
template <class F, class Out>
void exclusive_scan(F f, uint64_t n, Out* out, bool write_total, Pool& pool, hipStream_t s) {
  if (n == 0) {
    if (write_total) device_zero(out, sizeof(Out), s);
    return;
  }
  const uint64_t tiles = ceil_div(n, SCAN_TILE);
  if (tiles == 1) {
    k_scan_down<<<1, BLK, 0, s>>>(f, n, (const uint64_t*)nullptr, out, write_total ? 1 : 0);
    LAUNCH_CHECK();
    return;
  }
  DBuf<uint64_t> sums(&pool, s, tiles), offs(&pool, s, tiles);
  k_scan_reduce<<<(unsigned)tiles, BLK, 0, s>>>(f, n, sums.get());
  LAUNCH_CHECK();
  exclusive_scan(ArrayU64{sums.get()}, tiles, offs.get(), false, pool, s);
  k_scan_down<<<(unsigned)tiles, BLK, 0, s>>>(f, n, offs.get(), out, write_total ? 1 : 0);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ radix sort --
// Stable LSD radix sort, 8-bit digits over key bits [begin_bit, end_bit).
// Sorts (keys, vals) of n < 2^32 elements; uses (tmp_keys, tmp_vals) as the
// second buffer.  Returns true if the result is in the tmp buffers.
template <class V>
bool radix_sort_pairs(uint64_t* keys, V* vals, uint64_t* tmp_keys, V* tmp_vals, uint64_t n,
                      int begin_bit, int end_bit, Pool& pool, hipStream_t s);

}  // namespace lmgp
