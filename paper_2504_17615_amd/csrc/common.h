// Shared device/host definitions of the MI355X (gfx950) library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace lmgp {

#define LMGP_HD __host__ __device__ __forceinline__
#define LMGP_D __device__ __forceinline__

// ----------------------------------------------------------------- errors --
struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t c, const std::string& m) : std::runtime_error(m), code(c) {}
};
struct InvalidArg : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct OutOfMemory : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIP_CHECK(x)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      throw ::lmgp::HipError(e_, std::string(#x) + ": " + hipGetErrorString(e_) + " at " + \
                                     __FILE__ + ":" + std::to_string(__LINE__));          \
  } while (0)

// Counts a kernel launch for the profiler (a relaxed atomic add while it
// records, nothing otherwise).
void note_launch();

#define LAUNCH_CHECK()                 \
  do {                                 \
    HIP_CHECK(hipGetLastError());      \
    ::lmgp::note_launch();             \
  } while (0)

// ------------------------------------------------------------------ hashing --
// Counter-based hash: H(seed, tag, x1..xj) = mix(..mix(mix(mix(seed) ^ tag) ^ x1)..^ xj)
// with mix the SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).  Host
// code folds the leading arguments into a prefix; kernels fold in node and
// cluster ids with hash_add.
LMGP_HD uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
LMGP_HD uint64_t hash_add(uint64_t s, uint64_t x) { return mix64(s ^ x); }
inline uint64_t hash_prefix(uint64_t seed, uint64_t tag) { return mix64(mix64(seed) ^ tag); }

enum HashTag : uint64_t {
  TAG_SUB = 1,     // LP sub-round of a node (clustering)
  TAG_TIE = 2,     // LP target tie-break
  TAG_ADM = 3,     // LP admission order
  TAG_FAV = 4,     // 2-hop favourite tie-break
  TAG_TWOHOP = 5,  // 2-hop order inside a favourite segment
  TAG_SPARS = 6,   // threshold sampling among equal-weight edges
  TAG_IP = 7,      // initial bipartitioning start nodes
  TAG_RSUB = 8,    // refinement sub-round
  TAG_RTIE = 9,    // refinement tie-break
  TAG_RADM = 10,   // refinement admission order
  TAG_FFSTART = 11,  // (Weighted) Forest Fire: start node of a fire
  TAG_FFDRAW = 12,   // a frontier node's draw among its unvisited neighbours
  TAG_FFBREAK = 13,  // whether the node stops drawing after a draw
  TAG_FFCLAIM = 14   // which of several draws of one node burns it
};

// Sub-round of a node: floor(hi32(h) * S / 2^32).
LMGP_HD uint32_t subround_of(uint64_t h, uint32_t S) {
  return (uint32_t)(((h >> 32) * (uint64_t)S) >> 32);
}

constexpr uint32_t EMPTY_KEY = 0xFFFFFFFFu;

// ---------------------------------------------------------- wave helpers --
constexpr int WAVE = 64;

LMGP_D int lane_id() { return __lane_id(); }

// Make this wave's LDS writes visible to its other lanes.
LMGP_D void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

LMGP_D uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Edge-weight accessors: unit (no array), int32 or int64 per entry.
enum EwKind : int { EW_UNIT = 0, EW_I32 = 1, EW_I64 = 2 };

template <int K>
LMGP_D int64_t edge_w(const void* ew, uint64_t e);
template <>
LMGP_D int64_t edge_w<EW_UNIT>(const void*, uint64_t) { return 1; }
template <>
LMGP_D int64_t edge_w<EW_I32>(const void* ew, uint64_t e) {
  return (int64_t)((const int32_t*)ew)[e];
}
template <>
LMGP_D int64_t edge_w<EW_I64>(const void* ew, uint64_t e) {
  return ((const int64_t*)ew)[e];
}
// The weights of a row starting at entry `beg` (NULL for unit weights), read
// with 32-bit offsets by edge_w.
template <int K>
LMGP_D const void* edge_row(const void* ew, uint64_t beg) {
  return K == EW_I32 ? (const void*)((const int32_t*)ew + beg)
       : K == EW_I64 ? (const void*)((const int64_t*)ew + beg) : nullptr;
}

LMGP_HD uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

inline unsigned grid_for(uint64_t n, unsigned block) {
  uint64_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  if (g > 0x7fffffffull) g = 0x7fffffffull;
  return (unsigned)g;
}

}  // namespace lmgp
