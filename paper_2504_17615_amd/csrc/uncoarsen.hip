// Uncoarsening helpers: projection of blocks to the finer level (Sec. 2),
// block weights c(V_i) and the edge cut cut(Pi) = sum_{i<j} omega(E_ij).
#include "contract.h"
#include "profiler.h"

namespace lmgp {

namespace {

__global__ void k_project(const uint32_t* map, const uint32_t* cblock, uint64_t n,
                          uint32_t* block) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const uint32_t x = map[u];
  if (x != EMPTY_KEY) block[u] = cblock[x];
}

// Block weights; with at most 4096 blocks the sums are privatised in LDS.
constexpr uint64_t BW_LDS = 4096;

__global__ __launch_bounds__(256) void k_block_weights(const uint32_t* block, const int64_t* nw,
                                                       uint64_t n, int64_t* BW, uint64_t K) {
  __shared__ unsigned long long h[BW_LDS];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (K <= BW_LDS) {
    for (uint64_t i = threadIdx.x; i < K; i += 256) h[i] = 0;
    __syncthreads();
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
      atomicAdd(&h[block[u]], (unsigned long long)nw[u]);
    __syncthreads();
    for (uint64_t i = threadIdx.x; i < K; i += 256)
      if (h[i]) atomicAdd((unsigned long long*)&BW[i], h[i]);
  } else {
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
      atomicAdd((unsigned long long*)&BW[block[u]], (unsigned long long)nw[u]);
  }
}

template <int EWK>
__global__ __launch_bounds__(256) void k_cut(const uint32_t* src, const uint32_t* adj,
                                             const void* ew, const uint32_t* block,
                                             const uint32_t* gid, uint64_t nnz, int64_t* cut) {
  __shared__ int64_t sm[NWAVE];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  int64_t local = 0;
  uint32_t g0 = 0;
  bool single = gid == nullptr;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const uint32_t u = src[e], v = adj[e];
    if (u < v && block[u] != block[v]) {
      const int64_t w = edge_w<EWK>(ew, e);
      if (single) local += w;
      else atomicAdd((unsigned long long*)&cut[gid[u]], (unsigned long long)w);
    }
  }
  if (single) {
    const int64_t t = block_reduce_sum(local, sm);
    if (threadIdx.x == 0 && t) atomicAdd((unsigned long long*)&cut[g0], (unsigned long long)t);
  }
}

}  // namespace

void project_blocks(const uint32_t* map, const uint32_t* cblock, uint64_t n, uint32_t* block,
                    hipStream_t s) {
  if (!n) return;
  // map[u] and block[u] read and written per node, the coarse block gathered
  ProfScope prof("rf:project", 12 * n, s);
  k_project<<<grid_for(n, 256), 256, 0, s>>>(map, cblock, n, block);
  LAUNCH_CHECK();
}

void block_weights(const uint32_t* block, const int64_t* nw, uint64_t n, int64_t* BW, uint64_t K,
                   hipStream_t s) {
  if (!n) return;
  unsigned g = grid_for(n, 256);
  if (g > 1024) g = 1024;
  ProfScope prof("ev:block_weights", 12 * n, s);  // block + node weight per node
  k_block_weights<<<g, 256, 0, s>>>(block, nw, n, BW, K);
  LAUNCH_CHECK();
}

void edge_cut(const uint32_t* src, const uint32_t* adj, const void* ew, int ew_kind,
              const uint32_t* block, const uint32_t* gid, uint64_t nnz, int64_t* cut,
              hipStream_t s) {
  if (!nnz) return;
  unsigned g = grid_for(nnz, 256);
  if (g > 4096) g = 4096;
  // per entry: row, neighbour, its block (4 B each) and the stored weight
  const uint64_t bw = ew_kind == EW_UNIT ? 0 : ew_kind == EW_I32 ? 4 : 8;
  ProfScope prof("ev:cut", (12 + bw) * nnz, s);
  switch (ew_kind) {
    case EW_UNIT: k_cut<EW_UNIT><<<g, 256, 0, s>>>(src, adj, ew, block, gid, nnz, cut); break;
    case EW_I32: k_cut<EW_I32><<<g, 256, 0, s>>>(src, adj, ew, block, gid, nnz, cut); break;
    default: k_cut<EW_I64><<<g, 256, 0, s>>>(src, adj, ew, block, gid, nnz, cut); break;
  }
  LAUNCH_CHECK();
}

}  // namespace lmgp
