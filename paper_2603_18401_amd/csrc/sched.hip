// Work distribution for the tile kernels when many pairs of uneven size run
// together: a longest-first (LPT) order of the angle tiles, and clears of the
// scheduling counters by kernel (so a whole pipeline can be captured in a HIP
// graph without memset nodes).
//
// Tile cost (written by the window pass): queries x window records of the
// tile, plus pair size x brute-force queries.  Tiles are bucketed by
// floor(log2 cost) and laid out bucket by bucket, most expensive first; the
// order inside a bucket is arbitrary (results never depend on the order in
// which tiles run, only the finishing time does).
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
static_assert(kLptXcd == kNumXcd, "the XCD order follows xcd_tile");
static_assert(kCostBuckets == 65, "cost_bucket: 1 + 2 x 31 + 1 is the largest bucket");

__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t* __restrict__ p, int64_t n,
                                                       uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    p[i] = v;
}

// Bucket histogram: per-workgroup counts in LDS, one global add per
// non-empty bucket.
__global__ __launch_bounds__(kThreads) void k_lpt_hist(const uint32_t* __restrict__ cost, int n,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kCostBuckets];
  if (threadIdx.x < kCostBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const int t = (int)blockIdx.x * kThreads + (int)threadIdx.x;
  if (t < n) atomicAdd(&h[cost_bucket(cost[t])], 1u);
  __syncthreads();
  if (threadIdx.x < kCostBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Scatter: the workgroup reserves a run inside each of its buckets, every
// tile takes the next place of its run.  Bucket b starts after all buckets
// above it.
__global__ __launch_bounds__(kThreads) void k_lpt_scatter(const uint32_t* __restrict__ cost,
                                                          int n,
                                                          const uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ cursor,
                                                          uint32_t* __restrict__ order) {
  __shared__ uint32_t h[kCostBuckets], base[kCostBuckets];
  const int tid = (int)threadIdx.x;
  if (tid < kCostBuckets) h[tid] = 0u;
  __syncthreads();
  const int t = (int)blockIdx.x * kThreads + tid;
  int b = 0;
  uint32_t rank = 0;
  if (t < n) {
    b = cost_bucket(cost[t]);
    rank = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (tid < kCostBuckets && h[tid]) {
    uint32_t start = 0;
    for (int k = kCostBuckets - 1; k > tid; --k) start += hist[k];
    base[tid] = start + atomicAdd(&cursor[tid], h[tid]);
  }
  __syncthreads();
  if (t < n) order[base[b] + rank] = (uint32_t)t;
}

// Per-XCD longest-first layout: workgroup x handles the tiles that
// xcd_tile gives XCD x, counts them per cost bucket, and deals them out most
// expensive bucket first: the tile of rank k goes to workgroup k * 8 + x of
// the tile launch (any order inside a bucket).
constexpr int kXcdThreads = 1024;

// i-th tile (0 <= i < tiles of XCD x) that xcd_tile sends to XCD x.
__device__ __forceinline__ int xcd_member(int i, int x, int n) {
  constexpr int round = kNumXcd * kXcdGroup;
  const int full = (n / round) * round;
  const int head = full / kNumXcd;  // XCD x's tiles among the first `full`
  if (i < head) return ((i / kXcdGroup) * kNumXcd + x) * kXcdGroup + i % kXcdGroup;
  return full + (i - head) * kNumXcd + x;
}

__global__ __launch_bounds__(kXcdThreads) void k_xcd_lpt_order(const uint32_t* __restrict__ cost,
                                                               int n,
                                                               uint32_t* __restrict__ block_tile) {
  __shared__ uint32_t h[kCostBuckets], cursor[kCostBuckets];
  const int x = (int)blockIdx.x, tid = (int)threadIdx.x;
  constexpr int round = kNumXcd * kXcdGroup;
  const int full = (n / round) * round;
  const int rest = n - full - x;
  const int nx = full / kNumXcd + (rest > 0 ? (rest + kNumXcd - 1) / kNumXcd : 0);
  if (tid < kCostBuckets) h[tid] = 0u;
  __syncthreads();
  for (int i = tid; i < nx; i += kXcdThreads)
    atomicAdd(&h[cost_bucket(cost[xcd_member(i, x, n)])], 1u);
  __syncthreads();
  if (tid < kCostBuckets) {
    uint32_t start = 0;
    for (int c = kCostBuckets - 1; c > tid; --c) start += h[c];
    cursor[tid] = start;
  }
  __syncthreads();
  for (int i = tid; i < nx; i += kXcdThreads) {
    const int t = xcd_member(i, x, n);
    const uint32_t k = atomicAdd(&cursor[cost_bucket(cost[t])], 1u);
    block_tile[k * kNumXcd + (uint32_t)x] = (uint32_t)t;
  }
}

}  // namespace

hipError_t launch_xcd_lpt_order(const uint32_t* cost, int num_tiles, uint32_t* block_tile,
                                hipStream_t s) {
  if (num_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_xcd_lpt_order, dim3(kNumXcd), dim3(kXcdThreads), 0, s, cost, num_tiles,
                     block_tile);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_lpt_order(const uint32_t* cost, int num_tiles, uint32_t* sched,
                            uint32_t* order, hipStream_t s) {
  if (num_tiles == 0) return hipSuccess;
  const int blocks = (num_tiles + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_lpt_hist, dim3(blocks), dim3(kThreads), 0, s, cost, num_tiles,
                     sched + kSchedHist);
  hipLaunchKernelGGL(k_lpt_scatter, dim3(blocks), dim3(kThreads), 0, s, cost, num_tiles,
                     sched + kSchedHist, sched + kSchedCursor, order);
  return hipGetLastError();
}

}  // namespace epm
