// GMS validation of guided matches (grid-based motion statistics, the filter
// of the paper's experiments, threshold 6; the method is cited in Sec. 4.3).
// Single-grid form over a batch of pairs:
//   1. every query with a match gets its image-1 cell a and the image-2 cell
//      b of its match (G x G cells per image, floor(x G / W) in FP64,
//      clamped); matches are counted per (pair, a);
//   2. after an exclusive scan of the counts, the matches are listed by
//      (pair, a) with an atomic cursor per cell (order within a cell does
//      not matter: only counts are used);
//   3. one wavefront per (pair, a): a histogram of b in LDS gives the cell's
//      motion (most frequent b, ties to the lowest index); the score sums,
//      over the 3 x 3 cells around a, the matches going to the cell at the
//      same offset around b; the cell passes when score^2 * cells >
//      alpha^2 * (matches in those cells), evaluated in FP64; the matches of
//      a that go to b are kept, the others set to -1.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

__device__ __forceinline__ int grid_cell(float x, float y, double w, double h, int G) {
  double cx = floor((double)x * (double)G / w);
  double cy = floor((double)y * (double)G / h);
  cx = !(cx >= 0.0) ? 0.0 : (cx > G - 1 ? (double)(G - 1) : cx);  // NaN to cell 0
  cy = !(cy >= 0.0) ? 0.0 : (cy > G - 1 ? (double)(G - 1) : cy);
  return (int)cy * G + (int)cx;
}

__global__ __launch_bounds__(kThreads) void k_gms_cells(GmsArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= A.n1) return;
  const int32_t j = A.best[i];
  A.out[i] = -1;
  A.key[i] = -1;
  if (j < 0) return;
  const int p = find_pair(A.qstart, A.num_pairs, i);
  const GmsPair g = A.pairs[p];
  const int64_t jg = A.kstart[p] + j;
  const int a = grid_cell(A.kp1[2 * i], A.kp1[2 * i + 1], g.w1, g.h1, A.grid);
  const int b = grid_cell(A.kp2[2 * jg], A.kp2[2 * jg + 1], g.w2, g.h2, A.grid);
  const int32_t key = p * A.grid * A.grid + a;
  A.key[i] = key;
  A.rcell[i] = b;
  atomicAdd(&A.count[key], 1u);
}

__global__ __launch_bounds__(kThreads) void k_gms_scatter(GmsArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= A.n1) return;
  const int32_t key = A.key[i];
  if (key < 0) return;
  const uint32_t at = atomicAdd(&A.cursor[key], 1u);
  A.list[A.offsets[key] + at] = (uint32_t)i;
}

// Matches from cell (pair, a2) whose image-2 cell is b2 (wavefront-wide).
__device__ __forceinline__ uint32_t count_to(const GmsArgs& A, int32_t key2, int b2) {
  const int lane = lane_id();
  const int64_t o = A.offsets[key2];
  const uint32_t n = A.count[key2];
  uint32_t c = 0;
  for (uint32_t t = 0; t < n; t += kWave) {
    const bool hit = t + lane < n && A.rcell[A.list[o + t + lane]] == b2;
    c += (uint32_t)__popcll(ballot(hit));
  }
  return c;
}

__global__ __launch_bounds__(kThreads) void k_gms_score(GmsArgs A) {
  __shared__ uint32_t hist[kWaves][kGmsMaxCells];
  const int lane = lane_id(), wave = wave_id();
  const int G = A.grid, GG = G * G;
  const int64_t cell = (int64_t)blockIdx.x * kWaves + wave;
  if (cell >= (int64_t)A.num_pairs * GG) return;
  const int32_t key = (int32_t)cell;
  const uint32_t n = A.count[key];
  if (n == 0) return;
  const int p = key / GG, a = key % GG;
  const int64_t o = A.offsets[key];
  uint32_t* h = hist[wave];
  for (int t = lane; t < GG; t += kWave) h[t] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (uint32_t t = lane; t < n; t += kWave) atomicAdd(&h[A.rcell[A.list[o + t]]], 1u);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // the cell's motion: most frequent image-2 cell, ties to the lowest index
  uint32_t bc = 0;
  int bi = GG;
  for (int t = lane; t < GG; t += kWave) {
    if (h[t] > bc) {
      bc = h[t];
      bi = t;
    }
  }
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t oc = __shfl_xor(bc, off);
    const int oi = __shfl_xor(bi, off);
    if (oc > bc || (oc == bc && oi < bi)) {
      bc = oc;
      bi = oi;
    }
  }
  const int ax = a % G, ay = a / G, bx = bi % G, by = bi / G;
  uint64_t score = 0, total = 0, ncell = 0;
  for (int dy = -1; dy <= 1; ++dy) {
    for (int dx = -1; dx <= 1; ++dx) {
      const int x1 = ax + dx, y1 = ay + dy;
      if (x1 < 0 || x1 >= G || y1 < 0 || y1 >= G) continue;
      const int32_t k2 = p * GG + y1 * G + x1;
      total += A.count[k2];
      ncell += 1;
      const int x2 = bx + dx, y2 = by + dy;
      if (x2 < 0 || x2 >= G || y2 < 0 || y2 >= G) continue;
      score += count_to(A, k2, y2 * G + x2);
    }
  }
  const double s = (double)score;
  const bool pass = s * s * (double)ncell > (double)A.alpha * (double)A.alpha * (double)total;
  for (uint32_t t = lane; t < n; t += kWave) {
    const uint32_t i = A.list[o + t];
    A.out[i] = pass && A.rcell[i] == bi ? A.best[i] : -1;
  }
}

}  // namespace

hipError_t launch_gms(const GmsArgs& a, int64_t* partials, hipStream_t s) {
  if (a.n1 == 0) return hipSuccess;
  const int64_t cells = (int64_t)a.num_pairs * a.grid * a.grid;
  const int64_t qb = (a.n1 + kThreads - 1) / kThreads;
  hipError_t e = launch_fill_u32(a.count, cells, 0u, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(a.cursor, cells, 0u, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gms_cells, dim3((unsigned)qb), dim3(kThreads), 0, s, a);
  e = launch_scan_counts(a.count, 1, cells, const_cast<int64_t*>(a.offsets), partials, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gms_scatter, dim3((unsigned)qb), dim3(kThreads), 0, s, a);
  const int64_t cb = (cells + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k_gms_score, dim3((unsigned)cb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace epm
