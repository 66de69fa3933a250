// Tiled descriptor matching over the candidate CSR (Sec. 4.3).
//
// One workgroup per angle tile of 64 queries (the tiles of the stabbing
// pass), tiles dispatched in XCD-aware order: neighbouring queries share most
// of their candidates, so the candidate rows one wavefront gathers are hit in
// L1/L2 by the next.  Each wavefront takes 16 of the tile's queries one after
// another, one lane per candidate; distances, selection and outputs are those
// of the plain kernel (canonical FP32 order, lowest-j ties).
#include "device_common.h"
#include "launch.h"
#include "match_common.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kQPerWave = kTileQ / kWaves;

__global__ __launch_bounds__(kThreads) void k_match_tile_f32(MatchArgs A) {
  __shared__ float4 qdesc[kWaves][32];
  const int lane = lane_id(), wave = wave_id();
  const StabTile T = A.tiles[xcd_tile(blockIdx.x, A.num_tiles)];
  const int64_t kb = A.kstart[T.pair];
  for (int qq = 0; qq < kQPerWave; ++qq) {
    const int q = wave * kQPerWave + qq;
    if (q >= T.count) break;
    const int64_t i = (int64_t)A.qperm[T.begin + q];
    const float4* d1 = reinterpret_cast<const float4*>(A.desc1) + i * 32;
    if (lane < 32) qdesc[wave][lane] = d1[lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t o0 = A.row_offsets[i], o1 = A.row_offsets[i + 1];
    Top2 t;
    for (int64_t e = o0 + lane; e < o1; e += kWave) {
      const int32_t j = A.cols[e];
      const float4* d2 = reinterpret_cast<const float4*>(A.desc2) + (kb + j) * 32;
      float acc = 0.0f;
      #pragma unroll 8
      for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qdesc[wave][k], d2[k]);
      t.insert(acc, j);
    }
    t = wave_merge_top2(t);
    if (lane == 0) write_match(A, i, t, false);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(kThreads) void k_match_tile_bin256(MatchArgs A) {
  const int lane = lane_id(), wave = wave_id();
  const StabTile T = A.tiles[xcd_tile(blockIdx.x, A.num_tiles)];
  const int64_t kb = A.kstart[T.pair];
  for (int qq = 0; qq < kQPerWave; ++qq) {
    const int q = wave * kQPerWave + qq;
    if (q >= T.count) break;
    const int64_t i = (int64_t)A.qperm[T.begin + q];
    const uint4* d1 = reinterpret_cast<const uint4*>(A.desc1) + i * 2;
    const uint4 qa = d1[0], qb = d1[1];
    const int64_t o0 = A.row_offsets[i], o1 = A.row_offsets[i + 1];
    Top2 t;
    for (int64_t e = o0 + lane; e < o1; e += kWave) {
      const int32_t j = A.cols[e];
      const uint4* d2 = reinterpret_cast<const uint4*>(A.desc2) + (kb + j) * 2;
      const uint4 ba = d2[0], bb = d2[1];
      const uint32_t h = __popc(qa.x ^ ba.x) + __popc(qa.y ^ ba.y) + __popc(qa.z ^ ba.z) +
                         __popc(qa.w ^ ba.w) + __popc(qb.x ^ bb.x) + __popc(qb.y ^ bb.y) +
                         __popc(qb.z ^ bb.z) + __popc(qb.w ^ bb.w);
      t.insert((float)h, j);
    }
    t = wave_merge_top2(t);
    if (lane == 0) write_match(A, i, t, true);
  }
}

}  // namespace

hipError_t launch_match_tiled_f32(const MatchArgs& a, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_match_tile_f32, dim3(a.num_tiles), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_match_tiled_bin256(const MatchArgs& a, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_match_tile_bin256, dim3(a.num_tiles), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace epm
