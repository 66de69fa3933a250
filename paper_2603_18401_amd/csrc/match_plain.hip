// Plain descriptor matching over the candidate CSR (Sec. 4.3): one wavefront
// per query, one lane per candidate, the candidate's descriptor gathered from
// global memory.  This is the reference GPU path the tiled kernels are
// measured against.
//
// Float distance: canonical FP32 squared L2, t = a_k - b_k then
// acc = fmaf(t, t, acc) for k = 0..127 in order, so every distance is
// bit-reproducible.  Binary distance: popcount of the XOR over 8 words.
// Selection: smallest (distance, j), then the next one; optional ratio test.
#include "device_common.h"
#include "launch.h"
#include "match_common.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

__global__ __launch_bounds__(kThreads) void k_match_plain_f32(MatchArgs A) {
  __shared__ float4 qdesc[kWaves][32];
  if (csr_overflow(A)) return;
  const int lane = lane_id(), wave = wave_id();
  const int64_t blk = A.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t qs = blk * kWaves + wave;
  if (qs >= A.n1) return;
  const int64_t i = A.qperm ? (int64_t)A.qperm[qs] : qs;
  const int pair = find_pair(A.qstart, A.num_pairs, i);
  const int64_t kb = A.kstart[pair];
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
    for (int k = 0; k < 32; ++k) {
      const float4 a = qdesc[wave][k];
      const float4 b = d2[k];
      acc = canonical_step4(acc, a, b);
    }
    t.insert(acc, j);
  }
  t = wave_merge_top2(t);
  if (lane == 0) write_match(A, i, t, false);
}

__global__ __launch_bounds__(kThreads) void k_match_plain_bin256(MatchArgs A) {
  if (csr_overflow(A)) return;
  const int lane = lane_id(), wave = wave_id();
  const int64_t qs = (int64_t)blockIdx.x * kWaves + wave;
  if (qs >= A.n1) return;
  const int64_t i = A.qperm ? (int64_t)A.qperm[qs] : qs;
  const int pair = find_pair(A.qstart, A.num_pairs, i);
  const int64_t kb = A.kstart[pair];
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

// Listed queries (the ones the fused stab + match pass left over): one
// wavefront per listed query, grid-stride over a list whose length only the
// device knows.
__global__ __launch_bounds__(kThreads) void k_match_listed_f32(MatchArgs A,
                                                               const uint32_t* __restrict__ list,
                                                               const unsigned long long* __restrict__ count) {
  __shared__ float4 qdesc[kWaves][32];
  if (csr_overflow(A)) return;
  const int lane = lane_id(), wave = wave_id();
  const uint64_t n = *count;
  for (uint64_t t = (uint64_t)blockIdx.x * kWaves + wave; t < n;
       t += (uint64_t)gridDim.x * kWaves) {
    const int64_t i = (int64_t)list[t];
    const int pair = find_pair(A.qstart, A.num_pairs, i);
    const int64_t kb = A.kstart[pair];
    if (lane < 32) qdesc[wave][lane] = reinterpret_cast<const float4*>(A.desc1)[i * 32 + lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t o0 = A.row_offsets[i], o1 = A.row_offsets[i + 1];
    Top2 tp;
    for (int64_t e = o0 + lane; e < o1; e += kWave) {
      const int32_t j = A.cols[e];
      const float4* d2 = reinterpret_cast<const float4*>(A.desc2) + (kb + j) * 32;
      float acc = 0.0f;
      #pragma unroll 8
      for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qdesc[wave][k], d2[k]);
      tp.insert(acc, j);
    }
    tp = wave_merge_top2(tp);
    if (lane == 0) write_match(A, i, tp, false);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace

hipError_t launch_match_listed_f32(const MatchArgs& a, const uint32_t* list,
                                   const unsigned long long* count, int64_t max_count,
                                   hipStream_t s) {
  if (max_count <= 0) return hipSuccess;
  // the list is usually short and its rows latency-bound: enough
  // workgroups that every listed query has its own wavefront up to 16384
  int64_t blocks = (max_count + kWaves - 1) / kWaves;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_match_listed_f32, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, list,
                     count);
  return hipGetLastError();
}

hipError_t launch_match_plain_f32(const MatchArgs& a, hipStream_t s) {
  if (a.n1 == 0) return hipSuccess;
  const int64_t blocks = (a.n1 + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k_match_plain_f32, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_match_plain_bin256(const MatchArgs& a, hipStream_t s) {
  if (a.n1 == 0) return hipSuccess;
  const int64_t blocks = (a.n1 + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k_match_plain_bin256, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace epm
