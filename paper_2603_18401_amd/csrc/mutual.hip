// Mutual guided matching (Sec. 4.3: guided matching combined with a standard
// matching strategy).  Matching in both directions -- image 1 against image 2
// with F, image 2 against image 1 with the transposed matrix (Eq. 1 read from
// the other camera) -- and keeping a pair only when each keypoint is the
// other's match is the classical cross-check; this kernel is that check over
// the two match arrays of a batch.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

__global__ __launch_bounds__(256) void k_mutual(const int64_t* __restrict__ qstart,
                                                const int64_t* __restrict__ kstart, int num_pairs,
                                                int64_t n1, const int32_t* __restrict__ best12,
                                                const int32_t* __restrict__ best21,
                                                int32_t* __restrict__ mutual) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  const int p = find_pair(qstart, num_pairs, i);
  const int32_t j = best12[i];
  int32_t out = -1;
  if (j >= 0 && (int64_t)j < kstart[p + 1] - kstart[p] &&
      (int64_t)best21[kstart[p] + j] == i - qstart[p])
    out = j;
  mutual[i] = out;
}

}  // namespace

hipError_t launch_mutual(const int64_t* qstart, const int64_t* kstart, int num_pairs, int64_t n1,
                         const int32_t* best12, const int32_t* best21, int32_t* mutual,
                         hipStream_t s) {
  if (n1 == 0) return hipSuccess;
  const int64_t blocks = (n1 + 255) / 256;
  hipLaunchKernelGGL(k_mutual, dim3((unsigned)blocks), dim3(256), 0, s, qstart, kstart, num_pairs,
                     n1, best12, best21, mutual);
  return hipGetLastError();
}

}  // namespace epm
