// Diagnostic: both sides of the Eq. 3 test for listed (query, keypoint)
// pairs, computed with the device arithmetic of the candidate search.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

struct F9 {
  double v[9];
};

__global__ __launch_bounds__(256) void k_point_line_terms(F9 F, const float* __restrict__ kp1,
                                                          const float* __restrict__ kp2,
                                                          const float* __restrict__ eps2,
                                                          float eps_scalar,
                                                          const int64_t* __restrict__ qi,
                                                          const int64_t* __restrict__ kj,
                                                          int64_t count, double* __restrict__ num,
                                                          double* __restrict__ rhs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int64_t i = qi[t], j = kj[t];
  double a, b, c;
  epipolar_line(F.v, kp1[2 * i], kp1[2 * i + 1], a, b, c);
  const float ef = eps2 ? eps2[j] : eps_scalar;
  num[t] = fabs(__dadd_rn(__dadd_rn(__dmul_rn(a, (double)kp2[2 * j]), __dmul_rn(b, (double)kp2[2 * j + 1])), c));
  rhs[t] = __dmul_rn((double)ef, __dsqrt_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b))));
}

}  // namespace

hipError_t launch_point_line_terms(const double* F9in, const float* kp1, const float* kp2,
                                   const float* eps2, float eps_scalar, const int64_t* qi,
                                   const int64_t* kj, int64_t count, double* num, double* rhs,
                                   hipStream_t s) {
  if (count == 0) return hipSuccess;
  F9 F;
  for (int k = 0; k < 9; ++k) F.v[k] = F9in[k];
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_point_line_terms, dim3((unsigned)blocks), dim3(256), 0, s, F, kp1, kp2,
                     eps2, eps_scalar, qi, kj, count, num, rhs);
  return hipGetLastError();
}

}  // namespace epm
