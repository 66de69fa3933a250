// Diagnostic: both sides of the Eq. 3 test for listed (query, keypoint)
// pairs, computed with the device arithmetic of the candidate search.
#include "device_common.h"
#include "launch.h"
#include "match_common.h"
#include "mfma_bounds.h"

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

// Descriptor distances of listed (query, keypoint) pairs as the matching
// kernels compute them: FMT 0 / 1 (BF16 / FP8 codes): the MFMA approximation
// |q^|^2 + |w^|^2 - 2 s1 s2 (q^ . w^) (norms k-ascending in FP32, the dot
// product on v_mfma_f32_16x16x32 with FP32 accumulation, combined in FP64);
// FMT -1: the canonical FP32 chain of FP32 rows.  One wavefront per 16 pairs:
// A = their query rows, B = their image-2 rows, the diagonal of the 16 x 16
// block is the pairs' dot products.
template <int FMT>
__global__ __launch_bounds__(kWave) void k_pair_distances(const void* __restrict__ desc1,
                                                          const void* __restrict__ desc2,
                                                          const float* __restrict__ scale1,
                                                          const float* __restrict__ scale2,
                                                          const int64_t* __restrict__ qi,
                                                          const int64_t* __restrict__ kj,
                                                          int64_t count, float* __restrict__ out) {
  const int lane = lane_id();
  const int64_t t0 = (int64_t)blockIdx.x * 16;
  const int p = lane & 15;
  const int64_t t = t0 + p;
  const bool live = t < count;
  const int64_t i = live ? qi[t] : 0, j = live ? kj[t] : 0;
  if constexpr (FMT < 0) {
    if (lane < 16 && live)
      out[t] = exact_distance(reinterpret_cast<const float4*>(desc1) + i * 32,
                              reinterpret_cast<const float4*>(desc2) + j * 32);
  } else {
    constexpr int RB = Fmt<FMT>::kRowBytes;
    const uint8_t* q = reinterpret_cast<const uint8_t*>(desc1) + i * RB;
    const uint8_t* w = reinterpret_cast<const uint8_t*>(desc2) + j * RB;
    const int g = lane >> 4;
    f32x4 acc = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int koff = kk * 32 + g * 8;  // this lane's 8 values of pair p's rows
      if (FMT == 0) {
        const bf16x8 a = live ? *reinterpret_cast<const bf16x8*>(q + koff * 2) : bf16x8{};
        const bf16x8 b = live ? *reinterpret_cast<const bf16x8*>(w + koff * 2) : bf16x8{};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
      } else {
        const long a = live ? *reinterpret_cast<const long*>(q + koff) : 0l;
        const long b = live ? *reinterpret_cast<const long*>(w + koff) : 0l;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc, 0, 0, 0);
      }
    }
    // D[m][n] sits in lane n + 16 (m >> 2), element m & 3: pair p's own
    // product is D[p][p]
    if (live && g == (p >> 2)) {
      const float dot = acc[p & 3];
      const float s1 = FMT == 1 ? scale1[i] : 1.0f, s2 = FMT == 1 ? scale2[j] : 1.0f;
      const float nq = row_sqnorm<FMT>(q) * s1 * s1, nw = row_sqnorm<FMT>(w) * s2 * s2;
      const double s = (double)dot * (double)s1 * (double)s2;
      out[t] = (float)((double)nq + (double)nw - 2.0 * s);
    }
  }
}

}  // namespace

hipError_t launch_pair_distances(int fmt, const void* desc1, const void* desc2,
                                 const float* scale1, const float* scale2, const int64_t* qi,
                                 const int64_t* kj, int64_t count, float* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const dim3 grid((unsigned)((count + 15) / 16));
  if (fmt == 0)
    hipLaunchKernelGGL((k_pair_distances<0>), grid, dim3(kWave), 0, s, desc1, desc2, scale1, scale2,
                       qi, kj, count, out);
  else if (fmt == 1)
    hipLaunchKernelGGL((k_pair_distances<1>), grid, dim3(kWave), 0, s, desc1, desc2, scale1, scale2,
                       qi, kj, count, out);
  else
    hipLaunchKernelGGL((k_pair_distances<-1>), grid, dim3(kWave), 0, s, desc1, desc2, scale1,
                       scale2, qi, kj, count, out);
  return hipGetLastError();
}

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
