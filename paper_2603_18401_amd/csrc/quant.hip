// Storage formats of the reduced-precision matching path: FP32 descriptor
// rows to BF16 (round to nearest even) or to OCP FP8-E4M3FN codes with one
// FP32 scale per row (s = amax / 448, 1 for an all-zero row; code =
// round-to-nearest-even of x / s, saturated at 448).  One wavefront per row.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr float kFp8Max = 448.0f;

__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;  // NaN
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits; subnormals step 2^-9
__device__ __forceinline__ uint8_t to_e4m3(float v) {
  const uint32_t sign = __float_as_uint(v) >> 31;
  const float a = fminf(fabsf(v), kFp8Max);
  uint32_t code;
  if (a < 0.015625f) {  // 2^-6: subnormal range (8 encodes the smallest normal)
    code = (uint32_t)rintf(a * 512.0f);
  } else {
    const uint32_t ua = __float_as_uint(a);
    int e = (int)(ua >> 23) - 127;
    const uint32_t m = ua & 0x7FFFFFu;
    uint32_t keep = m >> 20;
    const uint32_t rem = m & 0xFFFFFu;
    if (rem > 0x80000u || (rem == 0x80000u && (keep & 1u))) ++keep;
    if (keep == 8u) {
      keep = 0u;
      ++e;
    }
    code = ((uint32_t)(e + 7) << 3) | keep;
    if (code > 0x7Eu) code = 0x7Eu;  // 448, the largest finite value
  }
  return (uint8_t)(code | (sign << 7));
}

__device__ __forceinline__ float wave_max(float v) {
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

__global__ __launch_bounds__(kThreads) void k_quant_bf16(const float* __restrict__ src,
                                                         int64_t n, uint16_t* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    dst[i] = to_bf16(src[i]);
}

__global__ __launch_bounds__(kThreads) void k_quant_fp8(const float* __restrict__ src,
                                                        int64_t rows, int dim,
                                                        uint8_t* __restrict__ dst,
                                                        float* __restrict__ scale) {
  const int lane = lane_id();
  for (int64_t r = (int64_t)blockIdx.x * kWaves + wave_id(); r < rows;
       r += (int64_t)gridDim.x * kWaves) {
    const float* x = src + r * dim;
    float amax = 0.0f;
    for (int k = lane; k < dim; k += kWave) amax = fmaxf(amax, fabsf(x[k]));
    amax = wave_max(amax);
    float s = amax / kFp8Max;
    if (!(s > 0.0f)) s = 1.0f;
    for (int k = lane; k < dim; k += kWave) dst[r * dim + k] = to_e4m3(x[k] / s);
    if (lane == 0) scale[r] = s;
  }
}

// Norm of each row's rounding error, err[r] >= |x_r - dequant(code_r)|
// (FP64 sums, inflated by 1e-6 for their rounding): the tight per-row term
// that the reduced-precision bounds can use in place of the format's
// worst case.  One wavefront per row.
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_round_err(const float* __restrict__ src,
                                                        int64_t rows, int dim,
                                                        const void* __restrict__ codes,
                                                        const float* __restrict__ scale,
                                                        float* __restrict__ err) {
  const int lane = lane_id();
  for (int64_t r = (int64_t)blockIdx.x * kWaves + wave_id(); r < rows;
       r += (int64_t)gridDim.x * kWaves) {
    double acc = 0.0;
    const double s = FMT == 1 ? (double)scale[r] : 1.0;
    for (int k = lane; k < dim; k += kWave) {
      double y;
      if (FMT == 0) {
        y = (double)__uint_as_float((uint32_t)static_cast<const uint16_t*>(codes)[r * dim + k] << 16);
      } else {
        const uint32_t c = static_cast<const uint8_t*>(codes)[r * dim + k];
        const uint32_t e = (c >> 3) & 15u, m = c & 7u;
        double v = e == 0 ? (double)m * 0.001953125
                          : (double)__uint_as_float(((e + 120u) << 23) | (m << 20));
        y = ((c & 0x80u) ? -v : v) * s;
      }
      const double d = (double)src[r * dim + k] - y;
      acc += d * d;
    }
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) err[r] = (float)(sqrt(acc) * (1.0 + 1e-6)) + 1e-30f;
  }
}

}  // namespace

hipError_t launch_round_err(const float* src, int64_t rows, int dim, int fmt, const void* codes,
                            const float* scale, float* err, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  int64_t blocks = (rows + kWaves - 1) / kWaves;
  if (blocks > 65536) blocks = 65536;
  if (fmt == 0)
    hipLaunchKernelGGL((k_round_err<0>), dim3((unsigned)blocks), dim3(kThreads), 0, s, src, rows,
                       dim, codes, scale, err);
  else
    hipLaunchKernelGGL((k_round_err<1>), dim3((unsigned)blocks), dim3(kThreads), 0, s, src, rows,
                       dim, codes, scale, err);
  return hipGetLastError();
}

hipError_t launch_quantize(const float* src, int64_t rows, int dim, int fmt, void* dst,
                           float* scale, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  if (fmt == 0) {
    const int64_t n = rows * dim;
    int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_quant_bf16, dim3((unsigned)blocks), dim3(kThreads), 0, s, src, n,
                       static_cast<uint16_t*>(dst));
  } else {
    int64_t blocks = (rows + kWaves - 1) / kWaves;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_quant_fp8, dim3((unsigned)blocks), dim3(kThreads), 0, s, src, rows,
                       dim, static_cast<uint8_t*>(dst), scale);
  }
  return hipGetLastError();
}

}  // namespace epm
