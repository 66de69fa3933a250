// Rounding bounds of the reduced-precision descriptor formats and the
// certified lower bound on a canonical FP32 distance that the MFMA scores
// give (Sec. 4.3 selection, exact final results).  Shared by the window and
// wide-row MFMA kernels.
#pragma once

#include <hip/hip_fp16.h>

#include "device_common.h"
#include "match_common.h"

namespace epm {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

template <int FMT>
struct Fmt;
template <>
struct Fmt<0> {  // BF16: 8 significant bits, round to nearest even
  static constexpr int kRowBytes = 256;
  static constexpr double kUnit = 1.0 / 256.0;  // |x^ - x| <= u |x|
  static constexpr double kAbs = 0.0;
  __device__ static float decode(const uint8_t* row, int k) {
    const uint16_t h = reinterpret_cast<const uint16_t*>(row)[k];
    return __uint_as_float((uint32_t)h << 16);
  }
};
template <>
struct Fmt<1> {  // OCP E4M3FN with a per-row scale: 4 significant bits
  static constexpr int kRowBytes = 128;
  static constexpr double kUnit = 1.0 / 16.0;
  static constexpr double kAbs = 1.0 / 1024.0;  // half the subnormal spacing, times scale
  __device__ static float decode(const uint8_t* row, int k) {
    const uint32_t c = row[k];
    const uint32_t e = (c >> 3) & 15u, m = c & 7u;
    float v = e == 0 ? (float)m * 0.001953125f : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return (c & 0x80u) ? -v : v;
  }
};
// LDS row stride: 16 extra bytes start consecutive rows 4 banks apart, so the
// 16-byte (BF16) or 8-byte (FP8) fragment reads of 16 rows are conflict free.
template <int FMT>
constexpr int row_stride() { return Fmt<FMT>::kRowBytes + 16; }

__device__ __forceinline__ float exact_distance(const float4* __restrict__ a,
                                                const float4* __restrict__ b) {
  float acc = 0.0f;
  #pragma unroll 8
  for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, a[k], b[k]);
  return acc;
}

// Squared norm of a quantised row in LDS, k ascending, read 16 bytes at a time.
template <int FMT>
__device__ __forceinline__ float row_sqnorm(const uint8_t* row) {
  constexpr int kElemBytes = Fmt<FMT>::kRowBytes / 128;  // 2 (BF16) or 1 (FP8)
  constexpr int kPer = 16 / kElemBytes;                    // elements per 16 bytes
  static_assert(kPer * kElemBytes == 16 && 128 % kPer == 0, "row layout");
  float n = 0.0f;
  #pragma unroll 1
  for (int c = 0; c < 128 / kPer; ++c) {
    const uint4 w = reinterpret_cast<const uint4*>(row)[c];
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    #pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int byte = k * kElemBytes;
      const uint32_t bits = words[byte >> 2] >> ((byte & 3) * 8);
      float x;
      if (FMT == 0) {
        x = __uint_as_float((bits & 0xFFFFu) << 16);
      } else {
        const uint8_t code = (uint8_t)(bits & 0xFFu);
        x = Fmt<FMT>::decode(&code, 0);
      }
      n = __builtin_fmaf(x, x, n);
    }
  }
  return n;
}

// Quantisation error bound of a row from its quantised norm:
// |x^ - x|_2 <= (u |x^| + a s sqrt(128)) / (1 - u), slightly inflated.
template <int FMT>
__device__ __forceinline__ double row_delta(double norm_hat, double scale) {
  const double u = Fmt<FMT>::kUnit;
  return (u * norm_hat + Fmt<FMT>::kAbs * scale * 11.313708498984761) / (1.0 - u) *
         (1.0 + 1e-6) + 1e-30;
}

// Lower bound on the exact canonical FP32 distance of a candidate whose
// approximate squared distance is dt (norms are of the quantised rows):
//   |dt - |q^ - w^|^2| <= em = 3e-5 (|q^| + |w^|)^2   (FP32 accumulation),
//   | |q^ - w^| - |q - w| | <= dq + dw,
//   canonical >= (1 - 1e-5) |q - w|^2               (130 roundings of 2^-24).
__device__ __forceinline__ double lower_bound(double dt, double nq, double nw, double dq,
                                              double dw) {
  const double s = nq + nw;
  const double em = 3e-5 * s * s;
  const double root = sqrt(fmax(dt - em, 0.0));
  const double r = fmax(root - (dq + dw), 0.0);
  return (1.0 - 1e-5) * r * r;
}

// Upper bound on the exact canonical FP32 distance (the counterpart of
// lower_bound): |q - w| <= sqrt(dt + em) + dq + dw, canonical <= (1 + 1e-5) |q - w|^2.
__device__ __forceinline__ double upper_bound(double dt, double nq, double nw, double dq,
                                              double dw) {
  const double s = nq + nw;
  const double em = 3e-5 * s * s;
  const double r = sqrt(fmax(dt + em, 0.0)) + (dq + dw);
  return (1.0 + 1e-5) * r * r;
}

// Non-negative float to the nearest IEEE half at or below it (down) or at or
// above it (up); NaN gives 0 (down) and +inf (up).
__device__ __forceinline__ uint32_t half_down(float x) {
  if (!(x > 0.0f)) return 0u;
  uint32_t h = (uint32_t)__half_as_ushort(__float2half_rn(x));
  if (__half2float(__ushort_as_half((unsigned short)h)) > x) h -= 1u;
  return h;
}
__device__ __forceinline__ uint32_t half_up(float x) {
  if (!(x >= 0.0f)) return x < 0.0f ? 0u : 0x7C00u;
  uint32_t h = (uint32_t)__half_as_ushort(__float2half_rn(x));
  if (h < 0x7C00u && __half2float(__ushort_as_half((unsigned short)h)) < x) h += 1u;
  return h;
}
__device__ __forceinline__ float half_value(uint32_t h) {
  return __half2float(__ushort_as_half((unsigned short)(h & 0xFFFFu)));
}

}  // namespace epm
