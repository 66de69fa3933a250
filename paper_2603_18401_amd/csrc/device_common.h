// Device helpers shared by the libepm kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "epm_internal.h"

namespace epm {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This maps dispatch order to a logical tile order in which groups of
// kXcdGroup consecutive logical tiles -- neighbouring angle ranges that share
// candidates -- run on one XCD, while successive groups rotate over the XCDs
// so uneven work stays balanced.  A bijection of [0, n): the tail that does
// not fill a whole round of groups keeps the identity order.
constexpr int kNumXcd = 8;
constexpr int kXcdGroup = 16;
__device__ __forceinline__ int xcd_tile(int block, int n) {
  constexpr int round = kNumXcd * kXcdGroup;
  const int full = (n / round) * round;
  if (block >= full) return block;
  const int x = block % kNumXcd, k = block / kNumXcd;
  const int g = k / kXcdGroup, o = k % kXcdGroup;
  return (g * kNumXcd + x) * kXcdGroup + o;
}

// XCD that xcd_tile gives tile t: the inverse of the mapping above, mod 8.
__device__ __forceinline__ int xcd_of_tile(int t, int n) {
  constexpr int round = kNumXcd * kXcdGroup;
  const int full = (n / round) * round;
  return t >= full ? t % kNumXcd : (t / kXcdGroup) % kNumXcd;
}

// Cost bucket of the longest-first orders: 0 for no work, else two buckets
// per power of two (the bit below the leading one splits an octave).
__device__ __forceinline__ int cost_bucket(uint32_t c) {
  if (c == 0) return 0;
  const int msb = 31 - __clz(c);
  const int half = msb > 0 ? (int)((c >> (msb - 1)) & 1u) : 0;
  return 1 + 2 * msb + half;
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Last pair p with starts[p] <= idx (pairs own contiguous, ordered slices).
__device__ __forceinline__ int find_pair(const int64_t* __restrict__ starts, int num_pairs,
                                         int64_t idx) {
  int lo = 0, hi = num_pairs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= idx) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Eq. 2: the epipolar line of (x, y), every product and sum rounded once,
// left to right -- the same operations as the definition of the candidate set.
__device__ __forceinline__ void epipolar_line(const double* __restrict__ F, float xf, float yf,
                                              double& a, double& b, double& c) {
  const double x = (double)xf, y = (double)yf;
  a = __dadd_rn(__dadd_rn(__dmul_rn(F[0], x), __dmul_rn(F[1], y)), F[2]);
  b = __dadd_rn(__dadd_rn(__dmul_rn(F[3], x), __dmul_rn(F[4], y)), F[5]);
  c = __dadd_rn(__dadd_rn(__dmul_rn(F[6], x), __dmul_rn(F[7], y)), F[8]);
}

// sqrt(a^2 + b^2) of a line, correctly rounded (the denominator of Eq. 3).
__device__ __forceinline__ double line_norm(double a, double b) {
  return __dsqrt_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b)));
}

// Eq. 3-4 multiplied through by sqrt(a^2 + b^2): the only FP64 step of the
// per-candidate path.  Closed boundary.  nrm = line_norm(a, b), computed once
// per query; the decision is the same bit for bit as with the norm inline.
__device__ __forceinline__ bool within_tolerance_d(double a, double b, double c, double nrm,
                                                   double x, double y, double e) {
  const double num = fabs(__dadd_rn(__dadd_rn(__dmul_rn(a, x), __dmul_rn(b, y)), c));
  return num <= __dmul_rn(e, nrm);
}

// (x, y, eps) are FP32 inputs widened exactly.
__device__ __forceinline__ bool within_tolerance_n(double a, double b, double c, double nrm,
                                                   float xf, float yf, float ef) {
  return within_tolerance_d(a, b, c, nrm, (double)xf, (double)yf, (double)ef);
}

__device__ __forceinline__ bool within_tolerance(double a, double b, double c, float xf,
                                                 float yf, float ef) {
  return within_tolerance_n(a, b, c, line_norm(a, b), xf, yf, ef);
}

// Circular distance between two angle keys (mod 2^32 == mod pi).
__device__ __forceinline__ uint32_t key_distance(uint32_t p, uint32_t c) {
  const uint32_t d = p - c;
  const uint32_t e = c - p;
  return d < e ? d : e;
}

__device__ __forceinline__ int width_class(uint32_t half) {
  const int c = 32 - __clz(half);
  return c > kWideClass ? kWideClass : c;
}

// First index in [lo, hi) whose key is >= target (keys ascending); the whole
// wavefront cooperates, every lane gets the result.
__device__ __forceinline__ int64_t wave_lower_bound(const uint32_t* __restrict__ keys,
                                                    int64_t lo, int64_t hi, uint32_t target) {
  const int lane = lane_id();
  while (hi - lo > kWave) {
    const int64_t len = hi - lo;
    // 64 probes splitting [lo, hi) into 65 parts
    const int64_t pos = lo + (len * (lane + 1)) / (kWave + 1);
    const bool below = keys[pos] < target;
    const uint64_t m = ballot(below);
    const int cnt = __popcll(m);  // probes are ascending: a prefix is below
    const int64_t nlo = cnt == 0 ? lo : lo + (len * cnt) / (kWave + 1) + 1;
    const int64_t nhi = cnt == kWave ? hi : lo + (len * (cnt + 1)) / (kWave + 1) + 1;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  const int64_t pos = lo + lane;
  const bool below = pos < hi && keys[pos] < target;
  return lo + __popcll(ballot(below));
}

}  // namespace epm
