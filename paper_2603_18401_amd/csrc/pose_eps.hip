// Per-keypoint tolerance from the uncertainty of the relative pose (the
// paper's noise experiment widens one tolerance for all keypoints; Sec. 6
// names per-keypoint tolerances as future work).
//
// With the pose theta = (w, tau) around its estimate -- R = Exp([w]x) R0,
// t = t0 + tau -- of covariance Sigma, the signed distance of Eq. 3,
//     d(theta; x1, x2) = x2^T F(theta) x1 / |(F(theta) x1)_12|,
// of an image-2 keypoint x2 from the epipolar line of its image-1 partner x1
// spreads to first order by s^2 = g^T Sigma g, g = grad_theta d at 0.  The
// partner lies on the reverse epipolar line F^T x2 inside image 1 and, with a
// scene depth range, is the projection of the point seen at x2 at a depth in
// that range; the keypoint's tolerance covers k standard deviations at the
// worst of 16 such partners -- inverse depths evenly spaced over the range,
// else points evenly spaced over the segment:
// eps_j = min(eps0 + k max s, eps_max).
// The derivatives of F are exact (dF/dw_k = K2^-T [t]x [e_k]x R K1^-1,
// dF/dtau_k = K2^-T [e_k]x R K1^-1, from the host), the rest FP64.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kPoseSamples = 16;

__device__ __forceinline__ void mat3_vec(const double* M, double x, double y, double* out) {
  out[0] = M[0] * x + M[1] * y + M[2];
  out[1] = M[3] * x + M[4] * y + M[5];
  out[2] = M[6] * x + M[7] * y + M[8];
}

// g^T Sigma g at image-1 point (x, y) for image-2 keypoint (u, v); -1 where
// the epipolar line of (x, y) has no direction.
__device__ double spread_at(const PosePair& P, double x, double y, double u, double v) {
  double l[3];
  mat3_vec(P.F0, x, y, l);
  const double n = hypot(l[0], l[1]);
  if (!(n > 1e-12 * P.fmax)) return -1.0;
  const double N = l[0] * u + l[1] * v + l[2];
  double g[6];
  for (int k = 0; k < 6; ++k) {
    double lk[3];
    mat3_vec(P.dF[k], x, y, lk);
    const double Nk = lk[0] * u + lk[1] * v + lk[2];
    const double nk = (l[0] * lk[0] + l[1] * lk[1]) / n;
    g[k] = Nk / n - N * nk / (n * n);  // derivative of N / n
  }
  double s2 = 0.0;
  for (int r = 0; r < 6; ++r) {
    double row = 0.0;
    for (int k = 0; k < 6; ++k) row += P.cov[6 * r + k] * g[k];
    s2 += g[r] * row;
  }
  return s2;
}

// Largest spread over the partners of the depth range; -1 when none of them
// lies in front of camera 1 and inside image 1.
__device__ double depth_spread(const PosePair& P, double u, double v) {
  double ray[3];
  mat3_vec(P.K2i, u, v, ray);
  double best = -1.0;
  for (int s = 0; s < kPoseSamples; ++s) {
    const double rho = P.rho_lo + (P.rho_hi - P.rho_lo) * s / (kPoseSamples - 1);
    const double d[3] = {ray[0] - rho * P.t[0], ray[1] - rho * P.t[1], ray[2] - rho * P.t[2]};
    double X[3];
    for (int r = 0; r < 3; ++r) X[r] = P.Rt[3 * r] * d[0] + P.Rt[3 * r + 1] * d[1] + P.Rt[3 * r + 2] * d[2];
    if (!(X[2] > 0.0)) continue;
    double p[3];
    for (int r = 0; r < 3; ++r) p[r] = P.K1[3 * r] * X[0] + P.K1[3 * r + 1] * X[1] + P.K1[3 * r + 2] * X[2];
    const double x = p[0] / p[2], y = p[1] / p[2];
    if (!(x >= 0.0 && x <= P.w1 && y >= 0.0 && y <= P.h1)) continue;
    const double s2 = spread_at(P, x, y, u, v);
    if (s2 >= 0.0) best = fmax(best, s2);
  }
  return best;
}

// Largest spread over the sample points of the reverse epipolar segment.
__device__ double segment_spread(const PosePair& P, double u, double v) {
  const double* F = P.F0;
  // reverse epipolar line F^T x2 in image 1
  const double a = F[0] * u + F[3] * v + F[6];
  const double b = F[1] * u + F[4] * v + F[7];
  const double c = F[2] * u + F[5] * v + F[8];
  // its part inside [0, w1] x [0, h1]: the farthest pair of border crossings
  double px[4], py[4];
  int np = 0;
  if (b != 0.0) {
    for (int s = 0; s < 2; ++s) {
      const double x = s ? P.w1 : 0.0, y = -(a * x + c) / b;
      if (y >= 0.0 && y <= P.h1) { px[np] = x; py[np] = y; ++np; }
    }
  }
  if (a != 0.0) {
    for (int s = 0; s < 2; ++s) {
      const double y = s ? P.h1 : 0.0, x = -(b * y + c) / a;
      if (x >= 0.0 && x <= P.w1) { px[np] = x; py[np] = y; ++np; }
    }
  }
  double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0, far = 0.0;
  int S = 1;
  for (int i = 0; i < np; ++i)
    for (int j = i + 1; j < np; ++j) {
      const double d = hypot(px[i] - px[j], py[i] - py[j]);
      if (d > far) { far = d; ax = px[i]; ay = py[i]; bx = px[j]; by = py[j]; S = kPoseSamples; }
    }
  if (S == 1) {  // the line misses the image: its point nearest the centre
    const double cx = 0.5 * P.w1, cy = 0.5 * P.h1;
    const double t = (a * cx + b * cy + c) / (a * a + b * b);
    ax = cx - a * t;
    ay = cy - b * t;
  }
  double best = 0.0;
  for (int s = 0; s < S; ++s) {
    const double x = S == 1 ? ax : ax + (bx - ax) * s / (S - 1);
    const double y = S == 1 ? ay : ay + (by - ay) * s / (S - 1);
    best = fmax(best, spread_at(P, x, y, u, v));
  }
  return best;
}

__global__ __launch_bounds__(256) void k_pose_eps(const PosePair* __restrict__ pairs,
                                                  const int64_t* __restrict__ kstart,
                                                  int num_pairs, int64_t n2,
                                                  const float* __restrict__ kp2, float eps0,
                                                  float k_sigma, float eps_max,
                                                  float* __restrict__ eps2) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n2) return;
  const int p = find_pair(kstart, num_pairs, j);
  const PosePair& P = pairs[p];
  const double u = kp2[2 * j], v = kp2[2 * j + 1];
  double s2 = P.rho_hi > 0.0 ? depth_spread(P, u, v) : -1.0;
  if (s2 < 0.0) s2 = segment_spread(P, u, v);
  const double e = (double)eps0 + (double)k_sigma * sqrt(s2);
  eps2[j] = (float)fmin(e, (double)eps_max);
}

}  // namespace

hipError_t launch_pose_eps(const PosePair* pairs, const int64_t* kstart, int num_pairs,
                           int64_t n2, const float* kp2, float eps0, float k_sigma,
                           float eps_max, float* eps2, hipStream_t s) {
  if (n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pose_eps, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, pairs,
                     kstart, num_pairs, n2, kp2, eps0, k_sigma, eps_max, eps2);
  return hipGetLastError();
}

}  // namespace epm
