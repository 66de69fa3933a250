// Angular intervals of the image-2 tolerance circles and the angle keys of
// the image-1 epipolar lines.
//
// Sec. 4.1-4.2 (Eq. 5-6): seen from the epipole, the circle of radius eps_j
// around p_j subtends the interval of line directions between its two
// tangents.  The kernels express line directions in a pencil basis (u, v) of
// the lines through the epipole e (u, v, e orthonormal in normalised line
// space), which covers a finite epipole inside or outside the image and an
// epipole at infinity with one formula: the pencil line at angle phi is
// l(phi) = cos(phi) u + sin(phi) v, and p_j lies within eps of it iff
//     (w_j . c)^2 <= eps^2 c^T G c,   c = (cos phi, sin phi),
// with w_j = (u . p~_j, v . p~_j) and G the Gram matrix of (u_12, v_12).
// The solution set is the arc around the eigenvector of the negative
// eigenvalue of M_j = w_j w_j^T - eps^2 G, half-width atan(sqrt(-l-/l+));
// with an orthonormal basis of a finite epipole this is theta_j +- delta_j of
// Eq. 5-6.  A circle containing the epipole gives a negative semidefinite
// M_j: the full interval (Sec. 4.4).  Angles are stored mod pi as u32 keys,
// which makes the 0/pi wrap-around implicit.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

__device__ __forceinline__ uint32_t angle_key(double phi) {
  // phi in [0, pi) -> round(phi * 2^32 / pi) mod 2^32
  const double k = nearbyint(phi * kKeyPerRad);
  const uint64_t u = (uint64_t)(int64_t)k;
  return (uint32_t)u;
}

// Conservative interval of one keypoint: centre key and half-width key.
__device__ void circle_interval(const PairDev& pd, float xf, float yf, float ef, uint32_t& C,
                                uint32_t& H) {
  if (pd.kappa < 0.0) {  // no pencil: the pair's queries scan every record
    C = 0;
    H = kFullHalf;
    return;
  }
  const double px = pd.s * ((double)xf - pd.cx);
  const double py = pd.s * ((double)yf - pd.cy);
  const double w1 = pd.u[0] * px + pd.u[1] * py + pd.u[2];
  const double w2 = pd.v[0] * px + pd.v[1] * py + pd.v[2];
  const double ep = fabs(pd.e[0] * px + pd.e[1] * py + pd.e[2]);
  // tolerance in normalised units, inflated by the rounding slack and by the
  // largest line-to-epipole miss a query may have before it scans the pair
  double epsn = pd.s * ((double)ef * (1.0 + kEpsRelSlack) + kEpsAbsSlackPx);
  epsn += pd.kappa * (epsn * pd.e12 + ep);
  const double e2 = epsn * epsn;
  const double A = w1 * w1 - e2 * pd.G11;
  const double B = w1 * w2 - e2 * pd.G12;
  const double D = w2 * w2 - e2 * pd.G22;
  const double detG = pd.G11 * pd.G22 - pd.G12 * pd.G12;
  const double wadj = pd.G22 * w1 * w1 - 2.0 * pd.G12 * w1 * w2 + pd.G11 * w2 * w2;
  const double det = e2 * (e2 * detG - wadj);  // det M without cancellation
  if (!(det < 0.0)) {
    // both eigenvalues <= 0: the circle holds the epipole, every line hits it
    // (a positive definite M cannot occur; it is also treated as full)
    C = 0;
    H = kFullHalf;
    return;
  }
  const double half = 0.5 * (A - D);
  const double disc = sqrt(half * half + B * B);
  const double lp = 0.5 * (A + D) + disc;  // > 0
  const double lm = det / lp;              // < 0
  double vx, vy;                           // eigenvector of lp
  if (A >= D) {
    vx = half + disc;
    vy = B;
  } else {
    vx = B;
    vy = disc - half;
  }
  // interval centre: the eigenvector of lm, (-vy, vx)
  double psi = atan2(vx, -vy);
  if (psi < 0.0) psi += M_PI;
  if (psi >= M_PI) psi -= M_PI;
  const double h = atan(sqrt(-lm / lp));
  const double hk = ceil(h * kKeyPerRad) + (double)kGuard;
  if (!(hk < (double)(kFullHalf - 2 * kGuard))) {
    C = 0;
    H = kFullHalf;
    return;
  }
  C = angle_key(psi);
  H = (uint32_t)hk;
}

}  // namespace

// ------------------------------------------------------------ pair setup
// Algorithm 1, preprocessing, on the device: the image-2 epipole e2 = null(F^T)
// in normalised line coordinates and an orthonormal basis (u, v) of the
// pencil of lines through it, from F in device memory (one thread per pair).
// The normalisation (s, cx, cy from the image size) and the slices are kept
// from the pair record.  A pair without a pencil (F non-finite, zero, or of
// rank <= 1) gets kappa = -1: its queries are then tested against every
// keypoint of the pair, which keeps the result exact.
__device__ __forceinline__ void dcross(const double* a, const double* b, double* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dnorm3(const double* a) {
  return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

__device__ bool pencil_of(PairDev& pd) {
  const double* F = pd.F;
  double fn = 0.0;
  for (int k = 0; k < 9; ++k) {
    if (!isfinite(F[k])) return false;
    fn += F[k] * F[k];
  }
  if (!(fn > 0.0) || !isfinite(fn)) return false;
  // M = N F T^-1 (lines in normalised image-2 coordinates as functions of
  // normalised image-1 coordinates), scaled to a largest entry of 1
  double M[3][3];
  const double is = 1.0 / pd.s;
  double mx = 0.0;
  for (int r = 0; r < 3; ++r) {
    double NF[3];
    for (int k = 0; k < 3; ++k)
      NF[k] = r == 0 ? F[k] : r == 1 ? F[3 + k] : pd.s * (F[k] * pd.cx + F[3 + k] * pd.cy + F[6 + k]);
    // T^-1 = [[1/s, 0, cx], [0, 1/s, cy], [0, 0, 1]]
    M[r][0] = NF[0] * is;
    M[r][1] = NF[1] * is;
    M[r][2] = NF[0] * pd.cx + NF[1] * pd.cy + NF[2];
    for (int k = 0; k < 3; ++k) mx = fmax(mx, fabs(M[r][k]));
  }
  if (!(mx > 0.0) || !isfinite(mx)) return false;
  double col[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) col[k][d] = M[d][k] / mx;
  // the left null vector is orthogonal to every column: the largest cross
  // product of two columns
  double best[3] = {0.0, 0.0, 0.0}, bn = 0.0;
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int t = 0; t < 3; ++t) {
    double cr[3];
    dcross(col[pa[t]], col[pb[t]], cr);
    const double cn = dnorm3(cr);
    if (cn > bn) {
      bn = cn;
      for (int d = 0; d < 3; ++d) best[d] = cr[d];
    }
  }
  if (!(bn > 1e-12)) return false;
  for (int d = 0; d < 3; ++d) pd.e[d] = best[d] / bn;
  int ax = 0;
  for (int d = 1; d < 3; ++d)
    if (fabs(pd.e[d]) < fabs(pd.e[ax])) ax = d;
  double axis[3] = {0.0, 0.0, 0.0};
  axis[ax] = 1.0;
  dcross(pd.e, axis, pd.u);
  const double un = dnorm3(pd.u);
  for (int d = 0; d < 3; ++d) pd.u[d] /= un;
  dcross(pd.e, pd.u, pd.v);
  const double vn = dnorm3(pd.v);
  for (int d = 0; d < 3; ++d) pd.v[d] /= vn;
  pd.G11 = pd.u[0] * pd.u[0] + pd.u[1] * pd.u[1];
  pd.G12 = pd.u[0] * pd.v[0] + pd.u[1] * pd.v[1];
  pd.G22 = pd.v[0] * pd.v[0] + pd.v[1] * pd.v[1];
  pd.e12 = sqrt(pd.e[0] * pd.e[0] + pd.e[1] * pd.e[1]);
  pd.kappa = kKappaBuild;
  return true;
}

__global__ __launch_bounds__(64) void k_pair_setup(PairDev* __restrict__ pairs,
                                                   const double* __restrict__ F, int num_pairs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= num_pairs) return;
  PairDev pd = pairs[p];
  for (int k = 0; k < 9; ++k) pd.F[k] = F[9 * (int64_t)p + k];
  if (!pencil_of(pd)) {
    // no pencil: every query scans its pair, every record is a full interval
    for (int d = 0; d < 3; ++d) pd.u[d] = pd.v[d] = pd.e[d] = 0.0;
    pd.G11 = pd.G12 = pd.G22 = pd.e12 = 0.0;
    pd.kappa = -1.0;
  }
  pairs[p] = pd;
}

constexpr int kRadixDigits = 256;  // digits of one 8-bit radix pass

// Per-tile digit counts of the first radix pass of the keys this workgroup
// wrote (tile blockIdx.x), and zero counts for the next zero_passes passes:
// the segmented sort then starts with its scatter.
__device__ __forceinline__ void first_pass_counts(uint32_t* h, uint32_t* __restrict__ hist,
                                                  int num_tiles, int zero_passes) {
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid >= kRadixDigits) return;
  hist[(int64_t)blockIdx.x * kRadixDigits + tid] = h[tid];
  for (int p = 1; p <= zero_passes; ++p)
    hist[((int64_t)p * num_tiles + blockIdx.x) * kRadixDigits + tid] = 0u;
}

// One workgroup per record sort tile (kSortTile keypoints of one pair, one
// per thread).
__global__ __launch_bounds__(kSortTile) void k_intervals(
    const PairDev* __restrict__ pairs, const SortTile* __restrict__ tiles, int num_tiles,
    const float* __restrict__ kp2, const float* __restrict__ eps2, float eps_scalar,
    uint32_t* __restrict__ sort_key, uint32_t* __restrict__ sort_val, uint32_t* __restrict__ recC,
    uint32_t* __restrict__ recH, uint32_t* __restrict__ hist, int zero_passes) {
  __shared__ uint32_t h[kRadixDigits];
  if (threadIdx.x < kRadixDigits) h[threadIdx.x] = 0u;
  __syncthreads();
  const SortTile t = tiles[blockIdx.x];
  const PairDev& pd = pairs[t.seg];
  for (int k = threadIdx.x; k < t.count; k += kSortTile) {
    const int64_t r = t.begin + k;
    const float xf = kp2[2 * r], yf = kp2[2 * r + 1];
    const float ef = eps2 ? eps2[r] : eps_scalar;
    uint32_t C = 0, H = kFullHalf;
    // keypoints the interval formula cannot describe are always scanned and
    // left to the exact test
    if (ef > 0.0f && isfinite(ef) && isfinite(xf) && isfinite(yf))
      circle_interval(pd, xf, yf, ef, C, H);
    const uint32_t cls = (uint32_t)width_class(H);
    const uint32_t key = (cls << kCentreBits) | (C >> kCentreShift);
    sort_key[r] = key;
    sort_val[r] = (uint32_t)r;
    recC[r] = C;
    recH[r] = H;
    atomicAdd(&h[key & (kRadixDigits - 1)], 1u);
  }
  first_pass_counts(h, hist, num_tiles, zero_passes);
}

// Eq. 2 and Eq. 7: the angle of each query's epipolar line in the pencil,
// reduced mod pi (an undirected line).
// One workgroup per query sort tile (kSortTile queries of one pair, one per
// thread).
__global__ __launch_bounds__(kSortTile) void k_query_keys(
    const PairDev* __restrict__ pairs, const SortTile* __restrict__ tiles, int num_tiles,
    const float* __restrict__ kp1, uint32_t* __restrict__ qkey, uint32_t* __restrict__ qflag,
    uint32_t* __restrict__ sort_key, uint32_t* __restrict__ sort_val,
    double4* __restrict__ qline, uint32_t* __restrict__ hist, int zero_passes,
    unsigned long long* __restrict__ stats, uint32_t* __restrict__ sched,
    unsigned long long* __restrict__ match_stats) {
  __shared__ uint32_t h[kRadixDigits];
  if (threadIdx.x < kRadixDigits) h[threadIdx.x] = 0u;
  if (blockIdx.x == 0) {  // the query's counters start from zero
    if (stats && threadIdx.x < kNumStats) stats[threadIdx.x] = 0ull;
    if (match_stats && threadIdx.x < kMatchStatWords) match_stats[threadIdx.x] = 0ull;
    if (sched)
      for (int k = (int)threadIdx.x; k < kSchedWords; k += (int)blockDim.x) sched[k] = 0u;
  }
  __syncthreads();
  const SortTile t = tiles[blockIdx.x];
  const PairDev& pd = pairs[t.seg];
  for (int kk = threadIdx.x; kk < t.count; kk += kSortTile) {
    const int64_t i = t.begin + kk;
    double a, b, c;
    epipolar_line(pd.F, kp1[2 * i], kp1[2 * i + 1], a, b, c);
    uint32_t flag = kQueryNormal, key = 0;
    if (a == 0.0 && b == 0.0) {
      flag = kQueryEmpty;
    } else if (!isfinite(a) || !isfinite(b) || !isfinite(c)) {
      flag = kQueryBrute;
    } else {
      // the same line in normalised image-2 coordinates (scaled by 1/s)
      const double l3 = pd.s * (a * pd.cx + b * pd.cy + c);
      const double lam = pd.u[0] * a + pd.u[1] * b + pd.u[2] * l3;
      const double mu = pd.v[0] * a + pd.v[1] * b + pd.v[2] * l3;
      const double nu = pd.e[0] * a + pd.e[1] * b + pd.e[2] * l3;
      const double n1c = lam * pd.u[0] + mu * pd.v[0];
      const double n2c = lam * pd.u[1] + mu * pd.v[1];
      const double nrm = sqrt(n1c * n1c + n2c * n2c);
      if (pd.kappa < 0.0 || !(fabs(nu) <= pd.kappa * nrm)) {
        flag = kQueryBrute;  // the line misses the epipole by more than absorbed
      } else {
        double phi = atan2(mu, lam);
        if (phi < 0.0) phi += M_PI;
        if (phi >= M_PI) phi -= M_PI;
        key = angle_key(phi);
      }
    }
    qkey[i] = key;
    qflag[i] = flag;
    sort_key[i] = key >> (32 - kQuerySortBits);
    sort_val[i] = (uint32_t)i;
    // the line and its norm for the tile passes (the denominator of Eq. 3)
    qline[i] = flag == kQueryEmpty ? make_double4(0.0, 0.0, 0.0, 0.0)
                                   : make_double4(a, b, c, line_norm(a, b));
    atomicAdd(&h[(key >> (32 - kQuerySortBits)) & (kRadixDigits - 1)], 1u);
  }
  first_pass_counts(h, hist, num_tiles, zero_passes);
}

// Sorted layout: structure-of-arrays in angle order, plus the inverse
// permutation (record -> sorted position).
__global__ __launch_bounds__(256) void k_gather_records(
    const int64_t* __restrict__ kstart, int num_pairs, int64_t n2,
    const uint32_t* __restrict__ sorted_val, const float* __restrict__ kp2,
    const float* __restrict__ eps2, float eps_scalar, const uint32_t* __restrict__ recC,
    const uint32_t* __restrict__ recH, uint32_t* __restrict__ rC, uint32_t* __restrict__ rH,
    int32_t* __restrict__ rj, float2* __restrict__ rxy, float* __restrict__ reps,
    uint32_t* __restrict__ rinv, const uint32_t* __restrict__ digit_base,
    int64_t* __restrict__ class_begin) {
  // blocks of neighbouring sorted positions run on one XCD (xcd_tile): the
  // scattered reads and rinv writes of a pair's records then meet in one L2
  const int64_t pos = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
  if (digit_base && pos < (int64_t)num_pairs * kClassSlots) {
    // the start of width class c of pair p: the last radix pass's digit
    // (class, top centre bits) starts, as the sort left them
    const int p = (int)(pos / kClassSlots), c = (int)(pos % kClassSlots);
    class_begin[pos] = c == kNumClasses
                           ? kstart[p + 1]
                           : (int64_t)digit_base[(int64_t)p * 256 + (c << (kSortBits - 16 - kClassBits))];
  }
  if (pos >= n2) return;
  const uint32_t r = sorted_val[pos];
  const int p = find_pair(kstart, num_pairs, (int64_t)r);
  rC[pos] = recC[r];
  rH[pos] = recH[r];
  rj[pos] = (int32_t)((int64_t)r - kstart[p]);
  rxy[pos] = make_float2(kp2[2 * (int64_t)r], kp2[2 * (int64_t)r + 1]);
  reps[pos] = eps2 ? eps2[r] : eps_scalar;
  rinv[r] = (uint32_t)pos;
}

// Start of every width class inside each pair's sorted segment.
__global__ __launch_bounds__(64) void k_class_bounds(const int64_t* __restrict__ kstart,
                                                     const uint32_t* __restrict__ skey,
                                                     int64_t* __restrict__ class_begin) {
  const int p = blockIdx.x;
  const int64_t lo = kstart[p], hi = kstart[p + 1];
  const int c = lane_id();
  // every lane runs the same cooperative search for its own class in turn
  for (int cc = 0; cc < kClassSlots; ++cc) {
    const int64_t b = cc == kNumClasses ? hi : wave_lower_bound(skey, lo, hi, (uint32_t)cc << kCentreBits);
    if (c == 0) class_begin[(int64_t)p * kClassSlots + cc] = b;
  }
}

hipError_t launch_pair_setup(PairDev* pairs, const double* F, int num_pairs, hipStream_t s) {
  if (num_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_setup, dim3((unsigned)((num_pairs + 63) / 64)), dim3(64), 0, s, pairs,
                     F, num_pairs);
  return hipGetLastError();
}

hipError_t launch_intervals(const PairDev* pairs, const SortTile* tiles, int num_tiles,
                            const float* kp2, const float* eps2, float eps_scalar,
                            uint32_t* sort_key, uint32_t* sort_val, uint32_t* recC,
                            uint32_t* recH, uint32_t* hist, int zero_passes, hipStream_t s) {
  if (num_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_intervals, dim3((unsigned)num_tiles), dim3(kSortTile), 0, s, pairs,
                     tiles, num_tiles, kp2, eps2, eps_scalar, sort_key, sort_val, recC, recH,
                     hist, zero_passes);
  return hipGetLastError();
}

hipError_t launch_query_keys(const PairDev* pairs, const SortTile* tiles, int num_tiles,
                             const float* kp1, uint32_t* qkey, uint32_t* qflag,
                             uint32_t* sort_key, uint32_t* sort_val, double4* qline,
                             uint32_t* hist, int zero_passes, unsigned long long* stats,
                             uint32_t* sched, unsigned long long* match_stats, hipStream_t s) {
  if (num_tiles == 0) return launch_clear_stats(stats, s, sched, match_stats);
  hipLaunchKernelGGL(k_query_keys, dim3((unsigned)num_tiles), dim3(kSortTile), 0, s, pairs,
                     tiles, num_tiles, kp1, qkey, qflag, sort_key, sort_val, qline, hist,
                     zero_passes, stats, sched, match_stats);
  return hipGetLastError();
}

hipError_t launch_gather_records(const int64_t* kstart, int num_pairs, int64_t n2,
                                 const uint32_t* sorted_val, const float* kp2, const float* eps2,
                                 float eps_scalar, const uint32_t* recC, const uint32_t* recH,
                                 uint32_t* rC, uint32_t* rH, int32_t* rj, float2* rxy,
                                 float* reps, uint32_t* rinv, const uint32_t* digit_base,
                                 int64_t* class_begin, hipStream_t s) {
  if (n2 == 0) return hipSuccess;
  const int64_t items = n2 > (int64_t)num_pairs * kClassSlots ? n2 : (int64_t)num_pairs * kClassSlots;
  const int64_t blocks = (items + 255) / 256;
  hipLaunchKernelGGL(k_gather_records, dim3((unsigned)blocks), dim3(256), 0, s, kstart,
                     num_pairs, n2, sorted_val, kp2, eps2, eps_scalar, recC, recH, rC, rH, rj,
                     rxy, reps, rinv, digit_base, class_begin);
  return hipGetLastError();
}

hipError_t launch_class_bounds(const int64_t* kstart, int num_pairs, const uint32_t* skey,
                               int64_t* class_begin, hipStream_t s) {
  if (num_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_class_bounds, dim3(num_pairs), dim3(64), 0, s, kstart, skey, class_begin);
  return hipGetLastError();
}

}  // namespace epm
