// Learned per-keypoint tolerance (the paper's future-work item of Sec. 6):
// a 6 -> 64 -> 64 -> 1 ReLU network maps image-2 keypoint attributes to
// eps_j = clamp(softplus(z), 0.5, 8) px, trained with a pinball (quantile)
// loss on point-line residuals (Eq. 3) of the method's own matches.
//
//   k_eps_features   per keypoint: (scale, response, orientation, x^, y^,
//                    log1p(min(|p - e2| / diag, 1000)))
//   k_eps_infer      BF16 weights (rounded on the device from the FP32
//                    masters), FP32 activations and accumulation
//   k_eps_grad       FP32 forward + backward of a minibatch; every workgroup
//                    owns a fixed slice of the batch and writes its partial
//                    gradient, so the sums have a fixed order
//   k_eps_reduce     partial gradients summed over workgroups in order
//   k_eps_adam       Adam update, one thread per parameter
//   k_residuals      point-line distance (FP64, same evaluation as the
//                    candidate test) of each query's selected match
//
// Parameter vector (4673 floats): W1 [64][6], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3; matrices row-major with one row per output unit.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kIn = 6, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH,
              kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH;
constexpr int kParams = kOffB3 + 1;
static_assert(kParams == kEpsParams, "parameter layout");
constexpr float kEpsMin = 0.5f, kEpsMax = 8.0f;
constexpr double kDistClip = 1000.0;

__device__ __forceinline__ float softplus_f(float z) {
  return z > 0.0f ? z + log1pf(expf(-z)) : log1pf(expf(z));
}

__device__ __forceinline__ float sigmoid_f(float z) {
  return z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
}

// float -> nearest bfloat16 (ties to even), as a float
__device__ __forceinline__ float bf16_round(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(r);
}

// ---------------------------------------------------------------- features
constexpr int kFeatThreads = 256;

__global__ __launch_bounds__(kFeatThreads) void k_eps_features(const EpsPair* __restrict__ pairs,
                                                               const int64_t* __restrict__ kstart,
                                                               int num_pairs, int64_t n2,
                                                               const float* __restrict__ kp2,
                                                               const float* __restrict__ attrs,
                                                               float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * kFeatThreads + threadIdx.x;
  if (j >= n2) return;
  const EpsPair P = pairs[find_pair(kstart, num_pairs, j)];
  const double x = kp2[2 * j], y = kp2[2 * j + 1];
  double rel = kDistClip;
  if (P.finite) {
    const double d = hypot(x - P.ex, y - P.ey);
    rel = fmin(d / P.diag, kDistClip);
  }
  const double half = 0.5 * P.w;
  float* o = out + 6 * j;
  o[0] = attrs[3 * j];
  o[1] = attrs[3 * j + 1];
  o[2] = attrs[3 * j + 2];
  o[3] = (float)((x - half) / half);
  o[4] = (float)((y - 0.5 * P.h) / half);
  o[5] = (float)log1p(rel);
}

// --------------------------------------------------------------- inference
constexpr int kInferThreads = 256;

__global__ __launch_bounds__(kInferThreads) void k_eps_infer(const float* __restrict__ feat,
                                                             int64_t n,
                                                             const float* __restrict__ params,
                                                             float* __restrict__ eps) {
  __shared__ float w[kParams];
  for (int p = threadIdx.x; p < kParams; p += kInferThreads) w[p] = bf16_round(params[p]);
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kInferThreads + threadIdx.x;
  if (j >= n) return;
  float x[kIn];
  #pragma unroll
  for (int c = 0; c < kIn; ++c) x[c] = feat[kIn * j + c];
  float h1[kH];
  #pragma unroll
  for (int u = 0; u < kH; ++u) {
    float a = w[kOffB1 + u];
    #pragma unroll
    for (int c = 0; c < kIn; ++c) a = fmaf(w[kOffW1 + u * kIn + c], x[c], a);
    h1[u] = fmaxf(a, 0.0f);
  }
  float z = w[kOffB3];
  for (int r = 0; r < kH; ++r) {
    float a = w[kOffB2 + r];
    #pragma unroll
    for (int c = 0; c < kH; ++c) a = fmaf(w[kOffW2 + r * kH + c], h1[c], a);
    z = fmaf(w[kOffW3 + r], fmaxf(a, 0.0f), z);
  }
  eps[j] = fminf(fmaxf(softplus_f(z), kEpsMin), kEpsMax);
}

// ---------------------------------------------------------------- training
// 256 threads = 64 samples x 4 quarters of the hidden units per pass.
constexpr int kGradThreads = 256;
constexpr int kPass = 64;
constexpr int kQuarter = kH / 4;
constexpr int kOwn = (kParams + kGradThreads - 1) / kGradThreads;  // parameters per thread
constexpr int kLd = kH + 1;  // padded row of the per-sample buffers

__global__ __launch_bounds__(kGradThreads) void k_eps_grad(EpsGradArgs A) {
  __shared__ float w[kParams];
  __shared__ float xs[kPass][kIn];
  __shared__ float h1s[kPass][kLd], h2s[kPass][kLd], d1s[kPass][kLd], d2s[kPass][kLd];
  __shared__ float dzs[kPass], ls[kPass];
  const int tid = threadIdx.x;
  for (int p = tid; p < kParams; p += kGradThreads) w[p] = A.params[p];
  const int s = tid >> 2, k = tid & 3;
  const int u0 = k * kQuarter;
  const int64_t chunk = (A.batch + gridDim.x - 1) / gridDim.x;
  const int64_t begin = (int64_t)blockIdx.x * chunk;
  const int64_t end = begin + chunk < A.batch ? begin + chunk : A.batch;
  float acc[kOwn];
  #pragma unroll
  for (int t = 0; t < kOwn; ++t) acc[t] = 0.0f;
  float loss_acc = 0.0f;
  __syncthreads();

  for (int64_t base = begin; base < end; base += kPass) {
    const int64_t sid = base + s;
    bool valid = sid < end;
    float x[kIn] = {0, 0, 0, 0, 0, 0};
    float y = 0.0f;
    if (valid) {
      // indices outside the caller's arrays make the sample count as absent
      const int64_t slot = A.sample_idx[sid];
      const int64_t fi = slot >= 0 && slot < A.num_slots ? (A.feat_index ? A.feat_index[slot] : slot)
                                                         : -1;
      valid = fi >= 0 && fi < A.num_rows;
      if (valid) {
        #pragma unroll
        for (int c = 0; c < kIn; ++c) x[c] = A.features[kIn * fi + c];
        y = A.target[slot];
      }
    }
    if (k == 0) {
      #pragma unroll
      for (int c = 0; c < kIn; ++c) xs[s][c] = x[c];
    }
    // layer 1, this thread's 16 units
    #pragma unroll
    for (int i = 0; i < kQuarter; ++i) {
      const int u = u0 + i;
      float a = w[kOffB1 + u];
      #pragma unroll
      for (int c = 0; c < kIn; ++c) a = fmaf(w[kOffW1 + u * kIn + c], x[c], a);
      h1s[s][u] = fmaxf(a, 0.0f);
    }
    __syncthreads();
    // layer 2 and this thread's share of z
    float zp = 0.0f;
    #pragma unroll 1
    for (int i = 0; i < kQuarter; ++i) {
      const int r = u0 + i;
      float a = w[kOffB2 + r];
      #pragma unroll 8
      for (int c = 0; c < kH; ++c) a = fmaf(w[kOffW2 + r * kH + c], h1s[s][c], a);
      const float h = fmaxf(a, 0.0f);
      h2s[s][r] = h;
      zp = fmaf(w[kOffW3 + r], h, zp);
    }
    // the four quarters of a sample are adjacent lanes
    float z = zp + __shfl_xor(zp, 1);
    z = z + __shfl_xor(z, 2);
    z += w[kOffB3];
    const float yhat = softplus_f(z);
    const float uu = y - yhat;
    float dz = 0.0f, li = 0.0f;
    if (valid) {
      li = uu >= 0.0f ? A.q * uu : (A.q - 1.0f) * uu;
      const float dyhat = (yhat >= y ? 1.0f - A.q : -A.q) * A.inv_batch;
      dz = dyhat * sigmoid_f(z);
    }
    for (int i = 0; i < kQuarter; ++i) {
      const int r = u0 + i;
      d2s[s][r] = h2s[s][r] > 0.0f ? dz * w[kOffW3 + r] : 0.0f;
    }
    if (k == 0) {
      dzs[s] = dz;
      ls[s] = li;
    }
    __syncthreads();
    // back through layer 2
    #pragma unroll 1
    for (int i = 0; i < kQuarter; ++i) {
      const int u = u0 + i;
      float g = 0.0f;
      #pragma unroll 8
      for (int r = 0; r < kH; ++r) g = fmaf(w[kOffW2 + r * kH + u], d2s[s][r], g);
      d1s[s][u] = h1s[s][u] > 0.0f ? g : 0.0f;
    }
    __syncthreads();
    // this workgroup's sums, samples in order
    #pragma unroll
    for (int t = 0; t < kOwn; ++t) {
      const int p = tid + t * kGradThreads;
      if (p >= kParams) break;
      float a = acc[t];
      if (p < kOffB1) {
        const int r = p / kIn, c = p % kIn;
        #pragma unroll 8
        for (int q = 0; q < kPass; ++q) a = fmaf(d1s[q][r], xs[q][c], a);
      } else if (p < kOffW2) {
        const int r = p - kOffB1;
        for (int q = 0; q < kPass; ++q) a += d1s[q][r];
      } else if (p < kOffB2) {
        const int r = (p - kOffW2) / kH, c = (p - kOffW2) % kH;
        #pragma unroll 8
        for (int q = 0; q < kPass; ++q) a = fmaf(d2s[q][r], h1s[q][c], a);
      } else if (p < kOffW3) {
        const int r = p - kOffB2;
        for (int q = 0; q < kPass; ++q) a += d2s[q][r];
      } else if (p < kOffB3) {
        const int r = p - kOffW3;
        for (int q = 0; q < kPass; ++q) a = fmaf(dzs[q], h2s[q][r], a);
      } else {
        for (int q = 0; q < kPass; ++q) a += dzs[q];
      }
      acc[t] = a;
    }
    if (tid == 0)
      for (int q = 0; q < kPass; ++q) loss_acc += ls[q];
    __syncthreads();
  }
  float* out = A.partials + (int64_t)blockIdx.x * (kParams + 1);
  #pragma unroll
  for (int t = 0; t < kOwn; ++t) {
    const int p = tid + t * kGradThreads;
    if (p < kParams) out[p] = acc[t];
  }
  if (tid == 0) out[kParams] = loss_acc;
}

__global__ void k_eps_reduce(const float* __restrict__ partials, int blocks, float inv_batch,
                             float* __restrict__ grad, float* __restrict__ loss) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p > kParams) return;
  float a = 0.0f;
  for (int b = 0; b < blocks; ++b) a += partials[(int64_t)b * (kParams + 1) + p];
  if (p < kParams) grad[p] = a;
  else if (loss) *loss = a * inv_batch;
}

__global__ void k_eps_adam(float* __restrict__ theta, float* __restrict__ m,
                           float* __restrict__ v, const float* __restrict__ grad, float lr,
                           float beta1, float beta2, float eps, float c1, float c2) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= kParams) return;
  const float g = grad[p];
  const float mm = beta1 * m[p] + (1.0f - beta1) * g;
  const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// --------------------------------------------------------------- residuals
__global__ __launch_bounds__(256) void k_residuals(const PairDev* __restrict__ pairs,
                                                   const int64_t* __restrict__ qstart,
                                                   int num_pairs, int64_t n1,
                                                   const float* __restrict__ kp1,
                                                   const float* __restrict__ kp2,
                                                   const int32_t* __restrict__ best,
                                                   float* __restrict__ residual,
                                                   int64_t* __restrict__ feat_index) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n1) return;
  const PairDev& pd = pairs[find_pair(qstart, num_pairs, i)];
  const int32_t j = best[i];
  if (j < 0 || j >= pd.n) {
    residual[i] = -1.0f;
    if (feat_index) feat_index[i] = -1;
    return;
  }
  double a, b, c;
  epipolar_line(pd.F, kp1[2 * i], kp1[2 * i + 1], a, b, c);
  const int64_t g = pd.k_begin + j;
  const double num = fabs(__dadd_rn(__dadd_rn(__dmul_rn(a, (double)kp2[2 * g]),
                                              __dmul_rn(b, (double)kp2[2 * g + 1])), c));
  const double den = __dsqrt_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b)));
  residual[i] = (float)__ddiv_rn(num, den);
  if (feat_index) feat_index[i] = g;
}

}  // namespace

hipError_t launch_eps_features(const EpsPair* pairs, const int64_t* kstart, int num_pairs,
                               int64_t n2, const float* kp2, const float* attrs, float* out,
                               hipStream_t s) {
  if (n2 == 0) return hipSuccess;
  const int64_t blocks = (n2 + kFeatThreads - 1) / kFeatThreads;
  hipLaunchKernelGGL(k_eps_features, dim3((unsigned)blocks), dim3(kFeatThreads), 0, s, pairs,
                     kstart, num_pairs, n2, kp2, attrs, out);
  return hipGetLastError();
}

hipError_t launch_eps_infer(const float* feat, int64_t n, const float* params, float* eps,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + kInferThreads - 1) / kInferThreads;
  hipLaunchKernelGGL(k_eps_infer, dim3((unsigned)blocks), dim3(kInferThreads), 0, s, feat, n,
                     params, eps);
  return hipGetLastError();
}

int eps_grad_blocks(int64_t batch) {
  const int64_t b = (batch + kPass - 1) / kPass;
  return (int)(b < kEpsGradMaxBlocks ? (b > 0 ? b : 1) : kEpsGradMaxBlocks);
}

hipError_t launch_eps_grad(const EpsGradArgs& a, float* grad, float* loss, hipStream_t s) {
  const int blocks = eps_grad_blocks(a.batch);
  hipLaunchKernelGGL(k_eps_grad, dim3(blocks), dim3(kGradThreads), 0, s, a);
  hipLaunchKernelGGL(k_eps_reduce, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, a.partials,
                     blocks, a.inv_batch, grad, loss);
  return hipGetLastError();
}

hipError_t launch_eps_adam(float* theta, float* m, float* v, const float* grad, float lr,
                           float beta1, float beta2, float eps, float c1, float c2,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_eps_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, theta, m, v, grad,
                     lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_residuals(const PairDev* pairs, const int64_t* qstart, int num_pairs,
                            int64_t n1, const float* kp1, const float* kp2, const int32_t* best,
                            float* residual, int64_t* feat_index, hipStream_t s) {
  if (n1 == 0) return hipSuccess;
  const int64_t blocks = (n1 + 255) / 256;
  hipLaunchKernelGGL(k_residuals, dim3((unsigned)blocks), dim3(256), 0, s, pairs, qstart,
                     num_pairs, n1, kp1, kp2, best, residual, feat_index);
  return hipGetLastError();
}

}  // namespace epm
