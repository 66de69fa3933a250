// Stabbing query (Sec. 4.2, Algorithm 1 match loop): every query's angle key
// is tested against the angle-sorted intervals of its pair; each angular hit
// is confirmed by the FP64 point-line test (Eq. 3), so the rows are exactly
// the candidate sets of Eq. 4.
//
// One wavefront per query, queries taken in angle order so that neighbouring
// wavefronts read neighbouring windows.  For width class c the only centres
// that can hold the key lie within 2^c - 1 key units of it; the window is
// found with a cooperative 64-way search and scanned 64 records at a time,
// one lane per record.  Hits are compacted with a ballot and a lane prefix
// count.  The count pass writes the row lengths; the fill pass repeats the
// scan, gathers the hits in LDS, sorts them by j and writes the CSR row.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

// Bitonic sort of one value per lane, ascending over the wavefront.
__device__ __forceinline__ int32_t wave_sort64(int32_t v) {
  const int lane = lane_id();
  #pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
    #pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int32_t o = __shfl_xor(v, j);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const int32_t mn = v < o ? v : o, mx = v < o ? o : v;
      v = (lower == up) ? mn : mx;
    }
  }
  return v;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort of buf[0..len) (len a power of two, 128..kRowSortMax) by one
// wavefront.
__device__ void wave_sort_lds(int32_t* buf, int len) {
  const int lane = lane_id();
  for (int k = 2; k <= len; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < len / 2; t += kWave) {
        // comparator t: element pair (lo, lo + j)
        const int lo = ((t / j) * 2 * j) + (t % j);
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const int32_t a = buf[lo], b = buf[hi];
        if ((a > b) == up) {
          buf[lo] = b;
          buf[hi] = a;
        }
      }
      wave_sync_lds();
    }
  }
}

struct QueryCtx {
  double a, b, c;
  uint32_t key;
  bool brute;
};

// Scans sorted records [r0, r1): returns the number of hits; in the fill
// pass appends the hit image-2 indices to buf (up to kRowSortMax).
template <bool FILL>
__device__ __forceinline__ uint32_t scan_range(const StabArgs& A, const QueryCtx& q, int64_t r0,
                                               int64_t r1, int32_t* buf, uint32_t total) {
  const int lane = lane_id();
  for (int64_t base = r0; base < r1; base += kWave) {
    const int64_t pos = base + lane;
    bool hit = false;
    if (pos < r1) {
      const uint32_t C = A.rC[pos], H = A.rH[pos];
      if (q.brute || key_distance(q.key, C) <= H) {
        const float2 xy = A.rxy[pos];
        hit = within_tolerance(q.a, q.b, q.c, xy.x, xy.y, A.reps[pos]);
      }
    }
    const uint64_t m = ballot(hit);
    if (FILL && hit) {
      const uint32_t slot = total + lanes_below(m);
      if (slot < (uint32_t)kRowSortMax) buf[slot] = A.rj[pos];
    }
    total += (uint32_t)__popcll(m);
  }
  return total;
}

template <bool FILL>
__device__ uint32_t stab_query(const StabArgs& A, const PairDev& pd, int pair, const QueryCtx& q,
                               int32_t* buf) {
  const int64_t* cb = A.class_begin + (int64_t)pair * kClassSlots;
  uint32_t total = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    const int64_t beg = cb[c], end = cb[c + 1];
    if (beg == end) continue;
    if (q.brute || c == kWideClass) {
      total = scan_range<FILL>(A, q, beg, end, buf, total);
      continue;
    }
    const uint32_t span = (1u << c) - 1u;
    const uint32_t lo = q.key - span, hi = q.key + span;
    const uint32_t cls = (uint32_t)c << kCentreBits;
    const uint32_t blo = cls | (lo >> kCentreShift), bhi = cls | (hi >> kCentreShift);
    if (lo <= hi) {
      const int64_t r0 = wave_lower_bound(A.skey, beg, end, blo);
      const int64_t r1 = wave_lower_bound(A.skey, r0, end, bhi + 1u);
      total = scan_range<FILL>(A, q, r0, r1, buf, total);
    } else {
      // the window wraps through angle 0 == pi
      const int64_t r0 = wave_lower_bound(A.skey, beg, end, blo);
      total = scan_range<FILL>(A, q, r0, end, buf, total);
      const int64_t r1 = wave_lower_bound(A.skey, beg, r0, bhi + 1u);
      total = scan_range<FILL>(A, q, beg, r1, buf, total);
    }
  }
  return total;
}

template <bool FILL>
__global__ __launch_bounds__(kThreads) void k_stab(StabArgs A) {
  __shared__ int32_t rowbuf[FILL ? kWaves : 1][FILL ? kRowSortMax : 1];
  const int lane = lane_id(), wave = wave_id();
  const int64_t qs = (int64_t)blockIdx.x * kWaves + wave;
  if (qs >= A.n1) return;
  const int64_t i = A.qperm ? (int64_t)A.qperm[qs] : qs;
  const int pair = find_pair(A.qstart, A.num_pairs, i);
  const PairDev& pd = A.pairs[pair];
  const uint32_t flag = A.qflag[i];
  int32_t* buf = rowbuf[FILL ? wave : 0];

  if (!FILL) {
    uint32_t total = 0;
    if (flag != kQueryEmpty) {
      QueryCtx q;
      epipolar_line(pd.F, A.kp1[2 * i], A.kp1[2 * i + 1], q.a, q.b, q.c);
      q.key = A.qkey[i];
      q.brute = flag == kQueryBrute;
      total = stab_query<false>(A, pd, pair, q, buf);
    }
    if (lane == 0) A.counts[i] = total;
    return;
  }

  const int64_t o0 = A.row_offsets[i];
  const int64_t len = A.row_offsets[i + 1] - o0;
  if (len == 0 || flag == kQueryEmpty) return;
  QueryCtx q;
  epipolar_line(pd.F, A.kp1[2 * i], A.kp1[2 * i + 1], q.a, q.b, q.c);
  q.key = A.qkey[i];
  q.brute = flag == kQueryBrute;

  if (len > kRowSortMax) {
    // long row: rebuild it in ascending j directly from the definition
    const int64_t kb = pd.k_begin;
    uint32_t total = 0;
    for (int64_t j0 = 0; j0 < pd.n; j0 += kWave) {
      const int64_t j = j0 + lane;
      bool hit = false;
      if (j < pd.n) {
        const uint32_t pos = A.rinv[kb + j];
        const float2 xy = A.rxy[pos];
        hit = within_tolerance(q.a, q.b, q.c, xy.x, xy.y, A.reps[pos]);
      }
      const uint64_t m = ballot(hit);
      const int64_t dst = o0 + total + lanes_below(m);
      if (hit && dst < A.capacity) A.cols[dst] = (int32_t)j;
      total += (uint32_t)__popcll(m);
    }
    return;
  }

  const uint32_t total = stab_query<true>(A, pd, pair, q, buf);
  wave_sync_lds();
  const int n = (int)(total < (uint32_t)len ? total : (uint32_t)len);
  if (n <= kWave) {
    const int32_t v = wave_sort64(lane < n ? buf[lane] : INT32_MAX);
    if (lane < n && o0 + lane < A.capacity) A.cols[o0 + lane] = v;
  } else {
    int p2 = 128;
    while (p2 < n) p2 <<= 1;
    for (int t = n + lane; t < p2; t += kWave) buf[t] = INT32_MAX;
    wave_sync_lds();
    wave_sort_lds(buf, p2);
    for (int t = lane; t < n; t += kWave)
      if (o0 + t < A.capacity) A.cols[o0 + t] = buf[t];
  }
}

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int64_t o = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += o;
    __syncthreads();
  }
  const int64_t incl = sh[tid];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(const uint32_t* __restrict__ counts,
                                                                int64_t n,
                                                                int64_t* __restrict__ partials) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (idx < n) s += counts[idx];
  }
  int64_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t* __restrict__ partials,
                                                           int64_t nb) {
  __shared__ int64_t sh[kScanThreads];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int64_t idx = b0 + threadIdx.x;
    const int64_t v = idx < nb ? partials[idx] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, sh, &tot);
    if (idx < nb) partials[idx] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) partials[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_final(const uint32_t* __restrict__ counts,
                                                             int64_t n,
                                                             const int64_t* __restrict__ partials,
                                                             int64_t nb,
                                                             int64_t* __restrict__ offsets) {
  __shared__ int64_t sh[kScanThreads];
  // thread t owns items [base + t*kScanItems, +kScanItems): blocked order
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? counts[base + k] : 0u;
    s += v[k];
  }
  int64_t tot;
  int64_t run = partials[blockIdx.x] + block_exclusive_scan(s, sh, &tot);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) offsets[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) offsets[n] = partials[nb];
}

}  // namespace

hipError_t launch_stab_count(const StabArgs& a, hipStream_t s) {
  if (a.n1 == 0) return hipSuccess;
  const int64_t blocks = (a.n1 + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k_stab<false>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stab_fill(const StabArgs& a, hipStream_t s) {
  if (a.n1 == 0) return hipSuccess;
  const int64_t blocks = (a.n1 + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k_stab<true>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

int64_t scan_partials_count(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan_counts(const uint32_t* counts, int64_t n, int64_t* offsets,
                              int64_t* partials, hipStream_t s) {
  if (n == 0) {
    // offsets[0] = 0 is written by the caller
    return hipSuccess;
  }
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, n,
                     partials);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, n,
                     partials, nb, offsets);
  return hipGetLastError();
}

}  // namespace epm
