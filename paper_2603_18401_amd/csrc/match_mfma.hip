// Reduced-precision descriptor matching with exact final results (Sec. 4.3).
//
// Descriptors stored as BF16 or as OCP FP8-E4M3 with a per-row FP32 scale are
// compared on MFMA (dense query-tile x window-row score blocks, FP32
// accumulation); the FP32 masters are used only for the exact distances of a
// few candidates.  Per workgroup (one angle tile of 64 queries):
//   1. the tile's CSR rows are mapped to window indices (as in the FP32 window
//      kernel);
//   2. quantised query rows and, chunk by chunk, quantised window rows are
//      staged in LDS; S = Q W^T on v_mfma_f32_16x16x32_{bf16,fp8_fp8};
//   3. every candidate gets certified bounds LB <= D <= UB on its exact
//      canonical FP32 distance D from the approximate distance
//      |q^|^2 + |w^|^2 - 2 s S and the format's rounding bound, kept as two
//      outward-rounded halves in the candidate's 32-bit list entry;
//   4. with U2 the second smallest UB of a row, two candidates have D <= U2,
//      so a candidate with LB > U2 is neither best nor second: every other
//      candidate of the row is evaluated exactly on the masters (all threads
//      over the tile's entries) and the row's top-2 is taken over those;
//   5. rows that do not fit the tile's dense list of 8192 entries are
//      evaluated exactly by gathers -- counted in the match statistics.
// Final outputs therefore equal the FP32 path bit for bit, with no separate
// certificate: the bounds only decide which candidates need exact distances.
#include "device_common.h"
#include "launch.h"
#include "match_common.h"
#include "mfma_bounds.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kChunkRows = 64;
constexpr int kMaxPairs = 8192;  // dense (query, candidate) entries per tile
constexpr uint32_t kPending = kEntPending;
constexpr uint32_t kNoWindow = kEntNoWindow;

template <int FMT, bool PERSIST>
__global__ __launch_bounds__(kThreads) void k_match_window_mfma(MatchArgs A) {
  constexpr int RS = row_stride<FMT>();
  // the query rows, and after the last MFMA the list of exact distances to take
  constexpr int kQBytes = kTileQ * RS > kMaxPairs * 2 ? kTileQ * RS : kMaxPairs * 2;
  __shared__ __attribute__((aligned(16))) uint8_t qrows[kQBytes];
  constexpr int kScoreBytes = kTileQ * (kChunkRows + 1) * 4;
  constexpr int kWBytes = kChunkRows * RS > kScoreBytes ? kChunkRows * RS : kScoreBytes;
  __shared__ __attribute__((aligned(16))) uint8_t wrows[kWBytes];
  __shared__ uint32_t ent[kMaxPairs];
  __shared__ uint32_t slot_b[kSlots], slot_pref[kSlots + 1];
  __shared__ uint32_t ss_b[kSlots], ss_v[kSlots], ss_len[kSlots];
  __shared__ int64_t q_i[kTileQ], q_o0[kTileQ];
  __shared__ uint32_t q_k[kTileQ], q_off[kTileQ + 1], q_in[kTileQ];
  __shared__ float q_norm[kTileQ], q_scale[kTileQ], w_norm[kChunkRows], w_scale[kChunkRows];
  // per-row terms of the bound: inflated norm and quantisation error bound
  __shared__ double q_nb[kTileQ], q_db[kTileQ], w_nb[kChunkRows], w_db[kChunkRows];
  __shared__ int32_t row_j[kChunkRows];
  __shared__ uint32_t n_sorted_slots;
  __shared__ float4 qdesc[kWaves][32];
  __shared__ float lb5[kTileQ];  // the second smallest upper bound of each row
  __shared__ uint32_t wave_total[kWaves];

  __shared__ int next_tile;
  if (csr_overflow(A)) return;
  // one tile per workgroup, or (persistent) tiles from the queue until it is
  // exhausted; every workgroup leaves once the counter passes the last tile
  for (int iter = 0;; ++iter) {
    int tile;
    if (PERSIST) {
      if (threadIdx.x == 0) next_tile = (int)atomicAdd(A.queue, 1u);
      __syncthreads();
      const int t = next_tile;
      if (t >= A.num_tiles) break;
      tile = A.order ? (int)A.order[t] : t;
    } else {
      if (iter > 0) break;
      tile = A.block_tile ? (int)A.block_tile[blockIdx.x] : xcd_tile(blockIdx.x, A.num_tiles);
    }
    if (A.skip_tiles && A.skip_tiles[tile]) {  // matched by the wide-row pass
      if (PERSIST) __syncthreads();            // next_tile is read before it is rewritten
      continue;
    }
    const StabTile T = A.tiles[tile];
    const int64_t kb = A.kstart[T.pair];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    const TileWindow* W = A.windows + tile;
    const uint8_t* d1 = reinterpret_cast<const uint8_t*>(A.desc1);
    const uint8_t* d2 = reinterpret_cast<const uint8_t*>(A.desc2);
    constexpr int RB = Fmt<FMT>::kRowBytes;

    if (wave == 0) {
      const int q = lane;
      int64_t i = 0, o0 = 0, k = 0;
      if (q < T.count) {
        i = (int64_t)A.qperm[T.begin + q];
        o0 = A.row_offsets[i];
        k = A.row_offsets[i + 1] - o0;
      }
      q_i[q] = i;
      q_o0[q] = o0;
      q_k[q] = (uint32_t)k;
      // rows enter the dense list in order while they fit; the rest are
      // evaluated by gathers
      uint32_t incl = (uint32_t)(k < kMaxPairs ? k : kMaxPairs);
      #pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      const bool fits = incl <= (uint32_t)kMaxPairs;
      const uint64_t fit_mask = ballot(fits);
      // the fitting rows are a prefix: recompute the offsets over that prefix
      const int nfit = __popcll(fit_mask);
      uint32_t kk = lane < nfit ? (uint32_t)k : 0u;
      incl = kk;
      #pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      q_off[q + 1] = incl;
      q_in[q] = lane < nfit ? 1u : 0u;
      if (lane == 0) q_off[0] = 0;
      const uint32_t b = W->slot_b[lane];
      const uint32_t p0 = W->slot_pref[lane], p1 = W->slot_pref[lane + 1];
      slot_b[lane] = b;
      slot_pref[lane] = p0;
      if (lane == 0) slot_pref[kSlots] = W->slot_pref[kSlots];
      const bool nonempty = p1 > p0;
      const uint64_t ne = ballot(nonempty);
      uint32_t rank = 0;
      for (int s = 0; s < kWave; ++s) {
        const uint32_t bs = __builtin_amdgcn_readlane(b, s);
        if (((ne >> s) & 1ull) && (bs < b || (bs == b && s < lane))) ++rank;
      }
      if (nonempty) {
        ss_b[rank] = b;
        ss_v[rank] = p0;
        ss_len[rank] = p1 - p0;
      }
      if (lane == 0) n_sorted_slots = (uint32_t)__popcll(ne);
    }
    __syncthreads();

    // quantised query rows (zero rows past the tile end), their norms and scales
    for (int f = tid; f < kTileQ * (RB / 16); f += kThreads) {
      const int q = f / (RB / 16), c = f % (RB / 16);
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < T.count) v = reinterpret_cast<const uint4*>(d1 + q_i[q] * RB)[c];
      *reinterpret_cast<uint4*>(qrows + q * RS + c * 16) = v;
    }
    // dense (query, candidate, window index) list
    const uint32_t npairs = q_off[kTileQ];
    const uint32_t nss = n_sorted_slots;
    build_dense_list<kThreads>(A, kb, npairs, q_off, q_o0, ss_b, ss_v, ss_len, nss, ent, nullptr,
                               tid);
    __syncthreads();
    if (tid < kTileQ) {
      const float n = row_sqnorm<FMT>(qrows + tid * RS);
      const float s = (FMT == 1 && tid < T.count) ? A.scale1[q_i[tid]] : 1.0f;
      q_scale[tid] = s;
      q_norm[tid] = n * s * s;  // squared norm of the dequantised row
      const double nb = sqrt((double)q_norm[tid]) * (1.0 + 1e-5);
      q_nb[tid] = nb;
      q_db[tid] = A.qerr1 && tid < T.count ? (double)A.qerr1[q_i[tid]] : row_delta<FMT>(nb, s);
    }

    const uint32_t wlen = slot_pref[kSlots];
    float* score = reinterpret_cast<float*>(wrows);  // reused after the MFMA reads
    for (uint32_t c0 = 0; c0 < wlen; c0 += kChunkRows) {
      const uint32_t nr = wlen - c0 < (uint32_t)kChunkRows ? wlen - c0 : (uint32_t)kChunkRows;
      for (uint32_t r = tid; r < kChunkRows; r += kThreads) {
        int32_t j = -1;
        if (r < nr) {
          const uint32_t v = c0 + r;
          uint32_t s = 0;
          #pragma unroll
          for (int step = 32; step > 0; step >>= 1)
            if (s + step <= kSlots && slot_pref[s + step] <= v) s += step;
          j = A.rj[slot_b[s] + (v - slot_pref[s])];
        }
        row_j[r] = j;
      }
      __syncthreads();
      for (int f = tid; f < kChunkRows * (RB / 16); f += kThreads) {
        const int r = f / (RB / 16), c = f % (RB / 16);
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row_j[r] >= 0) v = reinterpret_cast<const uint4*>(d2 + (kb + row_j[r]) * RB)[c];
        *reinterpret_cast<uint4*>(wrows + r * RS + c * 16) = v;
      }
      __syncthreads();
      if (tid < kChunkRows) {
        const float n = row_sqnorm<FMT>(wrows + tid * RS);
        const float s = (FMT == 1 && row_j[tid] >= 0) ? A.scale2[kb + row_j[tid]] : 1.0f;
        w_scale[tid] = s;
        w_norm[tid] = n * s * s;
        const double nb = sqrt((double)w_norm[tid]) * (1.0 + 1e-5);
        w_nb[tid] = nb;
        w_db[tid] = A.qerr2 && row_j[tid] >= 0 ? (double)A.qerr2[kb + row_j[tid]]
                                               : row_delta<FMT>(nb, s);
      }
      // S = Q W^T: wavefront w owns queries 16w..16w+15 against all 64 rows
      f32x4 acc[4];
      #pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
      const int arow = wave * 16 + (lane & 15);
      #pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int koff = kk * 32 + (lane >> 4) * 8;  // element offset of this lane's 8 values
        if (FMT == 0) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(qrows + arow * RS + koff * 2);
          #pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(wrows + (cb * 16 + (lane & 15)) * RS + koff * 2);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
          }
        } else {
          const long a = *reinterpret_cast<const long*>(qrows + arow * RS + koff);
          #pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const long b = *reinterpret_cast<const long*>(wrows + (cb * 16 + (lane & 15)) * RS + koff);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc[cb], 0, 0, 0);
          }
        }
      }
      __syncthreads();  // every wave has read wrows; the scores go there now
      #pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = wave * 16 + (lane >> 4) * 4 + i;
          const int r = cb * 16 + (lane & 15);
          score[q * (kChunkRows + 1) + r] = acc[cb][i];
        }
      }
      __syncthreads();
      for (uint32_t e = tid; e < npairs; e += kThreads) {
        const uint32_t x = ent[e];
        if (!(x & kPending)) continue;
        const uint32_t v = (x >> 6) & kNoWindow;
        if (v < c0 || v >= c0 + nr) continue;
        const uint32_t q = x & 63u, r = v - c0;
        const double s = (double)score[q * (kChunkRows + 1) + r] * (double)q_scale[q] * (double)w_scale[r];
        const double dt = (double)q_norm[q] + (double)w_norm[r] - 2.0 * s;
        const double lb = lower_bound(dt, q_nb[q], w_nb[r], q_db[q], w_db[r]);
        const double ub = upper_bound(dt, q_nb[q], w_nb[r], q_db[q], w_db[r]);
        // both bounds as halves, rounded outward: upper << 16 | lower
        ent[e] = half_up((float)(ub * (1.0 + 1e-7))) << 16 | half_down((float)(lb * (1.0 - 1e-7)));
      }
      __syncthreads();
    }
    // candidates outside the window: bounds 0 and +inf (always evaluated)
    for (uint32_t e = tid; e < npairs; e += kThreads)
      if (ent[e] & kPending) ent[e] = 0x7C00u << 16;
    __syncthreads();

    // per query the second smallest upper bound U2: two candidates lie at
    // or below it, so one whose lower bound exceeds U2 is neither best nor
    // second
    if (tid < T.count && q_in[tid]) {
      const int q = tid;
      float u1 = __builtin_inff(), u2 = __builtin_inff();
      for (uint32_t e = q_off[q]; e < q_off[q + 1]; ++e) {
        const float ub = half_value(ent[e] >> 16);
        if (ub < u1) {
          u2 = u1;
          u1 = ub;
        } else if (ub < u2) {
          u2 = ub;
        }
      }
      lb5[q] = u2;
    }
    __syncthreads();
    // every candidate within U2 of its row is listed (entry indices, in the
    // query rows' area, dead since the last MFMA), then all threads take the
    // list in turn for its exact canonical distances; a result replaces its
    // entry with the distance's bits and the top bit set
    uint16_t* todo = reinterpret_cast<uint16_t*>(qrows);
    uint32_t mine = 0;
    for (uint32_t e = tid; e < npairs; e += kThreads)
      mine += half_value(ent[e]) <= lb5[entry_query(q_off, e)] ? 1u : 0u;
    uint32_t incl = mine;
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
      if (lane >= off) incl += o;
    }
    if (lane == kWave - 1) wave_total[wave] = incl;
    __syncthreads();
    uint32_t pos = incl - mine, nexact = 0;
    for (int w = 0; w < kWaves; ++w) {
      pos += w < wave ? wave_total[w] : 0u;
      nexact += wave_total[w];
    }
    for (uint32_t e = tid; e < npairs; e += kThreads)
      if (half_value(ent[e]) <= lb5[entry_query(q_off, e)]) todo[pos++] = (uint16_t)e;
    __syncthreads();
    for (uint32_t k = tid; k < nexact; k += kThreads) {
      const uint32_t e = todo[k];
      const uint32_t q = entry_query(q_off, e);
      const int32_t j = A.cols[q_o0[q] + (e - q_off[q])];
      const float d = exact_distance(reinterpret_cast<const float4*>(A.desc1_f32) + q_i[q] * 32,
                                     reinterpret_cast<const float4*>(A.desc2_f32) + (kb + j) * 32);
      ent[e] = __float_as_uint(d) | 0x80000000u;
    }
    __syncthreads();
    if (tid < T.count && q_in[tid]) {
      const int q = tid;
      Top2 t;
      for (uint32_t e = q_off[q]; e < q_off[q + 1]; ++e) {
        const uint32_t x = ent[e];
        if (x & 0x80000000u) t.insert(__uint_as_float(x & 0x7FFFFFFFu), A.cols[q_o0[q] + (e - q_off[q])]);
      }
      write_match(A, q_i[q], t, false);
    }
    if (A.match_stats && tid == 0 && nexact)
      atomicAdd(&A.match_stats[3], (unsigned long long)nexact);
    __syncthreads();
    if (A.match_stats && tid == 0) {
      uint32_t longs = 0, reranked = 0;
      for (int q = 0; q < T.count; ++q) {
        longs += !q_in[q] && q_k[q] > 0;
        reranked += q_in[q] && q_k[q] > 0;
      }
      atomicAdd(&A.match_stats[0], (unsigned long long)reranked);
      atomicAdd(&A.match_stats[2], (unsigned long long)longs);
    }
    // fallback and long rows: every candidate exactly, one wavefront per query
    for (int t0 = wave; t0 < T.count; t0 += kWaves) {
      const int q = t0;
      if (q_in[q]) continue;
      const int64_t i = q_i[q];
      if (lane < 32) qdesc[wave][lane] = reinterpret_cast<const float4*>(A.desc1_f32)[i * 32 + lane];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      Top2 t;
      for (int64_t e = q_o0[q] + lane; e < q_o0[q] + q_k[q]; e += kWave) {
        const int32_t j = A.cols[e];
        const float4* r2 = reinterpret_cast<const float4*>(A.desc2_f32) + (kb + j) * 32;
        float acc = 0.0f;
        #pragma unroll 8
        for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qdesc[wave][k], r2[k]);
        t.insert(acc, j);
      }
      t = wave_merge_top2(t);
      if (lane == 0) write_match(A, i, t, false);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (PERSIST) __syncthreads();  // the tile's LDS is dead before the next one starts
  }
}

}  // namespace

hipError_t launch_match_window_mfma(const MatchArgs& a, int fmt, int grid, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  if (grid > 0 && !a.queue) return hipErrorInvalidValue;
  const dim3 g(grid > 0 ? (grid < a.num_tiles ? grid : a.num_tiles) : a.num_tiles);
  if (fmt == 0) {
    if (grid > 0)
      hipLaunchKernelGGL((k_match_window_mfma<0, true>), g, dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL((k_match_window_mfma<0, false>), g, dim3(kThreads), 0, s, a);
  } else {
    if (grid > 0)
      hipLaunchKernelGGL((k_match_window_mfma<1, true>), g, dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL((k_match_window_mfma<1, false>), g, dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace epm
