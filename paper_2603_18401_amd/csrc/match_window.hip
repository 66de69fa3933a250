// Window-staged FP32 descriptor matching over the candidate CSR (Sec. 4.3).
//
// Neighbouring angle-sorted queries share most of their candidates, and all
// candidates of a stabbing tile lie in the tile's record window.  One
// workgroup per tile:
//   1. maps every candidate j of the tile's rows to its window index (inverse
//      angle permutation, then the tile's window slots) and builds a dense
//      list of (query, candidate, window index) entries in LDS;
//   2. stages the window's descriptor rows once, coalesced, in LDS (row
//      stride 132 floats so 16-byte LDS reads by different rows are bank
//      conflict free);
//   3. every thread evaluates whole canonical FP32 distances for list entries
//      (query row from L1, candidate row from LDS, k ascending, fmaf);
//   4. one thread per query selects (distance, j) best and second.
// Rows that do not fit the tile's dense list, and candidates outside the
// window (a CSR that did not come from this index's last query), use
// per-candidate gathers.  Every
// distance is the canonical one, so results equal the plain kernel's bit for
// bit.
#include "device_common.h"
#include "launch.h"
#include "match_common.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kRowStride = 132;  // floats
constexpr int kWinRows = 64;     // rows staged per pass
constexpr int kMaxPairs = 4096;  // dense (query, candidate) entries per tile
constexpr uint32_t kPending = kEntPending;
constexpr uint32_t kNoWindow = kEntNoWindow;

__device__ __forceinline__ float row_distance_global(const float4* __restrict__ qr,
                                                     const float4* __restrict__ wr) {
  float acc = 0.0f;
  #pragma unroll 8
  for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qr[k], wr[k]);
  return acc;
}

template <bool PERSIST>
__global__ __launch_bounds__(kThreads) void k_match_window_f32(MatchArgs A) {
  __shared__ float4 rows4[kWinRows * kRowStride / 4];
  __shared__ uint32_t ent[kMaxPairs];
  __shared__ int32_t ent_j[kMaxPairs];
  __shared__ uint32_t slot_b[kSlots], slot_pref[kSlots + 1];
  __shared__ uint32_t ss_b[kSlots], ss_v[kSlots], ss_len[kSlots];
  __shared__ int64_t q_i[kTileQ], q_o0[kTileQ];
  __shared__ uint32_t q_k[kTileQ], q_off[kTileQ + 1], q_in[kTileQ];
  __shared__ int32_t row_j[kWinRows];
  __shared__ uint32_t n_sorted_slots;
  __shared__ float4 qdesc[kWaves][32];

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

    if (wave == 0) {
      // rows of the tile's queries
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
      // window slots, and the non-empty ones ordered by start position
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

    // 1. dense (query, candidate, window index) list
    const uint32_t npairs = q_off[kTileQ];
    const uint32_t nss = n_sorted_slots;
    build_dense_list<kThreads>(A, kb, npairs, q_off, q_o0, ss_b, ss_v, ss_len, nss, ent, ent_j,
                               tid);
    __syncthreads();

    // 2-3. stage window rows and evaluate the entries that fall in them
    const uint32_t wlen = slot_pref[kSlots];
    const float* rows = reinterpret_cast<const float*>(rows4);
    for (uint32_t c0 = 0; c0 < wlen; c0 += kWinRows) {
      const uint32_t nr = wlen - c0 < (uint32_t)kWinRows ? wlen - c0 : (uint32_t)kWinRows;
      for (uint32_t r = tid; r < nr; r += kThreads) {
        const uint32_t v = c0 + r;
        uint32_t s = 0;  // last slot with slot_pref[s] <= v
        #pragma unroll
        for (int step = 32; step > 0; step >>= 1)
          if (s + step <= kSlots && slot_pref[s + step] <= v) s += step;
        row_j[r] = A.rj[slot_b[s] + (v - slot_pref[s])];
      }
      __syncthreads();
      for (uint32_t f = tid; f < nr * 32; f += kThreads) {
        const uint32_t r = f >> 5, c4 = f & 31;
        const float4* src = reinterpret_cast<const float4*>(A.desc2) + (kb + row_j[r]) * 32;
        rows4[r * (kRowStride / 4) + c4] = src[c4];
      }
      __syncthreads();
      for (uint32_t e = tid; e < npairs; e += kThreads) {
        const uint32_t x = ent[e];
        if (!(x & kPending)) continue;
        const uint32_t v = (x >> 6) & kNoWindow;
        if (v < c0 || v >= c0 + nr) continue;
        const uint32_t q = x & 63u;
        const float4* qr = reinterpret_cast<const float4*>(A.desc1) + q_i[q] * 32;
        const float4* wr = reinterpret_cast<const float4*>(rows + (v - c0) * kRowStride);
        float acc = 0.0f;
        #pragma unroll 8
        for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qr[k], wr[k]);
        ent[e] = __float_as_uint(acc);
      }
      __syncthreads();
    }
    // candidates outside the window: gathered rows
    for (uint32_t e = tid; e < npairs; e += kThreads) {
      const uint32_t x = ent[e];
      if (!(x & kPending)) continue;
      const uint32_t q = x & 63u;
      const int32_t j = ent_j[e];
      const float4* qr = reinterpret_cast<const float4*>(A.desc1) + q_i[q] * 32;
      const float4* wr = reinterpret_cast<const float4*>(A.desc2) + (kb + j) * 32;
      ent[e] = __float_as_uint(row_distance_global(qr, wr));
    }
    __syncthreads();

    // 4. selection, one thread per query
    if (tid < T.count && q_in[tid]) {
      const int q = tid;
      Top2 best;
      for (uint32_t e = q_off[q]; e < q_off[q + 1]; ++e) best.insert(__uint_as_float(ent[e]), ent_j[e]);
      write_match(A, q_i[q], best, false);
    }
    // long rows: one wavefront each, one lane per candidate (gathers)
    for (int q = wave; q < T.count; q += kWaves) {
      if (q_in[q]) continue;
      const int64_t i = q_i[q];
      if (lane < 32) qdesc[wave][lane] = reinterpret_cast<const float4*>(A.desc1)[i * 32 + lane];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      Top2 t;
      for (int64_t e = q_o0[q] + lane; e < q_o0[q] + q_k[q]; e += kWave) {
        const int32_t j = A.cols[e];
        const float4* d2 = reinterpret_cast<const float4*>(A.desc2) + (kb + j) * 32;
        float acc = 0.0f;
        #pragma unroll 8
        for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qdesc[wave][k], d2[k]);
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

hipError_t launch_match_window_f32(const MatchArgs& a, int grid, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  if (grid > 0) {
    if (!a.queue) return hipErrorInvalidValue;
    const int g = grid < a.num_tiles ? grid : a.num_tiles;
    hipLaunchKernelGGL(k_match_window_f32<true>, dim3(g), dim3(kThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_match_window_f32<false>, dim3(a.num_tiles), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace epm
