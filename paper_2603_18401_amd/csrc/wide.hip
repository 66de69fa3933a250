// Wide rows: queries with more than kStage candidates (Sec. 4.2 query and
// Sec. 4.3 selection at the tolerances of the paper's experiments, where a
// query keeps hundreds to thousands of candidates).
//
// One workgroup per stabbing tile that has such rows.  The tile's record
// window (every width class, as found by the window pass) is enumerated in
// ascending image-2 index j: its j are marked in an LDS bitmap over a slab of
// 65536 j values, and an exclusive prefix count of the bitmap's words maps
// the e-th marked j to its word and bit.  Chunks of 64 window entries are
// then taken in j order:
//   1. every entry is tested against every wide query of the tile (angle
//      test, then the FP64 test of Eq. 3: the decisions of the counting
//      pass); one ballot per entry gives its 64-bit query mask;
//   2. one ballot per query over the chunk's masks appends the query's hits
//      to its CSR row -- in ascending j by construction, so no row is sorted;
//   3. (match) the entries' FP32 descriptor rows are rounded to BF16 in LDS
//      and scored against the tile's BF16 query rows on MFMA; every hit gets
//      the approximate key |w^|^2 - 2 q^.w^ and each query keeps the five
//      smallest keys.
// The four best keys of a query are re-ranked with canonical FP32 chains on
// the FP32 rows.  The fifth key bounds every other candidate from below
// (the rounding bound of the BF16 rows, of the MFMA accumulation and of the
// key itself, with the largest row terms of the window); when that bound
// exceeds the exact second distance the match is certified, otherwise the
// query is listed for the exact listed-query match.  Final outputs therefore
// equal the FP32 canonical selection bit for bit.
#include "device_common.h"
#include "launch.h"
#include "match_common.h"
#include "mfma_bounds.h"

namespace epm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kSlabWords = 1024;                         // bitmap words per slab
constexpr int64_t kSlabBits = (int64_t)kSlabWords * 64;  // j values per slab
constexpr int kL = 64;                                   // window entries per chunk
constexpr int kRS = 256 + 16;  // LDS bytes per BF16 row: fragment reads of 16 rows hit distinct banks
constexpr int kPicks = 4;
constexpr int kQPerWave = kTileQ / kWaves;
static_assert(kL == kWave, "one chunk entry per lane in the CSR step");
static_assert(kThreads * 4 == kSlabWords, "four bitmap words per thread in the prefix count");

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void store_bf16x4(uint8_t* dst, const float4& v) {
  uint2 w;
  w.x = bf16_bits(v.x) | (bf16_bits(v.y) << 16);
  w.y = bf16_bits(v.z) | (bf16_bits(v.w) << 16);
  *reinterpret_cast<uint2*>(dst) = w;
}

// Position of the k-th set bit (k from 0) of w, which has more than k bits set.
__device__ __forceinline__ int select_bit(uint64_t w, uint32_t k) {
  int pos = 0;
  uint32_t c = (uint32_t)__popc((uint32_t)w);
  if (k >= c) { k -= c; w >>= 32; pos += 32; }
  c = (uint32_t)__popc((uint32_t)w & 0xFFFFu);
  if (k >= c) { k -= c; w >>= 16; pos += 16; }
  c = (uint32_t)__popc((uint32_t)w & 0xFFu);
  if (k >= c) { k -= c; w >>= 8; pos += 8; }
  c = (uint32_t)__popc((uint32_t)w & 0xFu);
  if (k >= c) { k -= c; w >>= 4; pos += 4; }
  c = (uint32_t)__popc((uint32_t)w & 0x3u);
  if (k >= c) { k -= c; w >>= 2; pos += 2; }
  if (k >= ((uint32_t)w & 1u)) pos += 1;
  return pos;
}

__device__ __forceinline__ double wave_max_f64(double v) {
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Five smallest keys (ascending) with their image-2 indices.
struct Top5 {
  float k[kPicks + 1];
  int32_t j[kPicks + 1];
  __device__ __forceinline__ void init() {
    #pragma unroll
    for (int u = 0; u <= kPicks; ++u) {
      k[u] = __builtin_inff();
      j[u] = -1;
    }
  }
  __device__ __forceinline__ void insert(float d, int32_t jj) {
    if (!(d < k[kPicks])) return;
    #pragma unroll
    for (int u = 0; u <= kPicks; ++u) {
      if (d < k[u]) {
        const float td = k[u];
        const int32_t tj = j[u];
        k[u] = d;
        j[u] = jj;
        d = td;
        jj = tj;
      }
    }
  }
};

template <bool MATCH>
__global__ __launch_bounds__(kThreads) void k_wide_tile(StabArgs A) {
  __shared__ unsigned long long bits[kSlabWords];
  __shared__ uint32_t wpref[kSlabWords];
  __shared__ uint32_t wsum[kWaves], n_entries;
  __shared__ int32_t lj[kL];
  __shared__ uint32_t lC[kL], lH[kL];
  __shared__ float2 lXY[kL];
  __shared__ float lE[kL];
  __shared__ uint64_t lmask[kL];
  __shared__ double qa[kTileQ], qb[kTileQ], qc[kTileQ], qn[kTileQ];
  __shared__ uint32_t qk[kTileQ], q_run[kTileQ];
  __shared__ int64_t q_i[kTileQ], q_o0[kTileQ];
  __shared__ uint32_t slot_b[kSlots], slot_pref[kSlots + 1];
  __shared__ uint64_t wide_mask_s;
  // matching only
  constexpr int kQ = MATCH ? kTileQ : 1;
  constexpr int kW = MATCH ? kL : 1;
  __shared__ __attribute__((aligned(16))) uint8_t qrows[kQ * kRS];
  __shared__ __attribute__((aligned(16))) uint8_t wrows[kW * kRS];
  __shared__ float w_norm[kW], q_norm[kQ];
  __shared__ double q_nb[kQ], q_db[kQ];
  __shared__ double w_nbmax, w_dbmax;  // largest row terms of the bound over the window
  __shared__ float pk[kQ][kPicks + 1];
  __shared__ int32_t pj[kQ][kPicks];
  __shared__ float pdist[kQ][kPicks];
  __shared__ uint32_t n_cert, n_fallback;

  const int tile = xcd_tile(blockIdx.x, A.num_tiles);
  if (A.tile_wide[tile] == 0u) return;
  const StabTile T = A.tiles[tile];
  const PairDev& pd = A.pairs[T.pair];
  const int64_t kb = pd.k_begin, n2 = pd.n;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();

  if (wave == 0) {
    const bool live = lane < T.count;
    int64_t i = 0, o0 = 0, len = 0;
    uint32_t flag = kQueryEmpty, key = 0;
    double a = 0.0, b = 0.0, c = 0.0;
    if (live) {
      i = A.qperm[T.begin + lane];
      flag = A.qflag[i];
      key = A.qkey[i];
      o0 = A.row_offsets[i];
      len = A.row_offsets[i + 1] - o0;
      if (flag == kQueryNormal) epipolar_line(pd.F, A.kp1[2 * i], A.kp1[2 * i + 1], a, b, c);
    }
    const bool wide = live && flag == kQueryNormal && len > kStage;
    qa[lane] = a;
    qb[lane] = b;
    qc[lane] = c;
    qn[lane] = line_norm(a, b);
    qk[lane] = key;
    q_i[lane] = i;
    q_o0[lane] = o0;
    q_run[lane] = 0u;
    const uint64_t wm = ballot(wide);
    const TileWindow* W = A.windows + tile;
    slot_b[lane] = W->slot_b[lane];
    slot_pref[lane] = W->slot_pref[lane];
    if (lane == 0) {
      slot_pref[kSlots] = W->slot_pref[kSlots];
      wide_mask_s = wm;
      if (MATCH) {
        w_nbmax = 0.0;
        w_dbmax = 0.0;
        n_cert = 0u;
        n_fallback = 0u;
      }
    }
  }
  __syncthreads();
  const uint64_t wide_mask = wide_mask_s;
  // lane = query in the entry tests
  const double my_a = qa[lane], my_b = qb[lane], my_c = qc[lane], my_n = qn[lane];
  const uint32_t my_k = qk[lane];
  const bool my_wide = (wide_mask >> lane) & 1ull;

  Top5 best[4];  // this lane's four queries of the MFMA layout
  if (MATCH) {
    #pragma unroll
    for (int i = 0; i < 4; ++i) best[i].init();
    // BF16 query rows (zero rows for the queries that are not wide)
    for (int f = tid; f < kTileQ * 32; f += kThreads) {
      const int q = f >> 5, c = f & 31;
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if ((wide_mask >> q) & 1ull) v = reinterpret_cast<const float4*>(A.desc1)[q_i[q] * 32 + c];
      store_bf16x4(qrows + q * kRS + c * 8, v);
    }
    __syncthreads();
    if (tid < kTileQ) {
      const float n = row_sqnorm<0>(qrows + tid * kRS);
      q_norm[tid] = n;
      const double nb = sqrt((double)n) * (1.0 + 1e-5);
      q_nb[tid] = nb;
      q_db[tid] = row_delta<0>(nb, 1.0);
    }
  }

  const int64_t total_len = slot_pref[kSlots];
  const int64_t nslabs = (n2 + kSlabBits - 1) / kSlabBits;
  for (int64_t sb = 0; sb < nslabs; ++sb) {
    const int64_t j0 = sb * kSlabBits;
    const int64_t jn = n2 - j0 < kSlabBits ? n2 - j0 : kSlabBits;
    const int nwords = (int)((jn + 63) >> 6);
    for (int w = tid; w < kSlabWords; w += kThreads) bits[w] = 0ull;
    __syncthreads();
    // mark the window's j that fall in this slab
    for (int64_t v = tid; v < total_len; v += kThreads) {
      int s = 0;  // last slot with slot_pref[s] <= v
      #pragma unroll
      for (int step = 32; step > 0; step >>= 1)
        if (s + step <= kSlots && slot_pref[s + step] <= v) s += step;
      const int64_t j = (int64_t)A.rj[slot_b[s] + (v - slot_pref[s])] - j0;
      if (j >= 0 && j < jn) atomicOr(&bits[j >> 6], 1ull << (j & 63));
    }
    __syncthreads();
    // exclusive prefix count of the words: thread t owns words 4t .. 4t + 3
    {
      uint32_t c[4], tot = 0;
      #pragma unroll
      for (int u = 0; u < 4; ++u) {
        c[u] = (uint32_t)__popcll(bits[tid * 4 + u]);
        tot += c[u];
      }
      uint32_t incl = tot;
      #pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      if (lane == kWave - 1) wsum[wave] = incl;
      __syncthreads();
      uint32_t base = 0, all = 0;
      #pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        base += w < wave ? wsum[w] : 0u;
        all += wsum[w];
      }
      uint32_t run = base + incl - tot;
      #pragma unroll
      for (int u = 0; u < 4; ++u) {
        wpref[tid * 4 + u] = run;
        run += c[u];
      }
      if (tid == 0) n_entries = all;
    }
    __syncthreads();
    const uint32_t E = n_entries;

    for (uint32_t e0 = 0; e0 < E; e0 += kL) {
      // the chunk's entries in ascending j, with their records
      if (tid < kL) {
        const uint32_t e = e0 + tid;
        int32_t j = -1;
        if (e < E) {
          int w = 0;  // last word with wpref[w] <= e (it holds entry e)
          #pragma unroll
          for (int step = kSlabWords / 2; step > 0; step >>= 1)
            if (w + step < nwords && wpref[w + step] <= e) w += step;
          j = (int32_t)(j0 + ((int64_t)w << 6) + select_bit(bits[w], e - wpref[w]));
          const uint32_t pos = A.rinv[kb + j];
          lC[tid] = A.rC[pos];
          lH[tid] = A.rH[pos];
          lXY[tid] = A.rxy[pos];
          lE[tid] = A.reps[pos];
        }
        lj[tid] = j;
      }
      __syncthreads();
      if (MATCH) {
        // BF16 copies of the entries' FP32 rows (zero rows past the end)
        for (int f = tid; f < kL * 32; f += kThreads) {
          const int r = f >> 5, c = f & 31;
          const int32_t j = lj[r];
          float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          if (j >= 0) v = reinterpret_cast<const float4*>(A.desc2)[(kb + j) * 32 + c];
          store_bf16x4(wrows + r * kRS + c * 8, v);
        }
      }
      // 1. entry masks: wavefront w tests entries w, w + 4, ... (lane = query)
      for (int r = wave; r < kL; r += kWaves) {
        bool hit = false;
        if (my_wide && lj[r] >= 0 && key_distance(my_k, lC[r]) <= lH[r]) {
          const float2 xy = lXY[r];
          hit = within_tolerance_n(my_a, my_b, my_c, my_n, xy.x, xy.y, lE[r]);
        }
        const uint64_t m = ballot(hit);
        if (lane == 0) lmask[r] = m;
      }
      __syncthreads();
      // 2. CSR rows: wavefront w appends the hits of its queries (lane = entry)
      {
        const uint64_t em = lmask[lane];
        const int32_t ej = lj[lane];
        for (int qq = 0; qq < kQPerWave; ++qq) {
          const int q = wave * kQPerWave + qq;
          if (!((wide_mask >> q) & 1ull)) continue;
          const bool hit = (em >> q) & 1ull;
          const uint64_t b = ballot(hit);
          const uint32_t run = q_run[q];
          if (hit) {
            const int64_t dst = q_o0[q] + run + lanes_below(b);
            if (dst < A.capacity) A.cols[dst] = ej;
          }
          if (lane == 0) q_run[q] = run + (uint32_t)__popcll(b);
        }
      }
      if (MATCH) {
        if (tid < kL) {
          // norms of the staged rows; running maxima of their bound terms
          float n = 0.0f;
          double nb = 0.0, db = 0.0;
          if (lj[tid] >= 0) {
            n = row_sqnorm<0>(wrows + tid * kRS);
            nb = sqrt((double)n) * (1.0 + 1e-5);
            db = row_delta<0>(nb, 1.0);
          }
          w_norm[tid] = n;
          nb = wave_max_f64(nb);
          db = wave_max_f64(db);
          if (tid == 0) {
            w_nbmax = fmax(w_nbmax, nb);
            w_dbmax = fmax(w_dbmax, db);
          }
        }
        // 3. S = Q W^T: wavefront w owns queries 16w .. 16w + 15 against all 64 rows
        f32x4 acc[4];
        #pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
        const int arow = wave * 16 + (lane & 15);
        #pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int koff = kk * 32 + (lane >> 4) * 8;  // element offset of this lane's 8 values
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(qrows + arow * kRS + koff * 2);
          #pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const bf16x8 b =
                *reinterpret_cast<const bf16x8*>(wrows + (cb * 16 + (lane & 15)) * kRS + koff * 2);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
          }
        }
        __syncthreads();  // w_norm complete
        #pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int r = cb * 16 + (lane & 15);
          const uint64_t m = lmask[r];
          const float wn = w_norm[r];
          const int32_t j = lj[r];
          #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = wave * 16 + (lane >> 4) * 4 + i;
            if ((m >> q) & 1ull) best[i].insert(__builtin_fmaf(-2.0f, acc[cb][i], wn), j);
          }
        }
      }
      __syncthreads();  // the chunk's LDS is dead
    }
  }

  if (!MATCH) return;
  // merge the five smallest keys over the 16 lanes that share each query
  #pragma unroll
  for (int i = 0; i < 4; ++i) {
    #pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      float ok[kPicks + 1];
      int32_t oj[kPicks + 1];
      #pragma unroll
      for (int u = 0; u <= kPicks; ++u) {
        ok[u] = __shfl_xor(best[i].k[u], off);
        oj[u] = __shfl_xor(best[i].j[u], off);
      }
      #pragma unroll
      for (int u = 0; u <= kPicks; ++u) best[i].insert(ok[u], oj[u]);
    }
    if ((lane & 15) == 0) {
      const int q = wave * 16 + (lane >> 4) * 4 + i;
      #pragma unroll
      for (int u = 0; u < kPicks; ++u) {
        pk[q][u] = best[i].k[u];
        pj[q][u] = best[i].j[u];
      }
      pk[q][kPicks] = best[i].k[kPicks];
    }
  }
  __syncthreads();
  // exact canonical distances of the picks: thread = (query, pick)
  {
    const int q = tid >> 2, u = tid & 3;
    float d = __builtin_inff();
    if (((wide_mask >> q) & 1ull) && pj[q][u] >= 0)
      d = exact_distance(reinterpret_cast<const float4*>(A.desc1) + q_i[q] * 32,
                         reinterpret_cast<const float4*>(A.desc2) + (kb + pj[q][u]) * 32);
    pdist[q][u] = d;
  }
  __syncthreads();
  if (tid < kTileQ && ((wide_mask >> tid) & 1ull)) {
    const int q = tid;
    Top2 t;
    #pragma unroll
    for (int u = 0; u < kPicks; ++u)
      if (pj[q][u] >= 0) t.insert(pdist[q][u], pj[q][u]);
    // every other hit has a key >= the fifth key: its exact distance is at
    // least the bound of the smallest such approximate distance, taken with
    // the largest row terms of the window and a slack for the key's rounding
    const double nw = w_nbmax, s = q_nb[q] + nw;
    const double dt = (double)q_norm[q] + (double)pk[q][kPicks] - 1e-6 * s * s;
    const double lb = lower_bound(dt, q_nb[q], nw, q_db[q], w_dbmax);
    if (lb > (double)t.sd) {
      write_match_to(A.ratio, A.best_idx, A.best_dist, A.second_dist, q_i[q], t, false);
      atomicAdd(&n_cert, 1u);
    } else {
      const unsigned long long at = atomicAdd(&A.stats[kStatRest], 1ull);
      A.rest[at] = (uint32_t)q_i[q];
      atomicAdd(&n_fallback, 1u);
    }
  }
  if (A.match_stats) {
    __syncthreads();
    if (tid == 0) {
      if (n_cert + n_fallback)
        atomicAdd(&A.match_stats[0], (unsigned long long)(n_cert + n_fallback));
      if (n_fallback) atomicAdd(&A.match_stats[1], (unsigned long long)n_fallback);
    }
  }
}

}  // namespace

hipError_t launch_wide_tiles(const StabArgs& a, bool match, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  if (!a.tile_wide) return hipErrorInvalidValue;
  if (match && (!a.desc1 || !a.desc2 || !a.best_idx || !a.best_dist || !a.second_dist || !a.rest))
    return hipErrorInvalidValue;
  if (match)
    hipLaunchKernelGGL(k_wide_tile<true>, dim3(a.num_tiles), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_wide_tile<false>, dim3(a.num_tiles), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace epm
