// Selection helpers shared by the matching kernels.
#pragma once

#include "device_common.h"
#include "launch.h"

namespace epm {

// One step of the canonical FP32 squared distance over four dimensions,
// k ascending: t = a - b (rounded), acc = fmaf(t, t, acc).
__device__ __forceinline__ float canonical_step4(float acc, const float4& a, const float4& b) {
  float t = a.x - b.x;
  acc = __builtin_fmaf(t, t, acc);
  t = a.y - b.y;
  acc = __builtin_fmaf(t, t, acc);
  t = a.z - b.z;
  acc = __builtin_fmaf(t, t, acc);
  t = a.w - b.w;
  acc = __builtin_fmaf(t, t, acc);
  return acc;
}

// (distance, j) ordered lexicographically: the tie goes to the lower j.
__device__ __forceinline__ bool before(float d1, int32_t j1, float d2, int32_t j2) {
  return d1 < d2 || (d1 == d2 && j1 < j2);
}

struct Top2 {
  float bd = __builtin_inff();
  int32_t bj = INT32_MAX;
  float sd = __builtin_inff();
  int32_t sj = INT32_MAX;

  __device__ __forceinline__ void insert(float d, int32_t j) {
    if (before(d, j, bd, bj)) {
      sd = bd;
      sj = bj;
      bd = d;
      bj = j;
    } else if (before(d, j, sd, sj)) {
      sd = d;
      sj = j;
    }
  }
};

// Merge of two top-2 lists holding distinct candidates.
__device__ __forceinline__ Top2 merge_top2(const Top2& x, const Top2& y) {
  Top2 r;
  const bool xf = before(x.bd, x.bj, y.bd, y.bj);
  r.bd = xf ? x.bd : y.bd;
  r.bj = xf ? x.bj : y.bj;
  // runner-up: the other list's best or the winner list's second
  const float od = xf ? y.bd : x.bd;
  const int32_t oj = xf ? y.bj : x.bj;
  const float wd = xf ? x.sd : y.sd;
  const int32_t wj = xf ? x.sj : y.sj;
  const bool of = before(od, oj, wd, wj);
  r.sd = of ? od : wd;
  r.sj = of ? oj : wj;
  return r;
}

__device__ __forceinline__ Top2 wave_merge_top2(Top2 t) {
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    Top2 o;
    o.bd = __shfl_xor(t.bd, off);
    o.bj = __shfl_xor(t.bj, off);
    o.sd = __shfl_xor(t.sd, off);
    o.sj = __shfl_xor(t.sj, off);
    t = merge_top2(t, o);
  }
  return t;
}

// Dense (query, candidate) lists of the window kernels: entry e of query q is
// its t-th candidate, e = q_off[q] + t; an entry packs (pending bit, window
// position v, query q) as kEntPending | v << 6 | q, v = kEntNoWindow when the
// candidate lies outside the tile's window.
constexpr uint32_t kEntPending = 0x80000000u;
constexpr uint32_t kEntNoWindow = (1u << 25) - 1u;

__device__ __forceinline__ uint32_t entry_query(const uint32_t* q_off, uint32_t e) {
  uint32_t q = 0;  // last query with q_off[q] <= e
  #pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (q + step < kTileQ && q_off[q + step] <= e) q += step;
  return q;
}

// Builds ent[0 .. npairs) (and ent_j, the candidates' image-2 indices, when
// not NULL) for one tile.  Every thread handles entries tid, tid + NT, ...,
// kBatch of them at a time so that their CSR and inverse-permutation loads are
// in flight together; the caller synchronises afterwards.  The window is
// given by its non-empty slots sorted by start position (ss_*, nss of them).
template <int NT>
__device__ __forceinline__ void build_dense_list(const MatchArgs& A, int64_t kb, uint32_t npairs,
                                                 const uint32_t* q_off, const int64_t* q_o0,
                                                 const uint32_t* ss_b, const uint32_t* ss_v,
                                                 const uint32_t* ss_len, uint32_t nss,
                                                 uint32_t* ent, int32_t* ent_j, int tid) {
  constexpr int kBatch = 4;
  for (uint32_t e0 = tid; e0 < npairs; e0 += NT * kBatch) {
    int32_t j[kBatch];
    #pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t e = e0 + u * NT;
      if (e < npairs) {
        const uint32_t q = entry_query(q_off, e);
        j[u] = A.cols[q_o0[q] + (e - q_off[q])];
      }
    }
    uint32_t pos[kBatch];
    #pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (e0 + u * NT < npairs) pos[u] = A.rinv[kb + j[u]];
    #pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t e = e0 + u * NT;
      if (e >= npairs) continue;
      uint32_t v = kEntNoWindow;
      if (nss > 0) {
        uint32_t s = 0;  // last sorted slot with ss_b[s] <= pos
        #pragma unroll
        for (int step = 32; step > 0; step >>= 1)
          if (s + step < nss && ss_b[s + step] <= pos[u]) s += step;
        if (ss_b[s] <= pos[u] && pos[u] - ss_b[s] < ss_len[s]) v = ss_v[s] + (pos[u] - ss_b[s]);
      }
      if (v >= kEntNoWindow) v = kEntNoWindow;
      ent[e] = kEntPending | (v << 6) | entry_query(q_off, e);
      if (ent_j) ent_j[e] = j[u];
    }
  }
}

// Output convention: empty row -> -1 / +inf / +inf; ratio rejection -> -1
// with both distances kept.
// A CSR that did not fit its buffer (row_offsets[n1] beyond the caller's
// capacity) is incomplete: such a launch writes nothing.
__device__ __forceinline__ bool csr_overflow(const MatchArgs& A) {
  return A.capacity >= 0 && A.row_offsets[A.n1] > A.capacity;
}

__device__ __forceinline__ void write_match_to(float ratio, int32_t* __restrict__ best_idx,
                                               float* __restrict__ best_dist,
                                               float* __restrict__ second_dist, int64_t i,
                                               const Top2& t, bool binary) {
  int32_t idx = t.bj == INT32_MAX ? -1 : t.bj;
  if (idx >= 0 && ratio > 0.0f) {
    bool accept;
    if (binary) {
      accept = t.bd < ratio * t.sd;
    } else {
      const float thr = ratio * ratio;
      accept = t.bd < thr * t.sd;
    }
    if (!accept) idx = -1;
  }
  best_idx[i] = idx;
  best_dist[i] = t.bd;
  second_dist[i] = t.sd;
}

__device__ __forceinline__ void write_match(const MatchArgs& A, int64_t i, const Top2& t,
                                            bool binary) {
  write_match_to(A.ratio, A.best_idx, A.best_dist, A.second_dist, i, t, binary);
}

}  // namespace epm
