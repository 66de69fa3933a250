// Wide rows: queries with more than kStage candidates (Sec. 4.2 query and
// Sec. 4.3 selection at the tolerances of the paper's experiments, where a
// query keeps hundreds to thousands of candidates).
//
// One workgroup per stabbing tile that has such rows.  The tile's record
// window (every width class, as found by the window pass) is enumerated in
// ascending image-2 index j: its j are marked in an LDS bitmap over a slab of
// 65536 j values, and an exclusive prefix count of the bitmap's words maps
// the e-th marked j to its word and bit.  Chunks of 64 window entries are
// then taken in j order; each wavefront owns 16 queries of the tile:
//   1. every entry (one per lane) is tested against each of the wavefront's
//      wide queries (angle test, then the FP64 test of Eq. 3: the decisions
//      of the counting pass); one ballot per query gives its hit mask;
//   2. each mask appends the query's hits to its CSR row -- in ascending j
//      by construction, so no row is sorted;
//   3. (match) the entries' descriptor rows, as BF16 (copies rounded once
//      per call, or rounded on chip), are scored against the BF16 query rows
//      on MFMA; every hit gets the approximate key |w^|^2 - 2 q^.w^, and a
//      hit below the query's kPicks+1-th smallest key so far enters its list
//      of the kPicks+1 smallest keys.
// The kPicks best keys of a query are re-ranked with canonical FP32 chains on
// the FP32 rows.  The last kept key bounds every other candidate from below
// (the rounding bound of the BF16 rows, of the MFMA accumulation and of the
// key itself, with the largest row terms of the window); when that bound
// exceeds the exact second distance the match is certified, otherwise the
// query is listed for the exact listed-query match.  Final outputs therefore
// equal the FP32 canonical selection bit for bit.
//
// epm_match on a caller's CSR uses the same pass over the flagged tiles
// (every query of such a tile): the tile's candidate decisions are compared
// with the caller's rows instead of written, and a row that differs is left
// to the exact listed-query match.  BF16 descriptors given by the caller are
// staged as they are, with the format's worst-case rounding bound, and the
// picks re-ranked on the FP32 masters.
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
constexpr int kSC = kThreads;                            // window entries per super-chunk
constexpr int kL = 64;                                   // rows per block
constexpr int kSub = kSC / kL;                           // blocks per super-chunk
constexpr int kRS = 256 + 16;  // LDS bytes per BF16 row: fragment reads of 16 rows hit distinct banks
constexpr int kQS = 132;       // floats per FP32 query row of the re-rank (rows start 4 banks apart)
constexpr int kPicks = 5;      // exactly re-ranked candidates per query
constexpr int kMergeMin = 16;  // more survivors than this: merged by wavefront minima
constexpr int kQPerWave = kTileQ / kWaves;
constexpr int kRowPer = kL * 32 / kThreads;  // 16-byte pieces of a block's rows per thread
static_assert(kL == kWave && kQPerWave == 16, "one block row per lane, 16 queries per wavefront");
static_assert(kRowPer == 8 && kThreads == 256, "row sums: eight rows per half-wavefront");
static_assert(kPicks + 1 <= 16, "a query's kept keys are lanes 0 .. kPicks of the first DPP row");
static_assert(kThreads * 4 == kSlabWords, "four bitmap words per thread in the prefix count");
static_assert((kTileQ / 2) * kQS * 4 <= kL * kRS, "FP32 rows of half the queries fit the row area");
static_assert((kTileQ / 2) * kPicks <= kThreads, "one pick per thread in the re-rank");
static_assert(kTileQ * kPicks * 4 <= kSlabWords * 12, "exact distances fit the bitmap area");

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to BF16 (round to nearest even), packed low first.
__device__ __forceinline__ uint32_t bf16_pack(float lo, float hi) {
  const bf16x2_t b = __builtin_convertvector((float2_t){lo, hi}, bf16x2_t);
  return __builtin_bit_cast(uint32_t, b);
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

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  return __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(v), l));
}

// Value of the next lower lane within each row of 16 lanes (DPP row_shr:1;
// lane 0 of a row keeps its own value).
__device__ __forceinline__ int32_t row_shift_up(int32_t v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false);
}
__device__ __forceinline__ float row_shift_up(float v) {
  return __int_as_float(row_shift_up(__float_as_int(v)));
}

// Value of lane l ^ M (M < 32): DPP quad permutations for 1 and 2, the
// swizzle's bit mode (and 0x1F, xor M within each half) otherwise -- neither
// needs an address register.
template <int M>
__device__ __forceinline__ float xor_lanes(float v) {
  static_assert(M > 0 && M < 32 && (M & (M - 1)) == 0, "a single lane bit");
  const int x = __float_as_int(v);
  if (M == 1) return __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));
  if (M == 2) return __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));
  return __int_as_float(__builtin_amdgcn_ds_swizzle(x, 0x1F | (M << 10)));
}

// 64 FP32 rows (row r = piece f >> 5 of this thread, f = tid + kThreads u),
// loaded ahead of their use.
struct Rows {
  float4 v[kRowPer];
};

__device__ __forceinline__ Rows fetch_rows(const float* __restrict__ desc, const int64_t* row_of,
                                           int tid) {
  Rows R;
  #pragma unroll
  for (int u = 0; u < kRowPer; ++u) {
    const int f = tid + u * kThreads;
    const int64_t row = row_of[f >> 5];
    R.v[u] = row >= 0 ? reinterpret_cast<const float4*>(desc)[row * 32 + (f & 31)]
                      : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  return R;
}

// The same for the tile's queries: rows q_i[q] of the queries set in mask.
__device__ __forceinline__ Rows fetch_query_rows(const float* __restrict__ desc,
                                                 const int64_t* q_i, uint64_t mask, int tid) {
  Rows R;
  #pragma unroll
  for (int u = 0; u < kRowPer; ++u) {
    const int f = tid + u * kThreads, q = f >> 5;
    R.v[u] = (mask >> q) & 1ull ? reinterpret_cast<const float4*>(desc)[q_i[q] * 32 + (f & 31)]
                                : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  return R;
}

// Stores the BF16 copies of 64 rows (stride kRS) and, per row, the squared
// norm of the BF16 row and the squared norm of its rounding error, summed
// over the 32 lanes that hold the row's pieces by a transposing butterfly
// (each step halves the rows a lane keeps); optionally this thread's running
// maxima of both sums over the rows it summed.
__device__ __forceinline__ void stage_bf16(const Rows& R, uint8_t* dst, float* nrm, float* err,
                                           float* mx_n, float* mx_e, int tid) {
  float sn[kRowPer], se[kRowPer];
  #pragma unroll
  for (int u = 0; u < kRowPer; ++u) {
    const int f = tid + u * kThreads, r = f >> 5, c = f & 31;
    const float4 x = R.v[u];
    uint2 w;
    w.x = bf16_pack(x.x, x.y);
    w.y = bf16_pack(x.z, x.w);
    *reinterpret_cast<uint2*>(dst + r * kRS + c * 8) = w;
    const float y0 = __uint_as_float(w.x << 16), y1 = __uint_as_float(w.x & 0xFFFF0000u),
                y2 = __uint_as_float(w.y << 16), y3 = __uint_as_float(w.y & 0xFFFF0000u);
    // x - y is exact in FP32 (y is x rounded to fewer bits)
    const float e0 = x.x - y0, e1 = x.y - y1, e2 = x.z - y2, e3 = x.w - y3;
    sn[u] = __builtin_fmaf(y3, y3, __builtin_fmaf(y2, y2, __builtin_fmaf(y1, y1, y0 * y0)));
    se[u] = __builtin_fmaf(e3, e3, __builtin_fmaf(e2, e2, __builtin_fmaf(e1, e1, e0 * e0)));
  }
  const int lane = lane_id();
  const bool b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  float tn[4], te[4];
  #pragma unroll
  for (int v = 0; v < 4; ++v) {  // keep rows 4 b4 + v
    tn[v] = (b4 ? sn[4 + v] : sn[v]) + xor_lanes<16>(b4 ? sn[v] : sn[4 + v]);
    te[v] = (b4 ? se[4 + v] : se[v]) + xor_lanes<16>(b4 ? se[v] : se[4 + v]);
  }
  float un[2], ue[2];
  #pragma unroll
  for (int v = 0; v < 2; ++v) {  // keep rows 4 b4 + 2 b3 + v
    un[v] = (b3 ? tn[2 + v] : tn[v]) + xor_lanes<8>(b3 ? tn[v] : tn[2 + v]);
    ue[v] = (b3 ? te[2 + v] : te[v]) + xor_lanes<8>(b3 ? te[v] : te[2 + v]);
  }
  float vn = (b2 ? un[1] : un[0]) + xor_lanes<4>(b2 ? un[0] : un[1]);
  float ve = (b2 ? ue[1] : ue[0]) + xor_lanes<4>(b2 ? ue[0] : ue[1]);
  vn += xor_lanes<2>(vn);
  ve += xor_lanes<2>(ve);
  vn += xor_lanes<1>(vn);
  ve += xor_lanes<1>(ve);
  if ((lane & 3) == 0) {
    const int r = (tid >> 5) + 8 * (4 * b4 + 2 * b3 + b2);
    nrm[r] = vn;
    if (err) err[r] = ve;
  }
  if (mx_n) {  // every lane of the four holds the row's sums
    *mx_n = fmaxf(*mx_n, vn);
    *mx_e = fmaxf(*mx_e, ve);
  }
}

// 64 BF16 rows of 256 bytes given as codes (row r = piece f >> 4 of this
// thread, f = tid + kThreads u).
constexpr int kCodePer = kL * 16 / kThreads;
static_assert(kCodePer == 4, "row sums: four rows per 16-lane group");
struct Codes {
  uint4 v[kCodePer];
};

__device__ __forceinline__ Codes fetch_codes(const uint16_t* __restrict__ codes,
                                             const int64_t* row_of, int tid) {
  Codes C;
  #pragma unroll
  for (int u = 0; u < kCodePer; ++u) {
    const int f = tid + u * kThreads;
    const int64_t row = row_of[f >> 4];
    C.v[u] = row >= 0 ? reinterpret_cast<const uint4*>(codes)[row * 16 + (f & 15)]
                      : make_uint4(0u, 0u, 0u, 0u);
  }
  return C;
}

__device__ __forceinline__ Codes fetch_query_codes(const uint16_t* __restrict__ codes,
                                                   const int64_t* q_i, uint64_t mask, int tid) {
  Codes C;
  #pragma unroll
  for (int u = 0; u < kCodePer; ++u) {
    const int f = tid + u * kThreads, q = f >> 4;
    C.v[u] = (mask >> q) & 1ull ? reinterpret_cast<const uint4*>(codes)[q_i[q] * 16 + (f & 15)]
                                : make_uint4(0u, 0u, 0u, 0u);
  }
  return C;
}

__device__ __forceinline__ float bf16_sq4(uint32_t w0, uint32_t w1) {
  const float y0 = __uint_as_float(w0 << 16), y1 = __uint_as_float(w0 & 0xFFFF0000u),
              y2 = __uint_as_float(w1 << 16), y3 = __uint_as_float(w1 & 0xFFFF0000u);
  return y0 * y0 + y1 * y1 + y2 * y2 + y3 * y3;
}

// Stores 64 BF16 rows (stride kRS) and their squared norms (sums over the 16
// lanes of each row's pieces, transposing butterfly as in stage_bf16);
// optionally this thread's running maximum of the norms it summed.
__device__ __forceinline__ void stage_codes(const Codes& C, uint8_t* dst, float* nrm, float* mx_n,
                                            int tid) {
  float sn[kCodePer];
  #pragma unroll
  for (int u = 0; u < kCodePer; ++u) {
    const int f = tid + u * kThreads, r = f >> 4, c = f & 15;
    const uint4 w = C.v[u];
    *reinterpret_cast<uint4*>(dst + r * kRS + c * 16) = w;
    sn[u] = bf16_sq4(w.x, w.y) + bf16_sq4(w.z, w.w);
  }
  const int lane = lane_id();
  const bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  float t[2];
  #pragma unroll
  for (int v = 0; v < 2; ++v)  // keep rows 2 b3 + v of the group's four
    t[v] = (b3 ? sn[2 + v] : sn[v]) + xor_lanes<8>(b3 ? sn[v] : sn[2 + v]);
  float x = (b2 ? t[1] : t[0]) + xor_lanes<4>(b2 ? t[0] : t[1]);
  x += xor_lanes<2>(x);
  x += xor_lanes<1>(x);
  if ((lane & 3) == 0) {
    const int r = (tid >> 4) + 16 * (2 * b3 + b2);
    nrm[r] = x;
  }
  if (mx_n) *mx_n = fmaxf(*mx_n, x);
}

// Pairs whose image-2 rows get BF16 copies for the wide-row pass: those
// with at least one wide tile per kPreRows image-2 rows (each wide tile
// stages a window of more than kStage rows).
constexpr uint32_t kPreRows = 256;
__device__ __forceinline__ bool pair_pre(const StabArgs& A, int p) {
  return (uint64_t)A.pair_wide[p] * kPreRows >= (uint64_t)A.pairs[p].n;
}

// 64 pre-rounded BF16 rows (launch_round_rows) with their terms, held in the
// registers of a Rows: the codes as in Codes in v[0 .. kCodePer), and for
// thread r < 64 the terms of row r in v[kCodePer].
__device__ __forceinline__ void fetch_pre(Rows& R, const uint16_t* __restrict__ codes,
                                          const float2* __restrict__ terms,
                                          const int64_t* row_of, int tid) {
  const Codes C = fetch_codes(codes, row_of, tid);
  #pragma unroll
  for (int u = 0; u < kCodePer; ++u) R.v[u] = __builtin_bit_cast(float4, C.v[u]);
  float2 t = make_float2(0.0f, 0.0f);
  if (tid < kL) {
    const int64_t row = row_of[tid];
    if (row >= 0) t = terms[row];
  }
  R.v[kCodePer] = make_float4(t.x, t.y, 0.0f, 0.0f);
}

// Stores the rows of fetch_pre (stride kRS) and their squared norms; this
// thread's running maxima of the norms and rounding errors of its row.
__device__ __forceinline__ void stage_pre(const Rows& R, uint8_t* dst, float* nrm, float* mx_n,
                                          float* mx_e, int tid) {
  #pragma unroll
  for (int u = 0; u < kCodePer; ++u) {
    const int f = tid + u * kThreads;
    *reinterpret_cast<uint4*>(dst + (f >> 4) * kRS + (f & 15) * 16) =
        __builtin_bit_cast(uint4, R.v[u]);
  }
  if (tid < kL) {
    const float tn = R.v[kCodePer].x, te = R.v[kCodePer].y;
    nrm[tid] = tn;
    *mx_n = fmaxf(*mx_n, tn);
    *mx_e = fmaxf(*mx_e, te);
  }
}

// One window entry in ascending j: its image-2 index and record.
struct Entry {
  int32_t j;
  uint32_t C, H;
  float2 xy;
  float e;
};

// Signed-integer image of a float that keeps the order of non-NaN values
// (negative values get their magnitude bits flipped).
__device__ __forceinline__ int32_t order_key(float f) {
  const int32_t b = __float_as_int(f);
  return b >= 0 ? b : b ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float order_key_inv(int32_t k) {
  return __int_as_float(k >= 0 ? k : k ^ 0x7FFFFFFF);
}

// Minimum over the wavefront (uniform result): lanes take the minimum with a
// neighbour's value by DPP, INT32_MAX standing in where no neighbour is given.
__device__ __forceinline__ int32_t wave_min(int32_t v) {
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x141, 0xF, 0xF, false));  // half-row mirror
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x140, 0xF, 0xF, false));  // row mirror
  // every lane of a row holds the row's minimum: rows 1 and 3 take lane 15 of
  // the row below, rows 2 and 3 lane 31; lane 63 ends with the minimum of all
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x142, 0xA, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x143, 0xC, 0xF, false));
  return __builtin_amdgcn_readlane(v, kWave - 1);
}

// Maximum over the wavefront of non-negative floats (uniform result).
__device__ __forceinline__ float wave_max(float v) {
  return __int_as_float(-wave_min(-__float_as_int(v)));
}

// A 4 x 4 transpose of 16-lane rows across four registers: afterwards row g
// of register r holds what row r of register g held (v_permlane32_swap swaps
// the upper half of its first operand with the lower half of its second,
// v_permlane16_swap the odd rows of its first with the even rows of its second).
__device__ __forceinline__ void transpose_rows(float& r0, float& r1, float& r2, float& r3) {
  auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(r0), __float_as_uint(r2), false, false);
  auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(r1), __float_as_uint(r3), false, false);
  auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
  auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
  r0 = __uint_as_float(s01[0]);
  r1 = __uint_as_float(s01[1]);
  r2 = __uint_as_float(s23[0]);
  r3 = __uint_as_float(s23[1]);
}

// Merges a block's survivors into a query's kept list: lk / lj in lanes
// 0 .. kK - 1 hold the list (ascending keys, +inf and -1 past its end), the
// lanes of surv the survivors' keys kv and image-2 indices jv.  The kK
// smallest keys of both are taken one at a time by wavefront minima and
// leave lk / lj ascending; returns the largest kept key (+inf while fewer
// than kK are kept).  Equal keys may be taken in any order.
template <int kK>
__device__ __forceinline__ float merge_list(float& lk, int32_t& lj, uint64_t surv, float kv,
                                            int32_t jv) {
  const int lane = lane_id();
  constexpr int32_t kInf = 0x7F800000;  // order_key(+inf)
  int32_t ca = order_key(lk);
  int32_t cb = (surv >> lane) & 1ull ? order_key(kv) : INT32_MAX;
  float nk = __builtin_inff();
  int32_t nj = -1;
  #pragma unroll 1
  for (int r = 0; r < kK; ++r) {
    const int32_t mn = wave_min(min(ca, cb));
    if (mn >= kInf) break;  // uniform: nothing left
    const uint64_t at_a = ballot(ca == mn);
    int32_t js;
    if (at_a) {
      const int L = __builtin_ctzll(at_a);
      js = __builtin_amdgcn_readlane(lj, L);
      if (lane == L) ca = INT32_MAX;
    } else {
      const int L = __builtin_ctzll(ballot(cb == mn));
      js = __builtin_amdgcn_readlane(jv, L);
      if (lane == L) cb = INT32_MAX;
    }
    if (lane == r) {
      nk = order_key_inv(mn);
      nj = js;
    }
  }
  lk = nk;
  lj = nj;
  return readlane_f(nk, kK - 1);
}

// Copies of the image-2 rows (A.wcodes2, A.wterms2, for the pairs pair_pre
// picks) by PRE: kPreNone none (rounding on chip); kPreOnly the tiles of
// those pairs only, staging the copies; kPreOthers the other tiles only,
// rounding on chip; kPreMixed every tile, each as its pair has copies.
constexpr int kPreNone = 0, kPreOnly = 1, kPreOthers = 2, kPreMixed = 3;
template <int MODE, int PRE>
__global__ __launch_bounds__(kThreads, MODE == kWideFill ? 1 : 3) void k_wide_tile(StabArgs A) {
  constexpr bool MATCH = MODE != kWideFill;
  constexpr bool WRITE = MODE == kWideFill || MODE == kWideFused;  // writes the CSR
  constexpr bool CODES = MODE == kWideMatchBF16;                     // caller's BF16 codes
  static_assert(PRE == kPreNone || (MATCH && !CODES), "copies of FP32 rows only");
  // bitmap slab and word prefix; after the window sweep the picks live here
  __shared__ __attribute__((aligned(16))) unsigned char slab_raw[kSlabWords * 12];
  unsigned long long* bits = reinterpret_cast<unsigned long long*>(slab_raw);
  uint32_t* wpref = reinterpret_cast<uint32_t*>(slab_raw + kSlabWords * 8);
  __shared__ uint32_t wsum[kWaves], n_entries;
  // one super-chunk of window entries
  __shared__ int32_t lj[kSC];
  __shared__ uint32_t lC[kSC], lH[kSC];
  __shared__ float2 lXY[kSC];
  __shared__ float lE[kSC];
  __shared__ double4 qline_s[kTileQ];  // a, b, c and sqrt(a^2 + b^2) of each query's line
  __shared__ uint32_t qk[kTileQ], q_len[kTileQ], q_bad[kTileQ];
  __shared__ int64_t q_i[kTileQ], q_o0[kTileQ];
  __shared__ uint32_t slot_b[kSlots], slot_pref[kSlots + 1];
  __shared__ uint64_t wide_mask_s;
  // matching only
  constexpr int kQ = MATCH ? kTileQ : 1;
  constexpr int kRaw = MATCH ? kL * kRS : 16;
  // BF16 query rows, then block rows, then FP32 query rows of the re-rank
  __shared__ __attribute__((aligned(16))) uint8_t raw[kRaw];
  __shared__ int64_t row_of[MATCH ? kSC : 1];  // global image-2 row of each entry, -1 past the end
  __shared__ float w_norm[MATCH ? kL : 1];
  __shared__ float q_norm[kQ], q_err[kQ];
  __shared__ uint32_t max_nb, max_db;  // float bits of the largest window row terms
  __shared__ uint32_t n_cert, n_fallback;
  // per query the kPicks + 1 smallest keys so far, ascending, with their j
  constexpr int kK = kPicks + 1;
  __shared__ float tkl[kQ * kK];
  __shared__ int32_t tjl[kQ * kK];

  const int tile = A.block_tile ? (int)A.block_tile[blockIdx.x] : xcd_tile(blockIdx.x, A.num_tiles);
  if (A.tile_wide[tile] == 0u) return;
  // a caller's CSR that did not fit its buffer is incomplete: nothing is written
  if (!WRITE && A.row_offsets[A.n1] > A.capacity) return;
  const StabTile T = A.tiles[tile];
  const PairDev& pd = A.pairs[T.pair];
  const int64_t kb = pd.k_begin, n2 = pd.n;
  bool pre = false;  // uniform
  if (PRE == kPreOnly || PRE == kPreOthers) {
    if (pair_pre(A, T.pair) != (PRE == kPreOnly)) return;
    pre = PRE == kPreOnly;
  } else if (PRE == kPreMixed) {
    pre = pair_pre(A, T.pair);
  }
  const int tid = threadIdx.x, lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(wave_id());

  if (wave == 0) {
    const bool live = lane < T.count;
    int64_t i = 0, o0 = 0, len = 0;
    uint32_t flag = kQueryEmpty, key = 0;
    double4 L = make_double4(0.0, 0.0, 0.0, 0.0);
    if (live) {
      i = A.qperm[T.begin + lane];
      flag = A.qflag[i];
      key = A.qkey[i];
      o0 = A.row_offsets[i];
      len = A.row_offsets[i + 1] - o0;
      if (flag == kQueryNormal) L = A.qline[i];
    }
    // writing: the long rows of normal queries; matching a caller's CSR:
    // every normal query of the tile
    const bool wide = live && flag == kQueryNormal && (WRITE ? len > kStage : len > 0);
    if (!WRITE && live && !wide) {
      if (len == 0) {
        write_match_to(A.ratio, A.best_idx, A.best_dist, A.second_dist, i, Top2(), false);
      } else {  // a brute-force query: exact listed match
        const unsigned long long at = atomicAdd(A.rest_count, 1ull);
        A.rest[at] = (uint32_t)i;
        if (A.match_stats) atomicAdd(&A.match_stats[2], 1ull);
      }
    }
    // a NaN norm fails every test of Eq. 3: the queries that are not wide hit nothing
    if (!wide) L.w = __builtin_nan("");
    qline_s[lane] = L;
    qk[lane] = key;
    q_i[lane] = i;
    q_o0[lane] = o0;
    q_len[lane] = (uint32_t)len;
    const uint64_t wm = ballot(wide);
    const TileWindow* W = A.windows + tile;
    slot_b[lane] = W->slot_b[lane];
    slot_pref[lane] = W->slot_pref[lane];
    if (lane == 0) {
      slot_pref[kSlots] = W->slot_pref[kSlots];
      wide_mask_s = wm;
      if (MATCH) {
        max_nb = 0u;
        max_db = 0u;
        n_cert = 0u;
        n_fallback = 0u;
      }
    }
  }
  __syncthreads();
  const uint64_t wide_mask = wide_mask_s;
  const int q0 = wave * kQPerWave;  // this wavefront's queries
  // lane l < 16 holds query q0 + l's row start, its CSR write position and
  // (match) the largest kept key of its list -- read through readlane
  const int ql = q0 + (lane & (kQPerWave - 1));
  const int64_t qp_o0 = q_o0[ql];
  const uint32_t qp_len = q_len[ql];
  uint32_t run[kQPerWave];  // hits so far of each query of the wavefront (uniform)
  #pragma unroll
  for (int qq = 0; qq < kQPerWave; ++qq) run[qq] = 0u;
  // a CSR that fits the caller's buffer whole needs no check per hit
  const bool fits = A.row_offsets[A.n1] <= A.capacity;
  float thr[kQPerWave];  // (match) the largest kept key of each query's list (uniform)
  #pragma unroll
  for (int qq = 0; qq < kQPerWave; ++qq) thr[qq] = __builtin_inff();
  uint32_t badbits = 0u;  // matching a caller's CSR: queries whose row differs here
  // largest squared norm (and rounding error) of the window rows this thread summed
  float mx_n = 0.0f, mx_e = 0.0f;

  // the MFMA's A operand: BF16 rows of this wavefront's queries, k-slices
  // 32 kk + 8 (lane >> 4) .. + 7 of row q0 + (lane & 15)
  bf16x8 afrag[4];
  if (MATCH) {
    for (int t = tid; t < kTileQ * kK; t += kThreads) {
      tkl[t] = __builtin_inff();
      tjl[t] = -1;
    }
    if (CODES)  // zero rows for the queries that are not wide
      stage_codes(fetch_query_codes(A.codes1, q_i, wide_mask, tid), raw, q_norm, nullptr, tid);
    else
      stage_bf16(fetch_query_rows(A.desc1, q_i, wide_mask, tid), raw, q_norm, q_err, nullptr,
                 nullptr, tid);
    __syncthreads();
    #pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      afrag[kk] = *reinterpret_cast<const bf16x8*>(raw + ql * kRS + (kk * 32 + (lane >> 4) * 8) * 2);
    // the block rows overwrite these only after the slab set-up's barriers
  }
  uint8_t* wrows = raw;

  const int64_t total_len = slot_pref[kSlots];
  const int64_t nslabs = (n2 + kSlabBits - 1) / kSlabBits;
  for (int64_t sb = 0; sb < nslabs; ++sb) {
    const int64_t j0 = sb * kSlabBits;
    const int64_t jn = n2 - j0 < kSlabBits ? n2 - j0 : kSlabBits;
    const int nwords = (int)((jn + 63) >> 6);
    for (int w = tid; w < kSlabWords; w += kThreads) bits[w] = 0ull;
    __syncthreads();
    // mark the window's j that fall in this slab (four loads in flight per thread)
    for (int64_t v0 = tid; v0 < total_len; v0 += 4 * kThreads) {
      int64_t jj[4];
      #pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t v = v0 + u * kThreads;
        jj[u] = -1;
        if (v < total_len) {
          int s = 0;  // last slot with slot_pref[s] <= v
          #pragma unroll
          for (int step = 32; step > 0; step >>= 1)
            if (s + step <= kSlots && slot_pref[s + step] <= v) s += step;
          jj[u] = (int64_t)A.rj[slot_b[s] + (v - slot_pref[s])] - j0;
        }
      }
      #pragma unroll
      for (int u = 0; u < 4; ++u)
        if (jj[u] >= 0 && jj[u] < jn) atomicOr(&bits[jj[u] >> 6], 1ull << (jj[u] & 63));
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
      uint32_t r = base + incl - tot;
      #pragma unroll
      for (int u = 0; u < 4; ++u) {
        wpref[tid * 4 + u] = r;
        r += c[u];
      }
      if (tid == 0) n_entries = all;
    }
    __syncthreads();
    const uint32_t E = n_entries;

    // entry e of the slab: its j, then its record (the loads stay in flight
    // until the entry is stored)
    auto entry_j = [&](uint32_t e) -> int32_t {
      if (e >= E) return -1;
      int w = 0;  // last word with wpref[w] <= e (it holds entry e)
      #pragma unroll
      for (int step = kSlabWords / 2; step > 0; step >>= 1)
        if (w + step < nwords && wpref[w + step] <= e) w += step;
      return (int32_t)(j0 + ((int64_t)w << 6) + select_bit(bits[w], e - wpref[w]));
    };
    auto load_entry = [&](int32_t j) -> Entry {
      Entry en;
      en.j = j;
      if (j >= 0) {
        const uint32_t pos = A.rinv[kb + j];
        en.C = A.rC[pos];
        en.H = A.rH[pos];
        en.xy = A.rxy[pos];
        en.e = A.reps[pos];
      }
      return en;
    };
    auto store_entry = [&](const Entry& en) {
      lj[tid] = en.j;
      lC[tid] = en.C;
      lH[tid] = en.H;
      lXY[tid] = en.xy;
      lE[tid] = en.e;
      if (MATCH) row_of[tid] = en.j >= 0 ? kb + en.j : -1;
    };
    if (E > 0) store_entry(load_entry(entry_j(tid)));
    __syncthreads();

    for (uint32_t e0 = 0; e0 < E; e0 += kSC) {
      Rows rw;  // the next block's FP32 rows, or their copies (fetch_pre)
      Codes prc;
      if (CODES) prc = fetch_codes(A.codes2, row_of, tid);  // block 0
      else if (pre) fetch_pre(rw, A.wcodes2, A.wterms2, row_of, tid);
      else if (MATCH) rw = fetch_rows(A.desc2, row_of, tid);
      // the next super-chunk's entry: j now, its record during the blocks
      const int32_t nj = e0 + kSC < E ? entry_j(e0 + kSC + tid) : -1;
      Entry nxt;
      #pragma unroll 1
      for (int sub = 0; sub < kSub; ++sub) {
        const int base = sub * kL;
        if (e0 + base >= E) break;  // uniform
        float wn = 0.0f;
        if (MATCH) {
          if (CODES) stage_codes(prc, wrows, w_norm, &mx_n, tid);
          else if (pre) stage_pre(rw, wrows, w_norm, &mx_n, &mx_e, tid);
          else stage_bf16(rw, wrows, w_norm, nullptr, &mx_n, &mx_e, tid);
          __syncthreads();  // block rows and norms complete
          wn = w_norm[lane];
          if (sub + 1 < kSub && e0 + base + kL < E) {
            if (CODES) prc = fetch_codes(A.codes2, row_of + base + kL, tid);
            else if (pre) fetch_pre(rw, A.wcodes2, A.wterms2, row_of + base + kL, tid);
            else rw = fetch_rows(A.desc2, row_of + base + kL, tid);
          }
        }
        if (sub == 0 && nj >= 0) nxt = load_entry(nj);
        // this lane's entry of the block
        const int32_t ej = lj[base + lane];
        const uint32_t eC = lC[base + lane], eH = lH[base + lane];
        const float2 exy = lXY[base + lane];
        const double ex = (double)exy.x, ey = (double)exy.y, ee = (double)lE[base + lane];
        const bool live_e = ej >= 0;
        // 1. hit masks: every query of the wavefront against the block
        // (angle test, then the FP64 test of Eq. 3), one ballot per query
        // the queries' terms are read here and the lane tests made here, not
        // kept in registers across blocks
        int qb = q0, lsel = lane;
        asm volatile("" : "+s"(qb), "+v"(lsel));
        uint64_t hm[kQPerWave];
        #pragma unroll
        for (int qq = 0; qq < kQPerWave; ++qq) {
          const double4 L = qline_s[qb + qq];
          const uint32_t k = qk[qb + qq];
          const bool hit = live_e & (key_distance(k, eC) <= eH) &
                           within_tolerance_d(L.x, L.y, L.z, L.w, ex, ey, ee);
          hm[qq] = ballot(hit);
          if ((qq & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // four queries' terms at a time
        }
        // 2. the hits extend (or are checked against) the queries' CSR rows,
        // in ascending j
        #pragma unroll
        for (int qq = 0; qq < kQPerWave; ++qq) {
          const uint64_t m = hm[qq];
          if (m == 0ull) continue;  // uniform
          if ((m >> lane) & 1ull) {
            const uint32_t k = run[qq] + lanes_below(m);
            const int64_t dst = (int64_t)readlane_u64((uint64_t)qp_o0, qq) + k;
            if (WRITE) {
              if (fits || dst < A.capacity) A.cols[dst] = ej;
            } else {
              // the caller's row must hold this hit at this place
              const int32_t got =
                  k < (uint32_t)__builtin_amdgcn_readlane((int)qp_len, qq) ? A.cols[dst] : -2;
              if (got != ej) badbits |= 1u << qq;
            }
          }
          run[qq] += (uint32_t)__popcll(m);
        }
        // approximate keys |w^|^2 - 2 q^.w^ of this lane's entry base + lane
        // for the wavefront's 16 queries
        float kf[kQPerWave];
        if (MATCH) {
          // S = Q W^T: the wavefront's 16 queries against the 64 rows; lane
          // (g, c) = (lane >> 4, lane & 15) gets S[4 g + i][16 cb + c] in acc[cb][i]
          f32x4 acc[4];
          #pragma unroll
          for (int cb = 0; cb < 4; ++cb) acc[cb] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
          #pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int koff = kk * 32 + (lane >> 4) * 8;  // element offset of this lane's 8 values
            #pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
              const bf16x8 b = *reinterpret_cast<const bf16x8*>(
                  wrows + (cb * 16 + (lane & 15)) * kRS + koff * 2);
              acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag[kk], b, acc[cb], 0, 0, 0);
            }
          }
          __syncthreads();  // every wavefront has read the block rows
          // exchange rows and blocks: lane (g, c) then holds S[4 r + i][16 g + c],
          // the scores of its own entry 16 g + c, in acc[r][i]
          #pragma unroll
          for (int i = 0; i < 4; ++i) {
            float r0 = acc[0][i], r1 = acc[1][i], r2 = acc[2][i], r3 = acc[3][i];
            transpose_rows(r0, r1, r2, r3);
            kf[i] = __builtin_fmaf(-2.0f, r0, wn);
            kf[4 + i] = __builtin_fmaf(-2.0f, r1, wn);
            kf[8 + i] = __builtin_fmaf(-2.0f, r2, wn);
            kf[12 + i] = __builtin_fmaf(-2.0f, r3, wn);
          }
        }
        // 3. (match) hits below a query's kept (kPicks+1)-th key enter its list
        if (MATCH) {
          // this lane's slot of the wavefront's first list (constant offsets from here)
          float* const tk0 = tkl + q0 * kK + lane;
          int32_t* const tj0 = tjl + q0 * kK + lane;
          #pragma unroll
          for (int qq = 0; qq < kQPerWave; ++qq) {
            const uint64_t m = hm[qq];
            if (m == 0ull) continue;
            const float th0 = thr[qq];
            uint64_t surv = m & ballot(kf[qq] < th0);
            if (surv == 0ull) continue;
            const bool in = lane < kK;
            float lk = in ? tk0[qq * kK] : __builtin_inff();
            int32_t lji = in ? tj0[qq * kK] : -1;
            float th = th0;
            if (__popcll(surv) > kMergeMin) {
              th = merge_list<kK>(lk, lji, surv, kf[qq], ej);
            } else {
              do {  // one survivor at a time
                const int sl = __builtin_ctzll(surv);
                surv &= surv - 1;
                const float ks = readlane_f(kf[qq], sl);
                if (!(ks < th)) continue;
                const int32_t js = __builtin_amdgcn_readlane(ej, sl);
                // the new key goes after the kept keys that are <= it; the
                // ones above move up one lane
                const int pos = __popcll(ballot(in && lk <= ks));
                const float up_k = row_shift_up(lk);
                const int32_t up_j = row_shift_up(lji);
                if (lane == pos) {
                  lk = ks;
                  lji = js;
                } else if (lane > pos) {
                  lk = up_k;
                  lji = up_j;
                }
                th = readlane_f(lk, kPicks);
              } while (surv);
            }
            if (in) {
              tk0[qq * kK] = lk;
              tj0[qq * kK] = lji;
            }
            thr[qq] = th;
          }
        }
      }
      __syncthreads();  // the super-chunk's entries are dead
      if (nj >= 0 || e0 + kSC < E) {
        if (nj < 0) nxt.j = -1;
        store_entry(nxt);
      }
      __syncthreads();
    }
  }

  if (!MATCH) return;
  {
    // the largest row terms of the window (the bound terms are monotone in
    // the sums): relative slack 2e-5 covers the FP32 sums (at most 2^-24 per term)
    const float wn_max = wave_max(mx_n);
    const float we_max = wave_max(mx_e);
    if (lane == 0) {
      const double nb = sqrt((double)wn_max) * (1.0 + 2e-5);
      const double db = CODES ? row_delta<0>(nb, 1.0) * (1.0 + 1e-6)
                              : sqrt((double)we_max) * (1.0 + 2e-5) + 1e-30;
      atomicMax(&max_nb, __float_as_uint((float)nb));
      atomicMax(&max_db, __float_as_uint((float)db));
    }
  }
  if (!WRITE) {
    // rows that differ from the tile's candidate sets (a hit missing or out
    // of place, or a different length) are evaluated exactly
    #pragma unroll
    for (int qq = 0; qq < kQPerWave; ++qq) {
      const bool bad = ballot((badbits >> qq) & 1u) != 0ull;
      if (lane == qq) q_bad[q0 + qq] = bad || run[qq] != qp_len ? 1u : 0u;
    }
  }
  // the picks are the first kPicks of every list; the bitmap area holds their
  // exact distances, the row area the FP32 rows of half the queries at a time
  const float* pk = tkl;
  const int32_t* pj = tjl;
  float* pdist = reinterpret_cast<float*>(slab_raw);  // [kTileQ][kPicks]
  float* qf = reinterpret_cast<float*>(raw);          // [kTileQ / 2][kQS]
  constexpr int kHalf = kTileQ / 2;
  #pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    __syncthreads();  // the row area is free
    #pragma unroll
    for (int u = 0; u < kHalf * 32 / kThreads; ++u) {
      const int f = tid + u * kThreads, r = f >> 5, q = kHalf * h + r;
      reinterpret_cast<float4*>(qf + r * kQS)[f & 31] =
          (wide_mask >> q) & 1ull ? reinterpret_cast<const float4*>(A.desc1)[q_i[q] * 32 + (f & 31)]
                                  : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    // exact canonical distances of the picks: thread = (query, pick)
    const int r = tid / kPicks, u = tid % kPicks, sq = kHalf * h + r;
    if (r < kHalf) {
      float d = __builtin_inff();
      const int32_t j = pj[sq * kK + u];
      if (((wide_mask >> sq) & 1ull) && j >= 0)
        d = exact_distance(reinterpret_cast<const float4*>(qf + r * kQS),
                           reinterpret_cast<const float4*>(A.desc2) + (kb + j) * 32);
      pdist[sq * kPicks + u] = d;
    }
  }
  __syncthreads();
  if (tid < kTileQ && ((wide_mask >> tid) & 1ull)) {
    const int q = tid;
    Top2 t;
    #pragma unroll
    for (int u = 0; u < kPicks; ++u)
      if (pj[q * kK + u] >= 0) t.insert(pdist[q * kPicks + u], pj[q * kK + u]);
    // every other hit has a key >= the (kPicks+1)-th key: its exact distance
    // is at least the bound of the smallest such approximate distance, with
    // the largest row terms of the window and a slack for the key's rounding
    const double qnb = sqrt((double)q_norm[q]) * (1.0 + 2e-5);
    const double qdb = CODES ? row_delta<0>(qnb, 1.0) * (1.0 + 1e-6)
                             : sqrt((double)q_err[q]) * (1.0 + 2e-5) + 1e-30;
    const double nw = (double)__uint_as_float(max_nb), dw = (double)__uint_as_float(max_db);
    const double s = qnb + nw;
    const double dt = (double)q_norm[q] + (double)pk[q * kK + kPicks] - 1e-6 * s * s;
    const double lb = lower_bound(dt, qnb, nw, qdb, dw);
    if (lb > (double)t.sd && (WRITE || q_bad[q] == 0u)) {
      write_match_to(A.ratio, A.best_idx, A.best_dist, A.second_dist, q_i[q], t, false);
      atomicAdd(&n_cert, 1u);
    } else {
      const unsigned long long at = atomicAdd(A.rest_count, 1ull);
      A.rest[at] = (uint32_t)q_i[q];
      atomicAdd(&n_fallback, 1u);
    }
  }
  if (A.match_stats) {
    __syncthreads();
    if (tid == 0 && n_cert + n_fallback) {
      atomicAdd(&A.match_stats[0], (unsigned long long)(n_cert + n_fallback));
      if (n_fallback) atomicAdd(&A.match_stats[1], (unsigned long long)n_fallback);
    }
  }
}

// The pairs pair_pre picks, compacted: the k-th listed pair in pair_of[k],
// the exclusive prefix of their image-2 row counts in start[k] (start[count]
// the total); returns count.  The whole workgroup (kPreThreads) calls it.
constexpr int kPreThreads = 256;
template <typename Start, typename Pair>
__device__ int list_pre_pairs(const StabArgs& A, Start* start, Pair* pair_of, int64_t* sn, int* sc) {
  const int tid = threadIdx.x, P = A.num_pairs;
  int count = 0;
  int64_t rows = 0;
  for (int base = 0; base < P; base += kPreThreads) {
    const int p = base + tid;
    const bool take = p < P && pair_pre(A, p);
    const int64_t n = take ? A.pairs[p].n : 0;
    sn[tid] = n;
    sc[tid] = take ? 1 : 0;
    __syncthreads();
    for (int off = 1; off < kPreThreads; off <<= 1) {  // inclusive scans
      const int64_t on = tid >= off ? sn[tid - off] : 0;
      const int oc = tid >= off ? sc[tid - off] : 0;
      __syncthreads();
      sn[tid] += on;
      sc[tid] += oc;
      __syncthreads();
    }
    if (take) {
      const int k = count + sc[tid] - 1;
      start[k] = rows + sn[tid] - n;
      pair_of[k] = p;
    }
    count += sc[kPreThreads - 1];
    rows += sn[kPreThreads - 1];
    __syncthreads();  // the scan arrays are reused
  }
  if (tid == 0) start[count] = rows;
  __syncthreads();
  return count;
}

// The list of list_pre_pairs in global memory, for batches of more than
// kPreLocal pairs: pre[0] = count, pre[1 ..] the starts, pre[P + 2 ..] the pairs.
constexpr int kPreLocal = 1024;
__global__ __launch_bounds__(kPreThreads) void k_pre_pairs(StabArgs A, int64_t* __restrict__ pre) {
  __shared__ int64_t sn[kPreThreads];
  __shared__ int sc[kPreThreads];
  const int count = list_pre_pairs(A, pre + 1, pre + A.num_pairs + 2, sn, sc);
  if (threadIdx.x == 0) pre[0] = count;
}

// BF16 copies of the image-2 rows of the listed pairs: 32 threads per row,
// four values each, rounded as stage_bf16 rounds them, with the squared norm
// of the copy and of its rounding error (sums over the 32 threads).
// Grid-stride over the listed rows.  pre: the global list, or NULL for a
// batch of at most kPreLocal pairs, whose list each workgroup makes in LDS.
constexpr int kRoundRows = 8;  // rows per workgroup and step
static_assert(kRoundRows * 32 == kPreThreads, "one workgroup shape");
__global__ __launch_bounds__(kPreThreads) void k_round_rows(StabArgs A,
                                                            const int64_t* __restrict__ pre) {
  __shared__ int64_t l_start[kPreLocal + 1];
  __shared__ int l_pair[kPreLocal];
  __shared__ int64_t sn[kPreThreads];
  __shared__ int sc[kPreThreads];
  const int P = A.num_pairs;
  const int64_t* g_start = pre ? pre + 1 : nullptr;
  const int64_t* g_pair = pre ? pre + P + 2 : nullptr;
  const int count = pre ? (int)pre[0] : list_pre_pairs(A, l_start, l_pair, sn, sc);
  const int64_t total = pre ? g_start[count] : l_start[count];
  const int c = (int)(threadIdx.x & 31);
  for (int64_t r = (int64_t)blockIdx.x * kRoundRows + (threadIdx.x >> 5); r < total;
       r += (int64_t)gridDim.x * kRoundRows) {
    int lo = 0, hi = count - 1;  // the listed pair whose rows hold r
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((pre ? g_start[mid] : l_start[mid]) <= r) lo = mid;
      else hi = mid - 1;
    }
    const int p = pre ? (int)g_pair[lo] : l_pair[lo];
    const int64_t row = A.pairs[p].k_begin + (r - (pre ? g_start[lo] : l_start[lo]));
    const float4 x = reinterpret_cast<const float4*>(A.desc2)[row * 32 + c];
    uint2 w;
    w.x = bf16_pack(x.x, x.y);
    w.y = bf16_pack(x.z, x.w);
    reinterpret_cast<uint2*>(const_cast<uint16_t*>(A.wcodes2))[row * 32 + c] = w;
    const float y0 = __uint_as_float(w.x << 16), y1 = __uint_as_float(w.x & 0xFFFF0000u),
                y2 = __uint_as_float(w.y << 16), y3 = __uint_as_float(w.y & 0xFFFF0000u);
    const float e0 = x.x - y0, e1 = x.y - y1, e2 = x.z - y2, e3 = x.w - y3;  // exact
    float n = __builtin_fmaf(y3, y3, __builtin_fmaf(y2, y2, __builtin_fmaf(y1, y1, y0 * y0)));
    float e = __builtin_fmaf(e3, e3, __builtin_fmaf(e2, e2, __builtin_fmaf(e1, e1, e0 * e0)));
    n += xor_lanes<16>(n);
    e += xor_lanes<16>(e);
    n += xor_lanes<8>(n);
    e += xor_lanes<8>(e);
    n += xor_lanes<4>(n);
    e += xor_lanes<4>(e);
    n += xor_lanes<2>(n);
    e += xor_lanes<2>(e);
    n += xor_lanes<1>(n);
    e += xor_lanes<1>(e);
    if (c == 0) const_cast<float2*>(A.wterms2)[row] = make_float2(n, e);
  }
}

constexpr int kSplitTilesMin = 2048, kSplitTilesMax = 16384;

}  // namespace

hipError_t launch_wide_tiles(const StabArgs& a, int mode, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  if (!a.tile_wide || !a.qline) return hipErrorInvalidValue;
  if (mode != kWideFill &&
      (!a.desc1 || !a.desc2 || !a.best_idx || !a.best_dist || !a.second_dist || !a.rest ||
       !a.rest_count))
    return hipErrorInvalidValue;
  if (mode == kWideMatchBF16 && (!a.codes1 || !a.codes2)) return hipErrorInvalidValue;
  const dim3 g(a.num_tiles), b(kThreads);
  // with copies: one launch for the tiles of the pairs that have them and one
  // for the others (each kernel lean), or one launch that decides per tile,
  // where a second launch would cost more than it saves: a few microseconds
  // on small grids, about one workgroup slot per tile on large ones
  const bool copies = a.wcodes2 && a.wterms2;
  const bool split = copies && a.num_tiles > kSplitTilesMin && a.num_tiles <= kSplitTilesMax;
  switch (mode) {
    case kWideFill: hipLaunchKernelGGL((k_wide_tile<kWideFill, kPreNone>), g, b, 0, s, a); break;
    case kWideFused:
      if (split) {
        hipLaunchKernelGGL((k_wide_tile<kWideFused, kPreOnly>), g, b, 0, s, a);
        hipLaunchKernelGGL((k_wide_tile<kWideFused, kPreOthers>), g, b, 0, s, a);
      } else if (copies) {
        hipLaunchKernelGGL((k_wide_tile<kWideFused, kPreMixed>), g, b, 0, s, a);
      } else {
        hipLaunchKernelGGL((k_wide_tile<kWideFused, kPreNone>), g, b, 0, s, a);
      }
      break;
    case kWideMatchF32:
      if (split) {
        hipLaunchKernelGGL((k_wide_tile<kWideMatchF32, kPreOnly>), g, b, 0, s, a);
        hipLaunchKernelGGL((k_wide_tile<kWideMatchF32, kPreOthers>), g, b, 0, s, a);
      } else if (copies) {
        hipLaunchKernelGGL((k_wide_tile<kWideMatchF32, kPreMixed>), g, b, 0, s, a);
      } else {
        hipLaunchKernelGGL((k_wide_tile<kWideMatchF32, kPreNone>), g, b, 0, s, a);
      }
      break;
    case kWideMatchBF16:
      hipLaunchKernelGGL((k_wide_tile<kWideMatchBF16, kPreNone>), g, b, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_round_rows(const StabArgs& a, int64_t n2, int64_t* pre, hipStream_t s) {
  if (n2 == 0) return hipSuccess;
  if (!a.desc2 || !a.wcodes2 || !a.wterms2 || !a.pair_wide || !a.pairs || !pre)
    return hipErrorInvalidValue;
  const bool global_list = a.num_pairs > kPreLocal;
  if (global_list) hipLaunchKernelGGL(k_pre_pairs, dim3(1), dim3(kPreThreads), 0, s, a, pre);
  // grid-stride: enough workgroups to stream the rows of a large batch
  const int64_t want = (n2 + kRoundRows - 1) / kRoundRows;
  const int64_t blocks = want < 1024 ? want : 1024;
  hipLaunchKernelGGL(k_round_rows, dim3((unsigned)blocks), dim3(kPreThreads), 0, s, a,
                     global_list ? (const int64_t*)pre : nullptr);
  return hipGetLastError();
}

}  // namespace epm
