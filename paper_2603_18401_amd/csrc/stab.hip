// Stabbing query (Sec. 4.2, Algorithm 1 match loop): every query's angle key
// is tested against the angle-sorted intervals of its pair; each angular hit
// is confirmed by the FP64 point-line test (Eq. 3), so the rows are exactly
// the candidate sets of Eq. 4.
//
// Queries are taken in tiles of kTileQ angle-sorted queries of one pair.  For
// width class c the only centres that can hold a key lie within 2^c - 1 key
// units of it, so the window pass finds each tile's record window in every
// class; the tile pass tests every (query, record) pair of the window, writes
// the row lengths and parks short rows.  After the scan of the lengths the
// fill pass copies the parked rows and rebuilds the long rows of brute-force
// queries one wavefront per query (scan, LDS sort by j); long rows of normal
// queries are written tile by tile by the wide-row pass.  The tile pass can
// also select every short row's match (Sec. 4.3) while its hits are on chip:
// FP32 chains, or MFMA bounds over BF16 or FP8 rows with an exact FP32
// re-rank.
#include "device_common.h"
#include "launch.h"
#include "match_common.h"
#include "mfma_bounds.h"

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

// Writes query i's CSR row in ascending j (rows of any length).
__device__ void fill_row(const StabArgs& A, int64_t i, int32_t* buf) {
  const int lane = lane_id();
  const int pair = find_pair(A.qstart, A.num_pairs, i);
  const PairDev& pd = A.pairs[pair];
  const uint32_t flag = A.qflag[i];
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
    constexpr int kU = 4;  // blocks of 64 j whose gathers are in flight together
    for (int64_t j0 = 0; j0 < pd.n; j0 += kU * kWave) {
      uint32_t pos[kU];
      #pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int64_t j = j0 + u * kWave + lane;
        pos[u] = j < pd.n ? A.rinv[kb + j] : 0u;
      }
      float2 xy[kU];
      float ee[kU];
      #pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int64_t j = j0 + u * kWave + lane;
        xy[u] = j < pd.n ? A.rxy[pos[u]] : make_float2(0.0f, 0.0f);
        ee[u] = j < pd.n ? A.reps[pos[u]] : 0.0f;
      }
      #pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int64_t j = j0 + u * kWave + lane;
        const bool hit = j < pd.n && within_tolerance(q.a, q.b, q.c, xy[u].x, xy[u].y, ee[u]);
        const uint64_t m = ballot(hit);
        const int64_t dst = o0 + total + lanes_below(m);
        if (hit && dst < A.capacity) A.cols[dst] = (int32_t)j;
        total += (uint32_t)__popcll(m);
      }
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
  wave_sync_lds();
}

// The fused pass's record of a query: its row length and its match (as
// write_match_to would store it), or kMatchDeferred for a match that a later
// pass writes.
__device__ __forceinline__ uint4 query_record(uint32_t count, float ratio, const Top2& t,
                                              bool matched) {
  int32_t idx = t.bj == INT32_MAX ? -1 : t.bj;
  if (idx >= 0 && ratio > 0.0f && !(t.bd < ratio * ratio * t.sd)) idx = -1;
  if (!matched) idx = kMatchDeferred;
  return make_uint4(count, (uint32_t)idx, __float_as_uint(t.bd), __float_as_uint(t.sd));
}

// ------------------------------------------------------------- tiled pass
constexpr int kQPerWave = kTileQ / kWaves;
static_assert(kQPerWave == 16, "the pair test packs four records of 16 queries per wavefront");
static_assert(kTileQ == 64, "pair indexing uses a 6-bit query field");

// First index in [lo, hi) whose key is >= target (keys ascending), by one
// lane: seven probes in flight per step cut the range to an eighth.
__device__ __forceinline__ int64_t lower_bound_scalar(const uint32_t* __restrict__ keys,
                                                      int64_t lo, int64_t hi, uint32_t target) {
  // the answer lies in [lo, hi]
  while (hi - lo > 8) {
    const int64_t step = (hi - lo) / 8;
    uint32_t k[7];
    #pragma unroll
    for (int m = 0; m < 7; ++m) k[m] = keys[lo + (m + 1) * step];
    int c = 0;  // the probes below the target are a prefix
    #pragma unroll
    for (int m = 0; m < 7; ++m) c += k[m] < target ? 1 : 0;
    const int64_t nlo = c == 0 ? lo : lo + c * step + 1;
    const int64_t nhi = c == 7 ? hi : lo + (c + 1) * step;
    lo = nlo;
    hi = nhi;
  }
  int c = 0;
  #pragma unroll
  for (int m = 0; m < 8; ++m) c += lo + m < hi && keys[lo + m] < target ? 1 : 0;
  return lo + c;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

// Window pass: for tile t, the record ranges of every width class whose
// centres lie within [min key - 2^c + 1, max key + 2^c - 1] of the tile's
// queries; lane c searches class c.  No LDS, so every tile's searches are in
// flight at once.
constexpr int kWindowTiles = 4;  // tiles (one wavefront each) per workgroup
__global__ __launch_bounds__(kWave * kWindowTiles) void k_tile_windows(StabArgs A) {
  const int lane = lane_id();
  const int t = blockIdx.x * kWindowTiles + wave_id();
  if (t >= A.num_tiles) return;  // whole wavefronts
  const StabTile T = A.tiles[t];
  bool normal = false, brute = false;
  uint32_t key = 0;
  TileQuery tq;
  tq.a = tq.b = tq.c = tq.n = 0.0;
  tq.i = 0;
  tq.flag = kQueryEmpty;
  tq.key = 0;
  if (lane < T.count) {
    const int64_t i = A.qperm[T.begin + lane];
    const uint32_t flag = A.qflag[i];
    normal = flag == kQueryNormal;
    brute = flag == kQueryBrute;
    key = A.qkey[i];
    tq.i = i;
    tq.flag = flag;
    tq.key = key;
    const double4 L = A.qline[i];  // the line of Eq. 2 and its norm, from the key pass
    tq.a = L.x;
    tq.b = L.y;
    tq.c = L.z;
    tq.n = L.w;
  }
  A.tile_q[(int64_t)t * kTileQ + lane] = tq;
  if (lane == 0) {
    A.tile_wide[t] = 0u;  // set by the tile pass when a row is wide
    // the pair's flag likewise, cleared by the pair's first tile
    if (A.pair_wide && T.begin == A.qstart[T.pair]) A.pair_wide[T.pair] = 0u;
  }
  const uint32_t kmin = wave_min_u32(normal ? key : 0xFFFFFFFFu);
  const uint32_t kmax = wave_max_u32(normal ? key : 0u);
  const bool any = ballot(normal) != 0;
  // lane c < 32 searches the start of class c's window, lane c + 32 its end:
  // the two searches run side by side
  const int c = lane & (kNumClasses - 1);
  static_assert(2 * kNumClasses == kWave, "two lanes per width class");
  int64_t beg = 0, end = 0, r = 0;
  bool full = false, wrap = false;
  if (any) {
    const int64_t* cb = A.class_begin + (int64_t)T.pair * kClassSlots;
    beg = cb[c];
    end = cb[c + 1];
    if (beg < end) {
      const uint32_t span = c == kWideClass ? 0u : (1u << c) - 1u;
      const uint64_t width = (uint64_t)(kmax - kmin) + 2ull * span;
      full = c == kWideClass || width >= 0xFFFFE000ull;
      if (!full) {
        const uint32_t lo = kmin - span, hi = kmax + span;
        const uint32_t cls = (uint32_t)c << kCentreBits;
        const uint32_t blo = cls | (lo >> kCentreShift), bhi = cls | (hi >> kCentreShift);
        wrap = lo > hi;
        // bhi + 1 > blo without a wrap; through angle 0 the gap between hi
        // and lo is over 2^13 key units, so bhi + 1 <= blo
        r = lower_bound_scalar(A.skey, beg, end, lane < kNumClasses ? blo : bhi + 1u);
      }
    }
  }
  const int64_t r_end = __shfl(r, c + kNumClasses);
  int64_t b0 = 0, l0 = 0, b1 = 0, l1 = 0;
  if (lane < kNumClasses && any && beg < end) {
    if (full) {
      b0 = beg;
      l0 = end - beg;
    } else if (!wrap) {
      b0 = r;
      l0 = r_end - r;
    } else {
      b0 = r;
      l0 = end - r;
      b1 = beg;
      l1 = (r_end < r ? r_end : r) - beg;
    }
  }
  // slot s = class s/2, part s%2; inclusive scan of the 64 slot lengths
  const int src = lane >> 1;
  const int64_t be = __shfl(b0, src), bo = __shfl(b1, src);
  const int64_t le = __shfl(l0, src), lo_ = __shfl(l1, src);
  const int64_t myb = (lane & 1) ? bo : be;
  int64_t incl = (lane & 1) ? lo_ : le;
  #pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  TileWindow* w = A.windows + t;
  w->slot_b[lane] = (uint32_t)myb;
  w->slot_pref[lane + 1] = (uint32_t)incl;
  if (lane == 0) w->slot_pref[0] = 0u;
  if (A.tile_cost) {
    // work estimate: (query, record) pairs of the window scan, brute-force
    // scans, and one unit per query
    const uint64_t wlen = (uint64_t)__shfl(incl, kWave - 1);
    const uint64_t nn = (uint64_t)__popcll(ballot(normal));
    const uint64_t nb = (uint64_t)__popcll(ballot(brute));
    if (lane == 0) {
      const uint64_t c = nn * wlen + nb * (uint64_t)A.pairs[T.pair].n + (uint64_t)T.count;
      const uint32_t c32 = c > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)c;
      A.tile_cost[t] = c32;
    }
  }
}

// Counts every row of a tile of kTileQ angle-sorted queries and parks rows of
// up to kStage candidates in ascending j in the staging buffer.  The window
// records of the tile are staged in LDS; wavefront w owns queries 16w..16w+15
// (lane & 15), whose lines stay in registers, and tests them against four
// records per step (lane >> 4, LDS broadcasts): angle test, FP64 test, and the
// hit's slot from a ballot over the query's four lanes, so no atomics are
// needed and every row lists its hits in ascending window position.
//
// FUSE: the same pass also selects every query's match (Sec. 4.3) from its
// hit list while the list is still in LDS.  The hits are kept as 16-bit
// window positions (their j from the window's j, kept in LDS for windows of
// up to kKeepJ records); the window's descriptor rows are copied to LDS
// kFuseRows at a time (over the record chunk buffers, dead by then), and four
// lanes per query evaluate canonical FP32 distances of that query's hits in
// the chunk, each lane resuming where the last chunk left it, and keep a
// top-2, merged across the four lanes at the end.  Rows longer than kStage are
// matched by the wide-row pass; the rows this pass does not keep (brute-force
// queries, windows longer than kKeepJ) are marked for the fill pass to
// rebuild, and those queries are listed for the listed-query match after the
// CSR is complete; empty rows get their (-1, inf, inf) here.  The LDS and
// register budget allows three workgroups per CU.  After the pair test every
// wavefront works on its own 16 queries until the descriptor rows are staged,
// so the tile needs only the barriers of the record and row chunks; its
// counters gather in LDS and go to global memory once per tile (per-wavefront
// global atomics on the same counters cost more than a barrier).
constexpr int kFuseRows = 48;
constexpr int kFuseStride = 132;  // floats per staged row: 16-byte reads of rows hit distinct banks
// LDS bytes of a round of CH window records (C, H, x y, eps, j).
constexpr int rec_bytes(int CH) { return CH * (4 + 4 + 8 + 4 + 4); }
// The staged rows are copied straight from global memory to LDS (lane l of a
// wavefront copy writes 16-byte chunk l of it): kFuseCopies wavefront copies
// cover the rows with their padding, and the tail of the last one is slack.
constexpr int kFuseChunks = kFuseRows * (kFuseStride / 4);
constexpr int kFuseCopies = (kFuseChunks + kWave - 1) / kWave;
constexpr int kFuseBytes = kFuseCopies * kWave * 16;
// First entry of a parked row that was not parked: the fill pass rebuilds it.
constexpr int32_t kRowNotParked = -1;

// FUSE: the j of the first kKeepJ window positions stay in LDS; the hits
// are kept as 16-bit window positions, and tiles with longer windows are not
// fused (their rows are rebuilt by the fill pass and matched from the list)
constexpr int kKeepJ = 1024;
constexpr int64_t kFuseMaxWindow = kKeepJ;

// Starts the copy of rows [c0, c0 + nr) of the window (0 < nr <= kFuseRows)
// to LDS at a stride of kFuseStride floats.  Chunk p of the image is column
// p % 33 of row p / 33; the padding column and the rows past nr repeat real
// data.  The copies complete asynchronously: wait for them (vmcnt) before the
// barrier that publishes the rows.
__device__ __forceinline__ void fuse_stage(const StabArgs& A, int c0, int nr, int64_t kb,
                                           const int32_t* sJ, float4* rows4, int wave, int lane) {
  constexpr int kRowChunks = kFuseStride / 4;
  for (int g = wave; g < kFuseCopies; g += kWaves) {
    const int p = g * kWave + lane;
    int r = p / kRowChunks;
    int c = p - r * kRowChunks;
    r = r < nr ? r : nr - 1;
    c = c < 32 ? c : 31;
    const float4* src = reinterpret_cast<const float4*>(A.desc2) + (kb + sJ[c0 + r]) * 32 + c;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)(rows4 + g * kWave),
                                     16, 0, 0);
  }
}

// s_waitcnt vmcnt(0): this wavefront's copies to LDS have landed.
__device__ __forceinline__ void wait_lds_copies() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ------------------------------------------------ BF16 fused selection
// MODE kStabBF16: the caller's descriptors are BF16 codes with FP32 masters,
// and the final matches must be the canonical FP32 selection on the masters.
// The window's BF16 rows are staged kBfRows at a time; wavefront w scores its
// 16 queries against them on MFMA (A = the window rows, B = the queries, so
// lane l holds query l & 15 against rows 16 cb + 4 i + (l >> 4)).  Every hit
// gets certified bounds D_lo <= D <= D_hi on its exact canonical distance D:
//   |q^ - w^|^2 is within em = 3e-5 (|q^| + |w^|)^2 of |q^|^2 + |w^|^2 - 2 q^.w^
//   (FP32 accumulation), |q - w| is within eps_q + eps_w of |q^ - w^| (eps_q
//   the measured norm of the query's rounding error, exact in FP32 from its
//   master; eps_w the BF16 bound u |w^| / (1 - u), u = 2^-8, of a row rounded
//   to nearest even), and D is within 2e-5 (relative) of |q - w|^2 (130
//   roundings of 2^-24).
// Let U2 be the second smallest D_hi over any set of the row's candidates.
// Two candidates have D <= U2, so a candidate with D_lo > U2 is strictly
// worse than both and is neither best nor second: the candidates with
// D_lo <= U2 are evaluated exactly (canonical chains on the masters) and
// their top-2 is the row's.  Each lane keeps only the kBfKeep smallest
// approximate distances A of its hits, with their rows' bound norms; after
// the last chunk it works out D_lo and D_hi of those (U2 is taken over the
// row's kept candidates) and, since D_lo grows with A and shrinks with the
// row norm, a lower bound on D_lo of every pushed-out hit from the smallest
// pushed-out A and the largest row norm.  A row whose pushed-out bound is not
// above U2 is left to the listed-query match, exact either way.
constexpr int kBfRows = 32;  // window rows per chunk: with 256-record rounds, four workgroups per CU
constexpr int kBfBlocks = kBfRows / 16;     // 16-row MFMA blocks per chunk
constexpr int kBfStride = 256 + 16;         // LDS bytes per row: 16 rows' reads hit distinct banks
constexpr int kBfPieces = kBfStride / 16;   // 16-byte pieces per row (the last repeats one)
constexpr int kBfCopies = (kBfRows * kBfPieces + kWave - 1) / kWave;
constexpr int kBfRowBytes = kBfCopies * kWave * 16;
constexpr int kBfKeep = 3;
static_assert(kBfRows % 16 == 0 && kBfRows <= 64, "the hit mask of a chunk is one 64-bit word");
// MODE kStabFP8: the image-2 rows are 128 one-byte E4M3 codes c with a scale
// s per row (w^ = s c), staged at a stride of 144 bytes (the padding
// staggers the rows over the LDS banks) and decoded to BF16 for the MFMA,
// exactly; the queries are rounded to BF16 on chip from their masters (eps_q
// measured as above).  The score of the codes times s is q^.w^ within the
// same accumulation bound, |w^|^2 = s^2 |c|^2, and eps_w is the caller's
// bound on |w - w^| for the row, carried per kept candidate rounded up to
// FP16 (the accumulation term takes the lane's largest row norm).  These
// errors are an order of magnitude above BF16's, so more candidates per row
// fall within the row's second upper bound: each lane keeps six.
constexpr int kF8Stride = 128 + 16;
constexpr int kF8Pieces = kF8Stride / 16;
constexpr int kF8Copies = (kBfRows * kF8Pieces + kWave - 1) / kWave;
constexpr int kF8RowBytes = kF8Copies * kWave * 16;
constexpr int kF8Keep = 6;
// After the pair test the record chunk holds the chunk's row terms (a float4
// per row) and the per-query task lists (four lanes of `keep` entries).
constexpr int red_scratch(int keep) { return kBfRows * 16 + kTileQ * 4 * keep * 2; }

// Starts the copy of BF16 rows [c0, c0 + nr) of the window to LDS (stride
// kBfStride, 0 < nr <= kBfRows); rows past nr and the padding piece repeat
// real data.  The copies complete asynchronously (wait_lds_copies).
__device__ __forceinline__ void bf16_stage(const StabArgs& A, int c0, int nr, int64_t kb,
                                           const int32_t* sJ, uint8_t* rows, int wave, int lane) {
  for (int g = wave; g < kBfCopies; g += kWaves) {
    const int p = g * kWave + lane;
    int r = p / kBfPieces;
    int c = p - r * kBfPieces;
    r = r < nr ? r : nr - 1;
    c = c < 16 ? c : 15;
    const uint4* src = reinterpret_cast<const uint4*>(A.codes2) + (kb + sJ[c0 + r]) * 16 + c;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)(rows + g * kWave * 16),
                                     16, 0, 0);
  }
}

// Starts the copy of FP8 rows [c0, c0 + nr) of the window to LDS (stride
// kF8Stride, 0 < nr <= kBfRows), as bf16_stage.
__device__ __forceinline__ void f8_stage(const StabArgs& A, int c0, int nr, int64_t kb,
                                         const int32_t* sJ, uint8_t* rows, int wave, int lane) {
  for (int g = wave; g < kF8Copies; g += kWaves) {
    const int p = g * kWave + lane;
    int r = p / kF8Pieces;
    int c = p - r * kF8Pieces;
    r = r < nr ? r : nr - 1;
    c = c < 8 ? c : 7;
    const uint4* src = reinterpret_cast<const uint4*>(A.f8codes2) + (kb + sJ[c0 + r]) * 8 + c;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)(rows + g * kWave * 16),
                                     16, 0, 0);
  }
}

// Eight OCP E4M3FN codes (byte e is element e) as BF16 values.  Every E4M3
// value has at most four significant bits and an exponent inside BF16's
// range, so the upper half of the hardware's FP32 decode is the value itself.
__device__ __forceinline__ bf16x8 e4m3x8_bf16(uint2 v) {
  const uint32_t src[2] = {v.x, v.y};
  uint32_t w[4];
  #pragma unroll
  for (int h = 0; h < 2; ++h) {
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)src[h], false);  // bytes 0, 1
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)src[h], true);   // bytes 2, 3
    w[2 * h] = (__float_as_uint(lo[0]) >> 16) | (__float_as_uint(lo[1]) & 0xFFFF0000u);
    w[2 * h + 1] = (__float_as_uint(hi[0]) >> 16) | (__float_as_uint(hi[1]) & 0xFFFF0000u);
  }
  return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
}

// Sum of the squares of sixteen E4M3 codes (decoded exactly; each square is
// exact in FP32).
__device__ __forceinline__ float e4m3x16_sumsq(uint4 v, float acc) {
  const uint32_t src[4] = {v.x, v.y, v.z, v.w};
  #pragma unroll
  for (int h = 0; h < 4; ++h) {
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)src[h], false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)src[h], true);
    acc = __builtin_fmaf(lo[0], lo[0], acc);
    acc = __builtin_fmaf(lo[1], lo[1], acc);
    acc = __builtin_fmaf(hi[0], hi[0], acc);
    acc = __builtin_fmaf(hi[1], hi[1], acc);
  }
  return acc;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int off) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, off);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), off);
  return ((uint64_t)hi << 32) | lo;
}


// Per-lane state of one query's selection with deferred bounds (lane group g
// of its four lanes): the K smallest approximate distances
// A = |q^|^2 + |w^|^2 - 2 q^.w^ seen (FP32, as the bounds take them), with
// their window positions and a row bound term rounded up to FP16 (BF16 rows:
// the bound norm |w^|; FP8 rows: the norm of the row's rounding error), the
// smallest A pushed out of that list, the largest row bound norm and (FP8)
// the largest rounding-error term seen.  The certified bounds D_lo <= D <=
// D_hi of the kept candidates, and a lower bound on D_lo of every pushed-out
// one (D_lo grows with A and shrinks with the row's norm and error), are
// worked out once after the last chunk.
constexpr uint32_t kNoPick = 0xFFFFFFFFu;
template <int K>
struct BfKeep {
  float a[K];      // ascending
  uint32_t pk[K];  // window position | FP16 row term << 16, kNoPick: empty
  float a_drop = __builtin_inff();
  float nb_max = 0.0f;
  uint32_t ew_max = 0u;  // FP16 bits: positive halves order as their bit patterns
  bool bad = false;

  __device__ __forceinline__ BfKeep() {
    #pragma unroll
    for (int t = 0; t < K; ++t) {
      a[t] = __builtin_inff();
      pk[t] = kNoPick;
    }
  }

  // sorted insertion: entry t moves down one place when A goes before entry
  // t - 1, takes A when A goes between them, and the last entry drops out
  __device__ __forceinline__ void add(float at, uint32_t p, float nb, uint32_t ew) {
    bad |= !(at == at);
    nb_max = fmaxf(nb_max, nb);
    ew_max = ew_max > ew ? ew_max : ew;
    if constexpr (K == 3) {  // written out: the compiler keeps it free of branches
      const bool c0 = at < a[0], c1 = at < a[1], c2 = at < a[2];  // c0 => c1 => c2
      const float out = c2 ? a[2] : at;
      const bool out_real = c2 ? pk[2] != kNoPick : true;
      a[2] = c1 ? a[1] : (c2 ? at : a[2]);
      pk[2] = c1 ? pk[1] : (c2 ? p : pk[2]);
      a[1] = c0 ? a[0] : (c1 ? at : a[1]);
      pk[1] = c0 ? pk[0] : (c1 ? p : pk[1]);
      a[0] = c0 ? at : a[0];
      pk[0] = c0 ? p : pk[0];
      a_drop = out_real ? fminf(a_drop, out) : a_drop;
    } else {
      // new entry t: the old one, A, or the old entry t - 1, from the two
      // comparisons around it (selects only)
      float na[K];
      uint32_t np[K];
      bool prev = false;  // A goes before entry t - 1
      #pragma unroll
      for (int t = 0; t < K; ++t) {
        const bool ct = at < a[t];
        na[t] = prev ? a[t - (t > 0)] : (ct ? at : a[t]);
        np[t] = prev ? pk[t - (t > 0)] : (ct ? p : pk[t]);
        prev = ct;
      }
      const float out = prev ? a[K - 1] : at;
      const bool out_real = prev ? pk[K - 1] != kNoPick : true;
      a_drop = out_real ? fminf(a_drop, out) : a_drop;
      #pragma unroll
      for (int t = 0; t < K; ++t) {
        a[t] = na[t];
        pk[t] = np[t];
      }
    }
  }
};

// Certified bounds on the exact canonical distance of a candidate whose
// approximate distance is `at` and whose row bound norm is at most nb (query
// terms q_nb, q_db; see the comment above kBfRows).
// ew: a bound on |q - q^| + |w - w^|.
__device__ __forceinline__ void bounds_from(float at, float nb, float q_nb, float ew, float& dlo,
                                            float& dhi) {
  const float sum = q_nb + nb;
  const float em = 3e-5f * sum * sum;
  // sqrt(at +- em) from the hardware reciprocal square root (within a few
  // ulps): the 1e-6 factors cover it; arguments under 2^-100 take the
  // trivially valid bounds 0 and 2^-50
  const float th = fmaxf(at, 0.0f) + em;
  const float tl = at - em;
  const float r_hi = th > 0x1p-100f ? th * __builtin_amdgcn_rsqf(th) * (1.0f + 1e-6f) : 0x1p-50f;
  const float r_lo = tl > 0x1p-100f ? tl * __builtin_amdgcn_rsqf(tl) * (1.0f - 1e-6f) : 0.0f;
  // the 1e-6 r_lo term covers the rounding of the two subtractions
  const float e_lo = fmaxf(r_lo - ew - 1e-6f * r_lo, 0.0f);
  const float e_hi = r_hi + ew;
  dlo = e_lo * e_lo * (1.0f - 3e-5f);
  dhi = e_hi * e_hi * (1.0f + 3e-5f);
}

// BF16 rows: |w - w^| <= u |w^| / (1 - u) for a row rounded to nearest even.
__device__ __forceinline__ void bf_bounds(float at, float nb, float q_nb, float q_db, float& dlo,
                                          float& dhi) {
  bounds_from(at, nb, q_nb,
              q_db + nb * (float)(Fmt<0>::kUnit / (1.0 - Fmt<0>::kUnit) * (1.0 + 1e-6)) + 1e-30f,
              dlo, dhi);
}

// MODE: kStabCount (count and park rows), kStabF32 (FP32 selection fused),
// kStabBF16 / kStabFP8 (BF16 or FP8 image-2 rows: MFMA bounds with an exact
// FP32 re-rank, fused).
// Fused: three workgroups per CU (LDS and registers are sized for it; four
// for kStabBF16)
// CH: window records staged in LDS per round of the pair test.
template <bool PERSIST, int MODE, int CH>
__global__ __launch_bounds__(kThreads, MODE == kStabBF16 ? 4 : MODE != kStabCount ? 3 : 2) void k_stab_tile(StabArgs A) {
  constexpr bool FUSE = MODE != kStabCount;
  // BF16 / FP8: MFMA bounds and an exact re-rank on the masters
  constexpr bool RED = MODE == kStabBF16 || MODE == kStabFP8;
  // record chunk (sC, sH, sXY, sE; sJ too unless FUSE keeps the window's j
  // in sJ_keep), reused for descriptor rows in the match phase
  constexpr int kRecRaw = FUSE ? rec_bytes(CH) - CH * 4 : rec_bytes(CH);
  constexpr int kMatchRaw = MODE == kStabF32    ? kFuseBytes
                           : MODE == kStabBF16 ? red_scratch(kBfKeep)
                           : MODE == kStabFP8  ? red_scratch(kF8Keep)
                                               : 0;
  constexpr int kRaw = kMatchRaw > kRecRaw ? kMatchRaw : kRecRaw;
  __shared__ __attribute__((aligned(16))) unsigned char raw[kRaw];
  // BF16 / FP8: the window's reduced rows, kBfRows at a time (the first
  // chunk is copied in while the pair test runs)
  __shared__ __attribute__((aligned(16)))
  uint8_t bfrows[MODE == kStabBF16 ? kBfRowBytes : MODE == kStabFP8 ? kF8RowBytes : 16];
  __shared__ int32_t sJ_keep[FUSE ? kKeepJ : 1];
  uint32_t* sC = reinterpret_cast<uint32_t*>(raw);
  uint32_t* sH = sC + CH;
  float2* sXY = reinterpret_cast<float2*>(sH + CH);
  float* sE = reinterpret_cast<float*>(sXY + CH);
  int32_t* sJ = reinterpret_cast<int32_t*>(sE + CH);  // not FUSE
  // hit lists: image-2 indices, or (FUSE) 16-bit window positions
  __shared__ int32_t hits[FUSE ? 1 : kTileQ][FUSE ? 1 : kStage + 1];  // +1: rows in different banks
  __shared__ uint16_t hits_v[FUSE ? kTileQ : 1][FUSE ? kStage + 2 : 1];
  // image-2 index of hit u of query q
  const auto hit_j = [&](int q, uint32_t u) -> int32_t {
    if constexpr (FUSE)
      return sJ_keep[hits_v[q][u]];
    else
      return hits[q][u];
  };
  __shared__ double qa[kTileQ], qb[kTileQ], qc[kTileQ], qn[kTileQ];
  __shared__ uint32_t qk[kTileQ], qmode[kTileQ], cnt[kTileQ];
  __shared__ int64_t qidx[kTileQ];
  __shared__ uint32_t slot_b[kSlots], slot_pref[kSlots + 1];
  // scanned, angle hits, brute-force and empty queries; BF16 fused: rows
  // ranked on bounds, rows left uncertified, exact distances evaluated
  __shared__ uint32_t tile_stats[kTileCounts];
  __shared__ int next_tile;

  // one tile per workgroup, or (persistent) tiles from the queue until it is
  // exhausted; every workgroup leaves the loop once the counter passes the
  // last tile
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
    const StabTile T = A.tiles[tile];
    const PairDev& pd = A.pairs[T.pair];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();

    if (wave == 0) {
      // the tile's queries with their lines, from the window pass
      const TileQuery tq = A.tile_q[(int64_t)tile * kTileQ + lane];
      qa[lane] = tq.a;
      qb[lane] = tq.b;
      qc[lane] = tq.c;
      qn[lane] = tq.n;
      qk[lane] = tq.key;
      qmode[lane] = tq.flag;
      qidx[lane] = tq.i;
      cnt[lane] = 0;
      if (lane < kTileCounts) tile_stats[lane] = 0u;
    }
    {
      const TileWindow* w = A.windows + tile;
      if (tid < kSlots) slot_b[tid] = w->slot_b[tid];
      if (tid <= kSlots) slot_pref[tid] = w->slot_pref[tid];
    }
    __syncthreads();

    const int64_t total_len = slot_pref[kSlots];
    const bool fusable = total_len <= kFuseMaxWindow;
    uint32_t scanned = 0, angle_w = 0;  // angle_w: the wavefront's angle hits (uniform)
    // this lane's query of the pair test: its line stays in registers
    const int lq = wave * kQPerWave + (lane & (kQPerWave - 1));
    const bool line_live = qmode[lq] == kQueryNormal;
    const uint64_t live_mask = ballot(line_live);
    const bool any_live = ballot(line_live) != 0;
    const uint32_t lkey = qk[lq];
    const double la = qa[lq], lb = qb[lq], lc = qc[lq], ln = qn[lq];
    const uint64_t same_query = 0x0001000100010001ull << (lane & (kQPerWave - 1));
    // the wavefront's key span [kmn, kmx] over its live queries: a record
    // whose interval misses every key of the span (circular distance from the
    // span's middle beyond its half-width plus the span's half-length, by the
    // triangle inequality on the circle of keys) cannot meet any of them and
    // is skipped without the per-query test
    uint32_t kmn = line_live ? lkey : 0xFFFFFFFFu, kmx = line_live ? lkey : 0u;
    #pragma unroll
    for (int off = 1; off < kQPerWave; off <<= 1) {
      kmn = min(kmn, (uint32_t)__shfl_xor((int)kmn, off));
      kmx = max(kmx, (uint32_t)__shfl_xor((int)kmx, off));
    }
    const uint32_t kmid = kmn + ((kmx - kmn) >> 1);
    const uint64_t khalf = ((uint64_t)(kmx - kmn) + 1u) >> 1;
    uint32_t lcnt = 0;
    // BF16: the query rows are loaded before the pair test so that their
    // latency hides behind it.  Lane l of wavefront w holds query
    // 16 w + (l & 15): as MFMA B operands its BF16 values at dimensions
    // 32 kk + 8 g .. + 7 (g = l >> 4), and its quarter, dimensions
    // 32 g .. 32 g + 31, as BF16 codes and as the FP32 master (the exact
    // chains pass their sum from quarter to quarter)
    bf16x8 bq[4];
    uint4 qcode[4];
    float4 qx[8];
    // FP8: the master's values at the B operand's dimensions, rounded to
    // BF16 after the pair test (the quarter for the exact chains is loaded
    // then, behind the first chunk)
    float4 qraw[8];
    if constexpr (MODE == kStabFP8) {
      const int g = lane >> 4;
      const bool ld = line_live && lq < T.count && fusable;
      const float4* m = reinterpret_cast<const float4*>(A.desc1) + qidx[lq] * 32;
      #pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        qraw[2 * kk] = ld ? m[kk * 8 + g * 2] : make_float4(0.f, 0.f, 0.f, 0.f);
        qraw[2 * kk + 1] = ld ? m[kk * 8 + g * 2 + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    if constexpr (MODE == kStabBF16) {
      const int g = lane >> 4;
      const bool ld = line_live && lq < T.count && fusable;
      const int64_t qi = qidx[lq];
      #pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const uint4 c = ld ? reinterpret_cast<const uint4*>(A.codes1)[qi * 16 + kk * 4 + g]
                           : make_uint4(0u, 0u, 0u, 0u);
        bq[kk] = __builtin_bit_cast(bf16x8, c);
        qcode[kk] = ld ? reinterpret_cast<const uint4*>(A.codes1)[qi * 16 + g * 4 + kk]
                    : make_uint4(0u, 0u, 0u, 0u);
      }
      #pragma unroll
      for (int u = 0; u < 8; ++u)
        qx[u] = ld ? reinterpret_cast<const float4*>(A.desc1)[qi * 32 + g * 8 + u]
                   : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int64_t base = 0; base < total_len; base += CH) {
      const int clen = (int)(total_len - base < CH ? total_len - base : CH);
      for (int v = tid; v < clen; v += kThreads) {
        const int64_t virt = base + v;
        int s = 0;  // last slot with slot_pref[s] <= virt
        #pragma unroll
        for (int step = 32; step > 0; step >>= 1)
          if (s + step <= kSlots && slot_pref[s + step] <= virt) s += step;
        const int64_t pos = slot_b[s] + (virt - slot_pref[s]);
        sC[v] = A.rC[pos];
        sH[v] = A.rH[pos];
        sXY[v] = A.rxy[pos];
        sE[v] = A.reps[pos];
        if (!FUSE)
          sJ[v] = A.rj[pos];
        else if (virt < kKeepJ)
          sJ_keep[virt] = A.rj[pos];
      }
      __syncthreads();
      if constexpr (RED) {
        // the first reduced rows of the window go to LDS behind the pair test
        if (base == 0 && fusable && total_len > 0) {
          const int nr0 = total_len < kBfRows ? (int)total_len : kBfRows;
          if constexpr (MODE == kStabFP8)
            f8_stage(A, 0, nr0, pd.k_begin, sJ_keep, bfrows, wave, lane);
          else
            bf16_stage(A, 0, nr0, pd.k_begin, sJ_keep, bfrows, wave, lane);
        }
      }
      if (any_live) {
        // this wave's 16 queries (lane & 15) against four records per step
        // (lane >> 4), over the records of each group of 64 that can meet
        // the wave's key span; a hit's slot is the query's count plus its
        // rank among the query's lanes of the step, so every row lists its
        // hits in ascending window position
        const int g4 = lane >> 4;
        for (int g0 = 0; g0 < clen; g0 += kWave) {
          bool rel = false;
          if (g0 + lane < clen)
            rel = (uint64_t)key_distance(kmid, sC[g0 + lane]) <= (uint64_t)sH[g0 + lane] + khalf;
          uint64_t m = ballot(rel);
          if (line_live && lane < kQPerWave) scanned += (uint32_t)__popcll(m);
          while (m != 0ull) {
            // the next four of them, in ascending position, one per lane group
            int pick = kWave;
            #pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int b = m != 0ull ? (int)__builtin_ctzll(m) : kWave;
              pick = g4 == t ? b : pick;
              m &= m - 1ull;
            }
            const int r = g0 + pick;
            // branch-free: nearly every step has lanes that pass the angle
            // test, and the SIMD runs the FP64 test for all of its lanes
            // anyway; each test is balloted on its own (a ballot of one
            // comparison is its lane mask as it stands)
            const int rr = pick < kWave ? r : g0;  // an index inside the chunk
            const uint32_t C = sC[rr], H = sH[rr];
            const float2 xy = sXY[rr];
            const bool key_ok = key_distance(lkey, C) <= H;
            const bool fp_ok = within_tolerance_n(la, lb, lc, ln, xy.x, xy.y, sE[rr]);
            const uint64_t vm = live_mask & ballot(pick < kWave);
            const uint64_t am = vm & ballot(key_ok);
            angle_w += (uint32_t)__popcll(am);
            const uint64_t all_hits = am & ballot(fp_ok);
            const bool hit = line_live & (pick < kWave) & key_ok & fp_ok;  // this lane's bit
            const uint64_t hm = all_hits & same_query;
            if (hit) {
              const uint32_t slot = lcnt + lanes_below(hm);
              if (slot < (uint32_t)kStage) {
                if (FUSE)
                  hits_v[lq][slot] = (uint16_t)(base + r);
                else
                  hits[lq][slot] = sJ[r];
              }
            }
            lcnt += (uint32_t)__popcll(hm);
          }
        }
      }
      __syncthreads();
    }
    if (line_live && lane < kQPerWave) cnt[lq] = lcnt;

    // queries whose line misses the epipole too far: exact scan of the pair
    uint32_t brute = 0;
    for (int qq = 0; qq < kQPerWave; ++qq) {
      const int q = wave * kQPerWave + qq;
      if (qmode[q] != kQueryBrute) continue;
      const double a = qa[q], b = qb[q], c = qc[q], nrm = qn[q];
      uint32_t c0 = 0;
      brute += 1;
      for (int64_t base = pd.k_begin; base < pd.k_begin + pd.n; base += kWave) {
        const int64_t pos = base + lane;
        bool hit = false;
        if (pos < pd.k_begin + pd.n) {
          const float2 xy = A.rxy[pos];
          hit = within_tolerance_n(a, b, c, nrm, xy.x, xy.y, A.reps[pos]);
        }
        const uint64_t m = ballot(hit);
        if (!FUSE && hit) {  // FUSE: counted only, the row is rebuilt by the fill pass
          const uint32_t slot = c0 + lanes_below(m);
          if (slot < (uint32_t)kStage) hits[q][slot] = A.rj[pos];
        }
        c0 += (uint32_t)__popcll(m);
      }
      if (lane == 0) cnt[q] = c0;
    }
    // From here to the match phase every wavefront works on its own 16
    // queries only (their hits and counts were written by this wavefront),
    // so no barrier is needed.
    {
      // the tile's counters gather in LDS; one thread adds them to the
      // query's counters once every wavefront has passed a later barrier
      const bool own = lane < kQPerWave && lq < T.count;
      const uint32_t nbrute = (uint32_t)__popcll(ballot(own && qmode[lq] == kQueryBrute));
      const uint32_t empty = (uint32_t)__popcll(ballot(own && qmode[lq] == kQueryEmpty));
      scanned = wave_sum_u32(scanned);
      const uint32_t angle_hits = angle_w;
      // rows longer than kStage of normal queries are written (and, fused,
      // matched) by the wide-row pass over the tile; the window pass cleared
      // the flag
      const uint64_t wm = ballot(own && qmode[lq] == kQueryNormal && cnt[lq] > (uint32_t)kStage);
      if (lane == 0) {
        atomicAdd(&tile_stats[0], scanned);
        atomicAdd(&tile_stats[1], angle_hits);
        atomicAdd(&tile_stats[2], nbrute);
        atomicAdd(&tile_stats[3], empty);
        if (wm != 0ull) {
          A.tile_wide[tile] = 1u;
          if (A.pair_wide) atomicAdd(&A.pair_wide[T.pair], 1u);
        }
      }
    }
    (void)brute;

    // FUSE: four threads per query select its match
    const int q = tid >> 2, part = tid & 3;
    const bool mine = FUSE && q < T.count && qmode[q] == kQueryNormal &&
                      cnt[q] <= (uint32_t)kStage && fusable;

    // row lengths, and short rows parked in ascending j: four threads per
    // row, each placing a quarter of its hits by rank (the j of a row are
    // distinct, so a hit's place is the number of smaller hits); a thread
    // ranks up to four of its hits in one pass over the row
    // (the fused modes write the row length with the match, in one record)
    if (!FUSE && part == 0 && q < T.count)
      A.counts[qidx[q]] = qmode[q] == kQueryEmpty ? 0u : cnt[q];
    {
      const uint32_t n = q < T.count && qmode[q] != kQueryEmpty ? cnt[q] : 0u;
      // FUSE keeps only the hits of normal queries in fused windows; other
      // short rows are marked (first entry -1) for the fill pass to rebuild
      const bool here = !FUSE || (fusable && qmode[q] == kQueryNormal);
      int32_t* dst = A.staging + qidx[q] * kStage;
      if (n <= (uint32_t)kStage && here) {
        for (uint32_t t0 = part; t0 < n; t0 += 16) {
          int32_t v[4];
          uint32_t r[4];
          #pragma unroll
          for (int m = 0; m < 4; ++m) {
            v[m] = t0 + 4 * m < n ? hit_j(q, t0 + 4 * m) : INT32_MIN;
            r[m] = 0;
          }
          #pragma unroll 4
          for (uint32_t u = 0; u < n; ++u) {
            const int32_t h = hit_j(q, u);
            #pragma unroll
            for (int m = 0; m < 4; ++m) r[m] += h < v[m] ? 1u : 0u;
          }
          #pragma unroll
          for (int m = 0; m < 4; ++m)
            if (t0 + 4 * m < n) dst[r[m]] = v[m];
        }
      } else if (n > 0 && n <= (uint32_t)kStage && part == 0) {
        dst[0] = kRowNotParked;
      }
    }

    if (FUSE) {
      if (part == 0 && q < T.count) {
        const uint32_t mode = qmode[q];
        if (mode != kQueryEmpty &&
            (mode != kQueryNormal || (cnt[q] <= (uint32_t)kStage && !fusable))) {
          const unsigned long long at = atomicAdd(&A.stats[kStatRest], 1ull);
          A.rest[at] = (uint32_t)qidx[q];
        }
      }
    }
    if constexpr (MODE == kStabF32) {
      const int nq = mine ? (int)cnt[q] : 0;
      const int64_t kb = pd.k_begin;
      float4* rows4 = reinterpret_cast<float4*>(raw);
      // the query row stays in registers for all its hits
      float4 qreg[32];
      {
        const float4* qrow = reinterpret_cast<const float4*>(A.desc1) + qidx[q] * 32;
        #pragma unroll
        for (int k = 0; k < 32; ++k) qreg[k] = mine ? qrow[k] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      Top2 best;
      int cur = part;
      // the record chunk is dead since the pair test's last barrier, so the
      // first rows go in without one
      if (fusable && total_len > 0) {
        const int wlen = (int)total_len;
        for (int c0 = 0; c0 < wlen; c0 += kFuseRows) {
          const int nr = wlen - c0 < kFuseRows ? wlen - c0 : kFuseRows;
          if (c0 > 0) __syncthreads();  // the previous rows are no longer read
          fuse_stage(A, c0, nr, kb, sJ_keep, rows4, wave, lane);
          wait_lds_copies();
          __syncthreads();
          // the row's hits are in ascending window position: this lane's
          // hits in the chunk continue from where the previous chunk stopped
          for (; cur < nq; cur += 4) {
            const int v = hits_v[q][cur];
            if (v >= c0 + nr) break;
            const float4* wr = rows4 + (v - c0) * (kFuseStride / 4);
            float acc = 0.0f;
            #pragma unroll
            for (int k = 0; k < 32; ++k) acc = canonical_step4(acc, qreg[k], wr[k]);
            best.insert(acc, sJ_keep[v]);
          }
        }
      }
      // the four parts of a query are adjacent lanes and hold distinct hits
      #pragma unroll
      for (int off = 1; off < 4; off <<= 1) {
        Top2 o;
        o.bd = __shfl_xor(best.bd, off);
        o.bj = __shfl_xor(best.bj, off);
        o.sd = __shfl_xor(best.sd, off);
        o.sj = __shfl_xor(best.sj, off);
        best = merge_top2(best, o);
      }
      if (part == 0 && q < T.count) {
        const bool empty = qmode[q] == kQueryEmpty;
        A.qrec[qidx[q]] = query_record(empty ? 0u : cnt[q], A.ratio, best, mine || empty);
      }
    } else if constexpr (RED) {
      constexpr bool F8 = MODE == kStabFP8;
      constexpr int kKeep = F8 ? kF8Keep : kBfKeep;
      constexpr int kQTasks = 4 * kKeep;  // exact distances a query can list
      // lane l of wavefront w: query 16 w + (l & 15), lane group g = l >> 4
      const int q2 = wave * kQPerWave + (lane & (kQPerWave - 1));
      const int g = lane >> 4;
      const bool mine2 = q2 < T.count && qmode[q2] == kQueryNormal &&
                         cnt[q2] <= (uint32_t)kStage && fusable;
      const int nq = mine2 ? (int)cnt[q2] : 0;
      const int64_t kb = pd.k_begin;
      const int64_t qi2 = qidx[q2];
      // per chunk row: (|w^|^2, bound norm, rounding bound) -- the record
      // chunk is dead -- then the per-query task lists
      float4* w_terms = reinterpret_cast<float4*>(raw);
      uint16_t* qtask = reinterpret_cast<uint16_t*>(w_terms + kBfRows);  // [kTileQ][kQTasks]
      // the query's BF16 norm and the measured norm of its rounding error
      // (x - x^, exact in FP32), summed over its four quarters (FP8: the
      // query rounded to BF16 here, to nearest even, into the B operand)
      float qn_part = 0.0f, qe_part = 0.0f;
      #pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const float4 xa = F8 ? qraw[2 * kk] : qx[2 * kk];
        const float4 xb = F8 ? qraw[2 * kk + 1] : qx[2 * kk + 1];
        const float x[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
        uint32_t w[4];
        if constexpr (F8) {
          #pragma unroll
          for (int h = 0; h < 4; ++h) {
            const uint32_t u0 = __float_as_uint(x[2 * h]), u1 = __float_as_uint(x[2 * h + 1]);
            w[h] = ((u0 + 0x7FFFu + ((u0 >> 16) & 1u)) >> 16) |
                   ((u1 + 0x7FFFu + ((u1 >> 16) & 1u)) & 0xFFFF0000u);
          }
          bq[kk] = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
        } else {
          w[0] = qcode[kk].x;
          w[1] = qcode[kk].y;
          w[2] = qcode[kk].z;
          w[3] = qcode[kk].w;
        }
        #pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float y = __uint_as_float(e & 1 ? (w[e >> 1] & 0xFFFF0000u) : (w[e >> 1] << 16));
          qn_part = __builtin_fmaf(y, y, qn_part);
          const float d = x[e] - y;
          qe_part = __builtin_fmaf(d, d, qe_part);
        }
      }
      if constexpr (F8) {
        const bool ld = mine2;
        const float4* m = reinterpret_cast<const float4*>(A.desc1) + qi2 * 32 + g * 8;
        #pragma unroll
        for (int u = 0; u < 8; ++u) qx[u] = ld ? m[u] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      qn_part += __shfl_xor(qn_part, 16);
      qe_part += __shfl_xor(qe_part, 16);
      qn_part += __shfl_xor(qn_part, 32);
      qe_part += __shfl_xor(qe_part, 32);
      // per-query bound terms, inflated for the FP32 sums (2^-24 per term)
      const float q_nb = sqrtf(qn_part) * (1.0f + 2e-5f);
      const float q_db = sqrtf(qe_part) * (1.0f + 2e-5f) + 1e-30f;
      BfKeep<kKeep> st;
      int cur = g;
      Top2 best;
      uint32_t evals = 0;
      bool cert = mine2;  // a tile without window records has only empty rows
      if (fusable && total_len > 0) {
        const int wlen = (int)total_len;
        for (int c0 = 0; c0 < wlen; c0 += kBfRows) {
          const int nr = wlen - c0 < kBfRows ? wlen - c0 : kBfRows;
          if (c0 > 0) {
            __syncthreads();  // the previous rows are no longer read
            if constexpr (F8)
              f8_stage(A, c0, nr, kb, sJ_keep, bfrows, wave, lane);
            else
              bf16_stage(A, c0, nr, kb, sJ_keep, bfrows, wave, lane);
          }  // the first rows were started during the pair test
          // this query's hits in the chunk (the row is in ascending window
          // position; each lane resumes where the last chunk left it)
          uint64_t hmask = 0ull;
          for (; cur < nq; cur += 4) {
            const int v = hits_v[q2][cur];
            if (v >= c0 + nr) break;
            hmask |= 1ull << (v - c0);
          }
          hmask |= shfl_xor_u64(hmask, 16);
          hmask |= shfl_xor_u64(hmask, 32);
          // FP8: the scale and the rounding-error bound of the row whose
          // terms this thread works out below, read beside the copies
          float f8s = 1.0f, f8e = 0.0f;
          if constexpr (F8) {
            const int r = tid / (kThreads / kBfRows);
            if (tid % (kThreads / kBfRows) == 0) {
              const int64_t j = kb + sJ_keep[c0 + (r < nr ? r : nr - 1)];
              f8s = A.f8scale2[j];
              f8e = A.f8err2[j];
            }
          }
          wait_lds_copies();
          __syncthreads();
          {
            // norms of the chunk's rows: kTpr threads per row
            constexpr int kTpr = kThreads / kBfRows;
            const int r = tid / kTpr, part4 = tid % kTpr;
            float sn = 0.0f;
            if constexpr (F8) {
              static_assert(kTpr * 16 == 128, "sixteen codes per thread");
              sn = e4m3x16_sumsq(
                  *reinterpret_cast<const uint4*>(bfrows + r * kF8Stride + part4 * 16), 0.0f);
            } else {
              const uint4* rp =
                  reinterpret_cast<const uint4*>(bfrows + r * kBfStride + part4 * (256 / kTpr));
              #pragma unroll
              for (int t = 0; t < 16 / kTpr; ++t) {
                const uint4 c = rp[t];
                const uint32_t w[4] = {c.x, c.y, c.z, c.w};
                #pragma unroll
                for (int e = 0; e < 8; ++e) {
                  const float y =
                      __uint_as_float(e & 1 ? (w[e >> 1] & 0xFFFF0000u) : (w[e >> 1] << 16));
                  sn = __builtin_fmaf(y, y, sn);
                }
              }
            }
            #pragma unroll
            for (int off = 1; off < kTpr; off <<= 1) sn += __shfl_xor(sn, off);
            if (part4 == 0) {
              if constexpr (F8) {
                // w^ = s c: |w^|^2 = s^2 |c|^2, and the MFMA scores of the
                // codes are scaled by s; the last term is the row's
                // rounding-error bound rounded up to FP16
                const float wn = sn * (f8s * f8s);
                const float nb = sqrtf(wn) * (1.0f + 2e-5f);
                w_terms[r] = make_float4(wn, nb, f8s, __uint_as_float(half_up(f8e)));
              } else {
                const float nb = sqrtf(sn) * (1.0f + 2e-5f);
                // |w - w^| <= u |w^| / (1 - u) for a row rounded to nearest even
                const float db =
                    nb * (float)(Fmt<0>::kUnit / (1.0 - Fmt<0>::kUnit) * (1.0 + 1e-6)) + 1e-30f;
                w_terms[r] = make_float4(sn, nb, db, __uint_as_float(half_up(nb)));
              }
            }
          }
          __syncthreads();
          if (ballot(hmask != 0ull) != 0ull) {
            // S^T = W^ Q^T on MFMA, for the row blocks where one of the
            // wave's queries has a hit (the others are never read).  Block
            // position m of block cb holds window row 16 cb + 4 (m & 3) +
            // (m >> 2), so that the scores of consecutive rows -- a query's
            // hits come in runs of neighbouring window positions -- land in
            // its four lane groups in turn and the lanes share the work
            f32x4 acc[kBfBlocks];
            const int arow = ((lane & 3) << 2) | ((lane >> 2) & 3);
            #pragma unroll
            for (int cb = 0; cb < kBfBlocks; ++cb) {
              acc[cb] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
              if (ballot(((hmask >> (16 * cb)) & 0xFFFFull) != 0ull) == 0ull) continue;
              #pragma unroll
              for (int kk = 0; kk < 4; ++kk) {
                bf16x8 a;
                if constexpr (F8)
                  a = e4m3x8_bf16(*reinterpret_cast<const uint2*>(
                      bfrows + (cb * 16 + arow) * kF8Stride + kk * 32 + g * 8));
                else
                  a = *reinterpret_cast<const bf16x8*>(bfrows + (cb * 16 + arow) * kBfStride +
                                                       (kk * 32 + g * 8) * 2);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[kk], acc[cb], 0, 0, 0);
              }
            }
            // this lane's hits among its scores: slot 4 cb + i (element i of
            // acc[cb]) is window row 16 cb + 4 i + g; only set slots are
            // visited
            uint32_t slots = 0u;
            #pragma unroll
            for (int cb = 0; cb < kBfBlocks; ++cb)
              #pragma unroll
              for (int i = 0; i < 4; ++i)
                slots |= (uint32_t)((hmask >> (16 * cb + 4 * i + g)) & 1ull) << (4 * cb + i);
            // the slots in a fixed order, a block's four row terms read
            // together; a slot without a hit leaves the state unchanged
            #pragma unroll
            for (int cb = 0; cb < kBfBlocks; ++cb) {
              if (((slots >> (4 * cb)) & 0xFu) == 0u) continue;
              float4 wt[4];
              #pragma unroll
              for (int i = 0; i < 4; ++i) wt[i] = w_terms[16 * cb + 4 * i + g];
              #pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (!((slots >> (4 * cb + i)) & 1u)) continue;
                const float sc = F8 ? wt[i].z * acc[cb][i] : acc[cb][i];
                const float at = (qn_part + wt[i].x) - 2.0f * sc;
                const uint32_t term = __float_as_uint(wt[i].w);
                st.add(at, (uint32_t)(c0 + 16 * cb + 4 * i + g) | (term << 16), wt[i].y,
                       F8 ? term : 0u);
              }
            }
          }
        }
        // this lane's bounds: the kept candidates' D_lo and D_hi (two
        // smallest D_hi), and a lower bound on D_lo of the pushed-out ones
        float klo[kKeep];
        float u1 = __builtin_inff(), u2 = __builtin_inff();
        #pragma unroll
        for (int t = 0; t < kKeep; ++t) {
          float dlo = __builtin_inff(), dhi = __builtin_inff();
          if (st.pk[t] != kNoPick) {
            if constexpr (F8)  // the lane's largest row norm for the MFMA term
              bounds_from(st.a[t], st.nb_max, q_nb, q_db + half_value(st.pk[t] >> 16), dlo, dhi);
            else
              bf_bounds(st.a[t], half_value(st.pk[t] >> 16), q_nb, q_db, dlo, dhi);
          }
          klo[t] = dlo;
          u2 = fminf(u2, fmaxf(u1, dhi));
          u1 = fminf(u1, dhi);
        }
        float dmin = __builtin_inff();
        if (st.a_drop != __builtin_inff()) {
          float dhi_unused;
          if constexpr (F8)
            bounds_from(st.a_drop, st.nb_max, q_nb, q_db + half_value(st.ew_max), dmin,
                        dhi_unused);
          else
            bf_bounds(st.a_drop, st.nb_max, q_nb, q_db, dmin, dhi_unused);
        }
        bool bad = st.bad || !(u1 == u1) || !(u2 == u2) || !(dmin == dmin);
        // the row's U2 and smallest dropped bound over its four lanes
        #pragma unroll
        for (int off = 16; off < kWave; off <<= 1) {
          const float o1 = __shfl_xor(u1, off), o2 = __shfl_xor(u2, off);
          u2 = fminf(fmaxf(u1, o1), fminf(u2, o2));
          u1 = fminf(u1, o1);
          dmin = fminf(dmin, __shfl_xor(dmin, off));
          bad |= __shfl_xor((int)bad, off) != 0;
        }
        // nothing dropped (dmin = +inf): every candidate that can be best or
        // second is kept, including rows of fewer than two candidates (U2 = +inf)
        cert = mine2 && !bad && (dmin == __builtin_inff() || dmin > u2);
        // the row's exact distances (kept candidates within U2) are listed
        // per query and dealt to its four lanes
        uint32_t tmask = 0u;
        #pragma unroll
        for (int t = 0; t < kKeep; ++t)
          if (cert && st.pk[t] != kNoPick && klo[t] <= u2) tmask |= 1u << t;
        const uint32_t myn = (uint32_t)__popc(tmask);
        const int qlane = lane & (kQPerWave - 1);
        const uint32_t n0 = (uint32_t)__shfl((int)myn, qlane), n1 = (uint32_t)__shfl((int)myn, qlane + 16),
                       n2 = (uint32_t)__shfl((int)myn, qlane + 32), n3 = (uint32_t)__shfl((int)myn, qlane + 48);
        const uint32_t before = (g > 0 ? n0 : 0u) + (g > 1 ? n1 : 0u) + (g > 2 ? n2 : 0u);
        const uint32_t qtotal = n0 + n1 + n2 + n3;
        uint16_t* mylist = qtask + q2 * kQTasks;
        {
          uint32_t k = before;
          #pragma unroll
          for (int t = 0; t < kKeep; ++t)
            if ((tmask >> t) & 1u) mylist[k++] = (uint16_t)(st.pk[t] & 0xFFFFu);
        }
        wave_sync_lds();
        // one task of each query per round: the query's four lanes load their
        // quarters of the candidate's FP32 row (the next round's while this
        // one is summed) and pass the canonical sum on from quarter to
        // quarter, so it runs over dimensions 0 .. 127 in order
        const uint32_t rounds = wave_max_u32(qtotal);
        const float4* w2 = reinterpret_cast<const float4*>(A.desc2);
        auto wslice = [&](uint32_t k, float4* dst) {
          const bool has = k < qtotal;
          const int32_t j = has ? sJ_keep[mylist[k]] : 0;
          const float4* wr = w2 + (kb + j) * 32 + g * 8;
          #pragma unroll
          for (int u = 0; u < 8; ++u) dst[u] = has ? wr[u] : make_float4(0.f, 0.f, 0.f, 0.f);
        };
        float4 wcur[8], wnext[8];
        if (rounds > 0) wslice(0, wcur);
        for (uint32_t rd = 0; rd < rounds; ++rd) {
          if (rd + 1 < rounds) wslice(rd + 1, wnext);
          float sum = 0.0f;
          #pragma unroll
          for (int gp = 0; gp < 4; ++gp) {
            float acc = sum;
            #pragma unroll
            for (int u = 0; u < 8; ++u) acc = canonical_step4(acc, qx[u], wcur[u]);
            sum = __shfl(acc, qlane + 16 * gp);  // quarter gp's result
          }
          if (rd < qtotal && g == 0) {
            best.insert(sum, sJ_keep[mylist[rd]]);
            ++evals;
          }
          #pragma unroll
          for (int u = 0; u < 8; ++u) wcur[u] = wnext[u];
        }
      }
      if (g == 0 && q2 < T.count) {  // lane group 0 holds the query's selection
        const bool empty = qmode[q2] == kQueryEmpty;
        A.qrec[qi2] = query_record(empty ? 0u : cnt[q2], A.ratio, best, (mine2 && cert) || empty);
        if (mine2 && !cert) {
          const unsigned long long at = atomicAdd(&A.stats[kStatRest], 1ull);
          A.rest[at] = (uint32_t)qi2;
        }
      }
      const uint32_t n_rank = (uint32_t)__popcll(ballot(mine2 && g == 0));
      const uint32_t n_unc = (uint32_t)__popcll(ballot(mine2 && g == 0 && !cert));
      const uint32_t n_ev = wave_sum_u32(evals);
      if (lane == 0) {
        atomicAdd(&tile_stats[4], n_rank);
        atomicAdd(&tile_stats[5], n_unc);
        atomicAdd(&tile_stats[6], n_ev);
      }
    }
    // the tile's counters: complete once every wavefront has passed a barrier
    // after adding its share (the match phase has one unless it was skipped);
    // written per tile, summed on the host when they are asked for
    // (the BF16 phase adds its counters after its last barrier: one more)
    if (!FUSE || RED || !(fusable && total_len > 0)) __syncthreads();
    if (A.tile_counts && tid == 0) {
      const uint64_t nb = tile_stats[2];
      unsigned long long* tc = A.tile_counts + (int64_t)tile * kTileCounts;
      tc[0] = (unsigned long long)tile_stats[0] + nb * (uint64_t)pd.n;
      tc[1] = (unsigned long long)tile_stats[1] + nb * (uint64_t)pd.n;
      tc[2] = nb;
      tc[3] = tile_stats[3];
      tc[4] = tile_stats[4];
      tc[5] = tile_stats[5];
      tc[6] = tile_stats[6];
      tc[7] = 0ull;
    }
    if (PERSIST) __syncthreads();  // the tile's LDS is dead before the next one starts
  }
}

// Fill pass, part 1: sixteen lanes per query, queries in natural order, copy
// the parked (already sorted) short rows; short rows marked as not parked and
// longer rows of brute-force queries are queued for part 2 (long rows of
// normal queries go to the wide-row pass).
constexpr int kCopyLanes = 16;
constexpr int kCopyQueries = kThreads / kCopyLanes;
constexpr int kCopyUnroll = 4;  // rows per group
__global__ __launch_bounds__(kThreads) void k_copy_rows(StabArgs A) {
  static_assert(kCopyLanes <= kStage, "the first piece lies inside the staging slot");
  const int sub = (int)(threadIdx.x & (kCopyLanes - 1));
  // kCopyUnroll consecutive rows per group of kCopyLanes, their loads in flight together
  const int64_t i0 =
      ((int64_t)blockIdx.x * kCopyQueries + (threadIdx.x / kCopyLanes)) * kCopyUnroll;
  if (i0 >= A.n1) return;  // whole groups of kCopyLanes leave together
  // each slot's first piece is read beside the row offsets (before the row's
  // length is known); its first word tells whether the row was parked
  int32_t v[kCopyUnroll];
  int64_t o0[kCopyUnroll], o1[kCopyUnroll];
  #pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int64_t i = i0 + u;
    const bool in = i < A.n1;
    v[u] = in ? A.staging[i * kStage + sub] : 0;
    o0[u] = in ? A.row_offsets[i] : 0;
    o1[u] = in ? A.row_offsets[i + 1] : 0;
  }
  #pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int64_t i = i0 + u;
    if (i >= A.n1) break;  // uniform in the group
    const int64_t len = o1[u] - o0[u];
    const int32_t first = __shfl(v[u], 0, kCopyLanes);
    if (len <= kStage && (len == 0 || first != kRowNotParked)) {
      if (sub < len && o0[u] + sub < A.capacity) A.cols[o0[u] + sub] = v[u];
      const int32_t* src = A.staging + i * kStage;
      for (int k = sub + kCopyLanes; k < (int)len; k += kCopyLanes)
        if (o0[u] + k < A.capacity) A.cols[o0[u] + k] = src[k];
    } else if (sub == 0 && (len <= kStage || A.qflag[i] != kQueryNormal)) {
      // long rows of normal queries belong to the wide-row pass of their tile
      const unsigned long long slot = atomicAdd(&A.stats[kStatLongRows], 1ull);
      A.long_rows[slot] = (uint32_t)i;
    }
  }
}

// The fused pass's matches, from its per-query records to the caller's
// arrays (thread per query, all accesses coalesced), unless a later pass
// writes the query's match.
__global__ __launch_bounds__(kThreads) void k_write_matches(StabArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= A.n1) return;
  const uint4 r = A.qrec[i];
  if ((int32_t)r.y == kMatchDeferred) return;
  A.best_idx[i] = (int32_t)r.y;
  A.best_dist[i] = __uint_as_float(r.z);
  A.second_dist[i] = __uint_as_float(r.w);
}

// Fill pass, part 2: rebuilds the queued long rows (grid-stride over the
// queue, whose length only the device knows).
__global__ __launch_bounds__(kThreads) void k_fill_long(StabArgs A) {
  __shared__ int32_t rowbuf[kWaves][kRowSortMax];
  const int wave = wave_id();
  const uint64_t n = A.stats[kStatLongRows];
  for (uint64_t t = (uint64_t)blockIdx.x * kWaves + wave; t < n;
       t += (uint64_t)gridDim.x * kWaves)
    fill_row(A, (int64_t)A.long_rows[t], rowbuf[wave]);
}

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;
constexpr int64_t kScanDirectBlocks = 4096;  // up to 8 M counts: no top-level scan launch

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

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(const uint32_t* __restrict__ counts, int stride,
                                                                int64_t n,
                                                                int64_t* __restrict__ partials) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (idx < n) s += counts[idx * stride];
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

// Sum of partials[0 .. nb) by one workgroup (every thread gets it).
__device__ __forceinline__ int64_t block_sum(const int64_t* __restrict__ partials, int64_t nb,
                                             int64_t* sh) {
  int64_t v = 0;
  for (int64_t k = threadIdx.x; k < nb; k += kScanThreads) v += partials[k];
  int64_t tot;
  block_exclusive_scan(v, sh, &tot);
  return tot;
}

// Final pass without the top-level scan (few blocks): block b adds up the
// partial sums of blocks 0 .. b - 1 itself; the last block writes offsets[n].
__global__ __launch_bounds__(kScanThreads) void k_scan_final_direct(
    const uint32_t* __restrict__ counts, int stride, int64_t n, const int64_t* __restrict__ partials,
    int64_t nb, int64_t* __restrict__ offsets) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t before = block_sum(partials, (int64_t)blockIdx.x, sh);
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? counts[(base + k) * stride] : 0u;
    s += v[k];
  }
  int64_t tot;
  int64_t run = before + block_exclusive_scan(s, sh, &tot);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) offsets[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) offsets[n] = before + tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_final(const uint32_t* __restrict__ counts, int stride,
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
    v[k] = base + k < n ? counts[(base + k) * stride] : 0u;
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

__global__ __launch_bounds__(256) void k_clear_stats(unsigned long long* stats, uint32_t* sched,
                                                     unsigned long long* match_stats) {
  if (stats && threadIdx.x < kNumStats) stats[threadIdx.x] = 0ull;
  if (match_stats && threadIdx.x < kMatchStatWords) match_stats[threadIdx.x] = 0ull;
  if (sched)
    for (int k = (int)threadIdx.x; k < kSchedWords; k += 256) sched[k] = 0u;
}

hipError_t launch_clear_stats(unsigned long long* stats, hipStream_t s, uint32_t* sched,
                              unsigned long long* match_stats) {
  hipLaunchKernelGGL(k_clear_stats, dim3(1), dim3(256), 0, s, stats, sched, match_stats);
  return hipGetLastError();
}

hipError_t launch_tile_windows(const StabArgs& a, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_windows, dim3((a.num_tiles + kWindowTiles - 1) / kWindowTiles),
                     dim3(kWave * kWindowTiles), 0, s, a);
  return hipGetLastError();
}

namespace {

template <int MODE, int CH>
void launch_stab_mode(const StabArgs& a, int grid, const dim3& g, hipStream_t s) {
  if (grid > 0)
    hipLaunchKernelGGL((k_stab_tile<true, MODE, CH>), g, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_stab_tile<false, MODE, CH>), g, dim3(kThreads), 0, s, a);
}

template <int CH>
hipError_t launch_stab_chunk(const StabArgs& a, int grid, int mode, const dim3& g,
                             hipStream_t s) {
  switch (mode) {
    case kStabCount: launch_stab_mode<kStabCount, CH>(a, grid, g, s); break;
    case kStabF32: launch_stab_mode<kStabF32, CH>(a, grid, g, s); break;
    case kStabBF16: launch_stab_mode<kStabBF16, CH>(a, grid, g, s); break;
    case kStabFP8: launch_stab_mode<kStabFP8, CH>(a, grid, g, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stab_tiles(const StabArgs& a, int grid, int mode, int chunk, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  if (grid > 0 && !a.queue) return hipErrorInvalidValue;
  if (mode != kStabCount && (!a.desc1 || !a.desc2 || !a.best_idx || !a.best_dist ||
                             !a.second_dist || !a.rest || !a.qrec))
    return hipErrorInvalidValue;
  if (mode == kStabBF16 && (!a.codes1 || !a.codes2)) return hipErrorInvalidValue;
  // (FP8: the image-2 pointers are read only through window records, so they
  // may be NULL when image 2 is empty; the entry point checks them otherwise)
  const dim3 g(grid > 0 ? (grid < a.num_tiles ? grid : a.num_tiles) : a.num_tiles);
  // default: 256 records for the BF16 and FP8 passes (their LDS then allows
  // four workgroups per CU), kChunk otherwise
  if (chunk == 0) chunk = mode == kStabBF16 || mode == kStabFP8 ? 256 : kChunk;
  switch (chunk) {
    case 256: return launch_stab_chunk<256>(a, grid, mode, g, s);
    case 512: return launch_stab_chunk<512>(a, grid, mode, g, s);
    case 1024: return launch_stab_chunk<1024>(a, grid, mode, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_rows(const StabArgs& a, hipStream_t s) {
  if (a.n1 == 0) return hipSuccess;
  const int64_t blocks = (a.n1 + kWaves - 1) / kWaves;
  const int64_t rows_per_block = (int64_t)kCopyQueries * kCopyUnroll;
  const int64_t cblocks = (a.n1 + rows_per_block - 1) / rows_per_block;
  if (a.qrec)
    hipLaunchKernelGGL(k_write_matches, dim3((unsigned)((a.n1 + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)cblocks), dim3(kThreads), 0, s, a);
  // long rows are few and each is latency-bound: up to 2048 workgroups
  // (8192 wavefronts) take them from the queue
  const int64_t lblocks = blocks < 2048 ? blocks : 2048;
  hipLaunchKernelGGL(k_fill_long, dim3((unsigned)lblocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

int64_t scan_partials_count(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan_counts(const uint32_t* counts, int stride, int64_t n, int64_t* offsets,
                              int64_t* partials, hipStream_t s) {
  if (n == 0) {
    // offsets[0] = 0 is written by the caller
    return hipSuccess;
  }
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, stride,
                     n, partials);
  if (nb <= kScanDirectBlocks) {  // every block sums the partials before it
    hipLaunchKernelGGL(k_scan_final_direct, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts,
                       stride, n, partials, nb, offsets);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, stride,
                     n, partials, nb, offsets);
  return hipGetLastError();
}

}  // namespace epm
