// Segmented, stable LSD radix sort of (u32 key, u32 value) pairs.
//
// Builds the angle-sorted interval layout that replaces the paper's centred
// segment tree (Sec. 4.4): every pair's records are one segment.  Each
// segment is cut into tiles of kSortTile elements that never straddle two
// segments, so the per-pass digit offsets are a scan over (digit, tile)
// inside one segment and no cross-segment work is needed.
//
// Per 8-bit pass: k_sort_hist (per-tile digit counts), k_sort_offsets (one
// workgroup per segment turns the counts into global start offsets, in place)
// and k_sort_scatter (stable ranking with wavefront ballots, then the write).
// Workgroups take their tiles through xcd_tile: groups of consecutive tiles
// run on one XCD, so the short digit runs that neighbouring tiles of a
// segment write side by side in every bucket meet in one L2 before they are
// written back.
// When no segment has more than kFusedTiles tiles, a pass is one launch:
// k_sort_pass finds its tile's offsets from the per-tile counts of its
// segment itself and, while writing, counts the next pass's digits into the
// tiles the elements land in, so only the first pass needs counts, from
// k_sort_hist or from the kernel that wrote the keys.
#include "device_common.h"
#include "launch.h"

namespace epm {

namespace {

constexpr int kRadix = 256;
constexpr int kWavesPerBlock = kSortThreads / kWave;

// zero_passes > 0: also clears this tile's counts of the next zero_passes
// passes (the fused sort accumulates them with atomics).
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ keys,
                                                            const SortTile* __restrict__ tiles,
                                                            int shift,
                                                            uint32_t* __restrict__ hist,
                                                            int zero_passes) {
  __shared__ uint32_t h[kRadix];
  const int tid = threadIdx.x;
  const int tb = xcd_tile((int)blockIdx.x, (int)gridDim.x);  // this workgroup's tile
  h[tid] = 0;
  for (int p = 1; p <= zero_passes; ++p)
    hist[((int64_t)p * gridDim.x + tb) * kRadix + tid] = 0u;
  __syncthreads();
  const SortTile t = tiles[tb];
  for (int k = tid; k < t.count; k += kSortThreads)
    atomicAdd(&h[(keys[t.begin + k] >> shift) & (kRadix - 1)], 1u);
  __syncthreads();
  hist[(int64_t)tb * kRadix + tid] = h[tid];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_offsets(const SortSeg* __restrict__ segs,
                                                               uint32_t* __restrict__ hist,
                                                               uint32_t* __restrict__ seg_base) {
  __shared__ uint32_t sc[kRadix];
  const SortSeg sg = segs[blockIdx.x];
  const int d = threadIdx.x;
  constexpr int kBatch = 8;  // tiles whose counts are in flight at once
  const uint32_t* hd = hist + (int64_t)sg.tile_begin * kRadix + d;
  uint32_t total = 0;
  for (int t0 = 0; t0 < sg.tile_count; t0 += kBatch) {
    uint32_t c[kBatch];
    #pragma unroll
    for (int u = 0; u < kBatch; ++u)
      c[u] = t0 + u < sg.tile_count ? hd[(int64_t)(t0 + u) * kRadix] : 0u;
    #pragma unroll
    for (int u = 0; u < kBatch; ++u) total += c[u];
  }
  // exclusive scan over the 256 digits (Hillis-Steele in LDS)
  sc[d] = total;
  __syncthreads();
  for (int off = 1; off < kRadix; off <<= 1) {
    const uint32_t v = d >= off ? sc[d - off] : 0u;
    __syncthreads();
    sc[d] += v;
    __syncthreads();
  }
  uint32_t run = (uint32_t)sg.begin + sc[d] - total;
  // start of every digit inside the segment (after the last pass: the sorted
  // order's bucket boundaries)
  if (seg_base) seg_base[(int64_t)blockIdx.x * kRadix + d] = run;
  uint32_t* hw = hist + (int64_t)sg.tile_begin * kRadix + d;
  for (int t0 = 0; t0 < sg.tile_count; t0 += kBatch) {
    uint32_t c[kBatch];
    #pragma unroll
    for (int u = 0; u < kBatch; ++u)
      c[u] = t0 + u < sg.tile_count ? hw[(int64_t)(t0 + u) * kRadix] : 0u;
    #pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (t0 + u < sg.tile_count) hw[(int64_t)(t0 + u) * kRadix] = run;
      run += c[u];
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const SortTile* __restrict__ tiles,
    int shift, const uint32_t* __restrict__ offs) {
  __shared__ uint32_t run[kRadix];
  __shared__ uint32_t wcnt[kWavesPerBlock][kRadix];
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int tb = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const SortTile t = tiles[tb];
  run[tid] = offs[(int64_t)tb * kRadix + tid];
  for (int base = 0; base < t.count; base += kSortThreads) {
    const int idx = base + tid;
    const bool valid = idx < t.count;
    const uint32_t key = valid ? kin[t.begin + idx] : 0u;
    const uint32_t val = valid ? vin[t.begin + idx] : 0u;
    const uint32_t d = (key >> shift) & (kRadix - 1);
    // lanes of this wavefront holding the same digit
    uint64_t same = ballot(valid);
    #pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = ballot(valid && bit);
      same &= bit ? m : ~m;
    }
    const uint32_t rank = lanes_below(same);
    #pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    #pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][tid];
    run[tid] += add;
    __syncthreads();
  }
}

constexpr int kFusedTiles = 128;

// The tile lists of the record sort, the query sort and the stabbing pass,
// filled on the device from the per-pair tables (segments, query slice starts
// and the first stabbing tile of each pair), so that only those go up from
// the host; the host builds the same lists for its launch sizes.  One thread
// per tile: its segment (or pair) is the last one whose first tile is not
// after it, which skips empty ones.
__global__ __launch_bounds__(256) void k_expand_tiles(
    const SortSeg* __restrict__ rsegs, const SortSeg* __restrict__ qsegs,
    const int64_t* __restrict__ qstart, const int32_t* __restrict__ stile_begin, int num_pairs,
    SortTile* __restrict__ rtiles, int64_t tr, SortTile* __restrict__ qtiles, int64_t tq,
    StabTile* __restrict__ stiles, int64_t ts) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < tr + tq) {
    const bool rec = g < tr;
    const SortSeg* segs = rec ? rsegs : qsegs;
    const int64_t t = rec ? g : g - tr;
    int lo = 0, hi = num_pairs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)segs[mid].tile_begin <= t) lo = mid;
      else hi = mid - 1;
    }
    const SortSeg sg = segs[lo];
    const int64_t o = (t - sg.tile_begin) * kSortTile;
    SortTile st;
    st.begin = sg.begin + o;
    st.count = (int32_t)(sg.count - o < kSortTile ? sg.count - o : kSortTile);
    st.seg = lo;
    (rec ? rtiles : qtiles)[t] = st;
  } else if (g < tr + tq + ts) {
    const int64_t t = g - tr - tq;
    int lo = 0, hi = num_pairs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)stile_begin[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int64_t o = (t - stile_begin[lo]) * kTileQ;
    const int64_t m = qstart[lo + 1] - qstart[lo];
    StabTile st;
    st.begin = qstart[lo] + o;
    st.count = (int32_t)(m - o < kTileQ ? m - o : kTileQ);
    st.pair = lo;
    stiles[t] = st;
  }
}

// Sorts of more tiles than this take each pass's counts from LDS histograms
// of the keys (k_sort_hist) and the tile offsets from k_sort_offsets, three
// launches per pass: at that size the global atomics with which the one-launch
// pass counts the next pass's digits dominate it.  Smaller sorts keep the one
// launch per pass.
constexpr int kSplitPassTiles = 2048;

// One pass of the fused sort.  hist: this pass's per-tile digit counts, or
// (READY) the tiles' start offsets that k_sort_offsets made of them;
// hist_next: the next pass's counts (zero on entry), or NULL on the last pass.
template <bool READY>
__global__ __launch_bounds__(kSortThreads) void k_sort_pass(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const SortTile* __restrict__ tiles,
    const SortSeg* __restrict__ segs, int num_segs, int shift, const uint32_t* __restrict__ hist,
    uint32_t* __restrict__ hist_next, uint32_t* __restrict__ seg_base) {
  __shared__ uint32_t run[kRadix];
  __shared__ uint32_t wsum[kWavesPerBlock];
  __shared__ uint32_t wcnt[kWavesPerBlock][kRadix];
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int tb = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const SortTile t = tiles[tb];
  const SortSeg sg = segs[t.seg];
  static_assert(kSortThreads == kRadix, "one digit per thread");
  // the tile's keys and values, loaded while the offsets are worked out
  constexpr int kRounds = kSortTile / kSortThreads;
  uint32_t rk[kRounds], rv[kRounds];
  #pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int idx = r * kSortThreads + tid;
    rk[r] = idx < t.count ? kin[t.begin + idx] : 0u;
    rv[r] = idx < t.count ? vin[t.begin + idx] : 0u;
  }
  const int mine = tb - sg.tile_begin;
  if constexpr (READY) {
    run[tid] = hist[(int64_t)tb * kRadix + tid];
    __syncthreads();
  } else {
    // digit d = tid: count in the segment's earlier tiles, and in all of them
    uint32_t before = 0, total = 0;
    const uint32_t* hd = hist + (int64_t)sg.tile_begin * kRadix + tid;
    constexpr int kBatch = 16;  // tiles whose counts are in flight at once
    for (int t0 = 0; t0 < sg.tile_count; t0 += kBatch) {
      uint32_t c[kBatch];
      #pragma unroll
      for (int u = 0; u < kBatch; ++u)
        c[u] = t0 + u < sg.tile_count ? hd[(int64_t)(t0 + u) * kRadix] : 0u;
      #pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        total += c[u];
        before += t0 + u < mine ? c[u] : 0u;
      }
    }
    // exclusive scan of the totals over the digits: wavefront scans, then
    // the wavefront totals
    uint32_t incl = total;
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    #pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) incl += w < wave ? wsum[w] : 0u;
    const uint32_t start = (uint32_t)sg.begin + incl - total;
    run[tid] = start + before;
    if (seg_base && mine == 0) seg_base[(int64_t)t.seg * kRadix + tid] = start;
    // segments without elements have no tile: the first workgroup writes
    // their (empty) digit starts
    if (seg_base && blockIdx.x == 0) {
      for (int g = tid; g < num_segs; g += kSortThreads) {
        const SortSeg e = segs[g];
        if (e.count == 0)
          for (int dd = 0; dd < kRadix; ++dd) seg_base[(int64_t)g * kRadix + dd] = (uint32_t)e.begin;
      }
    }
    __syncthreads();
  }
  const int nshift = shift + 8;
  #pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int base = r * kSortThreads;
    if (base >= t.count) break;  // uniform
    const int idx = base + tid;
    const bool valid = idx < t.count;
    const uint32_t key = rk[r];
    const uint32_t val = rv[r];
    const uint32_t d = (key >> shift) & (kRadix - 1);
    uint64_t same = ballot(valid);
    #pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = ballot(valid && bit);
      same &= bit ? m : ~m;
    }
    const uint32_t rank = lanes_below(same);
    #pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
      if (hist_next) {
        // the tile of the segment that position pos belongs to next pass
        const int64_t nt = sg.tile_begin + ((int64_t)pos - sg.begin) / kSortTile;
        atomicAdd(&hist_next[nt * kRadix + ((key >> nshift) & (kRadix - 1))], 1u);
      }
    }
    __syncthreads();
    uint32_t add = 0;
    #pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][tid];
    run[tid] += add;
    __syncthreads();
  }
}

}  // namespace

int sort_passes(int bits) { return (bits + 7) / 8; }

hipError_t launch_expand_tiles(const SortSeg* rsegs, const SortSeg* qsegs, const int64_t* qstart,
                               const int32_t* stile_begin, int num_pairs, SortTile* rtiles,
                               int64_t tr, SortTile* qtiles, int64_t tq, StabTile* stiles,
                               int64_t ts, hipStream_t s) {
  const int64_t n = tr + tq + ts;
  if (n == 0 || num_pairs < 1) return hipSuccess;
  hipLaunchKernelGGL(k_expand_tiles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rsegs,
                     qsegs, qstart, stile_begin, num_pairs, rtiles, tr, qtiles, tq, stiles, ts);
  return hipGetLastError();
}

hipError_t segmented_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                                const SortTile* tiles, int num_tiles, const SortSeg* segs,
                                int num_segs, int max_seg_tiles, uint32_t* hist, int bits,
                                bool* sorted_in_1, hipStream_t s, uint32_t* last_digit_base,
                                bool first_counts_ready) {
  *sorted_in_1 = false;
  if (num_tiles == 0) return hipSuccess;
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  if (max_seg_tiles <= kFusedTiles) {
    const int npass = sort_passes(bits);
    // counts of passes 1 .. npass-1 are accumulated by the previous pass
    // into rows this launch clears (or the kernel that wrote the keys did
    // both)
    if (!first_counts_ready)
      hipLaunchKernelGGL(k_sort_hist, dim3(num_tiles), dim3(kSortThreads), 0, s, ki, tiles, 0,
                         hist, npass - 1);
    for (int p = 0; p < npass; ++p) {
      const bool last = p + 1 == npass;
      uint32_t* h = hist + (int64_t)p * num_tiles * kRadix;
      uint32_t* hn = last ? nullptr : h + (int64_t)num_tiles * kRadix;
      if (num_tiles > kSplitPassTiles) {
        // counts from LDS histograms of the keys (not global atomics in the
        // previous pass's scatter), then the tile offsets, then the scatter
        if (p > 0)
          hipLaunchKernelGGL(k_sort_hist, dim3(num_tiles), dim3(kSortThreads), 0, s, ki, tiles,
                             8 * p, h, 0);
        hipLaunchKernelGGL(k_sort_offsets, dim3(num_segs), dim3(kSortThreads), 0, s, segs, h,
                           last ? last_digit_base : nullptr);
        hipLaunchKernelGGL((k_sort_pass<true>), dim3(num_tiles), dim3(kSortThreads), 0, s, ki, vi,
                           ko, vo, tiles, segs, num_segs, 8 * p, h, nullptr, nullptr);
      } else {
        hipLaunchKernelGGL((k_sort_pass<false>), dim3(num_tiles), dim3(kSortThreads), 0, s, ki,
                           vi, ko, vo, tiles, segs, num_segs, 8 * p, h, hn,
                           last ? last_digit_base : nullptr);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      uint32_t* tk = ki; ki = ko; ko = tk;
      uint32_t* tv = vi; vi = vo; vo = tv;
      *sorted_in_1 = !*sorted_in_1;
    }
    return hipSuccess;
  }
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_sort_hist, dim3(num_tiles), dim3(kSortThreads), 0, s, ki, tiles, shift,
                       hist, 0);
    const bool last = shift + 8 >= bits;
    hipLaunchKernelGGL(k_sort_offsets, dim3(num_segs), dim3(kSortThreads), 0, s, segs, hist,
                       last ? last_digit_base : nullptr);
    hipLaunchKernelGGL(k_sort_scatter, dim3(num_tiles), dim3(kSortThreads), 0, s, ki, vi, ko, vo,
                       tiles, shift, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* tk = ki; ki = ko; ko = tk;
    uint32_t* tv = vi; vi = vo; vo = tv;
    *sorted_in_1 = !*sorted_in_1;
  }
  return hipSuccess;
}

}  // namespace epm
