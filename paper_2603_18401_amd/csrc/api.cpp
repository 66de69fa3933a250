// C ABI of libepm: argument validation, FP64 per-pair setup, workspace
// carving and kernel enqueue.  See include/epm.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "epm.h"
#include "epm_internal.h"
#include "launch.h"

using namespace epm;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Offsets of every device buffer inside the caller's workspace.
struct Layout {
  size_t pairs, qstart, kstart, rsegs, qsegs, stile_begin, head_end, rtiles, qtiles, stiles, hist,
      qhist;
  size_t rk0, rv0, rk1, rv1, recC, recH, rC, rH, rj, rxy, reps, rinv, class_begin;
  size_t qkey, qflag, qk0, qv0, qk1, qv1, counts, qrec, partials, staging, stats, long_rows;
  size_t digit_base, windows, match_stats, sched, tile_cost, order, block_tile, rest, tile_wide,
      pair_wide, pre_pairs, qline, tile_q, tile_counts;
  size_t total;
};

Layout make_layout(int P, int64_t n1, int64_t n2, int64_t tr, int64_t tq, int64_t ts) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes > 0 ? bytes : 1);
    return o;
  };
  const size_t N1 = (size_t)n1, N2 = (size_t)n2;
  // the host tables (one upload), then the tile lists made from them on the
  // device
  L.pairs = take(sizeof(PairDev) * P);
  L.qstart = take(sizeof(int64_t) * (P + 1));
  L.kstart = take(sizeof(int64_t) * (P + 1));
  L.rsegs = take(sizeof(SortSeg) * P);
  L.qsegs = take(sizeof(SortSeg) * P);
  L.stile_begin = take(sizeof(int32_t) * (P + 1));
  L.head_end = off;
  L.rtiles = take(sizeof(SortTile) * tr);
  L.qtiles = take(sizeof(SortTile) * tq);
  L.stiles = take(sizeof(StabTile) * ts);
  // per-tile digit counts of every pass of the record (3) and of the query
  // (2) sort: separate, so that the two sorts may run side by side
  L.hist = take(sizeof(uint32_t) * 256 * (size_t)sort_passes(kSortBits) * (size_t)tr);
  L.qhist = take(sizeof(uint32_t) * 256 * (size_t)sort_passes(kQuerySortBits) * (size_t)tq);
  L.rk0 = take(4 * N2);
  L.rv0 = take(4 * N2);
  L.rk1 = take(4 * N2);
  L.rv1 = take(4 * N2);
  L.recC = take(4 * N2);
  L.recH = take(4 * N2);
  L.rC = take(4 * N2);
  L.rH = take(4 * N2);
  L.rj = take(4 * N2);
  L.rxy = take(8 * N2);
  L.reps = take(4 * N2);
  L.rinv = take(4 * N2);
  L.class_begin = take(sizeof(int64_t) * kClassSlots * P);
  L.qkey = take(4 * N1);
  L.qflag = take(4 * N1);
  L.qk0 = take(4 * N1);
  L.qv0 = take(4 * N1);
  L.qk1 = take(4 * N1);
  L.qv1 = take(4 * N1);
  L.counts = take(4 * N1);
  L.qrec = take(16 * N1);
  L.partials = take(sizeof(int64_t) * (size_t)scan_partials_count(n1));
  L.staging = take(sizeof(int32_t) * kStage * N1);
  L.stats = take(sizeof(unsigned long long) * kNumStats);
  L.long_rows = take(sizeof(uint32_t) * N1);
  L.digit_base = take(sizeof(uint32_t) * 256 * P);
  L.windows = take(sizeof(TileWindow) * ts);
  L.match_stats = take(sizeof(unsigned long long) * kMatchStatWords);
  L.sched = take(sizeof(uint32_t) * kSchedWords);
  L.tile_cost = take(sizeof(uint32_t) * ts);
  L.order = take(sizeof(uint32_t) * ts);
  L.block_tile = take(sizeof(uint32_t) * ts);
  L.rest = take(sizeof(uint32_t) * N1);
  L.tile_wide = take(sizeof(uint32_t) * ts);
  L.pair_wide = take(sizeof(uint32_t) * P);
  L.pre_pairs = take(sizeof(int64_t) * (2 * (size_t)P + 2));
  L.qline = take(sizeof(double4) * N1);
  L.tile_q = take(sizeof(TileQuery) * kTileQ * (size_t)ts);
  L.tile_counts = take(sizeof(unsigned long long) * kTileCounts * (size_t)ts);
  L.total = off;
  return L;
}

int64_t tiles_of(int64_t count) { return (count + kSortTile - 1) / kSortTile; }

int max_tiles(const std::vector<SortSeg>& segs) {
  int m = 0;
  for (const SortSeg& g : segs) m = g.tile_count > m ? g.tile_count : m;
  return m;
}
int64_t stab_tiles_of(int64_t m) { return (m + kTileQ - 1) / kTileQ; }

bool validate_pairs(const epm_pair* pairs, int32_t num_pairs, int64_t* n1, int64_t* n2) {
  if (!pairs || num_pairs < 1 || num_pairs > 65535) return false;
  int64_t q = 0, k = 0;
  for (int p = 0; p < num_pairs; ++p) {
    const epm_pair& e = pairs[p];
    if (e.m < 0 || e.n < 0 || e.m >= (int64_t(1) << 31) || e.n >= (int64_t(1) << 31)) return false;
    if (e.q_begin != q || e.k_begin != k) return false;
    if (e.w2 <= 0 || e.h2 <= 0) return false;
    q += e.m;
    k += e.n;
  }
  if (q >= (int64_t(1) << 32) || k >= (int64_t(1) << 32)) return false;
  *n1 = q;
  *n2 = k;
  return true;
}

void cross3(const double* a, const double* b, double* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

double norm3(const double* a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// FP64 setup of one pair: image-2 normalisation, epipole e2 = null(F^T)
// (Algorithm 1, preprocessing) as a unit vector in normalised line space,
// and an orthonormal basis (u, v) of the pencil of lines through it.
epm_status setup_pair(const epm_pair& in, PairDev& pd) {
  const double* F = in.F;
  double fn = 0.0;
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(F[k])) return EPM_ERR_DEGENERATE_F;
    fn += F[k] * F[k];
  }
  if (!(fn > 0.0) || !std::isfinite(fn)) return EPM_ERR_DEGENERATE_F;
  std::memset(&pd, 0, sizeof(pd));
  for (int k = 0; k < 9; ++k) pd.F[k] = F[k];
  const double w = in.w2, h = in.h2;
  pd.s = 2.0 / (w > h ? w : h);
  pd.cx = 0.5 * w;
  pd.cy = 0.5 * h;
  // M = N F T^-1: lines in normalised image-2 coordinates, l^ = N l with
  // l^ = (a, b, s (a cx + b cy + c)), as functions of normalised image-1
  // coordinates (T^-1 undoes the same normalisation on the image-1 side, which
  // balances the columns; a right factor does not move the left null space)
  double M[3][3];
  {
    const double Ti[3][3] = {{1.0 / pd.s, 0.0, pd.cx}, {0.0, 1.0 / pd.s, pd.cy}, {0.0, 0.0, 1.0}};
    double NF[3][3];
    for (int k = 0; k < 3; ++k) {
      NF[0][k] = F[k];
      NF[1][k] = F[3 + k];
      NF[2][k] = pd.s * (F[k] * pd.cx + F[3 + k] * pd.cy + F[6 + k]);
    }
    double mx = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        M[r][k] = NF[r][0] * Ti[0][k] + NF[r][1] * Ti[1][k] + NF[r][2] * Ti[2][k];
        mx = std::fmax(mx, std::fabs(M[r][k]));
      }
    if (!(mx > 0.0) || !std::isfinite(mx)) return EPM_ERR_DEGENERATE_F;
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) M[r][k] /= mx;
  }
  double col[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) col[k][d] = M[d][k];
  // the left null vector is orthogonal to every column: the largest cross
  // product of two columns (a column that is only rounding residue never wins)
  double best[3] = {0, 0, 0}, bn = 0.0;
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int t = 0; t < 3; ++t) {
    double cr[3];
    cross3(col[pa[t]], col[pb[t]], cr);
    const double cn = norm3(cr);
    if (cn > bn) {
      bn = cn;
      for (int d = 0; d < 3; ++d) best[d] = cr[d];
    }
  }
  if (!(bn > 1e-12)) return EPM_ERR_DEGENERATE_F;  // rank <= 1: no pencil
  for (int d = 0; d < 3; ++d) pd.e[d] = best[d] / bn;
  // u: e x (the axis least aligned with e), v = e x u
  int ax = 0;
  for (int d = 1; d < 3; ++d)
    if (std::fabs(pd.e[d]) < std::fabs(pd.e[ax])) ax = d;
  double axis[3] = {0, 0, 0};
  axis[ax] = 1.0;
  cross3(pd.e, axis, pd.u);
  const double un = norm3(pd.u);
  for (int d = 0; d < 3; ++d) pd.u[d] /= un;
  cross3(pd.e, pd.u, pd.v);
  const double vn = norm3(pd.v);
  for (int d = 0; d < 3; ++d) pd.v[d] /= vn;
  pd.G11 = pd.u[0] * pd.u[0] + pd.u[1] * pd.u[1];
  pd.G12 = pd.u[0] * pd.v[0] + pd.u[1] * pd.v[1];
  pd.G22 = pd.v[0] * pd.v[0] + pd.v[1] * pd.v[1];
  pd.e12 = std::sqrt(pd.e[0] * pd.e[0] + pd.e[1] * pd.e[1]);
  pd.kappa = kKappaBuild;
  pd.q_begin = in.q_begin;
  pd.m = in.m;
  pd.k_begin = in.k_begin;
  pd.n = in.n;
  return EPM_OK;
}

void make_tiles(const std::vector<int64_t>& starts, int P, std::vector<SortTile>& tiles,
                std::vector<SortSeg>& segs) {
  tiles.clear();
  segs.resize(P);
  for (int p = 0; p < P; ++p) {
    const int64_t b = starts[p], cnt = starts[p + 1] - starts[p];
    segs[p].begin = b;
    segs[p].count = cnt;
    segs[p].tile_begin = (int32_t)tiles.size();
    for (int64_t o = 0; o < cnt; o += kSortTile) {
      SortTile t;
      t.begin = b + o;
      t.count = (int32_t)(cnt - o < kSortTile ? cnt - o : kSortTile);
      t.seg = p;
      tiles.push_back(t);
    }
    segs[p].tile_count = (int32_t)tiles.size() - segs[p].tile_begin;
  }
}

}  // namespace

struct epm_index {
  int P = 0;
  int64_t N1 = 0, N2 = 0;
  std::vector<PairDev> pairs;
  std::vector<int32_t> stile_begin;  // first stabbing tile of every pair, and the total
  std::vector<int64_t> qstart, kstart;
  std::vector<SortTile> rtiles, qtiles;
  std::vector<SortSeg> rsegs, qsegs;
  std::vector<StabTile> stiles;
  std::vector<char> head;  // host image of the table region of the workspace
  char* ws = nullptr;
  Layout L;
  size_t skey_off = 0;  // sorted record keys (one of the sort buffers)
  bool have_qperm = false;
  const uint32_t* qperm = nullptr;
  hipStream_t last_stream = nullptr;  // stream of the last query call
  const int64_t* last_offsets = nullptr;
  bool have_stats = false;
  bool have_match_stats = false;
  bool match_from_tiles = false;  // the last match was fused into the tile pass
  hipStream_t match_stream = nullptr;
  epm_sched sched{};         // work distribution of the tile kernels
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // around the dominant kernel of a call
  epm_timed_kernel timed = EPM_TIMED_STAB;           // which kernel of the query calls
  bool have_order = false;  // the last query wrote the longest-first tile order
  bool have_block_tile = false;  // ... or the per-XCD longest-first workgroup order

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

#define EPM_HIP(call)                         \
  do {                                        \
    if ((call) != hipSuccess) return EPM_ERR_HIP; \
  } while (0)

namespace {

// ------------------------------------------------------------ host stages
// Every stage below either does host work only or enqueues kernels only, so
// the enqueue stages can be recorded into a HIP graph as they are.

// Validation, FP64 pair setup, tiles, workspace layout and the host image of
// the table region.  No device work.
epm_status index_prepare(const epm_pair* pairs, int32_t num_pairs, void* workspace,
                         size_t workspace_bytes, epm_index** out) {
  *out = nullptr;
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2)) return EPM_ERR_ARG;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1))) return EPM_ERR_WORKSPACE;
  epm_index* idx = new (std::nothrow) epm_index();
  if (!idx) return EPM_ERR_ARG;
  idx->P = num_pairs;
  idx->N1 = n1;
  idx->N2 = n2;
  idx->pairs.resize(num_pairs);
  idx->qstart.resize(num_pairs + 1);
  idx->kstart.resize(num_pairs + 1);
  for (int p = 0; p < num_pairs; ++p) {
    const epm_status st = setup_pair(pairs[p], idx->pairs[p]);
    if (st != EPM_OK) {
      delete idx;
      return st;
    }
    idx->qstart[p] = pairs[p].q_begin;
    idx->kstart[p] = pairs[p].k_begin;
  }
  idx->qstart[num_pairs] = n1;
  idx->kstart[num_pairs] = n2;
  make_tiles(idx->kstart, num_pairs, idx->rtiles, idx->rsegs);
  make_tiles(idx->qstart, num_pairs, idx->qtiles, idx->qsegs);
  for (int p = 0; p < num_pairs; ++p) {
    PairDev& pd = idx->pairs[p];
    pd.rtile_begin = idx->rsegs[p].tile_begin;
    pd.rtile_count = idx->rsegs[p].tile_count;
    pd.qtile_begin = idx->qsegs[p].tile_begin;
    pd.qtile_count = idx->qsegs[p].tile_count;
  }
  idx->stile_begin.resize(num_pairs + 1);
  for (int p = 0; p < num_pairs; ++p) {
    idx->stile_begin[p] = (int32_t)idx->stiles.size();
    for (int64_t o = 0; o < pairs[p].m; o += kTileQ) {
      StabTile t;
      t.begin = pairs[p].q_begin + o;
      t.count = (int32_t)(pairs[p].m - o < kTileQ ? pairs[p].m - o : kTileQ);
      t.pair = p;
      idx->stiles.push_back(t);
    }
  }
  idx->stile_begin[num_pairs] = (int32_t)idx->stiles.size();
  idx->L = make_layout(num_pairs, n1, n2, (int64_t)idx->rtiles.size(), (int64_t)idx->qtiles.size(),
                       (int64_t)idx->stiles.size());
  if (workspace_bytes < idx->L.total) {
    delete idx;
    return EPM_ERR_WORKSPACE;
  }
  idx->ws = static_cast<char*>(workspace);
  const Layout& L = idx->L;
  // the host tables go up in one copy: they sit at the head of the
  // workspace, and the tile lists behind them are made on the device
  idx->head.assign(L.head_end, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(idx->head.data() + off, src, bytes);
  };
  put(L.pairs, idx->pairs.data(), sizeof(PairDev) * num_pairs);
  put(L.qstart, idx->qstart.data(), sizeof(int64_t) * (num_pairs + 1));
  put(L.kstart, idx->kstart.data(), sizeof(int64_t) * (num_pairs + 1));
  put(L.rsegs, idx->rsegs.data(), sizeof(SortSeg) * num_pairs);
  put(L.qsegs, idx->qsegs.data(), sizeof(SortSeg) * num_pairs);
  put(L.stile_begin, idx->stile_begin.data(), sizeof(int32_t) * (num_pairs + 1));
  *out = idx;
  return EPM_OK;
}

// The tile lists, from the uploaded tables (after their upload on `stream`).
hipError_t expand_tiles(const epm_index* idx, hipStream_t stream) {
  const Layout& L = idx->L;
  return launch_expand_tiles(idx->at<SortSeg>(L.rsegs), idx->at<SortSeg>(L.qsegs),
                             idx->at<int64_t>(L.qstart), idx->at<int32_t>(L.stile_begin), idx->P,
                             idx->at<SortTile>(L.rtiles), (int64_t)idx->rtiles.size(),
                             idx->at<SortTile>(L.qtiles), (int64_t)idx->qtiles.size(),
                             idx->at<StabTile>(L.stiles), (int64_t)idx->stiles.size(), stream);
}

epm_status index_upload(epm_index* idx, hipStream_t stream) {
  EPM_HIP(hipMemcpyAsync(idx->ws, idx->head.data(), idx->L.head_end, hipMemcpyHostToDevice,
                         stream));
  EPM_HIP(expand_tiles(idx, stream));
  return EPM_OK;
}

bool build_args_ok(int64_t n2, const float* kp2_xy, const float* eps2, float eps_scalar) {
  if (n2 > 0 && !kp2_xy) return false;
  return eps2 || (eps_scalar > 0.0f && std::isfinite(eps_scalar));
}

// Interval records, their segmented sort by (width class, centre) and the
// class bounds (Algorithm 1, preprocessing).
epm_status enqueue_build(epm_index* idx, const float* kp2_xy, const float* eps2,
                         float eps_scalar, hipStream_t stream) {
  const Layout& L = idx->L;
  const int P = idx->P;
  const int64_t n2 = idx->N2;
  const PairDev* dpairs = idx->at<PairDev>(L.pairs);
  const int64_t* dkstart = idx->at<int64_t>(L.kstart);
  EPM_HIP(launch_intervals(dpairs, idx->at<SortTile>(L.rtiles), (int)idx->rtiles.size(), kp2_xy,
                           eps2, eps_scalar, idx->at<uint32_t>(L.rk0), idx->at<uint32_t>(L.rv0),
                           idx->at<uint32_t>(L.recC), idx->at<uint32_t>(L.recH),
                           idx->at<uint32_t>(L.hist), sort_passes(kSortBits) - 1, stream));
  bool in1 = false;
  EPM_HIP(segmented_radix_sort(idx->at<uint32_t>(L.rk0), idx->at<uint32_t>(L.rv0),
                               idx->at<uint32_t>(L.rk1), idx->at<uint32_t>(L.rv1),
                               idx->at<SortTile>(L.rtiles), (int)idx->rtiles.size(),
                               idx->at<SortSeg>(L.rsegs), P, max_tiles(idx->rsegs),
                               idx->at<uint32_t>(L.hist), kSortBits, &in1, stream,
                               idx->at<uint32_t>(L.digit_base), true));
  const uint32_t* skey = idx->at<uint32_t>(in1 ? L.rk1 : L.rk0);
  const uint32_t* sval = idx->at<uint32_t>(in1 ? L.rv1 : L.rv0);
  EPM_HIP(launch_gather_records(dkstart, P, n2, sval, kp2_xy, eps2, eps_scalar,
                                idx->at<uint32_t>(L.recC), idx->at<uint32_t>(L.recH),
                                idx->at<uint32_t>(L.rC), idx->at<uint32_t>(L.rH),
                                idx->at<int32_t>(L.rj), idx->at<float2>(L.rxy),
                                idx->at<float>(L.reps), idx->at<uint32_t>(L.rinv),
                                idx->at<uint32_t>(L.digit_base), idx->at<int64_t>(L.class_begin),
                                stream));
  idx->skey_off = in1 ? L.rk1 : L.rk0;
  // with keypoints the gather wrote the class starts
  if (n2 == 0) EPM_HIP(launch_class_bounds(dkstart, P, skey, idx->at<int64_t>(L.class_begin), stream));
  return EPM_OK;
}

StabArgs stab_args(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                   int32_t* col_indices, int64_t capacity) {
  const Layout& L = idx->L;
  StabArgs A;
  A.pairs = idx->at<PairDev>(L.pairs);
  A.qstart = idx->at<int64_t>(L.qstart);
  A.num_pairs = idx->P;
  A.n1 = idx->N1;
  A.kp1 = kp1_xy;
  A.qkey = idx->at<uint32_t>(L.qkey);
  A.qflag = idx->at<uint32_t>(L.qflag);
  A.qperm = nullptr;
  A.class_begin = idx->at<int64_t>(L.class_begin);
  A.skey = idx->at<uint32_t>(idx->skey_off);
  A.rC = idx->at<uint32_t>(L.rC);
  A.rH = idx->at<uint32_t>(L.rH);
  A.rj = idx->at<int32_t>(L.rj);
  A.rxy = idx->at<float2>(L.rxy);
  A.reps = idx->at<float>(L.reps);
  A.rinv = idx->at<uint32_t>(L.rinv);
  A.counts = idx->at<uint32_t>(L.counts);
  A.qrec = nullptr;
  A.row_offsets = row_offsets;
  A.cols = col_indices;
  A.capacity = capacity;
  A.tiles = idx->at<StabTile>(L.stiles);
  A.num_tiles = (int)idx->stiles.size();
  A.staging = idx->at<int32_t>(L.staging);
  A.stats = idx->at<unsigned long long>(L.stats);
  A.long_rows = idx->at<uint32_t>(L.long_rows);
  A.windows = idx->at<TileWindow>(L.windows);
  A.tile_cost = nullptr;
  A.order = nullptr;
  A.queue = nullptr;
  A.tile_q = idx->at<TileQuery>(L.tile_q);
  A.tile_counts = idx->at<unsigned long long>(L.tile_counts);
  A.block_tile = nullptr;
  A.desc1 = nullptr;
  A.desc2 = nullptr;
  A.ratio = 0.0f;
  A.best_idx = nullptr;
  A.best_dist = nullptr;
  A.second_dist = nullptr;
  A.rest = idx->at<uint32_t>(L.rest);
  A.tile_wide = idx->at<uint32_t>(L.tile_wide);
  A.pair_wide = idx->at<uint32_t>(L.pair_wide);
  A.wcodes2 = nullptr;
  A.wterms2 = nullptr;
  A.match_stats = nullptr;
  A.qline = idx->at<double4>(L.qline);
  A.codes1 = nullptr;
  A.codes2 = nullptr;
  A.rest_count = A.stats + kStatRest;
  return A;
}

// Query keys and their sort, the tile windows, the stabbing pass and the
// scan of the row lengths into row_offsets (Algorithm 1, matching loop).
// records_ready: the record build runs on another stream and completes this
// event; the stream waits for it after the query sort, before the first
// kernel that reads the records.
epm_status enqueue_count(epm_index* idx, StabArgs& A, int64_t* row_offsets,
                         hipStream_t stream, int mode = kStabCount,
                         hipEvent_t records_ready = nullptr) {
  const Layout& L = idx->L;
  const int64_t n1 = idx->N1;
  idx->have_order = false;
  idx->have_block_tile = false;
  if (n1 == 0) {
    if (records_ready) EPM_HIP(hipStreamWaitEvent(stream, records_ready, 0));
    // row_offsets[0] = 0 (two zero words, by kernel); the counters read zero
    EPM_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(row_offsets), 2, 0u, stream));
    if (A.match_stats) EPM_HIP(launch_clear_stats(nullptr, stream, nullptr, A.match_stats));
    return EPM_OK;
  }
  EPM_HIP(launch_query_keys(A.pairs, idx->at<SortTile>(L.qtiles), (int)idx->qtiles.size(),
                            A.kp1, idx->at<uint32_t>(L.qkey), idx->at<uint32_t>(L.qflag),
                            idx->at<uint32_t>(L.qk0), idx->at<uint32_t>(L.qv0), A.qline,
                            idx->at<uint32_t>(L.qhist), sort_passes(kQuerySortBits) - 1, A.stats,
                            idx->at<uint32_t>(L.sched), A.match_stats, stream));
  bool in1 = false;
  EPM_HIP(segmented_radix_sort(idx->at<uint32_t>(L.qk0), idx->at<uint32_t>(L.qv0),
                               idx->at<uint32_t>(L.qk1), idx->at<uint32_t>(L.qv1),
                               idx->at<SortTile>(L.qtiles), (int)idx->qtiles.size(),
                               idx->at<SortSeg>(L.qsegs), idx->P, max_tiles(idx->qsegs),
                               idx->at<uint32_t>(L.qhist), kQuerySortBits, &in1, stream, nullptr,
                               true));
  idx->qperm = idx->at<uint32_t>(in1 ? L.qv1 : L.qv0);
  idx->have_qperm = true;
  A.qperm = idx->qperm;
  if (records_ready) EPM_HIP(hipStreamWaitEvent(stream, records_ready, 0));
  const epm_sched& S = idx->sched;
  const bool persistent = S.stab_workgroups > 0 || S.match_workgroups > 0;
  const bool lpt = persistent && S.lpt == 1;
  // one workgroup per tile: the tiles of every XCD run longest first
  const bool xcd_lpt = S.stab_workgroups == 0;
  uint32_t* sched = idx->at<uint32_t>(L.sched);  // cleared by the key pass
  A.tile_cost = lpt || xcd_lpt ? idx->at<uint32_t>(L.tile_cost) : nullptr;
  EPM_HIP(launch_tile_windows(A, stream));
  if (lpt) {
    EPM_HIP(launch_lpt_order(A.tile_cost, A.num_tiles, sched, idx->at<uint32_t>(L.order), stream));
    idx->have_order = true;
  }
  if (xcd_lpt) {
    EPM_HIP(launch_xcd_lpt_order(A.tile_cost, A.num_tiles, idx->at<uint32_t>(L.block_tile),
                                 stream));
    A.block_tile = idx->at<uint32_t>(L.block_tile);
    idx->have_block_tile = true;
  }
  if (S.stab_workgroups > 0) {
    A.queue = sched + kSchedStabQueue;
    A.order = lpt ? idx->at<uint32_t>(L.order) : nullptr;
  }
  const bool timed = idx->ev_start && idx->timed == EPM_TIMED_STAB;
  if (timed) EPM_HIP(hipEventRecord(idx->ev_start, stream));
  EPM_HIP(launch_stab_tiles(A, S.stab_workgroups, mode, S.stab_chunk, stream));
  if (timed) EPM_HIP(hipEventRecord(idx->ev_stop, stream));
  if (A.qrec)
    EPM_HIP(launch_scan_counts(reinterpret_cast<const uint32_t*>(A.qrec), 4, n1, row_offsets,
                               idx->at<int64_t>(L.partials), stream));
  else
    EPM_HIP(launch_scan_counts(A.counts, 1, n1, row_offsets, idx->at<int64_t>(L.partials), stream));
  return EPM_OK;
}

// CSR fill after the scan: parked short rows, brute-force long rows, then the
// wide-row pass (match: with its FP32 selection, see launch_wide_tiles).
// BF16 copies of the image-2 rows of the pairs with wide tiles, for a
// matching wide-row pass (A.desc2 set): they go to the staging area, whose
// parked rows the fill pass has copied out by then, when it holds 256 bytes
// of codes and 8 of terms per row; otherwise the pass rounds on chip.
hipError_t prepare_wide_rows(epm_index* idx, StabArgs& A, hipStream_t stream) {
  const size_t n2 = (size_t)idx->N2;
  const size_t codes = align_up(n2 * 256), terms = n2 * sizeof(float2);
  const size_t room = sizeof(int32_t) * kStage * (size_t)idx->N1;
  if (n2 == 0 || !A.desc2 || codes + terms > room) return hipSuccess;
  char* base = reinterpret_cast<char*>(idx->at<int32_t>(idx->L.staging));
  A.wcodes2 = reinterpret_cast<const uint16_t*>(base);
  A.wterms2 = reinterpret_cast<const float2*>(base + codes);
  return launch_round_rows(A, (int64_t)n2, idx->at<int64_t>(idx->L.pre_pairs), stream);
}

epm_status enqueue_fill(epm_index* idx, StabArgs& A, hipStream_t stream, bool match = false) {
  if (idx->N1 == 0) return EPM_OK;
  EPM_HIP(launch_fill_rows(A, stream));
  if (match) EPM_HIP(prepare_wide_rows(idx, A, stream));
  const bool timed = idx->ev_start && idx->timed == EPM_TIMED_WIDE;
  if (timed) EPM_HIP(hipEventRecord(idx->ev_start, stream));
  EPM_HIP(launch_wide_tiles(A, match ? kWideFused : kWideFill, stream));
  if (timed) EPM_HIP(hipEventRecord(idx->ev_stop, stream));
  return EPM_OK;
}

struct MatchCall {
  const int64_t* row_offsets;
  const int32_t* col_indices;
  epm_dtype dtype;
  int32_t dim;
  const void *desc1, *desc2;
  const float *scale1, *scale2, *desc1_f32, *desc2_f32;
  float ratio;
  int32_t* best_idx;
  float *best_dist, *second_dist;
  epm_algo algo;
  int64_t capacity;  // < 0: trusted
  const float* qerr1 = nullptr;  // measured rounding errors of the reduced rows, or NULL
  const float* qerr2 = nullptr;
  // FP8 image-2 rows only (epm_query_match_fp8): the queries are their FP32
  // masters, and the image-2 rows' measured rounding errors are required
  bool f8_rows2_only = false;
};

epm_status validate_match(const epm_index* idx, const MatchCall& c) {
  if (!idx || !c.row_offsets) return EPM_ERR_ARG;
  if (!(c.ratio >= 0.0f) || !std::isfinite(c.ratio)) return EPM_ERR_ARG;
  const int64_t n1 = idx->N1;
  if (n1 > 0 && (!c.best_idx || !c.best_dist || !c.second_dist || !c.desc1)) return EPM_ERR_ARG;
  if (idx->N2 > 0 && !c.desc2) return EPM_ERR_ARG;
  if (c.algo != EPM_ALGO_AUTO && c.algo != EPM_ALGO_PLAIN && c.algo != EPM_ALGO_TILED)
    return EPM_ERR_ARG;
  switch (c.dtype) {
    case EPM_F32:
    case EPM_BF16:
    case EPM_FP8_E4M3:
      if (c.dim != 128) return EPM_ERR_ARG;
      break;
    case EPM_BIN256:
      if (c.dim != 256) return EPM_ERR_ARG;
      break;
    default:
      return EPM_ERR_ARG;
  }
  const bool reduced = c.dtype == EPM_BF16 || c.dtype == EPM_FP8_E4M3;
  if (reduced && n1 > 0 && (!c.desc1_f32 || (idx->N2 > 0 && !c.desc2_f32))) return EPM_ERR_ARG;
  if (c.dtype == EPM_FP8_E4M3 && n1 > 0 &&
      ((!c.scale1 && !c.f8_rows2_only) || (idx->N2 > 0 && !c.scale2)))
    return EPM_ERR_ARG;
  if (c.f8_rows2_only && (c.dtype != EPM_FP8_E4M3 || (n1 > 0 && idx->N2 > 0 && !c.qerr2)))
    return EPM_ERR_ARG;
  return EPM_OK;
}

MatchArgs match_args(epm_index* idx, const MatchCall& c) {
  const Layout& L = idx->L;
  MatchArgs A;
  A.qstart = idx->at<int64_t>(L.qstart);
  A.kstart = idx->at<int64_t>(L.kstart);
  A.num_pairs = idx->P;
  A.n1 = idx->N1;
  A.qperm = idx->have_qperm ? idx->qperm : nullptr;
  A.row_offsets = c.row_offsets;
  A.cols = c.col_indices;
  A.desc1 = c.desc1;
  A.desc2 = c.desc2;
  A.ratio = c.ratio;
  A.best_idx = c.best_idx;
  A.best_dist = c.best_dist;
  A.second_dist = c.second_dist;
  A.tiles = idx->at<StabTile>(L.stiles);
  A.num_tiles = (int)idx->stiles.size();
  A.windows = idx->at<TileWindow>(L.windows);
  A.rinv = idx->at<uint32_t>(L.rinv);
  A.rj = idx->at<int32_t>(L.rj);
  A.xcd_order = false;
  A.scale1 = c.scale1;
  A.scale2 = c.scale2;
  A.desc1_f32 = c.desc1_f32;
  A.desc2_f32 = c.desc2_f32;
  A.match_stats = idx->at<unsigned long long>(L.match_stats);
  A.capacity = c.capacity;
  A.order = nullptr;
  A.queue = nullptr;
  A.skip_tiles = nullptr;
  A.block_tile = nullptr;
  A.qerr1 = c.qerr1;
  A.qerr2 = c.qerr2;
  return A;
}

epm_status enqueue_match_kernels(epm_index* idx, const MatchCall& c, hipStream_t stream);

epm_status enqueue_match(epm_index* idx, const MatchCall& c, hipStream_t stream) {
  if (idx->N1 == 0) return EPM_OK;
  if (idx->ev_start) EPM_HIP(hipEventRecord(idx->ev_start, stream));
  const epm_status st = enqueue_match_kernels(idx, c, stream);
  if (st == EPM_OK && idx->ev_stop) EPM_HIP(hipEventRecord(idx->ev_stop, stream));
  return st;
}

epm_status enqueue_match_kernels(epm_index* idx, const MatchCall& c, hipStream_t stream) {
  const int64_t n1 = idx->N1;
  const Layout& L = idx->L;
  MatchArgs A = match_args(idx, c);
  // the window kernels walk the angle tiles and windows of the last query
  const bool tiled = c.algo != EPM_ALGO_PLAIN && idx->have_qperm;
  const int grid = idx->sched.match_workgroups;
  if (tiled && grid > 0) {
    uint32_t* sched = idx->at<uint32_t>(L.sched);
    A.queue = sched + kSchedMatchQueue;
    A.order = idx->have_order ? idx->at<uint32_t>(L.order) : nullptr;
  }
  if (tiled && grid == 0 && idx->have_block_tile) A.block_tile = idx->at<uint32_t>(L.block_tile);
  auto tiled_launch = [&](int fmt) -> hipError_t {
    if (grid > 0) {
      const hipError_t e = launch_fill_u32(A.queue, 1, 0u, stream);
      if (e != hipSuccess) return e;
    }
    return fmt < 0 ? launch_match_window_f32(A, grid, stream)
                   : launch_match_window_mfma(A, fmt, grid, stream);
  };
  const bool reduced = c.dtype == EPM_BF16 || c.dtype == EPM_FP8_E4M3;
  // FP32 and BF16 on angle tiles: the tiles the last query flagged for rows
  // longer than kStage are matched by the wide-row pass, the rest by the
  // window kernels
  const bool wide = tiled && (c.dtype == EPM_F32 || c.dtype == EPM_BF16);
  if (reduced || wide) {
    idx->have_match_stats = true;
    idx->match_from_tiles = false;
    idx->match_stream = stream;
    EPM_HIP(launch_clear_stats(nullptr, stream, nullptr, A.match_stats));
  }
  if (wide) A.skip_tiles = idx->at<uint32_t>(L.tile_wide);
  auto wide_launch = [&]() -> hipError_t {
    const bool bf = c.dtype == EPM_BF16;
    StabArgs W = stab_args(idx, nullptr, const_cast<int64_t*>(c.row_offsets),
                           const_cast<int32_t*>(c.col_indices),
                           c.capacity >= 0 ? c.capacity : INT64_MAX);
    W.qperm = idx->qperm;
    W.desc1 = bf ? c.desc1_f32 : static_cast<const float*>(c.desc1);
    W.desc2 = bf ? c.desc2_f32 : static_cast<const float*>(c.desc2);
    W.codes1 = bf ? static_cast<const uint16_t*>(c.desc1) : nullptr;
    W.codes2 = bf ? static_cast<const uint16_t*>(c.desc2) : nullptr;
    W.ratio = c.ratio;
    W.best_idx = c.best_idx;
    W.best_dist = c.best_dist;
    W.second_dist = c.second_dist;
    W.match_stats = A.match_stats;
    W.rest_count = A.match_stats + kMatchStatRest;
    W.block_tile = A.block_tile;
    if (!bf) {
      const hipError_t pe = prepare_wide_rows(idx, W, stream);
      if (pe != hipSuccess) return pe;
    }
    hipError_t e = launch_wide_tiles(W, bf ? kWideMatchBF16 : kWideMatchF32, stream);
    if (e != hipSuccess) return e;
    // the rows the pass could not certify or trust, exactly on the FP32 rows
    MatchArgs M = A;
    M.desc1 = W.desc1;
    M.desc2 = W.desc2;
    M.skip_tiles = nullptr;
    return launch_match_listed_f32(M, W.rest, W.rest_count, n1, stream);
  };
  if (reduced) {
    if (!tiled) {
      // no angle tiles to stage: exact FP32 evaluation on the masters
      A.desc1 = c.desc1_f32;
      A.desc2 = c.desc2_f32;
      EPM_HIP(launch_match_plain_f32(A, stream));
      return EPM_OK;
    }
    EPM_HIP(tiled_launch(c.dtype == EPM_BF16 ? 0 : 1));
    if (wide) EPM_HIP(wide_launch());
    return EPM_OK;
  }
  switch (c.dtype) {
    case EPM_F32:
      if (!tiled) {
        EPM_HIP(launch_match_plain_f32(A, stream));
        return EPM_OK;
      }
      EPM_HIP(tiled_launch(-1));
      EPM_HIP(wide_launch());
      return EPM_OK;
    case EPM_BIN256:
      // 32-byte rows: per-candidate gathers are already line-efficient
      EPM_HIP(launch_match_plain_bin256(A, stream));
      return EPM_OK;
    default:
      return EPM_ERR_UNSUPPORTED;
  }
}

// Stabbing with fused FP32 selection, then the CSR fill with the wide-row
// selection, and the listed-query match of the rows the two passes left.
// nnz_host as in epm_query_candidates.
epm_status enqueue_query_match(epm_index* idx, StabArgs& A, int64_t* row_offsets,
                               int64_t* nnz_host, const MatchCall& c, hipStream_t stream,
                               hipEvent_t records_ready = nullptr) {
  const int64_t n1 = idx->N1;
  const bool bf = c.dtype == EPM_BF16;
  const bool f8 = c.dtype == EPM_FP8_E4M3 && c.f8_rows2_only;
  if (!bf && !f8 && c.dtype != EPM_F32) return EPM_ERR_UNSUPPORTED;
  // BF16 / FP8: the codes feed the bounds, the FP32 masters every exact
  // distance (and the wide-row pass, which rounds them to BF16 on chip itself)
  A.desc1 = static_cast<const float*>(bf || f8 ? c.desc1_f32 : c.desc1);
  A.desc2 = static_cast<const float*>(bf || f8 ? c.desc2_f32 : c.desc2);
  A.codes1 = bf ? static_cast<const uint16_t*>(c.desc1) : nullptr;
  A.codes2 = bf ? static_cast<const uint16_t*>(c.desc2) : nullptr;
  A.f8codes2 = f8 ? static_cast<const uint8_t*>(c.desc2) : nullptr;
  A.f8scale2 = f8 ? c.scale2 : nullptr;
  A.f8err2 = f8 ? c.qerr2 : nullptr;
  A.ratio = c.ratio;
  A.best_idx = c.best_idx;
  A.best_dist = c.best_dist;
  A.second_dist = c.second_dist;
  A.qrec = idx->at<uint4>(idx->L.qrec);
  // counters of the wide-row selection (certified / listed rows)
  A.match_stats = idx->at<unsigned long long>(idx->L.match_stats);  // cleared with the counters
  idx->have_match_stats = true;
  idx->match_from_tiles = true;
  idx->match_stream = stream;
  const epm_status st =
      enqueue_count(idx, A, row_offsets, stream, bf ? kStabBF16 : f8 ? kStabFP8 : kStabF32,
                    records_ready);
  if (st != EPM_OK) return st;
  if (n1 == 0) return EPM_OK;
  idx->last_stream = stream;
  idx->last_offsets = row_offsets;
  idx->have_stats = true;
  if (nnz_host) {
    int64_t nnz = 0;
    EPM_HIP(hipMemcpyAsync(&nnz, row_offsets + n1, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    EPM_HIP(hipStreamSynchronize(stream));
    *nnz_host = nnz;
    if (nnz > A.capacity) return EPM_ERR_CAPACITY;
  }
  const epm_status fs = enqueue_fill(idx, A, stream, true);
  if (fs != EPM_OK) return fs;
  MatchArgs M = match_args(idx, c);
  M.desc1 = A.desc1;  // FP32 rows (the masters for BF16)
  M.desc2 = A.desc2;
  EPM_HIP(launch_match_listed_f32(M, A.rest, A.stats + kStatRest, n1, stream));
  return EPM_OK;
}

}  // namespace

// ------------------------------------------------ allocation-free variant
// epm_query_match_noalloc keeps the whole index in this file-scope device
// array instead of a caller workspace.  Host code never passes the array's
// name to a kernel or a copy: on every device the library runs on, the first
// call (with that device current) looks its address up once with
// hipGetSymbolAddress and every later use goes through that pointer.
static __device__ __align__(256) unsigned char scratch[EPM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocMaxDevices = 64;

// Per-device state of the allocation-free variant.  The host image of the
// index tables is uploaded asynchronously, so it must stay untouched until
// the copy has run: two host images alternate, each with an event recorded
// after its upload, and a call waits for that event only before reusing an
// image (that is, when the host runs two calls ahead of the stream).
struct NoAllocDevice {
  bool ready = false;
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  std::vector<char> head[2];
  hipEvent_t uploaded[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int next = 0;
};

std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

// Host images of the per-call tables of epm_eps_features, epm_pose_eps and
// epm_gms.  Each upload keeps its image in a slot of a ring (one per device)
// until an event after the copy has completed, so those calls return without
// waiting for their stream; a call waits only when the slot it takes still
// holds an upload that has not run (more than kSlots calls in flight).
struct UploadRing {
  static constexpr int kSlots = 8;
  std::vector<char> img[kSlots];
  hipEvent_t done[kSlots] = {};
  bool pending[kSlots] = {};
  int next = 0;
};

std::mutex g_upload_mu;
UploadRing g_upload[kNoAllocMaxDevices];

// Copies `head` (taken over) to device address dst on `stream`, which must
// belong to the current device.
epm_status upload_table(std::vector<char>& head, void* dst, hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return EPM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_upload_mu);
  UploadRing& R = g_upload[dev];
  const int s = R.next;
  R.next = (s + 1) % UploadRing::kSlots;
  if (!R.done[s] && hipEventCreateWithFlags(&R.done[s], hipEventDisableTiming) != hipSuccess)
    return EPM_ERR_HIP;
  if (R.pending[s]) {
    if (hipEventSynchronize(R.done[s]) != hipSuccess) return EPM_ERR_HIP;
    R.pending[s] = false;
  }
  std::swap(R.img[s], head);
  if (hipMemcpyAsync(dst, R.img[s].data(), R.img[s].size(), hipMemcpyHostToDevice, stream) !=
      hipSuccess)
    return EPM_ERR_HIP;
  if (hipEventRecord(R.done[s], stream) != hipSuccess) return EPM_ERR_HIP;
  R.pending[s] = true;
  return EPM_OK;
}

// Set-up on the current device: the array's address and the two events.
epm_status noalloc_setup(NoAllocDevice& d) {
  if (d.ready) return EPM_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EPM_ERR_HIP;
  for (int k = 0; k < 2; ++k)
    if (!d.uploaded[k] &&
        hipEventCreateWithFlags(&d.uploaded[k], hipEventDisableTiming) != hipSuccess)
      return EPM_ERR_HIP;
  d.ptr = static_cast<unsigned char*>(p);
  d.ready = true;
  return EPM_OK;
}

}  // namespace

// A recorded pipeline: the index it runs on and the instantiated graph.
struct epm_batch {
  epm_index* idx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t* row_offsets = nullptr;
  int64_t capacity = 0;
  ~epm_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    delete idx;
  }
};

extern "C" {

size_t epm_workspace_bytes(const epm_pair* pairs, int32_t num_pairs) {
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2)) return 0;
  int64_t tr = 0, tq = 0, ts = 0;
  for (int p = 0; p < num_pairs; ++p) {
    tr += tiles_of(pairs[p].n);
    tq += tiles_of(pairs[p].m);
    ts += stab_tiles_of(pairs[p].m);
  }
  return make_layout(num_pairs, n1, n2, tr, tq, ts).total;
}

epm_status epm_build_intervals(const epm_pair* pairs, int32_t num_pairs, const float* kp2_xy,
                               const float* eps2, float eps_scalar, void* workspace,
                               size_t workspace_bytes, epm_index** out, hipStream_t stream) {
  if (!out) return EPM_ERR_ARG;
  *out = nullptr;
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2)) return EPM_ERR_ARG;
  if (!build_args_ok(n2, kp2_xy, eps2, eps_scalar)) return EPM_ERR_ARG;
  epm_index* idx = nullptr;
  const epm_status st = index_prepare(pairs, num_pairs, workspace, workspace_bytes, &idx);
  if (st != EPM_OK) return st;
  epm_status r = index_upload(idx, stream);
  if (r == EPM_OK) r = enqueue_build(idx, kp2_xy, eps2, eps_scalar, stream);
  if (r != EPM_OK) {
    delete idx;
    return r;
  }
  *out = idx;
  return EPM_OK;
}

epm_status epm_index_set_timing_events(epm_index* idx, hipEvent_t start, hipEvent_t stop) {
  if (!idx || (start == nullptr) != (stop == nullptr)) return EPM_ERR_ARG;
  idx->ev_start = start;
  idx->ev_stop = stop;
  return EPM_OK;
}

epm_status epm_index_set_timing_kernel(epm_index* idx, epm_timed_kernel kernel) {
  if (!idx || (kernel != EPM_TIMED_STAB && kernel != EPM_TIMED_WIDE)) return EPM_ERR_ARG;
  idx->timed = kernel;
  return EPM_OK;
}

epm_status epm_index_set_sched(epm_index* idx, const epm_sched* sched) {
  if (!idx || !sched) return EPM_ERR_ARG;
  if (sched->stab_workgroups < 0 || sched->match_workgroups < 0) return EPM_ERR_ARG;
  if (sched->lpt != 0 && sched->lpt != 1) return EPM_ERR_ARG;
  const int ch = sched->stab_chunk;
  if (ch != 0 && ch != 256 && ch != 512 && ch != 1024) return EPM_ERR_ARG;
  for (int k = 0; k < 4; ++k)
    if (sched->reserved[k] != 0) return EPM_ERR_ARG;
  idx->sched = *sched;
  return EPM_OK;
}

epm_status epm_query_candidates(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                                int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                                hipStream_t stream) {
  if (!idx || !row_offsets || capacity < 0) return EPM_ERR_ARG;
  if (idx->N1 > 0 && !kp1_xy) return EPM_ERR_ARG;
  if (capacity > 0 && !col_indices) return EPM_ERR_ARG;
  const int64_t n1 = idx->N1;
  StabArgs A = stab_args(idx, kp1_xy, row_offsets, col_indices, capacity);
  const epm_status st = enqueue_count(idx, A, row_offsets, stream);
  if (st != EPM_OK) return st;
  if (n1 > 0) {
    idx->last_stream = stream;
    idx->last_offsets = row_offsets;
    idx->have_stats = true;
  }
  if (nnz_host) {
    int64_t nnz = 0;
    EPM_HIP(hipMemcpyAsync(&nnz, row_offsets + n1, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    EPM_HIP(hipStreamSynchronize(stream));
    *nnz_host = nnz;
    if (nnz > capacity) return EPM_ERR_CAPACITY;
  }
  return enqueue_fill(idx, A, stream);
}

epm_status epm_match(const epm_index* idx, const int64_t* row_offsets,
                     const int32_t* col_indices, epm_dtype dtype, int32_t dim,
                     const void* desc1, const void* desc2, const float* scale1,
                     const float* scale2, const float* desc1_f32, const float* desc2_f32,
                     float ratio, int32_t* best_idx, float* best_dist, float* second_dist,
                     const epm_match_opts* opts, hipStream_t stream) {
  MatchCall c;
  c.row_offsets = row_offsets;
  c.col_indices = col_indices;
  c.dtype = dtype;
  c.dim = dim;
  c.desc1 = desc1;
  c.desc2 = desc2;
  c.scale1 = scale1;
  c.scale2 = scale2;
  c.desc1_f32 = desc1_f32;
  c.desc2_f32 = desc2_f32;
  c.ratio = ratio;
  c.best_idx = best_idx;
  c.best_dist = best_dist;
  c.second_dist = second_dist;
  c.algo = opts ? opts->algo : EPM_ALGO_AUTO;
  c.capacity = -1;
  if (opts) {
    if (opts->check_capacity != 0 && opts->check_capacity != 1) return EPM_ERR_ARG;
    for (int k = 0; k < 4; ++k)
      if (opts->reserved[k] != 0) return EPM_ERR_ARG;
    if (opts->check_capacity) {
      if (opts->col_capacity < 0) return EPM_ERR_ARG;
      c.capacity = opts->col_capacity;
    }
    if ((opts->qerr1 == nullptr) != (opts->qerr2 == nullptr)) return EPM_ERR_ARG;
    c.qerr1 = opts->qerr1;
    c.qerr2 = opts->qerr2;
  }
  const epm_status v = validate_match(idx, c);
  if (v != EPM_OK) return v;
  return enqueue_match(const_cast<epm_index*>(idx), c, stream);
}

epm_status epm_query_match(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                           int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                           const float* desc1, const float* desc2, float ratio,
                           int32_t* best_idx, float* best_dist, float* second_dist,
                           hipStream_t stream) {
  if (!idx || !row_offsets || capacity < 0) return EPM_ERR_ARG;
  if (idx->N1 > 0 && !kp1_xy) return EPM_ERR_ARG;
  if (capacity > 0 && !col_indices) return EPM_ERR_ARG;
  MatchCall c;
  c.row_offsets = row_offsets;
  c.col_indices = col_indices;
  c.dtype = EPM_F32;
  c.dim = 128;
  c.desc1 = desc1;
  c.desc2 = desc2;
  c.scale1 = c.scale2 = c.desc1_f32 = c.desc2_f32 = nullptr;
  c.ratio = ratio;
  c.best_idx = best_idx;
  c.best_dist = best_dist;
  c.second_dist = second_dist;
  c.algo = EPM_ALGO_TILED;
  // without a host check the leftover rows must not read past the buffer
  c.capacity = nnz_host ? -1 : capacity;
  const epm_status v = validate_match(idx, c);
  if (v != EPM_OK) return v;
  StabArgs A = stab_args(idx, kp1_xy, row_offsets, col_indices, capacity);
  return enqueue_query_match(idx, A, row_offsets, nnz_host, c, stream);
}

epm_status epm_query_match_bf16(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                                int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                                const uint16_t* desc1, const uint16_t* desc2,
                                const float* desc1_f32, const float* desc2_f32, float ratio,
                                int32_t* best_idx, float* best_dist, float* second_dist,
                                hipStream_t stream) {
  if (!idx || !row_offsets || capacity < 0) return EPM_ERR_ARG;
  if (idx->N1 > 0 && !kp1_xy) return EPM_ERR_ARG;
  if (capacity > 0 && !col_indices) return EPM_ERR_ARG;
  MatchCall c;
  c.row_offsets = row_offsets;
  c.col_indices = col_indices;
  c.dtype = EPM_BF16;
  c.dim = 128;
  c.desc1 = desc1;
  c.desc2 = desc2;
  c.scale1 = c.scale2 = nullptr;
  c.desc1_f32 = desc1_f32;
  c.desc2_f32 = desc2_f32;
  c.ratio = ratio;
  c.best_idx = best_idx;
  c.best_dist = best_dist;
  c.second_dist = second_dist;
  c.algo = EPM_ALGO_TILED;
  c.capacity = nnz_host ? -1 : capacity;
  const epm_status v = validate_match(idx, c);
  if (v != EPM_OK) return v;
  StabArgs A = stab_args(idx, kp1_xy, row_offsets, col_indices, capacity);
  return enqueue_query_match(idx, A, row_offsets, nnz_host, c, stream);
}

epm_status epm_query_match_fp8(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                               int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                               const uint8_t* desc2, const float* scale2, const float* err2,
                               const float* desc1_f32, const float* desc2_f32, float ratio,
                               int32_t* best_idx, float* best_dist, float* second_dist,
                               hipStream_t stream) {
  if (!idx || !row_offsets || capacity < 0) return EPM_ERR_ARG;
  if (idx->N1 > 0 && !kp1_xy) return EPM_ERR_ARG;
  if (capacity > 0 && !col_indices) return EPM_ERR_ARG;
  MatchCall c;
  c.row_offsets = row_offsets;
  c.col_indices = col_indices;
  c.dtype = EPM_FP8_E4M3;
  c.dim = 128;
  c.desc1 = desc1_f32;
  c.desc2 = desc2;
  c.scale1 = nullptr;
  c.scale2 = scale2;
  c.desc1_f32 = desc1_f32;
  c.desc2_f32 = desc2_f32;
  c.qerr2 = err2;
  c.f8_rows2_only = true;
  c.ratio = ratio;
  c.best_idx = best_idx;
  c.best_dist = best_dist;
  c.second_dist = second_dist;
  c.algo = EPM_ALGO_TILED;
  c.capacity = nnz_host ? -1 : capacity;
  const epm_status v = validate_match(idx, c);
  if (v != EPM_OK) return v;
  StabArgs A = stab_args(idx, kp1_xy, row_offsets, col_indices, capacity);
  return enqueue_query_match(idx, A, row_offsets, nnz_host, c, stream);
}

epm_status epm_query_match_noalloc(const epm_pair* pairs, int32_t num_pairs, const float* kp1_xy,
                                   const float* kp2_xy, const float* eps2, float eps_scalar,
                                   int64_t* row_offsets, int32_t* col_indices, int64_t capacity,
                                   int64_t* nnz_host, const float* desc1, const float* desc2,
                                   float ratio, int32_t* best_idx, float* best_dist,
                                   float* second_dist, hipStream_t stream) {
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2)) return EPM_ERR_ARG;
  if (!build_args_ok(n2, kp2_xy, eps2, eps_scalar)) return EPM_ERR_ARG;
  if (!row_offsets || capacity < 0 || (n1 > 0 && !kp1_xy)) return EPM_ERR_ARG;
  if (capacity > 0 && !col_indices) return EPM_ERR_ARG;
  {
    // the size limit is a host check: nothing runs when it fails
    int64_t tr = 0, tq = 0, ts = 0;
    for (int p = 0; p < num_pairs; ++p) {
      tr += tiles_of(pairs[p].n);
      tq += tiles_of(pairs[p].m);
      ts += stab_tiles_of(pairs[p].m);
    }
    if (make_layout(num_pairs, n1, n2, tr, tq, ts).total > (size_t)EPM_NOALLOC_SCRATCH_BYTES)
      return EPM_ERR_WORKSPACE;
  }
  MatchCall c;
  c.row_offsets = row_offsets;
  c.col_indices = col_indices;
  c.dtype = EPM_F32;
  c.dim = 128;
  c.desc1 = desc1;
  c.desc2 = desc2;
  c.scale1 = c.scale2 = c.desc1_f32 = c.desc2_f32 = nullptr;
  c.ratio = ratio;
  c.best_idx = best_idx;
  c.best_dist = best_dist;
  c.second_dist = second_dist;
  c.algo = EPM_ALGO_TILED;
  c.capacity = nnz_host ? -1 : capacity;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return EPM_ERR_HIP;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return EPM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& D = g_noalloc[dev];
  epm_status st = noalloc_setup(D);
  if (st != EPM_OK) return st;
  epm_index* idx = nullptr;
  st = index_prepare(pairs, num_pairs, D.ptr, (size_t)EPM_NOALLOC_SCRATCH_BYTES, &idx);
  if (st != EPM_OK) return st;
  st = validate_match(idx, c);
  if (st == EPM_OK) {
    // the table image goes up from one of the two host images
    const int slot = D.next;
    D.next ^= 1;
    if (D.pending[slot] && hipEventSynchronize(D.uploaded[slot]) != hipSuccess) st = EPM_ERR_HIP;
    if (st == EPM_OK) {
      std::swap(D.head[slot], idx->head);
      if (hipMemcpyAsync(D.ptr, D.head[slot].data(), idx->L.head_end, hipMemcpyHostToDevice,
                         stream) != hipSuccess ||
          hipEventRecord(D.uploaded[slot], stream) != hipSuccess ||
          expand_tiles(idx, stream) != hipSuccess)
        st = EPM_ERR_HIP;
      D.pending[slot] = true;
    }
  }
  if (st == EPM_OK) st = enqueue_build(idx, kp2_xy, eps2, eps_scalar, stream);
  if (st == EPM_OK) {
    StabArgs A = stab_args(idx, kp1_xy, row_offsets, col_indices, capacity);
    st = enqueue_query_match(idx, A, row_offsets, nnz_host, c, stream);
  }
  delete idx;
  return st;
}

epm_status epm_batch_create(const epm_pair* pairs, int32_t num_pairs, const epm_batch_desc* d,
                            void* workspace, size_t workspace_bytes, epm_batch** out,
                            hipStream_t stream) {
  if (!out) return EPM_ERR_ARG;
  *out = nullptr;
  if (!d) return EPM_ERR_ARG;
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2)) return EPM_ERR_ARG;
  if (!build_args_ok(n2, d->kp2_xy, d->eps2, d->eps_scalar)) return EPM_ERR_ARG;
  if (!d->row_offsets || d->capacity < 0 || (n1 > 0 && !d->kp1_xy)) return EPM_ERR_ARG;
  if (d->capacity > 0 && !d->col_indices) return EPM_ERR_ARG;
  epm_batch* b = new (std::nothrow) epm_batch();
  if (!b) return EPM_ERR_ARG;
  epm_status st = index_prepare(pairs, num_pairs, workspace, workspace_bytes, &b->idx);
  if (st != EPM_OK) {
    delete b;
    return st;
  }
  epm_index* idx = b->idx;
  st = epm_index_set_sched(idx, &d->sched);
  MatchCall c;
  c.row_offsets = d->row_offsets;
  c.col_indices = d->col_indices;
  c.dtype = d->dtype;
  c.dim = d->dim;
  c.desc1 = d->desc1;
  c.desc2 = d->desc2;
  c.scale1 = d->scale1;
  c.scale2 = d->scale2;
  c.desc1_f32 = d->desc1_f32;
  c.desc2_f32 = d->desc2_f32;
  c.ratio = d->ratio;
  c.best_idx = d->best_idx;
  c.best_dist = d->best_dist;
  c.second_dist = d->second_dist;
  c.algo = d->algo;
  c.capacity = d->capacity;
  // FP8 with the rows' error bounds: the fused FP8 pass (queries as masters)
  if (d->dtype == EPM_FP8_E4M3 && d->err2 && d->algo != EPM_ALGO_PLAIN) {
    c.f8_rows2_only = true;
    c.qerr2 = d->err2;
    c.desc1 = d->desc1_f32;
    c.scale1 = nullptr;
  }
  if (st == EPM_OK) st = validate_match(idx, c);
  if (st == EPM_OK) st = index_upload(idx, stream);
  if (st != EPM_OK) {
    delete b;
    return st;
  }
  b->row_offsets = d->row_offsets;
  b->capacity = d->capacity;

  // record on private streams, kernels only: the record build forks onto a
  // second stream beside the query keys and their sort, and joins before the
  // tile windows (two branches of the graph)
  hipStream_t cs = nullptr, cs2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  st = EPM_OK;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)
    st = EPM_ERR_HIP;
  if (st == EPM_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
    st = EPM_ERR_HIP;
  if (st == EPM_OK) {
    epm_status r = EPM_OK;
    // the pair setup on the device from F_dev heads the graph: both branches read it
    if (d->F_dev &&
        launch_pair_setup(idx->at<PairDev>(idx->L.pairs), d->F_dev, idx->P, cs) != hipSuccess)
      r = EPM_ERR_HIP;
    if (r == EPM_OK &&
        (hipEventRecord(fork, cs) != hipSuccess || hipStreamWaitEvent(cs2, fork, 0) != hipSuccess))
      r = EPM_ERR_HIP;
    if (r == EPM_OK) r = enqueue_build(idx, d->kp2_xy, d->eps2, d->eps_scalar, cs2);
    if (r == EPM_OK && hipEventRecord(join, cs2) != hipSuccess) r = EPM_ERR_HIP;
    // after the build: the stab arguments name the sorted key buffer it chose
    StabArgs A = stab_args(idx, d->kp1_xy, d->row_offsets, d->col_indices, d->capacity);
    // FP32, BF16 and FP8 with error bounds on the tiled path: selection fused
    // into the stabbing pass
    const bool fused = (c.dtype == EPM_F32 || c.dtype == EPM_BF16 || c.f8_rows2_only) &&
                       c.algo != EPM_ALGO_PLAIN;
    if (fused) {
      if (r == EPM_OK) r = enqueue_query_match(idx, A, d->row_offsets, nullptr, c, cs, join);
    } else {
      if (r == EPM_OK) r = enqueue_count(idx, A, d->row_offsets, cs, kStabCount, join);
      if (r == EPM_OK) r = enqueue_fill(idx, A, cs);
      if (r == EPM_OK) r = enqueue_match(idx, c, cs);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    b->graph = g;
    if (r != EPM_OK) st = r;
    else if (e != hipSuccess || !g) st = EPM_ERR_HIP;
  }
  if (st == EPM_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
    st = EPM_ERR_HIP;
  if (join) (void)hipEventDestroy(join);
  if (fork) (void)hipEventDestroy(fork);
  if (cs2) (void)hipStreamDestroy(cs2);
  if (cs) (void)hipStreamDestroy(cs);
  if (st != EPM_OK) {
    delete b;
    return st;
  }
  idx->have_stats = idx->N1 > 0;
  idx->last_offsets = d->row_offsets;
  idx->last_stream = stream;
  idx->match_stream = stream;
  *out = b;
  return EPM_OK;
}

epm_status epm_batch_launch(epm_batch* b, hipStream_t stream) {
  if (!b || !b->exec) return EPM_ERR_ARG;
  EPM_HIP(hipGraphLaunch(b->exec, stream));
  b->idx->last_stream = stream;
  b->idx->match_stream = stream;
  return EPM_OK;
}

epm_status epm_batch_nnz(epm_batch* b, int64_t* nnz, hipStream_t stream) {
  if (!b || !nnz) return EPM_ERR_ARG;
  int64_t v = 0;
  EPM_HIP(hipMemcpyAsync(&v, b->row_offsets + b->idx->N1, sizeof(int64_t), hipMemcpyDeviceToHost,
                         stream));
  EPM_HIP(hipStreamSynchronize(stream));
  *nnz = v;
  return v > b->capacity ? EPM_ERR_CAPACITY : EPM_OK;
}

const epm_index* epm_batch_index(const epm_batch* b) { return b ? b->idx : nullptr; }

void epm_batch_destroy(epm_batch* b) { delete b; }

size_t epm_eps_workspace_bytes(int32_t num_pairs) {
  if (num_pairs < 0) return 0;
  return align_up(sizeof(EpsPair) * (size_t)num_pairs) +
         align_up(sizeof(int64_t) * ((size_t)num_pairs + 1)) +
         align_up(sizeof(float) * (size_t)kEpsGradMaxBlocks * (kEpsParams + 1));
}

epm_status epm_eps_features(const epm_pair* pairs, int32_t num_pairs, const float* kp2_xy,
                            const float* attrs, float* features, void* workspace,
                            size_t workspace_bytes, hipStream_t stream) {
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2)) return EPM_ERR_ARG;
  if (n2 > 0 && (!kp2_xy || !attrs || !features)) return EPM_ERR_ARG;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) ||
      workspace_bytes < epm_eps_workspace_bytes(num_pairs))
    return EPM_ERR_WORKSPACE;
  // head: per-pair constants, then the image-2 slice starts
  const size_t off_k = align_up(sizeof(EpsPair) * (size_t)num_pairs);
  std::vector<char> head(off_k + sizeof(int64_t) * ((size_t)num_pairs + 1), 0);
  EpsPair* ep = reinterpret_cast<EpsPair*>(head.data());
  int64_t* ks = reinterpret_cast<int64_t*>(head.data() + off_k);
  for (int p = 0; p < num_pairs; ++p) {
    PairDev pd;
    const epm_status st = setup_pair(pairs[p], pd);
    if (st != EPM_OK) return st;
    // e is the epipole in normalised image-2 coordinates p^ = s (p - c)
    const double ew = pd.e[2];
    EpsPair& E = ep[p];
    E.w = pairs[p].w2;
    E.h = pairs[p].h2;
    E.diag = std::hypot(E.w, E.h);
    E.finite = 0;
    if (ew != 0.0) {
      E.ex = pd.e[0] / (pd.s * ew) + pd.cx;
      E.ey = pd.e[1] / (pd.s * ew) + pd.cy;
      E.finite = std::isfinite(E.ex) && std::isfinite(E.ey) ? 1 : 0;
    }
    ks[p] = pairs[p].k_begin;
  }
  ks[num_pairs] = n2;
  if (n2 == 0) return EPM_OK;
  char* ws = static_cast<char*>(workspace);
  const epm_status up = upload_table(head, ws, stream);
  if (up != EPM_OK) return up;
  EPM_HIP(launch_eps_features(reinterpret_cast<const EpsPair*>(ws),
                              reinterpret_cast<const int64_t*>(ws + off_k), num_pairs, n2, kp2_xy,
                              attrs, features, stream));
  return EPM_OK;
}

namespace {

void mat3_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

void skew3(const double* v, double* S) {
  S[0] = 0.0;   S[1] = -v[2]; S[2] = v[1];
  S[3] = v[2];  S[4] = 0.0;   S[5] = -v[0];
  S[6] = -v[1]; S[7] = v[0];  S[8] = 0.0;
}

bool inv3(const double* M, double* I) {
  const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                     M[2] * (M[3] * M[7] - M[4] * M[6]);
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  I[0] = (M[4] * M[8] - M[5] * M[7]) / det;
  I[1] = (M[2] * M[7] - M[1] * M[8]) / det;
  I[2] = (M[1] * M[5] - M[2] * M[4]) / det;
  I[3] = (M[5] * M[6] - M[3] * M[8]) / det;
  I[4] = (M[0] * M[8] - M[2] * M[6]) / det;
  I[5] = (M[2] * M[3] - M[0] * M[5]) / det;
  I[6] = (M[3] * M[7] - M[4] * M[6]) / det;
  I[7] = (M[1] * M[6] - M[0] * M[7]) / det;
  I[8] = (M[0] * M[4] - M[1] * M[3]) / det;
  return true;
}

// F = K2^-T [t]x R K1^-1 (Eq. 1) and its derivatives with respect to the
// rotation vector w (R = Exp([w]x) R0: dR/dw_k = [e_k]x R0) and to t.
bool pose_pair(const epm_pose_prior& pr, PosePair& P) {
  double K1i[9], K2i[9], K2iT[9];
  if (!inv3(pr.K1, K1i) || !inv3(pr.K2, K2i)) return false;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) K2iT[3 * r + c] = K2i[3 * c + r];
  double Tx[9], RK[9], T1[9];
  skew3(pr.t, Tx);
  mat3_mul(pr.R, K1i, RK);  // R K1^-1
  mat3_mul(K2iT, Tx, T1);   // K2^-T [t]x
  mat3_mul(T1, RK, P.F0);
  for (int k = 0; k < 3; ++k) {
    double e[3] = {0.0, 0.0, 0.0}, Ek[9], A[9], B[9];
    e[k] = 1.0;
    skew3(e, Ek);
    // rotation: K2^-T [t]x [e_k]x R K1^-1
    mat3_mul(T1, Ek, A);
    mat3_mul(A, RK, P.dF[k]);
    // translation: K2^-T [e_k]x R K1^-1
    mat3_mul(K2iT, Ek, B);
    mat3_mul(B, RK, P.dF[3 + k]);
  }
  for (int k = 0; k < 36; ++k) {
    if (!std::isfinite(pr.cov[k])) return false;
    P.cov[k] = pr.cov[k];
  }
  P.w1 = pr.w1;
  P.h1 = pr.h1;
  for (int k = 0; k < 9; ++k) {
    P.K1[k] = pr.K1[k];
    P.K2i[k] = K2i[k];
    P.Rt[k] = pr.R[3 * (k % 3) + k / 3];
  }
  for (int k = 0; k < 3; ++k) P.t[k] = pr.t[k];
  P.rho_lo = P.rho_hi = 0.0;
  if (pr.zmin > 0.0) {
    P.rho_hi = 1.0 / pr.zmin;
    P.rho_lo = std::isinf(pr.zmax) ? 0.0 : 1.0 / pr.zmax;
  }
  P.fmax = 0.0;
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(P.F0[k])) return false;
    P.fmax = std::fmax(P.fmax, std::fabs(P.F0[k]));
  }
  return P.fmax > 0.0;
}

}  // namespace

size_t epm_pose_eps_workspace_bytes(int32_t num_pairs) {
  if (num_pairs < 0) return 0;
  return align_up(sizeof(PosePair) * (size_t)num_pairs) +
         align_up(sizeof(int64_t) * ((size_t)num_pairs + 1));
}

epm_status epm_pose_eps(const epm_pair* pairs, const epm_pose_prior* priors, int32_t num_pairs,
                        const float* kp2_xy, float eps0, float k_sigma, float eps_max,
                        float* eps2, void* workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  int64_t n1, n2;
  if (!validate_pairs(pairs, num_pairs, &n1, &n2) || !priors) return EPM_ERR_ARG;
  if (n2 > 0 && (!kp2_xy || !eps2)) return EPM_ERR_ARG;
  if (!(eps0 >= 0.0f) || !(k_sigma >= 0.0f) || !(eps_max >= eps0) || !std::isfinite(eps_max))
    return EPM_ERR_ARG;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) ||
      workspace_bytes < epm_pose_eps_workspace_bytes(num_pairs))
    return EPM_ERR_WORKSPACE;
  const size_t off_k = align_up(sizeof(PosePair) * (size_t)num_pairs);
  std::vector<char> head(off_k + sizeof(int64_t) * ((size_t)num_pairs + 1), 0);
  PosePair* pp = reinterpret_cast<PosePair*>(head.data());
  int64_t* ks = reinterpret_cast<int64_t*>(head.data() + off_k);
  for (int p = 0; p < num_pairs; ++p) {
    if (priors[p].w1 <= 0 || priors[p].h1 <= 0) return EPM_ERR_ARG;
    const double zmin = priors[p].zmin, zmax = priors[p].zmax;
    if (!(zmin == 0.0 || (zmin > 0.0 && std::isfinite(zmin) && zmax > zmin)))
      return EPM_ERR_ARG;
    if (!pose_pair(priors[p], pp[p])) return EPM_ERR_DEGENERATE_F;
    ks[p] = pairs[p].k_begin;
  }
  ks[num_pairs] = n2;
  if (n2 == 0) return EPM_OK;
  char* ws = static_cast<char*>(workspace);
  const epm_status up = upload_table(head, ws, stream);
  if (up != EPM_OK) return up;
  EPM_HIP(launch_pose_eps(reinterpret_cast<const PosePair*>(ws),
                          reinterpret_cast<const int64_t*>(ws + off_k), num_pairs, n2, kp2_xy,
                          eps0, k_sigma, eps_max, eps2, stream));
  return EPM_OK;
}

epm_status epm_eps_infer(const float* features, int64_t n, const float* params, float* eps2,
                         hipStream_t stream) {
  if (n < 0) return EPM_ERR_ARG;
  if (n == 0) return EPM_OK;
  if (!features || !params || !eps2) return EPM_ERR_ARG;
  EPM_HIP(launch_eps_infer(features, n, params, eps2, stream));
  return EPM_OK;
}

epm_status epm_eps_grad(const float* features, int64_t num_rows, const int64_t* feat_index,
                        const float* target, int64_t num_slots, const int32_t* sample_idx,
                        int32_t batch, float q, const float* params, float* grad, float* loss,
                        void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!features || !target || !sample_idx || !params || !grad || batch < 1) return EPM_ERR_ARG;
  if (num_rows < 1 || num_slots < 1) return EPM_ERR_ARG;
  if (!(q > 0.0f && q < 1.0f)) return EPM_ERR_ARG;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) ||
      workspace_bytes < epm_eps_workspace_bytes(0))
    return EPM_ERR_WORKSPACE;
  EpsGradArgs a;
  a.features = features;
  a.num_rows = num_rows;
  a.feat_index = feat_index;
  a.target = target;
  a.num_slots = num_slots;
  a.sample_idx = sample_idx;
  a.batch = batch;
  a.q = q;
  a.inv_batch = 1.0f / (float)batch;
  a.params = params;
  a.partials = static_cast<float*>(workspace);
  EPM_HIP(launch_eps_grad(a, grad, loss, stream));
  return EPM_OK;
}

epm_status epm_eps_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                        float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  if (!params || !m || !v || !grad || step < 1) return EPM_ERR_ARG;
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps >= 0.0f))
    return EPM_ERR_ARG;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  EPM_HIP(launch_eps_adam(params, m, v, grad, lr, beta1, beta2, eps, c1, c2, stream));
  return EPM_OK;
}

namespace {

struct GmsLayout {
  size_t pairs, count, cursor, offsets, partials, key, rcell, list, total;
};

GmsLayout gms_layout(const epm_index* idx, int32_t grid) {
  GmsLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes > 0 ? bytes : 1);
    return o;
  };
  const size_t cells = (size_t)idx->P * (size_t)grid * (size_t)grid;
  const size_t n1 = (size_t)idx->N1;
  L.pairs = take(sizeof(GmsPair) * (size_t)idx->P);
  L.count = take(4 * cells);
  L.cursor = take(4 * cells);
  L.offsets = take(8 * (cells + 1));
  L.partials = take(8 * (size_t)scan_partials_count((int64_t)cells));
  L.key = take(4 * n1);
  L.rcell = take(4 * n1);
  L.list = take(4 * n1);
  L.total = off;
  return L;
}

}  // namespace

size_t epm_gms_workspace_bytes(const epm_index* idx, int32_t grid) {
  if (!idx || grid < 1 || grid > kGmsMaxGrid) return 0;
  return gms_layout(idx, grid).total;
}

epm_status epm_gms(const epm_index* idx, const int32_t* size1, int32_t grid, float alpha,
                   const float* kp1_xy, const float* kp2_xy, const int32_t* best_idx,
                   int32_t* out_idx, void* workspace, size_t workspace_bytes,
                   hipStream_t stream) {
  if (!idx || !size1 || grid < 1 || grid > kGmsMaxGrid || !(alpha > 0.0f) ||
      !std::isfinite(alpha))
    return EPM_ERR_ARG;
  for (int p = 0; p < idx->P; ++p)
    if (size1[2 * p] <= 0 || size1[2 * p + 1] <= 0) return EPM_ERR_ARG;
  if (idx->N1 == 0) return EPM_OK;
  if (!kp1_xy || !best_idx || !out_idx || (idx->N2 > 0 && !kp2_xy)) return EPM_ERR_ARG;
  const GmsLayout L = gms_layout(idx, grid);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) ||
      workspace_bytes < L.total)
    return EPM_ERR_WORKSPACE;
  std::vector<char> head(sizeof(GmsPair) * (size_t)idx->P);
  GmsPair* table = reinterpret_cast<GmsPair*>(head.data());
  for (int p = 0; p < idx->P; ++p) {
    table[p].w1 = size1[2 * p];
    table[p].h1 = size1[2 * p + 1];
    table[p].w2 = 2.0 * idx->pairs[p].cx;  // cx = w2 / 2 exactly
    table[p].h2 = 2.0 * idx->pairs[p].cy;
  }
  char* ws = static_cast<char*>(workspace);
  const epm_status up = upload_table(head, ws + L.pairs, stream);
  if (up != EPM_OK) return up;
  GmsArgs A;
  A.pairs = reinterpret_cast<const GmsPair*>(ws + L.pairs);
  A.qstart = idx->at<int64_t>(idx->L.qstart);
  A.kstart = idx->at<int64_t>(idx->L.kstart);
  A.num_pairs = idx->P;
  A.n1 = idx->N1;
  A.grid = grid;
  A.alpha = alpha;
  A.kp1 = kp1_xy;
  A.kp2 = kp2_xy;
  A.best = best_idx;
  A.out = out_idx;
  A.key = reinterpret_cast<int32_t*>(ws + L.key);
  A.rcell = reinterpret_cast<int32_t*>(ws + L.rcell);
  A.count = reinterpret_cast<uint32_t*>(ws + L.count);
  A.cursor = reinterpret_cast<uint32_t*>(ws + L.cursor);
  A.offsets = reinterpret_cast<const int64_t*>(ws + L.offsets);
  A.list = reinterpret_cast<uint32_t*>(ws + L.list);
  EPM_HIP(launch_gms(A, reinterpret_cast<int64_t*>(ws + L.partials), stream));
  return EPM_OK;
}

epm_status epm_mutual_check(const epm_index* idx, const int32_t* best12, const int32_t* best21,
                             int32_t* mutual, hipStream_t stream) {
  if (!idx) return EPM_ERR_ARG;
  if (idx->N1 == 0) return EPM_OK;
  if (!best12 || !mutual || (idx->N2 > 0 && !best21)) return EPM_ERR_ARG;
  EPM_HIP(launch_mutual(idx->at<int64_t>(idx->L.qstart), idx->at<int64_t>(idx->L.kstart), idx->P,
                        idx->N1, best12, best21, mutual, stream));
  return EPM_OK;
}

epm_status epm_match_residuals(const epm_index* idx, const float* kp1_xy, const float* kp2_xy,
                               const int32_t* best_idx, float* residual, int64_t* feat_index,
                               hipStream_t stream) {
  if (!idx) return EPM_ERR_ARG;
  if (idx->N1 == 0) return EPM_OK;
  if (!kp1_xy || !kp2_xy || !best_idx || !residual) return EPM_ERR_ARG;
  EPM_HIP(launch_residuals(idx->at<PairDev>(idx->L.pairs), idx->at<int64_t>(idx->L.qstart),
                           idx->P, idx->N1, kp1_xy, kp2_xy, best_idx, residual, feat_index,
                           stream));
  return EPM_OK;
}

epm_status epm_quantize(const float* src, int64_t rows, int32_t dim, epm_dtype dtype, void* dst,
                        float* scale, hipStream_t stream) {
  if (rows < 0 || dim < 1 || dim > 4096) return EPM_ERR_ARG;
  if (dtype != EPM_BF16 && dtype != EPM_FP8_E4M3) return EPM_ERR_ARG;
  if (rows == 0) return EPM_OK;
  if (!src || !dst || (dtype == EPM_FP8_E4M3 && !scale)) return EPM_ERR_ARG;
  EPM_HIP(launch_quantize(src, rows, dim, dtype == EPM_BF16 ? 0 : 1, dst, scale, stream));
  return EPM_OK;
}

epm_status epm_rounding_error(const float* src, int64_t rows, int32_t dim, epm_dtype dtype,
                              const void* codes, const float* scale, float* err,
                              hipStream_t stream) {
  if (rows < 0 || dim < 1 || dim > 4096) return EPM_ERR_ARG;
  if (dtype != EPM_BF16 && dtype != EPM_FP8_E4M3) return EPM_ERR_ARG;
  if (rows == 0) return EPM_OK;
  if (!src || !codes || !err || (dtype == EPM_FP8_E4M3 && !scale)) return EPM_ERR_ARG;
  EPM_HIP(launch_round_err(src, rows, dim, dtype == EPM_BF16 ? 0 : 1, codes, scale, err, stream));
  return EPM_OK;
}

epm_status epm_point_line_terms(const double* F, const float* kp1_xy, const float* kp2_xy,
                                const float* eps2, float eps_scalar, const int64_t* qi,
                                const int64_t* kj, int64_t count, double* num, double* rhs,
                                hipStream_t stream) {
  if (count < 0 || !F) return EPM_ERR_ARG;
  if (count == 0) return EPM_OK;
  if (!kp1_xy || !kp2_xy || !qi || !kj || !num || !rhs) return EPM_ERR_ARG;
  EPM_HIP(launch_point_line_terms(F, kp1_xy, kp2_xy, eps2, eps_scalar, qi, kj, count, num, rhs,
                                  stream));
  return EPM_OK;
}

epm_status epm_descriptor_distances(epm_dtype dtype, int32_t dim, const void* desc1,
                                    const void* desc2, const float* scale1, const float* scale2,
                                    const int64_t* qi, const int64_t* kj, int64_t count,
                                    float* out, hipStream_t stream) {
  if (count < 0 || dim != 128) return EPM_ERR_ARG;
  if (dtype != EPM_F32 && dtype != EPM_BF16 && dtype != EPM_FP8_E4M3) return EPM_ERR_ARG;
  if (count == 0) return EPM_OK;
  if (!desc1 || !desc2 || !qi || !kj || !out) return EPM_ERR_ARG;
  if (dtype == EPM_FP8_E4M3 && (!scale1 || !scale2)) return EPM_ERR_ARG;
  const int fmt = dtype == EPM_F32 ? -1 : dtype == EPM_BF16 ? 0 : 1;
  EPM_HIP(launch_pair_distances(fmt, desc1, desc2, scale1, scale2, qi, kj, count, out, stream));
  return EPM_OK;
}

epm_status epm_get_query_stats(const epm_index* idx, epm_query_stats* out) {
  if (!idx || !out) return EPM_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  out->queries = idx->N1;
  if (!idx->have_stats) return EPM_OK;
  // the tile pass leaves its counters per tile: summed here
  const size_t nt = idx->stiles.size();
  std::vector<unsigned long long> tc((size_t)kTileCounts * nt);
  int64_t nnz = 0;
  if (nt > 0)
    EPM_HIP(hipMemcpyAsync(tc.data(), idx->at<unsigned long long>(idx->L.tile_counts),
                           sizeof(unsigned long long) * tc.size(), hipMemcpyDeviceToHost,
                           idx->last_stream));
  EPM_HIP(hipMemcpyAsync(&nnz, idx->last_offsets + idx->N1, sizeof(nnz), hipMemcpyDeviceToHost,
                         idx->last_stream));
  EPM_HIP(hipStreamSynchronize(idx->last_stream));
  unsigned long long sum[kTileCounts] = {};
  for (size_t t = 0; t < nt; ++t)
    for (int k = 0; k < kTileCounts; ++k) sum[k] += tc[t * kTileCounts + k];
  out->candidates = nnz;
  out->records_scanned = (int64_t)sum[0];
  out->angle_hits = (int64_t)sum[1];
  out->scanned_queries = (int64_t)sum[2];
  out->empty_queries = (int64_t)sum[3];
  return EPM_OK;
}

epm_status epm_get_match_stats(const epm_index* idx, epm_match_stats* out) {
  if (!idx || !out) return EPM_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  out->queries = idx->N1;
  if (!idx->have_match_stats) return EPM_OK;
  unsigned long long c[kNumMatchStats] = {};
  EPM_HIP(hipMemcpyAsync(c, idx->at<unsigned long long>(idx->L.match_stats),
                         sizeof(unsigned long long) * kNumMatchStats, hipMemcpyDeviceToHost,
                         idx->match_stream));
  // a match fused into the tile pass leaves its BF16 counters per tile
  const size_t nt = idx->match_from_tiles ? idx->stiles.size() : 0;
  std::vector<unsigned long long> tc((size_t)kTileCounts * nt);
  if (nt > 0)
    EPM_HIP(hipMemcpyAsync(tc.data(), idx->at<unsigned long long>(idx->L.tile_counts),
                           sizeof(unsigned long long) * tc.size(), hipMemcpyDeviceToHost,
                           idx->match_stream));
  EPM_HIP(hipStreamSynchronize(idx->match_stream));
  unsigned long long ranked = 0, unc = 0, evals = 0;
  for (size_t t = 0; t < nt; ++t) {
    ranked += tc[t * kTileCounts + 4];
    unc += tc[t * kTileCounts + 5];
    evals += tc[t * kTileCounts + 6];
  }
  out->reranked_rows = (int64_t)(c[0] + ranked);
  out->fallback_rows = (int64_t)(c[1] + unc);
  out->long_rows = (int64_t)c[2];
  out->exact_distances = (int64_t)(c[3] + evals);
  return EPM_OK;
}

void epm_index_destroy(epm_index* idx) { delete idx; }

const char* epm_status_string(epm_status s) {
  switch (s) {
    case EPM_OK: return "EPM_OK";
    case EPM_ERR_ARG: return "EPM_ERR_ARG: invalid argument";
    case EPM_ERR_DEGENERATE_F: return "EPM_ERR_DEGENERATE_F: F has no epipole (non-finite, zero or rank <= 1)";
    case EPM_ERR_CAPACITY: return "EPM_ERR_CAPACITY: col_indices too small";
    case EPM_ERR_WORKSPACE: return "EPM_ERR_WORKSPACE: workspace too small or misaligned";
    case EPM_ERR_HIP: return "EPM_ERR_HIP: HIP runtime error";
    case EPM_ERR_UNSUPPORTED: return "EPM_ERR_UNSUPPORTED: not implemented in this build";
  }
  return "EPM_ERR_UNKNOWN";
}

const char* epm_version(void) { return "epm 0.2.0 (gfx950)"; }

}  // extern "C"
