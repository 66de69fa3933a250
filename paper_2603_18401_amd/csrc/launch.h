// Host-side launchers of the libepm kernels (one per kernel family).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "epm_internal.h"

namespace epm {

// Pair setup on the device (one thread per pair): F from F[9 p .. 9 p + 8]
// into the pair record, with the epipole, pencil basis and guard; a pair
// without a pencil gets kappa = -1 (its queries then scan the whole pair).
hipError_t launch_pair_setup(PairDev* pairs, const double* F, int num_pairs, hipStream_t s);

// One workgroup per record sort tile; also leaves the first radix pass's
// per-tile digit counts in hist (and zero counts for the later passes), so
// that segmented_radix_sort(..., first_counts_ready = true) skips its count.
hipError_t launch_intervals(const PairDev* pairs, const SortTile* tiles, int num_tiles,
                            const float* kp2, const float* eps2, float eps_scalar,
                            uint32_t* sort_key, uint32_t* sort_val, uint32_t* recC,
                            uint32_t* recH, uint32_t* hist, int zero_passes, hipStream_t s);

// One workgroup per query sort tile.  Also writes every query's line (a, b,
// c, sqrt(a^2 + b^2)) to qline (zero for a query without a line), the first
// radix pass's counts as launch_intervals does, and its first workgroup
// clears the counters as launch_clear_stats does (each pointer may be NULL).
hipError_t launch_query_keys(const PairDev* pairs, const SortTile* tiles, int num_tiles,
                             const float* kp1, uint32_t* qkey, uint32_t* qflag,
                             uint32_t* sort_key, uint32_t* sort_val, double4* qline,
                             uint32_t* hist, int zero_passes, unsigned long long* stats,
                             uint32_t* sched, unsigned long long* match_stats, hipStream_t s);

hipError_t launch_gather_records(const int64_t* kstart, int num_pairs, int64_t n2,
                                 const uint32_t* sorted_val, const float* kp2, const float* eps2,
                                 float eps_scalar, const uint32_t* recC, const uint32_t* recH,
                                 uint32_t* rC, uint32_t* rH, int32_t* rj, float2* rxy,
                                 float* reps, uint32_t* rinv, const uint32_t* digit_base,
                                 int64_t* class_begin, hipStream_t s);
// digit_base non-NULL: the gather also writes class_begin from the digit
// starts of the last sort pass (digit = class << 3 | top three centre bits).

hipError_t launch_class_bounds(const int64_t* kstart, int num_pairs, const uint32_t* skey,
                               int64_t* class_begin, hipStream_t s);

// Stable LSD radix sort of (key, value) u32 pairs inside every segment, over
// the low `bits` bits of the keys, 8 bits per pass.  Ping-pongs between
// (k0, v0) and (k1, v1); returns through *sorted_in_1 whether the result
// ended in (k1, v1).
// last_digit_base (optional, [num_segs][256]): global start of every digit
// value of the last pass inside each segment.
// hist: [sort_passes(bits)][num_tiles][256] words; max_seg_tiles: the most
// tiles of one segment (up to 64 a pass is a single launch).
int sort_passes(int bits);
// The sort tiles of the records (tr) and the queries (tq) and the stabbing
// tiles (ts), filled from the per-pair segments, the query slice starts and
// each pair's first stabbing tile (num_pairs + 1 entries).
hipError_t launch_expand_tiles(const SortSeg* rsegs, const SortSeg* qsegs, const int64_t* qstart,
                               const int32_t* stile_begin, int num_pairs, SortTile* rtiles,
                               int64_t tr, SortTile* qtiles, int64_t tq, StabTile* stiles,
                               int64_t ts, hipStream_t s);
hipError_t segmented_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                                const SortTile* tiles, int num_tiles, const SortSeg* segs,
                                int num_segs, int max_seg_tiles, uint32_t* hist, int bits,
                                bool* sorted_in_1, hipStream_t s,
                                uint32_t* last_digit_base = nullptr,
                                bool first_counts_ready = false);

struct StabArgs {
  const PairDev* pairs;
  const int64_t* qstart;
  int num_pairs;
  int64_t n1;
  const float* kp1;
  const uint32_t* qkey;
  const uint32_t* qflag;
  const uint32_t* qperm;
  const int64_t* class_begin;
  const uint32_t* skey;
  const uint32_t* rC;
  const uint32_t* rH;
  const int32_t* rj;
  const float2* rxy;
  const float* reps;
  const uint32_t* rinv;
  uint32_t* counts;
  // fused selection: per query (original index) one 16-byte record {row
  // length, best index, best distance, second distance} written in one store
  // (the count is read by the scan from it, the match by the copy pass);
  // best index kMatchDeferred: the match comes from a later pass.  NULL: the
  // counts array and no match.
  uint4* qrec;
  const int64_t* row_offsets;
  int32_t* cols;
  int64_t capacity;
  const StabTile* tiles;
  int num_tiles;
  int32_t* staging;  // [n1][kStage], indexed by the original query index
  unsigned long long* stats;  // kNumStats counters, cleared by launch_clear_stats
  // [num_tiles][kTileCounts] per-tile counters of the tile pass (records
  // scanned, angle hits, brute-force queries, empty queries), summed on the
  // host when asked for: no global atomics on shared counters in the pass
  unsigned long long* tile_counts;
  uint32_t* long_rows;        // [n1] queue of brute-force rows longer than kStage
  uint32_t* tile_wide;        // [num_tiles] 1: the tile has a normal row longer than kStage
  uint32_t* pair_wide;        // [num_pairs] the pair's wide tiles
  TileWindow* windows;        // [num_tiles], written by launch_tile_windows
  uint32_t* tile_cost;        // [num_tiles] work estimate per tile, or NULL
  const uint32_t* order;      // persistent launch: tile order (NULL = angle order)
  uint32_t* queue;            // persistent launch: next-tile counter, zero at launch
  TileQuery* tile_q;          // [num_tiles][kTileQ], written by launch_tile_windows
  const uint32_t* block_tile;  // one workgroup per tile: tile of each workgroup, or NULL
  // fused matching (FP32 descriptors), see launch_stab_tiles
  const float* desc1;
  const float* desc2;
  float ratio;
  int32_t* best_idx;
  float* best_dist;
  float* second_dist;
  uint32_t* rest;             // [n1] queries left to the listed-query match
  unsigned long long* match_stats;  // wide-row matching counters (kNumMatchStats), or NULL
  double4* qline;             // [n1] (a, b, c, sqrt(a^2 + b^2)) of every query, by the tile pass
  // wide-row matching of a caller's CSR (epm_match)
  const uint16_t* codes1;     // BF16 descriptor codes (desc1 / desc2 are then the FP32 masters)
  const uint16_t* codes2;
  // BF16 copies of the image-2 FP32 rows (desc2) and per row the squared norm
  // of the copy and of its rounding error, made by launch_round_rows for the
  // wide-row pass (NULL: the pass rounds the rows on chip)
  const uint16_t* wcodes2;
  const float2* wterms2;
  unsigned long long* rest_count;  // length of the rest list the wide-row pass appends to
  // FP8 selection fused into the stabbing pass (kStabFP8): the image-2 rows as
  // OCP E4M3FN codes [n2][128] with one FP32 scale per row and a bound on the
  // norm of each row's rounding error (desc1 / desc2 are the FP32 masters)
  const uint8_t* f8codes2 = nullptr;
  const float* f8scale2 = nullptr;
  const float* f8err2 = nullptr;
};

// Scheduling counters (u32 words of one workspace block).
constexpr int kCostBuckets = 65;  // cost 0, then two buckets per power of two
constexpr int kLptXcd = 8;        // XCDs the workgroups of a launch are dealt to in turn
constexpr int kSchedHist = 0, kSchedCursor = kCostBuckets, kSchedStabQueue = 2 * kCostBuckets,
              kSchedMatchQueue = 2 * kCostBuckets + 1;
constexpr int kSchedWords = 2 * kCostBuckets + 2;

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// Longest-first order of the tiles from their costs; the histogram and cursor
// words of `sched` must be zero.
hipError_t launch_lpt_order(const uint32_t* cost, int num_tiles, uint32_t* sched,
                            uint32_t* order, hipStream_t s);
// One workgroup per tile, longest first on every XCD: block_tile[b] for the
// workgroups b = x, x + 8, ... of XCD x lists the tiles that the XCD-grouped
// angle order gives that XCD, by decreasing cost bucket (cost from
// launch_tile_windows).
hipError_t launch_xcd_lpt_order(const uint32_t* cost, int num_tiles, uint32_t* block_tile,
                                hipStream_t s);

// One wavefront per tile finds the tile's window in every width class.
hipError_t launch_tile_windows(const StabArgs& a, hipStream_t s);

// Device-wide counters of a query: the lengths of its two queues (long rows
// for the fill pass, rows left to the listed-query match).
constexpr int kStatLongRows = 0, kStatRest = 1;
constexpr int kNumStats = 2;
// Clears the kNumStats counters unless stats is NULL, the kSchedWords
// scheduling words unless sched is NULL and the kMatchStatWords match counters
// unless match_stats is NULL.
hipError_t launch_clear_stats(unsigned long long* stats, hipStream_t s, uint32_t* sched = nullptr,
                              unsigned long long* match_stats = nullptr);

// Tiled count pass (also parks rows of <= kStage candidates).  grid 0: one
// workgroup per tile; grid > 0: that many workgroups take tiles from a.queue.
// mode kStabF32 / kStabBF16: also selects the FP32 matches of the rows it can
// (desc1/desc2 and the outputs in a); the other queries are appended to
// a.rest, counted in stats[kStatRest], for launch_match_listed_f32 once the
// CSR is complete.
// mode kStabBF16: BF16 codes in codes1/codes2 with the FP32 masters in
// desc1/desc2; the match is selected through certified MFMA bounds and an
// exact re-rank on the masters (rows it cannot certify go to a.rest).
// mode kStabFP8: likewise over the FP8 image-2 rows in f8codes2 (scales
// f8scale2, rounding-error bounds f8err2); the queries are rounded to BF16 on
// chip from their masters.
constexpr int kStabCount = 0, kStabF32 = 1, kStabBF16 = 2, kStabFP8 = 3;
// chunk: window records staged per round (256, 512 or 1024; 0 = 256 for the
// BF16 and FP8 passes, 512 for the others).
hipError_t launch_stab_tiles(const StabArgs& a, int grid, int mode, int chunk, hipStream_t s);
constexpr int32_t kMatchDeferred = INT32_MIN;
// Fill pass after launch_stab_tiles: copies parked rows, rebuilds the
// brute-force long rows.
hipError_t launch_fill_rows(const StabArgs& a, hipStream_t s);
// Wide-row pass over the tiles flagged in a.tile_wide.
//   kWideFill:  writes the rows longer than kStage of normal queries (after
//               the scan of the row lengths);
//   kWideFused: also selects their FP32 matches (desc1/desc2 and the outputs
//               in a) through a BF16 MFMA bound with a certified FP32 re-rank;
//   kWideMatchF32 / kWideMatchBF16: matches every query of the flagged tiles
//               over the caller's CSR (a.cols, trusted up to a.capacity),
//               FP32 rows rounded to BF16 on chip or the caller's BF16 codes
//               (codes1/codes2, FP32 masters in desc1/desc2); rows that differ
//               from the tile's candidate sets are not trusted to the bound.
// Queries it cannot certify (and, when matching, rows of brute-force queries
// or foreign rows) are appended to a.rest, counted in *a.rest_count, for the
// listed-query match.
constexpr int kWideFill = 0, kWideFused = 1, kWideMatchF32 = 2, kWideMatchBF16 = 3;
hipError_t launch_wide_tiles(const StabArgs& a, int mode, hipStream_t s);
// Rounds the FP32 image-2 rows (a.desc2) of the pairs with many wide tiles
// (a.pair_wide against the pair's size) to BF16 (round to nearest even) into
// a.wcodes2, with their terms in a.wterms2, for kWideFused and kWideMatchF32
// passes, whose tiles of those pairs stage the copies instead of rounding on
// chip.  n2 rows; pre: 2 * num_pairs + 2 int64 of scratch (the list of those
// pairs and their row prefix).
hipError_t launch_round_rows(const StabArgs& a, int64_t n2, int64_t* pre, hipStream_t s);

// Exclusive scan of counts[0..n) into offsets[0..n], offsets[n] = total.
// counts[stride * i] is the length of row i (stride 4: the count words of
// the fused pass's query records).
hipError_t launch_scan_counts(const uint32_t* counts, int stride, int64_t n, int64_t* offsets,
                              int64_t* partials, hipStream_t s);
int64_t scan_partials_count(int64_t n);

struct MatchArgs {
  const int64_t* qstart;
  const int64_t* kstart;
  int num_pairs;
  int64_t n1;
  const uint32_t* qperm;  // processing order (angle-sorted); NULL = natural order
  const int64_t* row_offsets;
  const int32_t* cols;
  const void* desc1;
  const void* desc2;
  float ratio;
  int32_t* best_idx;
  float* best_dist;
  float* second_dist;
  const StabTile* tiles;  // angle tiles of the last query pass (tiled kernels)
  int num_tiles;
  const TileWindow* windows;  // their record windows
  const uint32_t* rinv;       // record -> angle-sorted position
  const int32_t* rj;          // angle-sorted position -> image-2 index in the pair
  bool xcd_order;  // plain kernels: place consecutive blocks on one XCD
  const float* scale1;        // FP8 row scales
  const float* scale2;
  const float* desc1_f32;     // FP32 masters (re-rank and exact fallback)
  const float* desc2_f32;
  unsigned long long* match_stats;  // [kNumMatchStats], cleared before the launch
  int64_t capacity;            // size of cols; < 0: trusted.  Nothing is written
                               // when row_offsets[n1] exceeds it.
  const uint32_t* order;       // persistent tiled launch: tile order (NULL = angle order)
  uint32_t* queue;             // persistent tiled launch: next-tile counter, zero at launch
  const uint32_t* skip_tiles;  // tiled kernels: tiles left to the wide-row pass, or NULL
  const uint32_t* block_tile;  // one workgroup per tile: tile of each workgroup, or NULL
  // measured per-row rounding errors of the reduced rows (>= |x - dequant(x^)|),
  // or NULL for the format's worst case
  const float* qerr1;
  const float* qerr2;
};

// re-ranked rows, uncertified (exact fallback), long rows, exact distances of the re-rank
constexpr int kNumMatchStats = 4;
constexpr int kMatchStatRest = 4;  // internal: rest-list length of the wide-row match
constexpr int kMatchStatWords = kMatchStatRest + 1;
// fmt 0: BF16, 1: FP8-E4M3 with row scales.
// grid as for launch_stab_tiles.
hipError_t launch_match_window_mfma(const MatchArgs& a, int fmt, int grid, hipStream_t s);

hipError_t launch_match_plain_f32(const MatchArgs& a, hipStream_t s);
// FP32 matches of the queries list[0 .. *count) (count on the device, at most
// max_count).
hipError_t launch_match_listed_f32(const MatchArgs& a, const uint32_t* list,
                                   const unsigned long long* count, int64_t max_count,
                                   hipStream_t s);
hipError_t launch_match_plain_bin256(const MatchArgs& a, hipStream_t s);
// One workgroup per stabbing tile, window descriptor rows staged in LDS.
hipError_t launch_match_window_f32(const MatchArgs& a, int grid, hipStream_t s);

// ------------------------------------------------ learned tolerance network
constexpr int kEpsParams = 4673;       // 6-64-64-1 network, see mlp.hip
constexpr int kEpsGradMaxBlocks = 256;  // workgroups (and partial gradients) per batch

struct EpsPair {  // per-pair constants of the keypoint features
  double ex, ey;   // image-2 epipole in pixels (when finite)
  double diag;     // image-2 diagonal
  double w, h;     // image-2 size
  int32_t finite;  // 0: epipole at infinity
  int32_t pad;
};

struct EpsGradArgs {
  const float* features;    // [num_rows][6]
  int64_t num_rows;
  const int64_t* feat_index;  // [num_slots] sample slot -> feature row, or NULL (identity)
  const float* target;      // [num_slots] residuals
  int64_t num_slots;
  const int32_t* sample_idx;  // [batch] slots of this minibatch
  int64_t batch;
  float q;                  // quantile level of the pinball loss
  float inv_batch;
  const float* params;
  float* partials;          // [kEpsGradMaxBlocks][kEpsParams + 1]
};

hipError_t launch_eps_features(const EpsPair* pairs, const int64_t* kstart, int num_pairs,
                               int64_t n2, const float* kp2, const float* attrs, float* out,
                               hipStream_t s);
hipError_t launch_eps_infer(const float* feat, int64_t n, const float* params, float* eps,
                            hipStream_t s);
int eps_grad_blocks(int64_t batch);
hipError_t launch_eps_grad(const EpsGradArgs& a, float* grad, float* loss, hipStream_t s);
hipError_t launch_eps_adam(float* theta, float* m, float* v, const float* grad, float lr,
                           float beta1, float beta2, float eps, float c1, float c2,
                           hipStream_t s);
hipError_t launch_residuals(const PairDev* pairs, const int64_t* qstart, int num_pairs,
                            int64_t n1, const float* kp1, const float* kp2, const int32_t* best,
                            float* residual, int64_t* feat_index, hipStream_t s);

// Pose-uncertainty tolerance (see pose_eps.hip): per pair F, the six
// derivatives of F with respect to the pose (rotation vector, translation),
// their covariance and the image-1 size.
struct PosePair {
  double F0[9];
  double dF[6][9];
  double cov[36];
  double w1, h1;
  double fmax;  // largest |F0| entry
  // depth range: image-1 partners of x2 are K1 R^T (K2^-1 x2 - rho t) for
  // inverse depths rho in [rho_lo, rho_hi]; rho_hi = 0 when no range is given
  double K1[9], K2i[9], Rt[9], t[3];
  double rho_lo, rho_hi;
};
hipError_t launch_pose_eps(const PosePair* pairs, const int64_t* kstart, int num_pairs,
                           int64_t n2, const float* kp2, float eps0, float k_sigma,
                           float eps_max, float* eps2, hipStream_t s);

// GMS validation (see gms.hip).
constexpr int kGmsMaxGrid = 32;
constexpr int kGmsMaxCells = kGmsMaxGrid * kGmsMaxGrid;
struct GmsPair {
  double w1, h1, w2, h2;  // image sizes of the pair
};
struct GmsArgs {
  const GmsPair* pairs;
  const int64_t* qstart;
  const int64_t* kstart;
  int num_pairs;
  int64_t n1;
  int grid;
  float alpha;
  const float* kp1;
  const float* kp2;
  const int32_t* best;
  int32_t* out;
  int32_t* key;           // [n1] (pair, image-1 cell) of each match, -1 without one
  int32_t* rcell;         // [n1] image-2 cell of each match
  uint32_t* count;        // [pairs * grid^2] matches per (pair, cell)
  uint32_t* cursor;       // [pairs * grid^2]
  const int64_t* offsets; // [pairs * grid^2 + 1] exclusive scan of count
  uint32_t* list;         // [n1] matches listed by (pair, cell)
};
hipError_t launch_gms(const GmsArgs& a, int64_t* partials, hipStream_t s);

// mutual[i] = best12[i] when best21 (indexed by the global image-2 row) maps
// that keypoint back to query i of the same pair, else -1.
hipError_t launch_mutual(const int64_t* qstart, const int64_t* kstart, int num_pairs, int64_t n1,
                         const int32_t* best12, const int32_t* best21, int32_t* mutual,
                         hipStream_t s);

// err[r] >= |src_r - dequant(codes_r)| (fmt 0: BF16; 1: E4M3 with scales).
hipError_t launch_round_err(const float* src, int64_t rows, int dim, int fmt, const void* codes,
                            const float* scale, float* err, hipStream_t s);

// fmt 0: BF16 codes [rows][dim]; 1: E4M3 codes [rows][dim] and scales [rows].
hipError_t launch_quantize(const float* src, int64_t rows, int dim, int fmt, void* dst,
                           float* scale, hipStream_t s);

// fmt 0 / 1: MFMA approximate distances of BF16 / FP8 codes; -1: canonical
// FP32 distances of FP32 rows; for pairs (qi[t], kj[t]).
hipError_t launch_pair_distances(int fmt, const void* desc1, const void* desc2,
                                 const float* scale1, const float* scale2, const int64_t* qi,
                                 const int64_t* kj, int64_t count, float* out, hipStream_t s);

hipError_t launch_point_line_terms(const double* F9, const float* kp1, const float* kp2,
                                  const float* eps2, float eps_scalar, const int64_t* qi,
                                  const int64_t* kj, int64_t count, double* num, double* rhs,
                                  hipStream_t s);

}  // namespace epm
