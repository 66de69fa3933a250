// Internal layout shared by the host side and the HIP kernels of libepm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epm {

// ---------------------------------------------------------------- angle keys
// A pencil angle phi in [0, pi) is stored as the u32 key round(phi / pi * 2^32):
// 2^32 key units are pi, so a difference of keys taken mod 2^32 is the
// circular difference of undirected line angles and the wrap-around at 0/pi
// (Sec. 4.4) needs no splitting.
constexpr double kKeyPerRad = 4294967296.0 / 3.14159265358979323846;
// Key units added to every half-width on top of outward rounding.
constexpr uint32_t kGuard = 4;
// A half-width of 2^31 key units (pi/2) covers every angle: the "full"
// interval of a circle that contains the epipole (Sec. 4.4).
constexpr uint32_t kFullHalf = 0x80000000u;

// Records are sorted by (width class, top bits of the centre key).  Class c
// holds half-widths H with 2^(c-1) <= H < 2^c, so a query at key P only has
// to scan class-c centres in [P - 2^c + 1, P + 2^c - 1]; class 31 holds every
// half-width >= 2^30 and is scanned whole.
constexpr int kClassBits = 5;
constexpr int kNumClasses = 32;
constexpr int kCentreBits = 19;
constexpr int kCentreShift = 32 - kCentreBits;  // centre key >> 13
constexpr int kSortBits = kClassBits + kCentreBits;  // 24 -> three 8-bit passes
constexpr int kWideClass = 31;
// Queries are sorted by the top 16 bits of their key (two 8-bit passes).
constexpr int kQuerySortBits = 16;

// Query flags.
constexpr uint32_t kQueryNormal = 0;
constexpr uint32_t kQueryEmpty = 1;  // a = b = 0: no distance is defined
constexpr uint32_t kQueryBrute = 2;  // scan every record of the pair

// Relative miss of a query line from the epipole that the record intervals
// absorb; queries beyond it scan the whole pair (exact either way).
constexpr double kKappaBuild = 1.0 / (1 << 24);
// Tolerance inflation used when building intervals (pixels): relative and
// absolute slack that dominates every FP64 rounding in the key pipeline.
constexpr double kEpsRelSlack = 1.0 / (1 << 30);
constexpr double kEpsAbsSlackPx = 1e-7;

// ------------------------------------------------------------ pair records
struct PairDev {
  double F[9];          // row-major, pixel space, exactly as given
  double u[3], v[3], e[3];  // orthonormal pencil basis in normalised line space
  double s, cx, cy;     // image-2 normalisation p^ = s (p - c)
  double G11, G12, G22; // Gram matrix of (u_12, v_12)
  double e12;           // |e_12|
  double kappa;         // miss bound absorbed by the record intervals
  int64_t q_begin, m, k_begin, n;
  int32_t qtile_begin, qtile_count;  // query sort tiles
  int32_t rtile_begin, rtile_count;  // record sort tiles
};

struct SortTile {
  int64_t begin;  // global element index
  int32_t count;
  int32_t seg;
};

struct SortSeg {
  int64_t begin;
  int64_t count;
  int32_t tile_begin, tile_count;
};

constexpr int kSortTile = 512;      // elements per sort tile
constexpr int kSortThreads = 256;

constexpr int kClassSlots = kNumClasses + 1;  // class_begin entries per pair

// Longest row sorted in LDS by the fill kernel; longer rows are rebuilt in
// ascending j order by a direct scan of the pair.
constexpr int kRowSortMax = 2048;

// Stabbing tiles: kTileQ consecutive angle-sorted queries of one pair share
// one window search per width class; the window's records are staged in LDS
// a round at a time (256, 512 or 1024 records, a tile shape chosen per index;
// kChunk by default).  Rows of up to kStage candidates are parked in a staging
// buffer by the tile kernel and sorted by the copy pass; longer rows are
// rebuilt by the fill kernel.
constexpr int kTileQ = 64;
constexpr int kStage = 128;
constexpr int kChunk = 512;

// Per-tile record windows found by the window pass: up to two ranges of
// sorted positions per width class (the second one when the window wraps
// through angle 0), as start positions and a running prefix of lengths.
constexpr int kSlots = 2 * kNumClasses;
struct TileWindow {
  uint32_t slot_b[kSlots];
  uint32_t slot_pref[kSlots + 1];
};

// per-tile counters of the tile pass: records scanned, angle hits,
// brute-force queries, empty queries; BF16 fused selection: rows ranked on
// bounds, rows left uncertified, exact distances evaluated; one spare
constexpr int kTileCounts = 8;

struct StabTile {
  int64_t begin;  // first angle-sorted query position of the tile
  int32_t count;  // queries in the tile (<= kTileQ)
  int32_t pair;
};

// One query of a stabbing tile as the window pass leaves it for the tile
// pass: the epipolar line (a, b, c), sqrt(a^2 + b^2), the query's index, flag
// and key (slots past the tile's count: empty, index 0).
struct TileQuery {
  double a, b, c, n;
  int64_t i;
  uint32_t flag, key;
};

}  // namespace epm
