// Internal data shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffa {

// Consecutive columns a lane merges per row (odd, so that the 64 lanes of a
// wave reading consecutive column groups hit distinct LDS banks).
constexpr int kChunk = 5;
// A search-kernel workgroup has 16 waves of 64 (one per CU, all of the LDS)
// or 8 (two per CU, half of the LDS each).
constexpr int kWavesLarge = 16;
constexpr int kWavesSmall = 8;
// (row, column-group) slots a lane stages in registers per merge level.
constexpr int kStageMax = 8;
// Largest subtree a full tile folds; the host precomputes their schedules.
constexpr int kMaxFullRows = 192;
constexpr int kMaxFullLevels = 8;  // ceil(log2(kMaxFullRows))
// Full tiles fold their bottom nodes of at most kRegRows rows in registers
// (cross-lane shifts by one lane); log2 of it is the most register levels.
constexpr int kRegRows = 8;
constexpr int kRegLevels = 3;
// Most LDS merge levels of a full tile above its register levels (tiles of
// at most 128 rows: nodes of at most 8 rows at depth 4).
constexpr int kMaxTileLevels = 4;
static_assert(kWavesLarge * kStageMax <= (kRegRows << kMaxTileLevels),
              "a full tile's LDS levels fit kMaxTileLevels");
// Largest number of boxcar widths and of bins per profile.
constexpr int kMaxWidths = 32;
constexpr int kMaxBins = 1280;
constexpr int kSnrColsMax = (kMaxBins + 63) / 64;  // phases per lane, general S/N path
// Largest number of merge levels in one range pass (2^L source nodes).
constexpr int kMaxRangeLevels = 5;
constexpr int kMetaNodes = (2 << kMaxRangeLevels) - 1;
// Range-tile metadata in LDS: six arrays over the nodes, one over the levels.
constexpr int kMetaInts = 6 * kMetaNodes + kMaxRangeLevels + 4;
// LDS of a CU (gfx950: 160 KiB); a workgroup of w waves uses w / 16 of it.
constexpr int kLdsBytes = 160 * 1024;
// Downsampled octaves start on multiples of kDsGroup samples of their buffer:
// the downsampler emits kDsGroup consecutive outputs of an octave at a time,
// with whole 16-byte stores.
constexpr int kDsGroup = 8;
// Normalisation record of a series for the downsampler (FP32): mean rounded
// to FP32, 1 / std, the mean's FP32 rounding residual (mean - that float),
// and a pad word.
constexpr int kNormFloats = 4;
inline __host__ __device__ int wg_lds_bytes(int waves) { return kLdsBytes / kWavesLarge * waves; }
// LDS set aside for the S/N step; range tiles keep their pair-operation
// records of kOpInts ints here during the merges, so a range tile has at most
// kMaxTileOps operations.
constexpr int kSnrLdsBytes = 10 * 1024;
constexpr int kOpInts = 6;
constexpr int kMaxTileOps = kSnrLdsBytes / (kOpInts * 4);

// Bins past p that a row in LDS keeps as a copy of bins 0 .. kHalo - 1, so a
// rotated read of kChunk + 1 consecutive bins (the two rows of a merge pair)
// starting below p never wraps.
constexpr int kHalo = kChunk;

// Row stride in LDS (floats) of a profile of p bins. The stride covers every
// kChunk-column group that starts below p + kHalo (those groups compute the
// copy themselves) and is odd, so lanes reading the same column of different
// rows hit different banks.
inline __host__ __device__ int merge_groups(int p) {
  return (p + kHalo - 1) / kChunk + 1;
}
inline __host__ __device__ int lds_stride(int p) { return (merge_groups(p) * kChunk) | 1; }

// Column groups per lane for a p-bin row (one wave covers a row).
inline __host__ __device__ int col_iters(int p) { return (merge_groups(p) + 63) / 64; }

// Rows of a p-bin profile tile that fit in one workgroup's LDS next to the
// merge tables, the range-tile metadata, the S/N arrays, an all-zero row (the
// tail of plain copies) and a junk row (target of idle slots' writes); at most
// `cap` when cap > 0.
inline __host__ __device__ int rows_capacity(int p, int cap, int waves) {
  const int fixed = kSnrLdsBytes + kMetaInts * 4 + 64 + 2 * lds_stride(p) * 4;
  const int per_row = lds_stride(p) * 4 + 3 * 4;
  int r = (wg_lds_bytes(waves) - fixed) / per_row;
  const int rs = waves * (kStageMax / col_iters(p));
  r = r < rs ? r : rs;
  r = r < kMaxFullRows ? r : kMaxFullRows;
  if (cap > 0 && cap < r) r = cap;
  return r < 2 ? 2 : r;
}

// One folding transform of one series: the m x p row-major view of a
// downsampled series (Sec. 2.1).
struct XformDesc {
  int64_t in_off;    // element offset of the first row in the downsampled buffer
  int64_t scr_off;   // float offset of its m x p intermediate rows in a scratch buffer
  int64_t out_row0;  // periodogram row of trial s = 0 (S/N output) or, for raw
                     // transforms, float offset of row 0 in the output array
  int32_t m, p, keep;
  int32_t scale_off; // offset in the S/N scale table (num_widths floats)
};

enum TileFlags : uint8_t {
  kTileFull = 1,      // whole subtree: rows loaded from the input, all levels
  kTileFinal = 2,     // the tile's node is the root: emit results
  kTileOutRows = 4,   // final rows go to the raw-transform output, not to S/N
};

// A unit of work of a pass: output rows [s0, s1) of node `node` at depth
// d_dst of a transform's tree, computed from the rows at depth d_dst + L
// (range tiles) or from the input rows (full tiles).
struct TileDesc {
  int32_t xf;
  int32_t node;
  int32_t s0, s1;
  uint8_t d_dst;
  uint8_t levels;    // range tiles: merge levels in this pass
  uint8_t flags;
  uint8_t bufs;      // bit 0: scratch buffer read, bit 1: scratch buffer written
  // Persistent launches: the tile starts once counter `dep` reaches need[dep]
  // (-1: no wait) and adds one to counter `done` when finished (-1: none).
  int32_t dep;
  int32_t done;
  // Range tiles: position in PassArgs::src_rows of their source-row list (a
  // count, then the rows); set by attach_source_rows.
  int32_t rows_off;
};

// Arguments of one pass launch.
struct PassArgs {
  const TileDesc* tiles;
  const int32_t* src_rows;  // source-row lists of the range tiles (TileDesc::rows_off)
  int32_t ntiles;
  int32_t lds_rows_cap;    // cap on the rows of a tile (0 = what fits)
  int32_t waves;           // waves per workgroup (kWavesLarge or kWavesSmall)
  const XformDesc* xf;
  const void* in;          // downsampled series (or raw transform input)
  int32_t in_dtype;        // ffa_dtype
  int32_t num_widths;
  float* scr0;
  float* scr1;
  float* out_rows;         // raw transform output
  float* snr;              // periodogram S/N, rows x num_widths
  const float* scales;     // per transform and width: 1 / sqrt(m w var)
  int32_t widths[kMaxWidths];
  int32_t wmax;
  int32_t max_p;           // largest p of the launch
  int32_t width_set;       // 0: general widths; else a compiled width grid (WidthSet)
  int32_t pairs_only;      // every tile takes the pair-merge forms (pairs_only_launch)
                           // and is full (2) or a range tile (3); 0: any tile
  // Merge schedules of full subtrees of n rows (2 <= n <= kMaxFullRows):
  // entry full_off[n] + lev * n + q gives, for row q at relative depth lev,
  // the head row (low 16 bits) and tail row (high 16 bits; 0xffff: the row
  // is a one-row block and stays) and the rotation s - j.
  const uint32_t* full_ht;
  const uint16_t* full_rot;
  const int32_t* full_off;
  // Pair schedules of full subtrees: the merge operations of relative depth
  // lev of an n-row subtree are entries full_pops_off[n * (kMaxFullLevels + 1)
  // + lev] .. [.. + lev + 1] of full_pops, two words each: word 0 = output row
  // a | head row of a << 8 | head row of b << 16 | tail row << 24 (row b =
  // a + 1); word 1 = rotation of row a (row b: one more) | single << 16, a
  // single operation having no row b.
  const uint32_t* full_pops;
  const int32_t* full_pops_off;
  // Persistent launches: tile tickets, per-pass completion counters, and the
  // error word (bit 1: a dependency wait gave up after spin_limit polls).
  int32_t* ticket;
  int32_t* counters;
  const int32_t* need;
  int32_t* error_flag;
  int32_t spin_limit;
};

// Passes of one transform tracked by the persistent scheduler.
constexpr int kMaxPasses = 8;

// Width grids the S/N step is compiled for (registers instead of LDS for the
// prefix history).
enum WidthSet : int32_t {
  kWidthsGeneral = 0,
  kWidthsPaper9 = 1,   // 1,2,3,4,6,9,13,19,28: w0 = 1, w_{k+1} = max(floor(1.5 w_k), w_k + 1)
  kWidthsDuty9 = 2,    // 1,2,3,5,8,12,19,30,48: duty cycles 0.5 % .. 20 % of 240 bins
};

// Rows short enough for the pair-merge forms: one column group per lane, and
// room in the wave for the register levels of full tiles. Raw-transform
// launches (no S/N) of such rows run the kernels compiled for those forms.
// Launches in which every tile takes the pair-merge forms (one column group
// per lane, register levels in full tiles) and the register-window S/N of a
// compiled width grid: rows of 160 .. max bins with one column group per lane
// (the S/N window of 32 starts plus the widest boxcar then fits in a row and
// its copied bins, and the partial maxima fit in the row area of any tile of
// two or more rows). Such launches run a kernel compiled for those forms only.
inline __host__ __device__ bool pair_forms_fit(int max_p) {
  return col_iters(max_p) == 1 && merge_groups(max_p) + kRegLevels <= 64;
}
inline __host__ __device__ bool pairs_only_launch(int min_p, int max_p, int width_set) {
  return width_set != kWidthsGeneral && min_p >= 160 && pair_forms_fit(max_p);
}

}  // namespace ffa
