// Internal data shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffa {

// Columns handled by one merge item. Odd, so that 64 lanes reading
// consecutive items hit 64 distinct LDS banks.
constexpr int kChunk = 5;
// Threads of a search-kernel workgroup (16 waves of 64).
constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
// Merge items a thread stages in registers per level (rows x chunks of a
// tile must not exceed kItemsMax * kThreads).
constexpr int kItemsMax = 8;
// Largest number of boxcar widths and of bins per profile.
constexpr int kMaxWidths = 32;
constexpr int kMaxBins = 1280;
constexpr int kSnrColsMax = (kMaxBins + 63) / 64;  // phases per lane in the S/N step
// Largest number of merge levels in one range pass (2^L source nodes).
constexpr int kMaxRangeLevels = 4;
constexpr int kMetaNodes = (2 << kMaxRangeLevels) - 1;
// LDS available to one search workgroup (gfx950: 160 KiB per CU).
constexpr int kLdsBytes = 160 * 1024;
// LDS set aside for the S/N prefix arrays of the waves.
constexpr int kSnrLdsBytes = 24 * 1024;

// Row stride in LDS (floats) of a profile of p bins: the row is followed by a
// copy of its first kChunk - 1 bins, so a rotated read of kChunk consecutive
// bins starting below p never wraps.
inline __host__ __device__ int lds_stride(int p) { return p + kChunk - 1; }

// Rows of a p-bin profile tile that fit in one workgroup's LDS next to the
// merge tables, the range-tile metadata and the S/N prefix arrays; at most
// `cap` when cap > 0.
inline __host__ __device__ int rows_capacity(int p, int cap) {
  const int fixed = kSnrLdsBytes + kMetaNodes * 5 * 4 + 64;
  const int per_row = lds_stride(p) * 4 + 3 * 4;
  int r = (kLdsBytes - fixed) / per_row;
  const int nch = (p + kChunk - 1) / kChunk;
  const int ri = (kItemsMax * kThreads) / nch;
  r = r < ri ? r : ri;
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
};

// Arguments of one pass launch.
struct PassArgs {
  const TileDesc* tiles;
  int32_t ntiles;
  int32_t lds_rows_cap;    // cap on the rows of a tile (0 = what fits)
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
  int32_t max_p;           // largest p of the launch (sizes the S/N LDS arrays)
};

}  // namespace ffa
