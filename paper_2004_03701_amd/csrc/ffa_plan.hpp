// Host-side period plan and tile plan of the FFA search.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ffa.h"
#include "ffa_internal.hpp"

namespace ffa {

// One pseudo-octave (Sec. 5.3): the original series downsampled by
// ds = ds_fx / 2^32.
struct Octave {
  double ds;         // factor before quantisation
  uint64_t ds_fx;    // 32.32 fixed point
  double tau;        // sampling time after downsampling
  int64_t nsamp;     // downsampled samples
  double var;        // noise variance of a downsampled sample (App. A.4)
  int64_t ds_off;    // offset of this octave in the series' downsampled buffer
};

// One folding transform: bins p, m rows of the octave's series.
struct Transform {
  int32_t octave, p, m, keep;
  int64_t row0;      // periodogram row of s = 0
};

struct SeriesPlan {
  std::vector<Octave> oct;
  std::vector<Transform> tr;
  int64_t rows = 0;        // kept periodogram rows
  int64_t ds_total = 0;    // elements of the downsampled buffer (octaves padded to kDsGroup)
  int64_t ds_samples = 0;  // downsampled samples of all octaves
  uint64_t ds_fx_max = 0;
  int64_t cells = 0;       // sum of m * p over transforms
};

// Validates params and nsamp and builds the plan. Returns FFA_OK or an error
// status with a message in *err.
ffa_status build_series_plan(const ffa_search_params& params, int64_t nsamp, SeriesPlan* out,
                             std::string* err);

// Validates the parameters alone (no nsamp).
ffa_status validate_params(const ffa_search_params& params, std::string* err);

// Trial period of row s of an m-row transform (Eq. for P_s, Sec. 2.3).
double trial_period(int64_t s, int64_t m, int64_t p, double tau);

// Tile shapes.
struct Tiling {
  int32_t lds_rows = 0;         // 0: the largest that fits
  int32_t levels_per_pass = 5;  // 1..kMaxRangeLevels
  int32_t persistent = 0;       // 1: one persistent launch per group of series
  int32_t waves = kWavesSmall;  // waves per workgroup: 16 (one per CU) or 8 (two per CU)
  int32_t range_waves = 0;      // the same for the range passes (0: as `waves`)
  int32_t waves_of_range() const { return range_waves > 0 ? range_waves : waves; }
};

// Rows of a p-bin profile tile that fit in one workgroup's LDS: full tiles
// (first passes) and range tiles (later passes).
int32_t rows_capacity(int32_t p, const Tiling& t);
int32_t range_rows_capacity(int32_t p, const Tiling& t);

// Tiles of one transform, grouped by pass. `xf` is the transform's index in
// the launch's transform table. Appends to passes[k] for pass k. Full tiles
// hold at most rows_cap rows; the levels of a range pass are capped so that
// every range tile's rows fit range_rows_cap at every level; returns false (and
// the plan must not be used) if some tile would not.
bool plan_transform_tiles(int32_t xf, int32_t m, int32_t p, int32_t keep, int32_t rows_cap,
                          int32_t range_rows_cap, int32_t levels_per_pass, bool out_rows,
                          std::vector<std::vector<TileDesc>>* passes);

// Merge schedules of full subtrees of 2..kMaxFullRows rows (PassArgs).
void build_full_schedules(std::vector<uint32_t>* ht, std::vector<uint16_t>* rot,
                          std::vector<int32_t>* off);

// Pair schedules of full subtrees of 2..kMaxFullRows rows (PassArgs):
// consecutive output rows of a node that share their tail row (rotations k
// and k + 1) form one operation; a row without such a partner is a single.
void build_full_pair_ops(std::vector<uint32_t>* ops, std::vector<int32_t>* off);

// Compiled width grid matching `widths`, or kWidthsGeneral.
int32_t width_set_of(const int32_t* widths, int32_t n);

// Start row and size of node `node` at depth d of the m-row tree.
void node_geometry(int64_t m, int d, int64_t node, int64_t* r0, int64_t* n);

// Source rows of a range tile: rows [s0, s1) of node `node` at depth d_dst of
// the m-row tree are built from rows of its descendants `levels` levels
// below. Appends those rows (rows of the transform) to `out` in the order
// the tile keeps them in LDS: the descendants left to right, each one's rows
// ascending. Returns their count.
int32_t range_tile_source_rows(int64_t m, int d_dst, int64_t node, int64_t s0, int64_t s1,
                               int levels, std::vector<int32_t>* out);

// Sets rows_off of every range tile of `tiles` (transform table `xf`) to the
// position in `table` of its source-row list, stored as the count followed by
// the rows; tiles of the same geometry share one list. Full tiles get -1.
void attach_source_rows(std::vector<TileDesc>* tiles, const XformDesc* xf,
                        std::vector<int32_t>* table);

}  // namespace ffa
