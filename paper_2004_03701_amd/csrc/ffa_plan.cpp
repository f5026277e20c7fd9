// Host-side period plan (Sec. 2.3, 5.3) and tile plan of the FFA search.
#include "ffa_plan.hpp"

#include <math.h>

#include <algorithm>
#include <map>
#include <sstream>

namespace ffa {

namespace {

constexpr uint64_t kOne = uint64_t(1) << 32;

// i(s), j(s) of the merge rule for an n-row block (Sec. 2.2), nearest integer
// with ties rounded up, in exact integer arithmetic.
inline void merge_indices(int64_t n, int64_t s, int64_t* i, int64_t* j) {
  int64_t mh = n / 2, mt = n - mh;
  *i = (2 * (mh - 1) * s + (n - 1)) / (2 * (n - 1));
  *j = (2 * (mt - 1) * s + (n - 1)) / (2 * (n - 1));
}

}  // namespace

double trial_period(int64_t s, int64_t m, int64_t p, double tau) {
  double num = tau * (double)p * (double)p;
  double den = (double)p - (double)s / (double)(m - 1);
  return num / den;
}

ffa_status validate_params(const ffa_search_params& a, std::string* err) {
  std::ostringstream msg;
  if (!(a.tsamp > 0.0) || !isfinite(a.tsamp)) {
    *err = "tsamp must be positive and finite";
    return FFA_ERR_INVALID_ARG;
  }
  if (!(a.period_min > 0.0) || !(a.period_max > a.period_min) || !isfinite(a.period_max)) {
    *err = "need 0 < period_min < period_max < inf";
    return FFA_ERR_INVALID_ARG;
  }
  if (a.bins_min < 2 || a.bins_max < a.bins_min || a.bins_max > kMaxBins) {
    msg << "need 2 <= bins_min <= bins_max <= " << kMaxBins;
    *err = msg.str();
    return FFA_ERR_INVALID_ARG;
  }
  if (!a.widths || a.num_widths < 1 || a.num_widths > kMaxWidths) {
    msg << "need a widths array of 1.." << kMaxWidths << " entries";
    *err = msg.str();
    return FFA_ERR_INVALID_ARG;
  }
  for (int q = 0; q < a.num_widths; ++q) {
    if (a.widths[q] < 1 || a.widths[q] >= a.bins_min || (q > 0 && a.widths[q] <= a.widths[q - 1])) {
      *err = "widths must be strictly increasing with 1 <= w < bins_min";
      return FFA_ERR_INVALID_ARG;
    }
  }
  if (a.normalise != 0 && a.normalise != 1) {
    *err = "normalise must be 0 or 1";
    return FFA_ERR_INVALID_ARG;
  }
  if (a.dtype != FFA_F32 && a.dtype != FFA_BF16 && a.dtype != FFA_F16) {
    *err = "unknown dtype";
    return FFA_ERR_INVALID_ARG;
  }
  if (a.median_window < 0 || (a.median_window > 0 && a.median_window % 2 == 0)) {
    *err = "median_window must be 0 (none) or odd";
    return FFA_ERR_INVALID_ARG;
  }
  return FFA_OK;
}

ffa_status build_series_plan(const ffa_search_params& a, int64_t nsamp, SeriesPlan* out,
                             std::string* err) {
  ffa_status st = validate_params(a, err);
  if (st != FFA_OK) return st;
  if (nsamp < 1 || nsamp > INT32_MAX) {
    *err = "nsamp must be in [1, 2^31)";
    return FFA_ERR_INVALID_ARG;
  }
  // Sec. 5.3: the first octave brings P_min to bins_min bins; later octaves
  // downsample the original series by a factor f = (bins_max + 1) / bins_min
  // more each, covering the base periods [bins_min, bins_max + 1) tau_k.
  double ds = a.period_min / ((double)a.bins_min * a.tsamp);
  if (!(ds >= 1.0)) {
    *err = "period_min / (bins_min * tsamp) < 1: the series is too coarsely sampled";
    return FFA_ERR_RANGE;
  }
  const double f = (double)(a.bins_max + 1) / (double)a.bins_min;
  SeriesPlan plan;
  for (int k = 0;; ++k) {
    const uint64_t ds_fx = (uint64_t)floor(ds * (double)kOne + 0.5);
    const double tau = a.tsamp * ((double)ds_fx / (double)kOne);
    if ((double)a.bins_min * tau >= a.period_max) break;
    Octave o;
    o.ds = ds;
    o.ds_fx = ds_fx;
    o.tau = tau;
    o.nsamp = (int64_t)(((uint64_t)nsamp << 32) / ds_fx);
    const double dsq = (double)ds_fx / (double)kOne;
    // App. A.4: variance f - 1/3 of unit-variance noise downsampled by a
    // non-integer factor f; f for an integer factor.
    o.var = (ds_fx % kOne == 0) ? dsq : dsq - 1.0 / 3.0;
    o.ds_off = plan.ds_total;
    bool any = false;
    for (int32_t p = a.bins_min; p <= a.bins_max; ++p) {
      if ((double)p * tau >= a.period_max) break;
      const int64_t m = o.nsamp / p;
      if (m < 2) continue;  // the period of row s divides by m - 1
      // Row s is kept while s (p + 1) < p (m - 1), i.e. P_s < (p + 1) tau, and
      // P_s < P_max. Both bounds grow with s, so the kept rows are a prefix.
      int64_t keep = 0;
      int64_t lim = (p * (m - 1) - 1) / (p + 1) + 1;  // rows with s (p+1) < p (m-1)
      lim = std::min<int64_t>(lim, m);
      // largest prefix with P_s < P_max (P_s increases with s)
      int64_t lo = 0, hi = lim;  // answer in [0, lim]
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;  // is row `mid` below P_max?
        if (trial_period(mid, m, p, tau) < a.period_max)
          lo = mid + 1;
        else
          hi = mid;
      }
      keep = lo;
      if (keep == 0) continue;
      Transform t;
      t.octave = k;
      t.p = p;
      t.m = (int32_t)m;
      t.keep = (int32_t)keep;
      t.row0 = plan.rows;
      plan.rows += keep;
      plan.cells += m * p;
      plan.tr.push_back(t);
      any = true;
    }
    if (any) {
      plan.ds_total += (o.nsamp + kDsGroup - 1) / kDsGroup * kDsGroup;
      plan.ds_samples += o.nsamp;
      plan.ds_fx_max = std::max(plan.ds_fx_max, ds_fx);
    } else {
      o.nsamp = 0;  // nothing folded: no downsampled series needed
    }
    plan.oct.push_back(o);
    ds = ds * f;
  }
  if (plan.tr.empty()) {
    *err = "no transform has m >= 2 rows: the series is too short for the period range";
    return FFA_ERR_RANGE;
  }
  *out = std::move(plan);
  return FFA_OK;
}

int32_t rows_capacity(int32_t p, const Tiling& t) {
  return ffa::rows_capacity(p, t.lds_rows, t.waves);
}

int32_t range_rows_capacity(int32_t p, const Tiling& t) {
  return ffa::rows_capacity(p, t.lds_rows, t.waves_of_range());
}

void node_geometry(int64_t m, int d, int64_t node, int64_t* r0, int64_t* n) {
  int64_t base = 0, size = m;
  for (int b = d - 1; b >= 0; --b) {
    int64_t mh = size / 2;
    if ((node >> b) & 1) {
      base += mh;
      size -= mh;
    } else {
      size = mh;
    }
  }
  *r0 = base;
  *n = size;
}

void build_full_schedules(std::vector<uint32_t>* ht, std::vector<uint16_t>* rot,
                          std::vector<int32_t>* off) {
  ht->clear();
  rot->clear();
  off->assign(kMaxFullRows + 1, 0);
  for (int n = 2; n <= kMaxFullRows; ++n) {
    (*off)[n] = (int32_t)ht->size();
    int levels = 0;
    while ((1 << levels) < n) ++levels;
    for (int lev = 0; lev < levels; ++lev) {
      for (int q = 0; q < n; ++q) {
        // block holding row q at relative depth lev
        int b0 = 0, sz = n;
        for (int k = 0; k < lev; ++k) {
          const int mh = sz / 2;
          if (q - b0 < mh) {
            sz = mh;
          } else {
            b0 += mh;
            sz -= mh;
          }
        }
        if (sz < 2) {
          ht->push_back((uint32_t)q | (0xffffu << 16));
          rot->push_back(0);
        } else {
          const int s = q - b0, mh = sz / 2;
          int64_t i, j;
          merge_indices(sz, s, &i, &j);
          ht->push_back((uint32_t)(b0 + i) | ((uint32_t)(b0 + mh + j) << 16));
          rot->push_back((uint16_t)(s - j));
        }
      }
    }
  }
}

void build_full_pair_ops(std::vector<uint32_t>* ops, std::vector<int32_t>* off) {
  constexpr int K = kMaxFullLevels + 1;
  ops->clear();
  off->assign((size_t)(kMaxFullRows + 1) * K, 0);
  for (int n = 2; n <= kMaxFullRows; ++n) {
    int levels = 0;
    while ((1 << levels) < n) ++levels;
    for (int lev = 0; lev < K; ++lev) {
      (*off)[(size_t)n * K + lev] = (int32_t)(ops->size() / 2);
      if (lev >= levels) continue;
      for (int64_t b = 0; b < ((int64_t)1 << lev); ++b) {
        int64_t b0, sz;
        node_geometry(n, lev, b, &b0, &sz);
        if (sz < 2) continue;  // a one-row block stays in place
        const int64_t mh = sz / 2;
        int64_t s = 0;
        while (s < sz) {
          int64_t i, j, i2 = -1, j2 = -1;
          merge_indices(sz, s, &i, &j);
          if (s + 1 < sz) merge_indices(sz, s + 1, &i2, &j2);
          const bool pair = s + 1 < sz && j2 == j;
          const uint32_t w0 = (uint32_t)(b0 + s) | ((uint32_t)(b0 + i) << 8) |
                              ((uint32_t)(b0 + (pair ? i2 : i)) << 16) |
                              ((uint32_t)(b0 + mh + j) << 24);
          const uint32_t w1 = (uint32_t)(s - j) | (pair ? 0u : (1u << 16));
          ops->push_back(w0);
          ops->push_back(w1);
          s += pair ? 2 : 1;
        }
      }
    }
  }
}

int32_t width_set_of(const int32_t* w, int32_t n) {
  static const int32_t paper[9] = {1, 2, 3, 4, 6, 9, 13, 19, 28};
  static const int32_t duty[9] = {1, 2, 3, 5, 8, 12, 19, 30, 48};
  if (n == 9 && std::equal(w, w + 9, paper)) return kWidthsPaper9;
  if (n == 9 && std::equal(w, w + 9, duty)) return kWidthsDuty9;
  return kWidthsGeneral;
}

namespace {

// Rows needed at each of the `levels` levels below a node of n rows to
// produce its rows [lo, hi); tot[l] accumulates the count at level l.
void range_rows(int64_t n, int64_t lo, int64_t hi, int levels, int l, int64_t* tot) {
  tot[l] += hi - lo;
  if (l == levels || hi <= lo) return;
  if (n <= 1) {  // a one-row block is its own transform
    if (n == 1) range_rows(1, 0, 1, levels, l + 1, tot);
    return;
  }
  int64_t mh = n / 2, mt = n - mh, i0, j0, i1, j1;
  merge_indices(n, lo, &i0, &j0);
  merge_indices(n, hi - 1, &i1, &j1);
  range_rows(mh, i0, i1 + 1, levels, l + 1, tot);
  range_rows(mt, j0, j1 + 1, levels, l + 1, tot);
}

int64_t range_peak_rows(int64_t n, int64_t lo, int64_t hi, int levels) {
  int64_t tot[kMaxRangeLevels + 1] = {0};
  range_rows(n, lo, hi, levels, 0, tot);
  int64_t mx = 0;
  for (int l = 0; l <= levels; ++l) mx = std::max(mx, tot[l]);
  return mx;
}

// Pair operations that make rows [lo, hi) of an n-row node: rows s and s + 1
// share their tail row when s has the parity of n, so a leading row of the
// other parity and a trailing unpaired row are singles; a one-row block is
// one copy.
int64_t node_pair_ops(int64_t n, int64_t lo, int64_t hi) {
  if (hi <= lo || n <= 0) return 0;
  if (n == 1) return 1;
  const int64_t lead = ((lo & 1) != (n & 1)) ? 1 : 0;
  const int64_t rem = hi - lo - lead;
  return lead + (rem >> 1) + (rem & 1);
}

// Pair operations of every merge level of a range tile (rows [lo, hi) of an
// n-row node from the rows `levels` levels below).
int64_t range_ops(int64_t n, int64_t lo, int64_t hi, int levels) {
  if (levels == 0 || hi <= lo) return 0;
  int64_t ops = node_pair_ops(n, lo, hi);
  if (n <= 1) {
    if (n == 1) ops += range_ops(1, 0, 1, levels - 1);
    return ops;
  }
  int64_t mh = n / 2, mt = n - mh, i0, j0, i1, j1;
  merge_indices(n, lo, &i0, &j0);
  merge_indices(n, hi - 1, &i1, &j1);
  return ops + range_ops(mh, i0, i1 + 1, levels - 1) + range_ops(mt, j0, j1 + 1, levels - 1);
}

// Whether a range tile's rows fit the tile at every level and its pair
// operations fit the record area.
bool range_fits(int64_t n, int64_t lo, int64_t hi, int levels, int64_t rows_cap) {
  return range_peak_rows(n, lo, hi, levels) <= rows_cap &&
         range_ops(n, lo, hi, levels) <= kMaxTileOps;
}

}  // namespace

namespace {

// Walks the nodes below a node (r0, n rows, rows [lo, hi) wanted) down to
// `levels` levels, left child first, appending the rows wanted at the bottom.
// The children of a merge take the head and tail rows the wanted rows read
// (Sec. 2.2); a one-row block's tail child is the row itself.
void source_rows_rec(int64_t r0, int64_t n, int64_t lo, int64_t hi, int l, int levels,
                     std::vector<int32_t>* out) {
  if (l == levels) {
    for (int64_t k = lo; k < hi; ++k) out->push_back((int32_t)(r0 + k));
    return;
  }
  if (hi <= lo || n == 0) {
    source_rows_rec(r0, 0, 0, 0, l + 1, levels, out);
    source_rows_rec(r0, 0, 0, 0, l + 1, levels, out);
    return;
  }
  if (n == 1) {
    source_rows_rec(r0, 0, 0, 0, l + 1, levels, out);
    source_rows_rec(r0, 1, 0, 1, l + 1, levels, out);
    return;
  }
  const int64_t mh = n / 2;
  int64_t i0, j0, i1, j1;
  merge_indices(n, lo, &i0, &j0);
  merge_indices(n, hi - 1, &i1, &j1);
  source_rows_rec(r0, mh, i0, i1 + 1, l + 1, levels, out);
  source_rows_rec(r0 + mh, n - mh, j0, j1 + 1, l + 1, levels, out);
}

}  // namespace

int32_t range_tile_source_rows(int64_t m, int d_dst, int64_t node, int64_t s0, int64_t s1,
                               int levels, std::vector<int32_t>* out) {
  int64_t r0, n;
  node_geometry(m, d_dst, node, &r0, &n);
  const size_t before = out->size();
  source_rows_rec(r0, n, s0, s1, 0, levels, out);
  return (int32_t)(out->size() - before);
}

void attach_source_rows(std::vector<TileDesc>* tiles, const XformDesc* xf,
                        std::vector<int32_t>* table) {
  struct Key {
    int64_t m, node, s0, s1;
    int32_t d, levels;
    bool operator<(const Key& o) const {
      if (m != o.m) return m < o.m;
      if (node != o.node) return node < o.node;
      if (s0 != o.s0) return s0 < o.s0;
      if (s1 != o.s1) return s1 < o.s1;
      if (d != o.d) return d < o.d;
      return levels < o.levels;
    }
  };
  std::map<Key, int32_t> seen;
  std::vector<int32_t> rows;
  for (TileDesc& t : *tiles) {
    t.rows_off = -1;
    if (t.flags & kTileFull) continue;
    const Key k{xf[t.xf].m, t.node, t.s0, t.s1, t.d_dst, t.levels};
    auto it = seen.find(k);
    if (it != seen.end()) {
      t.rows_off = it->second;
      continue;
    }
    rows.clear();
    const int32_t cnt = range_tile_source_rows(k.m, t.d_dst, t.node, t.s0, t.s1, t.levels, &rows);
    t.rows_off = (int32_t)table->size();
    table->push_back(cnt);
    table->insert(table->end(), rows.begin(), rows.end());
    seen.emplace(k, t.rows_off);
  }
}

bool plan_transform_tiles(int32_t xf, int32_t m, int32_t p, int32_t keep, int32_t rows_cap,
                          int32_t range_rows_cap, int32_t levels_per_pass, bool out_rows,
                          std::vector<std::vector<TileDesc>>* passes) {
  (void)p;
  if (rows_cap < 2 || range_rows_cap < 2) return false;
  auto pass = [&](size_t k) -> std::vector<TileDesc>& {
    if (passes->size() <= k) passes->resize(k + 1);
    return (*passes)[k];
  };
  const uint8_t fin = kTileFinal | (out_rows ? kTileOutRows : 0);
  if (m <= rows_cap) {
    TileDesc t{xf, 0, 0, m, 0, 0, (uint8_t)(kTileFull | fin), 0, -1, -1};
    pass(0).push_back(t);
    return true;
  }
  // bottom depth: the shallowest whose nodes fit in LDS
  int db = 0;
  while ((((int64_t)m + (int64_t(1) << db) - 1) >> db) > rows_cap) ++db;
  for (int64_t nd = 0; nd < (int64_t(1) << db); ++nd) {
    int64_t r0, n;
    node_geometry(m, db, nd, &r0, &n);
    TileDesc t{xf, (int32_t)nd, 0, (int32_t)n, (uint8_t)db, 0, kTileFull, 0 /* writes buffer 0 */,
               -1, -1};
    pass(0).push_back(t);
  }
  // one output row of an L-level range tile reads up to 2^L rows at the
  // bottom level, so the levels of a pass are capped where 2^L <= rows_cap
  int L = std::max(1, std::min<int>(levels_per_pass, kMaxRangeLevels));
  while (L > 1 && (1 << L) > range_rows_cap) --L;
  const int npu = (db + L - 1) / L;
  int d_src = db;
  for (int k = 0; k < npu; ++k) {
    const int lv = db / npu + (k < db % npu ? 1 : 0);
    const int d_dst = d_src - lv;
    const bool last = (k == npu - 1);
    const int rd = k % 2, wr = (k + 1) % 2;
    for (int64_t nd = 0; nd < (int64_t(1) << d_dst); ++nd) {
      int64_t r0, n;
      node_geometry(m, d_dst, nd, &r0, &n);
      const int64_t end = last ? keep : n;
      int64_t s0 = 0;
      while (s0 < end) {
        if (!range_fits(n, s0, s0 + 1, lv, range_rows_cap)) return false;
        // largest s1 whose rows fit at every level of the pass
        int64_t lo = s0 + 1, hi = end;
        while (lo < hi) {
          int64_t mid = (lo + hi + 1) / 2;
          if (range_fits(n, s0, mid, lv, range_rows_cap))
            lo = mid;
          else
            hi = mid - 1;
        }
        TileDesc t{xf, (int32_t)nd, (int32_t)s0, (int32_t)lo, (uint8_t)d_dst, (uint8_t)lv,
                   (uint8_t)(last ? fin : 0), (uint8_t)(rd | (wr << 1)), -1, -1};
        pass(k + 1).push_back(t);
        s0 = lo;
      }
    }
    d_src = d_dst;
  }
  return true;
}

}  // namespace ffa
