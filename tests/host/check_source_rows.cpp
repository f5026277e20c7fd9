// Host checks of the tile plan.
//
// 1. The range tiles' source-row lists (range_tile_source_rows) against a
//    step-by-step emulation of the kernel's node metadata: for random trees,
//    tiles and depths, the rows each node of the bottom level keeps, in the
//    order the metadata places them in LDS (nodes left to right, rows
//    ascending), must be the host's list, and every row must lie in the tree.
// 2. Every tile the planner emits fits the workgroup's LDS: over a grid of
//    (m, p, tiling), a full tile holds at most rows_capacity rows, and a range
//    tile keeps at most rows_capacity rows at every level of its subtree and
//    at most kSnrLdsBytes of pair-operation records (kOpInts ints each).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "ffa_plan.hpp"
using namespace ffa;

static void merge_idx(int n, int s, int& i, int& j) {
  int mh = n >> 1, mt = n - mh;
  long long den = 2LL * (n - 1);
  i = (int)((2LL * (mh - 1) * s + (n - 1)) / den);
  j = (int)((2LL * (mt - 1) * s + (n - 1)) / den);
}

static int pair_ops(int n, int lo, int hi) {
  if (hi <= lo || n <= 0) return 0;
  if (n == 1) return 1;
  const int lead = ((lo & 1) != (n & 1)) ? 1 : 0;
  const int rem = hi - lo - lead;
  return lead + (rem >> 1) + (rem & 1);
}

// The kernel's metadata: every node of the subtree walks its path from the
// tile's node, taking at each merge the head or tail rows it reads.
struct Meta {
  std::vector<int> r0, n, lo, hi;
};
static Meta emulate(int64_t r0, int64_t n, int s0, int s1, int L) {
  const int nn = (2 << L) - 1;
  Meta M;
  M.r0.resize(nn);
  M.n.resize(nn);
  M.lo.resize(nn);
  M.hi.resize(nn);
  for (int lane = 0; lane < nn; ++lane) {
    int lv = 31 - __builtin_clz(lane + 1);
    int v = lane + 1 - (1 << lv);
    int a0 = (int)r0, an = (int)n, alo = s0, ahi = s1;
    for (int b = lv - 1; b >= 0; --b) {
      bool right = (v >> b) & 1;
      if (ahi <= alo || an == 0) {
        an = 0;
        alo = ahi = 0;
      } else if (an == 1) {
        an = right ? 1 : 0;
        alo = 0;
        ahi = right ? 1 : 0;
      } else {
        int mh = an >> 1;
        int i0, j0, i1, j1;
        merge_idx(an, alo, i0, j0);
        merge_idx(an, ahi - 1, i1, j1);
        int c0 = right ? j0 : i0, c1 = right ? j1 : i1;
        if (right) a0 += mh;
        an = right ? an - mh : mh;
        alo = c0;
        ahi = c1 + 1;
      }
    }
    M.r0[lane] = a0;
    M.n[lane] = an;
    M.lo[lane] = alo;
    M.hi[lane] = ahi;
  }
  return M;
}

static int check_lists() {
  std::mt19937 g(7);
  long checked = 0;
  for (int it = 0; it < 60000; ++it) {
    int m = 2 + g() % 50000;
    int L = 1 + g() % 5;
    int d = g() % 8;
    if ((m >> d) < 2) continue;
    int node = g() % (1 << d);
    int64_t r0, n;
    node_geometry(m, d, node, &r0, &n);
    if (n < 1) continue;
    int s0 = g() % n, s1 = s0 + 1 + g() % (n - s0);
    const Meta M = emulate(r0, n, s0, s1, L);
    std::vector<int> th;
    for (int v = 0; v < (1 << L); ++v) {
      int h = (1 << L) - 1 + v;
      for (int k = M.lo[h]; k < M.hi[h]; ++k) th.push_back(M.r0[h] + k);
    }
    std::vector<int32_t> host;
    int cnt = range_tile_source_rows(m, d, node, s0, s1, L, &host);
    if (cnt != (int)th.size() || host.size() != th.size()) {
      printf("count mismatch m=%d d=%d node=%d s=[%d,%d) L=%d: %d vs %zu\n", m, d, node, s0, s1, L,
             cnt, th.size());
      return 1;
    }
    for (size_t q = 0; q < th.size(); ++q) {
      if (host[q] != th[q]) {
        printf("row mismatch at %zu\n", q);
        return 1;
      }
      if (host[q] < 0 || host[q] >= m) {
        printf("row out of range\n");
        return 1;
      }
    }
    ++checked;
  }
  printf("ok: %ld tiles\n", checked);
  return 0;
}

constexpr int kOpBytes = kOpInts * 4;

static int check_plan_fits() {
  int max_range_ops = 0;
  std::vector<std::pair<int, int>> shapes = {
      {200, 1280}, {500, 600}, {497, 519}, {1000, 1000}, {300, 1280}, {500, 1000}, {1073, 259},
      {1500, 61},  {12000, 33}, {2048, 128}, {42406, 259}, {4000, 700}, {900, 1100}, {3, 1280}};
  std::mt19937 g(11);
  for (int q = 0; q < 60; ++q) shapes.push_back({2 + (int)(g() % 20000), 2 + (int)(g() % 1279)});
  long tiles = 0;
  for (auto [m, p] : shapes) {
    for (int waves : {kWavesSmall, kWavesLarge})
      for (int range_waves : {0, kWavesSmall + kWavesLarge - waves})
      for (int lds_rows : {0, 16, 24, 40})
        for (int levels = 1; levels <= kMaxRangeLevels; ++levels) {
          if ((int64_t)m * p > (int64_t(1) << 31)) continue;
          Tiling t;
          t.waves = waves;
          t.range_waves = range_waves;
          t.lds_rows = lds_rows;
          t.levels_per_pass = levels;
          const int R = rows_capacity(p, t), Rr = range_rows_capacity(p, t);
          std::vector<std::vector<TileDesc>> passes;
          if (!plan_transform_tiles(0, m, p, m, R, Rr, levels, false, &passes)) {
            printf("plan refused m=%d p=%d R=%d levels=%d\n", m, p, R, levels);
            return 1;
          }
          for (const auto& ps : passes)
            for (const TileDesc& tl : ps) {
              ++tiles;
              if (tl.flags & kTileFull) {
                if (tl.s1 > R) {
                  printf("full tile of %d rows > %d (m=%d p=%d)\n", tl.s1, R, m, p);
                  return 1;
                }
                continue;
              }
              int64_t r0, n;
              node_geometry(m, tl.d_dst, tl.node, &r0, &n);
              const Meta M = emulate(r0, n, tl.s0, tl.s1, tl.levels);
              int ops = 0;
              for (int l = 0; l <= tl.levels; ++l) {
                int rows = 0;
                for (int v = 0; v < (1 << l); ++v) {
                  const int h = (1 << l) - 1 + v;
                  rows += M.hi[h] - M.lo[h];
                  if (l < tl.levels) ops += pair_ops(M.n[h], M.lo[h], M.hi[h]);
                }
                if (rows > Rr) {
                  printf("range tile keeps %d rows > %d at level %d (m=%d p=%d L=%d)\n", rows, Rr,
                         l, m, p, tl.levels);
                  return 1;
                }
              }
              max_range_ops = std::max(max_range_ops, ops);
              if (ops * kOpBytes > kSnrLdsBytes) {
                printf("range tile has %d pair operations (m=%d p=%d)\n", ops, m, p);
                return 1;
              }
            }
        }
  }
  printf("ok: %ld planned tiles fit (most pair operations of a range tile %d, room for %d)\n",
         tiles, max_range_ops, kSnrLdsBytes / kOpBytes);
  return 0;
}

int main() {
  if (check_lists()) return 1;
  return check_plan_fits();
}
