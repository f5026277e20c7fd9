// Host check of the range tiles' source-row lists (range_tile_source_rows)
// against a step-by-step emulation of the kernel's node metadata: for random
// trees, tiles and depths, the rows each node of the bottom level keeps, in
// the order the metadata places them in LDS (nodes left to right, rows
// ascending), must be the host's list, and every row must lie in the tree.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <random>
#include "ffa_plan.hpp"
using namespace ffa;
static void merge_idx(int n, int s, int& i, int& j) {
  int mh = n >> 1, mt = n - mh;
  long long den = 2LL * (n - 1);
  i = (int)((2LL * (mh - 1) * s + (n - 1)) / den);
  j = (int)((2LL * (mt - 1) * s + (n - 1)) / den);
}
int main() {
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
    // the kernel's metadata: every node of the subtree walks its path from
    // the tile's node, taking at each merge the head or tail rows it reads
    int nn = (2 << L) - 1;
    std::vector<int> hr0(nn), hn(nn), hlo(nn), hhi(nn), lev(nn);
    for (int lane = 0; lane < nn; ++lane) {
      int lv = 31 - __builtin_clz(lane + 1);
      int v = lane + 1 - (1 << lv);
      int a0 = (int)r0, an = (int)n, alo = s0, ahi = s1;
      for (int b = lv - 1; b >= 0; --b) {
        bool right = (v >> b) & 1;
        if (ahi <= alo || an == 0) { an = 0; alo = ahi = 0; }
        else if (an == 1) { an = right ? 1 : 0; alo = 0; ahi = right ? 1 : 0; }
        else {
          int mh = an >> 1;
          int i0, j0, i1, j1;
          merge_idx(an, alo, i0, j0);
          merge_idx(an, ahi - 1, i1, j1);
          int c0 = right ? j0 : i0, c1 = right ? j1 : i1;
          if (right) a0 += mh;
          an = right ? an - mh : mh;
          alo = c0; ahi = c1 + 1;
        }
      }
      hr0[lane] = a0; hn[lane] = an; hlo[lane] = alo; hhi[lane] = ahi; lev[lane] = lv;
    }
    std::vector<int> th;
    for (int v = 0; v < (1 << L); ++v) {
      int h = (1 << L) - 1 + v;
      for (int k = hlo[h]; k < hhi[h]; ++k) th.push_back(hr0[h] + k);
    }
    std::vector<int32_t> host;
    int cnt = range_tile_source_rows(m, d, node, s0, s1, L, &host);
    if (cnt != (int)th.size() || host.size() != th.size()) { printf("count mismatch m=%d d=%d node=%d s=[%d,%d) L=%d: %d vs %zu\n", m, d, node, s0, s1, L, cnt, th.size()); return 1; }
    for (size_t q = 0; q < th.size(); ++q) {
      if (host[q] != th[q]) { printf("row mismatch at %zu\n", q); return 1; }
      if (host[q] < 0 || host[q] >= m) { printf("row out of range\n"); return 1; }
    }
    ++checked;
  }
  printf("ok: %ld tiles\n", checked);
  return 0;
}
