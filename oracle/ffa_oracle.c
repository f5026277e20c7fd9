/*
 * FP64 CPU oracle for the FFA periodicity search (Morello et al. 2020).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The GPU product path
 * never links, loads or calls it, and it shares no code with that path.
 *
 * Every routine here is the plain definition of a step, written for a reader
 * to check against the paper by eye: no blocking, no fusion, no reordering.
 * All arithmetic on sample values is double precision.
 *
 * Readings of the paper used here, where it is silent or ambiguous:
 *   - head/tail split of an n-row block: m_h = floor(n/2), m_t = n - m_h
 *     (Sec. 2.2 only asks for "similarly sized" blocks);
 *   - nearest-integer rounding of i and j is half-up, evaluated in exact
 *     integer arithmetic (Sec. 2.2, equation for i and j);
 *   - "T << k" is a left rotation: (T << k)[n] = T[(n + k) mod p]
 *     (Sec. 2.2, merge rule; Fig. 1 shows paths drifting to the right);
 *   - the boxcar S/N divides the best circular boxcar sum by
 *     sqrt(m * w * var), var being the per-sample variance of the
 *     (downsampled) series (Sec. 5.4; Sec. 3.3 for the unit-norm template).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* i(s) and j(s) of the merge rule for an n-row block (Sec. 2.2):
 * i = nint((m_h - 1) s / (n - 1)), j = nint((m_t - 1) s / (n - 1)),
 * half-up: nint(a/c) = floor((2a + c) / (2c)) for a, c >= 0. */
static void split_indices(int64_t n, int64_t s, int64_t* i, int64_t* j) {
  int64_t mh = n / 2, mt = n - mh;
  *i = (2 * (mh - 1) * s + (n - 1)) / (2 * (n - 1));
  *j = (2 * (mt - 1) * s + (n - 1)) / (2 * (n - 1));
}

/* D_m(s, r): phase offset (in bins) at which the integration path with total
 * drift s picks up row r of an m-row block. It follows from unrolling the
 * merge rule F_s = H_i + (T_j << (i + b)), b = s - (i + j): rows of the head
 * are reached through H_i, rows of the tail through T_j after a rotation by
 * i + b = s - j (Sec. 2.2). A single-row block is its own transform. */
int64_t oracle_path_offset(int64_t m, int64_t s, int64_t r) {
  int64_t acc = 0;
  while (m > 1) {
    int64_t mh = m / 2, i, j;
    split_indices(m, s, &i, &j);
    if (r < mh) {
      m = mh;
      s = i;
    } else {
      acc += s - j;
      r -= mh;
      m = m - mh;
      s = j;
    }
  }
  return acc;
}

/* Full m x m table of path offsets, D[s*m + r]. */
void oracle_path_table(int64_t m, int64_t* D) {
  for (int64_t s = 0; s < m; ++s)
    for (int64_t r = 0; r < m; ++r) D[s * m + r] = oracle_path_offset(m, s, r);
}

/* Folding transform by brute force (Sec. 2.1): row s integrates the m input
 * rows of X (m x p, row-major) along path s,
 *   F[s][n] = sum_r X[r][(n + D_m(s, r)) mod p].
 * O(p m^2) additions; rows summed in order r = 0..m-1. */
static void fold_bruteforce_rows(const double* X, int64_t m, int64_t p, int64_t s0, int64_t s1,
                                 double* F) {
  for (int64_t s = s0; s < s1; ++s) {
    double* out = F + s * p;
    for (int64_t n = 0; n < p; ++n) out[n] = 0.0;
    for (int64_t r = 0; r < m; ++r) {
      int64_t d = oracle_path_offset(m, s, r) % p;
      const double* row = X + r * p;
      for (int64_t n = 0; n < p; ++n) {
        int64_t c = n + d;
        if (c >= p) c -= p;
        out[n] += row[c];
      }
    }
  }
}

void oracle_fold_bruteforce(const double* X, int64_t m, int64_t p, double* F) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t s = 0; s < m; ++s) fold_bruteforce_rows(X, m, p, s, s + 1, F);
}

/* Depth-first FFA (Sec. 2.2): transform the head rows, then the tail rows,
 * then combine with F_s = H_i + (T_j << (s - j)). A one-row block is copied.
 * `work` must hold n*p doubles; the result is written to F (n x p). */
static void ffa_recursive(const double* X, int64_t n, int64_t p, double* F, double* work) {
  if (n == 1) {
    memcpy(F, X, (size_t)p * sizeof(double));
    return;
  }
  int64_t mh = n / 2, mt = n - mh;
  double* H = work;           /* mh x p */
  double* T = work + mh * p;  /* mt x p */
  /* F serves as the children's work space: it is overwritten below. */
  ffa_recursive(X, mh, p, H, F);
  ffa_recursive(X + mh * p, mt, p, T, F + mh * p);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i, j;
    split_indices(n, s, &i, &j);
    int64_t k = (s - j) % p;
    const double* h = H + i * p;
    const double* t = T + j * p;
    double* out = F + s * p;
    for (int64_t c = 0; c < p; ++c) {
      int64_t q = c + k;
      if (q >= p) q -= p;
      out[c] = h[c] + t[q];
    }
  }
}

/* Folding transform by the depth-first FFA. Returns 0, or -1 on allocation failure. */
int oracle_fold_ffa(const double* X, int64_t m, int64_t p, double* F) {
  double* work = (double*)malloc((size_t)(m * p) * sizeof(double));
  if (!work) return -1;
  ffa_recursive(X, m, p, F, work);
  free(work);
  return 0;
}

/* Downsampling by a real factor (Sec. 5.3 and App. A.4). The factor is
 * ds_fx / 2^32 input samples per output sample (32.32 fixed point), so window
 * edges are exact integers in units of 2^-32 samples. Output j integrates
 * the window [j ds, (j+1) ds); input sample i covers [i, i+1) and is weighted
 * by the length of its overlap with the window. */
void oracle_downsample(const double* x, int64_t n, uint64_t ds_fx, int64_t nout, double* y) {
  const uint64_t ONE = (uint64_t)1 << 32;
  const double scale = 1.0 / 4294967296.0;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nout; ++j) {
    uint64_t a = (uint64_t)j * ds_fx, b = (uint64_t)(j + 1) * ds_fx;
    double acc = 0.0;
    for (int64_t i = (int64_t)(a >> 32); i < n && (uint64_t)i * ONE < b; ++i) {
      uint64_t lo = (uint64_t)i * ONE, hi = lo + ONE;
      if (lo < a) lo = a;
      if (hi > b) hi = b;
      acc += (double)(hi - lo) * scale * x[i];
    }
    y[j] = acc;
  }
}

/* Boxcar matched-filter S/N of one profile P of p bins (Sec. 5.4): the
 * exclusive prefix sum S over two repeats of P gives every circular boxcar sum
 * C_n = S_{n+w} - S_n; the S/N for width w is max_n C_n / sqrt(m * w * var),
 * the boxcar having unit square sum over the m folded periods (Sec. 3.3).
 * S must hold 2p + 1 doubles. Requires w <= p. */
static void profile_snr(const double* P, int64_t p, int64_t m, double var, const int32_t* widths,
                        int32_t nw, double* S, double* out) {
  S[0] = 0.0;
  for (int64_t t = 0; t < 2 * p; ++t) S[t + 1] = S[t] + P[t % p];
  for (int32_t q = 0; q < nw; ++q) {
    int64_t w = widths[q];
    double best = -INFINITY;
    for (int64_t n0 = 0; n0 < p; ++n0) {
      double c = S[n0 + w] - S[n0];
      if (c > best) best = c;
    }
    out[q] = best / sqrt((double)m * (double)w * var);
  }
}

/* S/N of `rows` profiles (rows x p, row-major); out is rows x nw. */
void oracle_boxcar_snr(const double* F, int64_t rows, int64_t p, int64_t m, double var,
                       const int32_t* widths, int32_t nw, double* out) {
#pragma omp parallel
  {
    double* S = (double*)malloc((size_t)(2 * p + 1) * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t r = 0; r < rows; ++r) profile_snr(F + r * p, p, m, var, widths, nw, S, out + r * nw);
    free(S);
  }
}

/* Many transforms of one downsampled series, parallel over transforms:
 * transform q folds y + y_off[q] as m[q] x p[q] rows (by the FFA, or by brute
 * force when `brute` is set) and writes the S/N of its first keep[q] rows at
 * out + out_off[q] * nw. Returns 0, or -1 on allocation failure. */
int oracle_transforms_snr(const double* y, int64_t ntr, const int64_t* y_off, const int64_t* m,
                          const int64_t* p, const double* var, const int64_t* keep,
                          const int64_t* out_off, int32_t brute, const int32_t* widths, int32_t nw,
                          double* out) {
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t q = 0; q < ntr; ++q) {
    size_t cells = (size_t)(m[q] * p[q]);
    double* F = (double*)malloc(cells * sizeof(double));
    double* work = (double*)malloc(cells * sizeof(double));
    double* S = (double*)malloc((size_t)(2 * p[q] + 1) * sizeof(double));
    if (!F || !work || !S) {
      err |= 1;
    } else {
      if (brute)
        fold_bruteforce_rows(y + y_off[q], m[q], p[q], 0, m[q], F);
      else
        ffa_recursive(y + y_off[q], m[q], p[q], F, work);
      for (int64_t r = 0; r < keep[q]; ++r)
        profile_snr(F + r * p[q], p[q], m[q], var[q], widths, nw, S, out + (out_off[q] + r) * nw);
    }
    free(S);
    free(work);
    free(F);
  }
  return err ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * De-reddening by a running median (Sec. 5.2). Output i is x[i] minus the
 * median of the samples in the window of `window` (odd) samples centred on
 * i, the window cut at the ends of the series; the median of n samples is
 * their k-th smallest value, k = (n - 1) / 2 (0-based; for even n, at the
 * ends, the lower of the two middle values). The k-th smallest is found by
 * the textbook order-statistic method: every sample gets its rank in the
 * sort of the whole series by (value, index); a Fenwick tree counts the
 * ranks present in the window; the k-th present rank is found by descending
 * the tree.
 * ------------------------------------------------------------------------ */

static const double* g_sort_x;

static int cmp_value_index(const void* a, const void* b) {
  const int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
  const double xi = g_sort_x[i], xj = g_sort_x[j];
  if (xi < xj) return -1;
  if (xi > xj) return 1;
  return (i > j) - (i < j);
}

static void bit_add(int32_t* tree, int64_t n, int64_t pos, int32_t d) {
  for (int64_t q = pos + 1; q <= n; q += q & (-q)) tree[q] += d;
}

/* Smallest 0-based position whose prefix count reaches k + 1. */
static int64_t bit_kth(const int32_t* tree, int64_t n, int64_t k) {
  int64_t pos = 0, step = 1;
  while (step * 2 <= n) step *= 2;
  int64_t rem = k + 1;
  for (; step > 0; step /= 2) {
    if (pos + step <= n && tree[pos + step] < rem) {
      pos += step;
      rem -= tree[pos];
    }
  }
  return pos;  /* 1-based position pos + 1, i.e. 0-based pos */
}

/* med[i] = median of the window of output i; y[i] = x[i] - med[i]. Returns
 * 0, or -1 on allocation failure. */
int oracle_running_median(const double* x, int64_t n, int64_t window, double* med, double* y) {
  if (n <= 0) return 0;
  const int64_t h = window / 2;
  int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* rank = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* tree = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  if (!order || !rank || !tree) {
    free(order);
    free(rank);
    free(tree);
    return -1;
  }
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  g_sort_x = x;
  qsort(order, (size_t)n, sizeof(int64_t), cmp_value_index);
  for (int64_t r = 0; r < n; ++r) rank[order[r]] = r;
  int64_t s = 0, e = 0; /* samples [s, e) are in the tree */
  for (int64_t i = 0; i < n; ++i) {
    const int64_t ws = i - h < 0 ? 0 : i - h;
    const int64_t we = i + h + 1 > n ? n : i + h + 1;
    while (e < we) bit_add(tree, n, rank[e++], 1);
    while (s < ws) bit_add(tree, n, rank[s++], -1);
    const int64_t cnt = we - ws;
    const int64_t r = bit_kth(tree, n, (cnt - 1) / 2);
    med[i] = x[order[r]];
    y[i] = x[i] - med[i];
  }
  free(order);
  free(rank);
  free(tree);
  return 0;
}
