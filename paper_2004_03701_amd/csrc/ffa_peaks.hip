// Periodogram peak detection (Sec. 5.5). Every width trial of the
// periodogram is searched on its own: its S/N against trial frequency is cut
// into equal frequency segments; each segment gives a control point (median
// + k IQR / 1.349 at the segment's centre frequency); a polynomial in
// log(frequency) fitted to the control points by least squares is the
// selection threshold, and the points above it are clustered into peaks.
//
// Three steps:
//   k_peak_ctrl_seg (k_peak_ctrl_wave) / k_peak_ctrl_pair / k_peak_ctrl
//                the control points: one wave (segments of up to 1024 rows,
//                sorted in registers; one workgroup takes every width of a
//                segment when there are at most 12), two waves (up to 2048 rows, one stage
//                through LDS) or one workgroup (larger segments, sorted in
//                LDS) per (series, segment, width) sorts the segment's S/N
//                values with a bitonic network and reads the quantiles from
//                the order statistics;
//   k_peak_fit   one wave per (series, width): power sums of the control
//                points on a centred and scaled abscissa, reduced across the
//                wave, and the normal equations solved in FP64;
//   k_peak_flag / k_peak_cluster
//                every row's thresholds, the rows above them as one bit per
//                (row, width) from wave ballots (the S/N read as whole rows,
//                transposed through LDS); then one wave per (series,
//                width) lists the set rows in row (= frequency) order and
//                one lane walks them forming the clusters.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ffa_kernels.hpp"
#include "ffa_peaks.hpp"

namespace ffa {
namespace {

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Quantile f of n sorted values by linear interpolation between the order
// statistics around position f (n - 1).
__device__ __forceinline__ double quantile_sorted(const float* v, int n, double f) {
  const double pos = f * (n - 1);
  const int lo = (int)floor(pos);
  const int hi = lo + 1 < n ? lo + 1 : lo;
  const double t = pos - lo;
  const double a = v[lo], b = v[hi];
  return a + (b - a) * t;
}

// Segments of at most kWaveSortMax rows: one wave per (series, segment,
// width) sorts the values in registers, 16 per lane, with a bitonic network
// (exchanges inside a lane for partner distances below 16, across lanes with
// shuffles above); padding with +inf keeps the network fixed. Element e of
// the sorted order sits in register e % 16 of lane e / 16.
constexpr int kWaveSortMax = kPeakWaveSortMax;

template <int kCtrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, false));
}

// The value of lane ^ D: quad permutations for D = 1, 2, row shifts for
// 4, 8, a swizzle within 32 lanes for 16, a permute for 32.
template <int D>
__device__ __forceinline__ float from_lane_xor(float x, int lane) {
  if constexpr (D == 1) return dpp_move<0xb1>(x);  // quad_perm [1, 0, 3, 2]
  else if constexpr (D == 2) return dpp_move<0x4e>(x);  // quad_perm [2, 3, 0, 1]
  else if constexpr (D == 4 || D == 8) {
    // both moves run in every lane (a move reading a lane that a branch has
    // switched off gets no data), then each lane keeps its partner's:
    // row_shl:D reads lane + D, row_shr:D lane - D
    const float above = dpp_move<0x100 + D>(x);
    const float below = dpp_move<0x110 + D>(x);
    return (lane & D) ? below : above;
  }
  else if constexpr (D == 16)
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x1f | (16 << 10)));
  else return __shfl_xor(x, D, 64);
}

// One compare-exchange stage (block size K, partner distance J) of the
// bitonic network over element e = e0 + 16 lane + r (e0: the first element
// the wave holds).
template <int K, int J>
__device__ __forceinline__ void bitonic_stage(float (&v)[16], int lane, int e0) {
  if constexpr (J < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & J) continue;
      const bool up = ((e0 + lane * 16 + r) & K) == 0;
      const float x = v[r], y = v[r | J];
      const bool sw = (x > y) == up;
      v[r] = sw ? y : x;
      v[r | J] = sw ? x : y;
    }
  } else {
    constexpr int D = J >> 4;
    const bool lower = (lane & D) == 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool up = ((e0 + lane * 16 + r) & K) == 0;
      const float x = v[r], y = from_lane_xor<D>(x, lane);
      // the lower element of an ascending block keeps the minimum (values
      // are finite or +inf, so a compare and a select do it)
      const bool sw = (x > y) == (lower == up);
      v[r] = sw ? y : x;
    }
  }
}

// Stages J, J / 2, ..., 1 of block size K.
template <int K, int J>
__device__ __forceinline__ void bitonic_merge(float (&v)[16], int lane, int e0) {
  bitonic_stage<K, J>(v, lane, e0);
  if constexpr (J > 1) bitonic_merge<K, J / 2>(v, lane, e0);
}

// Block sizes K, 2K, ..., kWaveSortMax: the wave's 1024 elements end sorted
// ascending if bit 10 of e0 is clear, descending if set.
template <int K>
__device__ __forceinline__ void bitonic_sort(float (&v)[16], int lane, int e0) {
  bitonic_merge<K, K / 2>(v, lane, e0);
  if constexpr (K < kWaveSortMax) bitonic_sort<K * 2>(v, lane, e0);
}

__device__ __forceinline__ float pick16(const float (&v)[16], int r) {
  float x = v[0];
#pragma unroll
  for (int q = 1; q < 16; ++q) x = r == q ? v[q] : x;
  return x;
}

__device__ __forceinline__ double sorted_at(const float (&v)[16], int e) {
  return (double)__shfl(pick16(v, e & 15), e >> 4, 64);
}

__device__ __forceinline__ double wave_quantile(const float (&v)[16], int n, double f) {
  const double pos = f * (n - 1);
  const int lo = (int)floor(pos);
  const int hi = lo + 1 < n ? lo + 1 : lo;
  const double t = pos - lo;
  const double a = sorted_at(v, lo), b = sorted_at(v, hi);
  return a + (b - a) * t;
}

__global__ __launch_bounds__(64) void k_peak_ctrl_wave(PeakArgs a) {
  const int s = blockIdx.x / a.max_nseg, i = blockIdx.x - s * a.max_nseg, w = blockIdx.y;
  const int lane = threadIdx.x;
  const PeakSeriesDev sd = a.series[s];
  if (i >= sd.nseg) return;
  const int rb = a.seg_begin[sd.seg0 + i], n = a.seg_end[sd.seg0 + i] - rb;
  if (n > kWaveSortMax) return;  // the LDS form takes it
  double* out = a.ctrl + ((int64_t)s * a.num_widths + w) * a.max_nseg + i;
  if (n < a.min_points) {
    if (lane == 0) *out = NAN;
    return;
  }
  const float* col = a.snr + (sd.snr_row0 + rb) * a.num_widths + w;
  float v[16];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int e = r * 64 + lane;  // any assignment will do: the network sorts a multiset
    float x = INFINITY;
    if (e < n) {
      x = col[(int64_t)e * a.num_widths];
      if (!isfinite(x)) {
        bad = true;
        x = INFINITY;
      }
    }
    v[r] = x;
  }
  if (__ballot(bad)) {
    if (lane == 0) *out = NAN;
    return;
  }
  bitonic_sort<2>(v, lane, 0);
  const double med = wave_quantile(v, n, 0.5);
  const double iqr = wave_quantile(v, n, 0.75) - wave_quantile(v, n, 0.25);
  if (lane == 0) *out = med + a.k_sigma * iqr / 1.349;
}

// The same for every width of a segment at once (num_widths <= kSegWidths):
// the workgroup copies the segment's rows (contiguous, all widths) to LDS in
// one coalesced pass and wave w sorts width w from there.
constexpr int kSegWidths = 12;

__global__ __launch_bounds__(64 * kSegWidths) void k_peak_ctrl_seg(PeakArgs a) {
  extern __shared__ float seg[];  // n x num_widths
  const int s = blockIdx.x / a.max_nseg, i = blockIdx.x - s * a.max_nseg;
  const int nw = a.num_widths, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const PeakSeriesDev sd = a.series[s];
  if (i >= sd.nseg) return;
  const int rb = a.seg_begin[sd.seg0 + i], n = a.seg_end[sd.seg0 + i] - rb;
  if (n > kWaveSortMax) return;  // the two-wave and LDS forms take it
  double* out = a.ctrl + ((int64_t)s * nw + w) * a.max_nseg + i;
  if (n < a.min_points) {
    if (lane == 0) *out = NAN;
    return;
  }
  // n * nw <= 16 * blockDim words: every load of a thread in flight before
  // its first LDS store
  const float* src = a.snr + (sd.snr_row0 + rb) * nw;
  float buf[kWaveSortMax / 64];
#pragma unroll
  for (int k = 0; k < kWaveSortMax / 64; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    buf[k] = q < n * nw ? src[q] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < kWaveSortMax / 64; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    if (q < n * nw) seg[q] = buf[k];
  }
  __syncthreads();
  float v[16];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int e = r * 64 + lane;
    float x = INFINITY;
    if (e < n) {
      x = seg[e * nw + w];
      if (!isfinite(x)) {
        bad = true;
        x = INFINITY;
      }
    }
    v[r] = x;
  }
  if (__ballot(bad)) {  // per wave: no barrier follows
    if (lane == 0) *out = NAN;
    return;
  }
  bitonic_sort<2>(v, lane, 0);
  const double med = wave_quantile(v, n, 0.5);
  const double iqr = wave_quantile(v, n, 0.75) - wave_quantile(v, n, 0.25);
  if (lane == 0) *out = med + a.k_sigma * iqr / 1.349;
}

// Segments of kWaveSortMax + 1 .. 2 kWaveSortMax rows (the a.nmid pairs of
// a.mid): two waves of a workgroup hold 1024 elements each and sort them in
// opposite directions, the one stage of partner distance 1024 exchanges
// through LDS, and each wave finishes its half in registers.
__global__ __launch_bounds__(128) void k_peak_ctrl_pair(PeakArgs a) {
  __shared__ float xs[2 * kWaveSortMax];
  const int s = a.mid[2 * blockIdx.x], i = a.mid[2 * blockIdx.x + 1], w = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const PeakSeriesDev sd = a.series[s];
  double* out = a.ctrl + ((int64_t)s * a.num_widths + w) * a.max_nseg + i;
  const int rb = a.seg_begin[sd.seg0 + i], n = a.seg_end[sd.seg0 + i] - rb;
  if (n < a.min_points) {
    if (threadIdx.x == 0) *out = NAN;
    return;
  }
  const float* col = a.snr + (sd.snr_row0 + rb) * a.num_widths + w;
  const int e0 = wave * kWaveSortMax;
  float v[16];
  int bad = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int e = e0 + r * 64 + lane;  // a multiset: any assignment will do
    float x = INFINITY;
    if (e < n) {
      x = col[(int64_t)e * a.num_widths];
      if (!isfinite(x)) {
        bad = 1;
        x = INFINITY;
      }
    }
    v[r] = x;
  }
  if (__syncthreads_or(bad)) {
    if (threadIdx.x == 0) *out = NAN;
    return;
  }
  bitonic_sort<2>(v, lane, e0);  // wave 0 ascending, wave 1 descending
  // stage K = 2048, J = 1024: wave 0 keeps the minima, wave 1 the maxima
#pragma unroll
  for (int r = 0; r < 16; ++r) xs[e0 + lane * 16 + r] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float y = xs[(e0 ^ kWaveSortMax) + lane * 16 + r];
    v[r] = wave == 0 ? fminf(v[r], y) : fmaxf(v[r], y);
  }
  bitonic_merge<2 * kWaveSortMax, kWaveSortMax / 2>(v, lane, e0);
  __syncthreads();  // every wave has read the exchange
#pragma unroll
  for (int r = 0; r < 16; ++r) xs[e0 + lane * 16 + r] = v[r];
  __syncthreads();
  if (threadIdx.x == 0) {
    const double med = quantile_sorted(xs, n, 0.5);
    const double iqr = quantile_sorted(xs, n, 0.75) - quantile_sorted(xs, n, 0.25);
    *out = med + a.k_sigma * iqr / 1.349;
  }
}

// Segments of 2 kWaveSortMax + 1 .. kPeakSegMax rows (the a.nbig pairs of
// a.big): one workgroup sorts them in LDS.
__global__ __launch_bounds__(kPeakThreads) void k_peak_ctrl(PeakArgs a) {
  __shared__ float v[kPeakSegMax];
  const int s = a.big[2 * blockIdx.x], i = a.big[2 * blockIdx.x + 1], w = blockIdx.y;
  const PeakSeriesDev sd = a.series[s];
  double* out = a.ctrl + ((int64_t)s * a.num_widths + w) * a.max_nseg + i;
  const int rb = a.seg_begin[sd.seg0 + i], n = a.seg_end[sd.seg0 + i] - rb;
  if (n < a.min_points || n > kPeakSegMax) {
    if (threadIdx.x == 0) *out = NAN;
    return;
  }
  int npow = 1;
  while (npow < n) npow <<= 1;
  const float* col = a.snr + (sd.snr_row0 + rb) * a.num_widths + w;
  int bad = 0;
  for (int j = threadIdx.x; j < npow; j += kPeakThreads) {
    float x = INFINITY;  // padding sorts to the end
    if (j < n) {
      x = col[(int64_t)j * a.num_widths];
      if (!isfinite(x)) bad = 1;
    }
    v[j] = x;
  }
  if (__syncthreads_or(bad)) {  // a non-finite S/N: no control point
    if (threadIdx.x == 0) *out = NAN;
    return;
  }
  // ascending bitonic sort of npow values
  for (int k = 2; k <= npow; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < (npow >> 1); t += kPeakThreads) {
        const int lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const float x = v[lo], y = v[hi];
        if ((x > y) == up) {
          v[lo] = y;
          v[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const double med = quantile_sorted(v, n, 0.5);
    const double iqr = quantile_sorted(v, n, 0.75) - quantile_sorted(v, n, 0.25);
    *out = med + a.k_sigma * iqr / 1.349;
  }
}

__global__ __launch_bounds__(64) void k_peak_fit(PeakArgs a) {
  constexpr int D = kPeakMaxDegree;
  const int s = blockIdx.x / a.num_widths, w = blockIdx.x - s * a.num_widths;
  const int lane = threadIdx.x;
  const PeakSeriesDev sd = a.series[s];
  const double* y = a.ctrl + ((int64_t)s * a.num_widths + w) * a.max_nseg;
  const double* xs = a.seg_x + sd.seg0;
  const int d = a.degree;
  double sx = 0.0;
  int cnt = 0;
  for (int i = lane; i < sd.nseg; i += 64)
    if (isfinite(y[i])) {
      sx += xs[i];
      ++cnt;
    }
  cnt = wave_sum_i32(cnt);
  sx = wave_sum_f64(sx);
  PeakFitDev f{};
  f.npoints = cnt;
  if (cnt < d + 1) {
    if (lane == 0) a.fits[blockIdx.x] = f;  // ok = 0
    return;
  }
  const double xbar = sx / cnt;
  double mx = 0.0;
  for (int i = lane; i < sd.nseg; i += 64)
    if (isfinite(y[i])) mx = fmax(mx, fabs(xs[i] - xbar));
  mx = wave_max_f64(mx);
  const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
  // power sums S_j = sum u^j (j <= 2d) and B_j = sum y u^j (j <= d)
  double S[2 * D + 1], B[D + 1];
#pragma unroll
  for (int j = 0; j <= 2 * D; ++j) S[j] = 0.0;
#pragma unroll
  for (int j = 0; j <= D; ++j) B[j] = 0.0;
  for (int i = lane; i < sd.nseg; i += 64) {
    const double yi = y[i];
    if (!isfinite(yi)) continue;
    const double u = (xs[i] - xbar) * inv;
    double pw = 1.0;
#pragma unroll
    for (int j = 0; j <= 2 * D; ++j) {
      if (j <= 2 * d) S[j] += pw;
      if (j <= d) B[j] += yi * pw;
      pw *= u;
    }
  }
#pragma unroll
  for (int j = 0; j <= 2 * D; ++j) S[j] = wave_sum_f64(S[j]);
#pragma unroll
  for (int j = 0; j <= D; ++j) B[j] = wave_sum_f64(B[j]);
  if (lane != 0) return;
  // normal equations M c = B, M[j][l] = S[j + l], by Gaussian elimination
  // with partial pivoting
  double M[D + 1][D + 2];
  const int n = d + 1;
  for (int j = 0; j < n; ++j) {
    for (int l = 0; l < n; ++l) M[j][l] = S[j + l];
    M[j][n] = B[j];
  }
  bool ok = true;
  for (int c = 0; c < n && ok; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0) {
      ok = false;
      break;
    }
    if (piv != c)
      for (int l = 0; l <= n; ++l) {
        const double t = M[c][l];
        M[c][l] = M[piv][l];
        M[piv][l] = t;
      }
    for (int r = c + 1; r < n; ++r) {
      const double g = M[r][c] / M[c][c];
      for (int l = c; l <= n; ++l) M[r][l] -= g * M[c][l];
    }
  }
  if (ok)
    for (int c = n - 1; c >= 0; --c) {
      double t = M[c][n];
      for (int l = c + 1; l < n; ++l) t -= M[c][l] * f.c[l];
      f.c[c] = t / M[c][c];
    }
  f.xbar = xbar;
  f.inv_scale = inv;
  f.ok = ok ? 1 : 0;
  a.fits[blockIdx.x] = f;
}

__device__ __forceinline__ void emit_peak(const PeakArgs& a, int s, int w, int64_t row, float snr,
                                          double thr, int members) {
  const int slot = atomicAdd(&a.count[0], 1);
  atomicAdd(&a.count[1 + s], 1);
  if (slot < a.capacity) {
    PeakDev pk;
    pk.row = row;
    pk.threshold = thr;
    pk.snr = snr;
    pk.series = s;
    pk.width = w;
    pk.members = members;
    pk.pad = 0;
    a.peaks[slot] = pk;
  }
}

// Selection: every row's thresholds and the rows above them, as one bit per
// (row, width). A workgroup takes kFlagRows consecutive rows of one series;
// a wave takes 64 whole rows per step: it reads their 64 x num_widths S/N
// values as consecutive words (each load instruction covers 64 consecutive
// words), parks them in its own LDS area, reads back row = lane, and one
// ballot per width gives the 64 bits of that width.
constexpr int kFlagRows = 4096;
constexpr int kFlagSteps = 2;  // 64-row steps a wave loads together

__global__ __launch_bounds__(kPeakThreads) void k_peak_flag(PeakArgs a) {
  constexpr int kMaxW = 32;
  __shared__ PeakFitDev fit[kMaxW];
  extern __shared__ float stage[];  // per wave: kFlagSteps x 64 x num_widths
  const int nw = a.num_widths;
  const int chunks = (int)((a.nwords * 64 + kFlagRows - 1) / kFlagRows);
  const int s = blockIdx.x / chunks, c = blockIdx.x - s * chunks;
  const PeakSeriesDev sd = a.series[s];
  const int64_t r0 = (int64_t)c * kFlagRows;
  if (r0 >= sd.rows) return;
  if (threadIdx.x < nw) fit[threadIdx.x] = a.fits[(int64_t)s * nw + threadIdx.x];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* snr = a.snr + sd.snr_row0 * nw;
  const double* lx = a.lognu + sd.freq0;
  uint64_t* bits = a.flags + (int64_t)s * nw * a.nwords;
  float* my = stage + wave * kFlagSteps * 64 * nw;
  const int64_t rend = min(sd.rows, r0 + kFlagRows);
  for (int64_t rb = r0 + wave * 64; rb < rend; rb += kFlagSteps * kPeakThreads) {
    double x[kFlagSteps];
    // every load of both steps in flight before the first LDS store: up to
    // kLoadW words per lane and step at a time
    constexpr int kLoadW = 16;
    for (int i0 = 0; i0 < nw; i0 += kLoadW) {
      float buf[kFlagSteps][kLoadW];
#pragma unroll
      for (int q = 0; q < kFlagSteps; ++q) {
        const int64_t rq = rb + q * kPeakThreads;  // first row of this step
        const int words = rq < rend ? (int)min((int64_t)64, rend - rq) * nw : 0;
        const float* src = snr + rq * nw;
#pragma unroll
        for (int i = 0; i < kLoadW; ++i) {
          const int t = (i0 + i) * 64 + lane;
          buf[q][i] = (i0 + i < nw && t < words) ? src[t] : 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < kFlagSteps; ++q)
#pragma unroll
        for (int i = 0; i < kLoadW; ++i)
          if (i0 + i < nw) my[q * 64 * nw + (i0 + i) * 64 + lane] = buf[q][i];
    }
#pragma unroll
    for (int q = 0; q < kFlagSteps; ++q) {
      const int64_t rq = rb + q * kPeakThreads;
      x[q] = rq + lane < rend ? lx[rq + lane] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kFlagSteps; ++q) {
      const int64_t rq = rb + q * kPeakThreads;
      if (rq >= rend) break;  // uniform
      const bool in = rq + lane < rend;
      const float* row = my + q * 64 * nw + lane * nw;
      for (int w = 0; w < nw; ++w) {
        const PeakFitDev& f = fit[w];
        const double u = (x[q] - f.xbar) * f.inv_scale;
        // coefficients past the degree are zero, so the full-degree Horner
        // form gives the degree-d value exactly
        double t = f.c[kPeakMaxDegree];
#pragma unroll
        for (int j = kPeakMaxDegree - 1; j >= 0; --j) t = t * u + f.c[j];
        const bool flag = in && f.ok && (double)row[w] > t;  // false for a NaN S/N
        const unsigned long long m = __ballot(flag);
        if (lane == 0) bits[(int64_t)w * a.nwords + (rq >> 6)] = m;
      }
    }
  }
}

// Clustering: one wave per (series, width) reads the width's bits 64 words
// at a time, lists the set rows in order, gathers their S/N, threshold and
// frequency 64 rows at a time, and lane 0 walks them forming the clusters.
// Finished peaks are buffered and written out together.
constexpr int kPeakBuf = 128;

__global__ __launch_bounds__(64) void k_peak_cluster(PeakArgs a) {
  __shared__ int32_t list[64 * 64];
  __shared__ float bsnr[64];
  __shared__ double bthr[64], bnu[64];
  __shared__ int32_t prow[kPeakBuf], pmem[kPeakBuf];
  __shared__ float psnr[kPeakBuf];
  __shared__ double pthr[kPeakBuf];
  const int nw = a.num_widths;
  const int s = blockIdx.x / nw, w = blockIdx.x - s * nw;
  const int lane = threadIdx.x;
  const PeakFitDev f = a.fits[blockIdx.x];
  if (!f.ok) return;
  const PeakSeriesDev sd = a.series[s];
  const uint64_t* bits = a.flags + ((int64_t)s * nw + w) * a.nwords;
  const int nwords = (int)((sd.rows + 63) >> 6);
  const float* snr = a.snr + sd.snr_row0 * nw + w;
  const double* lx = a.lognu + sd.freq0;
  const double* nu = a.nu + sd.freq0;
  // cluster state and the count of buffered peaks, held by lane 0
  bool have = false;
  double nu_prev = 0.0, best_thr = 0.0;
  int32_t best_row = 0;
  float best = 0.0f;
  int members = 0, npk = 0;
  auto flush = [&](int n_out) {  // every lane: write buffered peaks 0 .. n_out - 1
    int base = 0;
    if (lane == 0) {
      base = atomicAdd(&a.count[0], n_out);
      atomicAdd(&a.count[1 + s], n_out);
    }
    base = __shfl(base, 0, 64);
    for (int q = lane; q < n_out; q += 64)
      if (base + (int64_t)q < a.capacity) {
        PeakDev pk;
        pk.row = prow[q];
        pk.threshold = pthr[q];
        pk.snr = psnr[q];
        pk.series = s;
        pk.width = w;
        pk.members = pmem[q];
        pk.pad = 0;
        a.peaks[base + q] = pk;
      }
  };
  auto finish = [&]() {  // lane 0: the current cluster is complete
    if (npk < kPeakBuf) {
      prow[npk] = best_row;
      psnr[npk] = best;
      pthr[npk] = best_thr;
      pmem[npk] = members;
      ++npk;
    } else {
      emit_peak(a, s, w, best_row, best, best_thr, members);
    }
  };
  for (int w0 = 0; w0 < nwords; w0 += 64) {
    const int wi = w0 + lane;
    const uint64_t m = wi < nwords ? bits[wi] : 0ull;
    const int cnt = __popcll(m);
    int pre = cnt;  // inclusive prefix over lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(pre, o, 64);
      if (lane >= o) pre += t;
    }
    const int total = __shfl(pre, 63, 64);
    if (total == 0) continue;
    int pos = pre - cnt;
    for (uint64_t mm = m; mm; mm &= mm - 1) list[pos++] = wi * 64 + __builtin_ctzll(mm);
    __syncthreads();
    for (int b0 = 0; b0 < total; b0 += 64) {
      const int k = b0 + lane;
      if (k < total) {
        const int32_t r = list[k];
        const double u = (lx[r] - f.xbar) * f.inv_scale;
        double t = f.c[kPeakMaxDegree];
#pragma unroll
        for (int j = kPeakMaxDegree - 1; j >= 0; --j) t = t * u + f.c[j];
        bsnr[lane] = snr[(int64_t)r * nw];
        bthr[lane] = t;
        bnu[lane] = nu[r];
      }
      __syncthreads();
      if (lane == 0) {
        const int nb = total - b0 < 64 ? total - b0 : 64;
        for (int q = 0; q < nb; ++q) {
          const double fr = bnu[q];
          if (have && nu_prev - fr > sd.gap) {
            finish();
            have = false;
          }
          if (!have) {
            have = true;
            members = 0;
            best = bsnr[q];
            best_row = list[b0 + q];
            best_thr = bthr[q];
          } else if (bsnr[q] > best) {  // the first of equal S/N stays
            best = bsnr[q];
            best_row = list[b0 + q];
            best_thr = bthr[q];
          }
          ++members;
          nu_prev = fr;
        }
      }
      __syncthreads();
    }
    const int n_out = __shfl(npk, 0, 64);
    if (n_out >= kPeakBuf / 2) {
      flush(n_out);
      npk = 0;
      __syncthreads();
    }
  }
  if (lane == 0 && have) finish();  // the last cluster
  __syncthreads();
  const int n_out = __shfl(npk, 0, 64);
  if (n_out > 0) flush(n_out);
}

}  // namespace

hipError_t launch_peak_ctrl(const PeakArgs& a, hipStream_t stream) {
  if (a.nseries <= 0 || a.max_nseg <= 0) return hipSuccess;
  if (a.num_widths <= kSegWidths)
    hipLaunchKernelGGL(k_peak_ctrl_seg, dim3(a.nseries * a.max_nseg), dim3(64 * a.num_widths),
                       kWaveSortMax * a.num_widths * sizeof(float), stream, a);
  else
    hipLaunchKernelGGL(k_peak_ctrl_wave, dim3(a.nseries * a.max_nseg, a.num_widths), dim3(64), 0,
                       stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.nmid > 0) {
    hipLaunchKernelGGL(k_peak_ctrl_pair, dim3(a.nmid, a.num_widths), dim3(128), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.nbig <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_peak_ctrl, dim3(a.nbig, a.num_widths), dim3(kPeakThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_peak_fit(const PeakArgs& a, hipStream_t stream) {
  if (a.nseries <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_peak_fit, dim3(a.nseries * a.num_widths), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_peak_scan(const PeakArgs& a, hipStream_t stream) {
  if (a.nseries <= 0 || a.nwords <= 0) return hipSuccess;
  const int chunks = (int)((a.nwords * 64 + kFlagRows - 1) / kFlagRows);
  static bool done[kMaxDevices] = {};  // up to 32 widths: 64 KiB of staging
  hipError_t e = set_lds_limit_once(reinterpret_cast<const void*>(k_peak_flag), 96 * 1024, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_peak_flag, dim3(a.nseries * chunks), dim3(kPeakThreads),
                     (kPeakThreads / 64) * kFlagSteps * 64 * a.num_widths * sizeof(float), stream,
                     a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_peak_cluster, dim3(a.nseries * a.num_widths), dim3(64), 0, stream, a);
  return hipGetLastError();
}

}  // namespace ffa
