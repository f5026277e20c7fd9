// Periodogram peak detection (Sec. 5.5). Every width trial of the
// periodogram is searched on its own: its S/N against trial frequency is cut
// into equal frequency segments; each segment gives a control point (median
// + k IQR / 1.349 at the segment's centre frequency); a polynomial in
// log(frequency) fitted to the control points by least squares is the
// selection threshold, and the points above it are clustered into peaks.
//
// Three steps:
//   k_peak_ctrl_wave / k_peak_ctrl
//                the control points: one wave (segments of up to 1024 rows,
//                sorted in registers) or one workgroup (larger segments,
//                sorted in LDS) per (series, segment, width) sorts the
//                segment's S/N values with a bitonic network and reads the
//                quantiles from the order statistics;
//   k_peak_fit   one wave per (series, width): power sums of the control
//                points on a centred and scaled abscissa, reduced across the
//                wave, and the normal equations solved in FP64;
//   k_peak_scan  one workgroup per (series, width): every row's threshold,
//                the rows above it compacted in row (= frequency) order and
//                walked by one thread that forms the clusters.
#include <hip/hip_runtime.h>
#include <math.h>

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
constexpr int kWaveSortMax = 1024;

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
#pragma unroll
  for (int k = 2; k <= kWaveSortMax; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if (r & j) continue;
          const int e = lane * 16 + r;
          const bool up = (e & k) == 0;
          const float x = v[r], y = v[r | j];
          const bool sw = (x > y) == up;
          v[r] = sw ? y : x;
          v[r | j] = sw ? x : y;
        }
      } else {
        const int d = j >> 4;
        const bool lower = (lane & d) == 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int e = lane * 16 + r;
          const bool up = (e & k) == 0;
          const float x = v[r], y = __shfl_xor(x, d, 64);
          v[r] = (lower == up) ? fminf(x, y) : fmaxf(x, y);
        }
      }
    }
  }
  const double med = wave_quantile(v, n, 0.5);
  const double iqr = wave_quantile(v, n, 0.75) - wave_quantile(v, n, 0.25);
  if (lane == 0) *out = med + a.k_sigma * iqr / 1.349;
}

// Segments of kWaveSortMax + 1 .. kPeakSegMax rows: one workgroup sorts them
// in LDS.
__global__ __launch_bounds__(kPeakThreads) void k_peak_ctrl(PeakArgs a) {
  __shared__ float v[kPeakSegMax];
  const int s = blockIdx.x / a.max_nseg, i = blockIdx.x - s * a.max_nseg, w = blockIdx.y;
  const PeakSeriesDev sd = a.series[s];
  if (i >= sd.nseg) return;
  double* out = a.ctrl + ((int64_t)s * a.num_widths + w) * a.max_nseg + i;
  const int rb = a.seg_begin[sd.seg0 + i], n = a.seg_end[sd.seg0 + i] - rb;
  if (n <= kWaveSortMax) return;  // the register form takes it
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

// Rows per thread and chunk of the scan: their loads are issued together.
constexpr int kScanRows = 4;

__global__ __launch_bounds__(kPeakThreads) void k_peak_scan(PeakArgs a) {
  constexpr int kWaves = kPeakThreads / 64, kChunkRows = kScanRows * kPeakThreads;
  __shared__ int64_t lrow[kChunkRows];
  __shared__ float lsnr[kChunkRows];
  __shared__ double lthr[kChunkRows];
  __shared__ int wcount[kScanRows][kWaves];
  const int s = blockIdx.x / a.num_widths, w = blockIdx.x - s * a.num_widths;
  const PeakFitDev f = a.fits[blockIdx.x];
  if (!f.ok) return;
  const PeakSeriesDev sd = a.series[s];
  const float* col = a.snr + sd.snr_row0 * a.num_widths + w;
  const double* nu = a.nu + sd.freq0;
  const double* lx = a.lognu + sd.freq0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // cluster state, held by thread 0
  bool have = false;
  double nu_prev = 0.0, best_thr = 0.0;
  int64_t best_row = 0;
  float best = 0.0f;
  int members = 0;
  for (int64_t base = 0; base < sd.rows; base += kChunkRows) {
    // row base + q * kPeakThreads + tid of the chunk, q = 0 .. kScanRows - 1
    float v[kScanRows];
    double x[kScanRows];
#pragma unroll
    for (int q = 0; q < kScanRows; ++q) {
      const int64_t r = base + q * kPeakThreads + tid;
      v[q] = r < sd.rows ? col[r * a.num_widths] : 0.0f;
      x[q] = r < sd.rows ? lx[r] : 0.0;
    }
    bool flag[kScanRows];
    double thr[kScanRows];
    int before[kScanRows];
#pragma unroll
    for (int q = 0; q < kScanRows; ++q) {
      const int64_t r = base + q * kPeakThreads + tid;
      const double u = (x[q] - f.xbar) * f.inv_scale;
      double t = f.c[a.degree];
      for (int j = a.degree - 1; j >= 0; --j) t = t * u + f.c[j];
      thr[q] = t;
      flag[q] = r < sd.rows && (double)v[q] > t;  // false for a NaN S/N
      const unsigned long long m = __ballot(flag[q]);
      before[q] = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[q][wave] = __popcll(m);
    }
    __syncthreads();
    // compaction in row order: sub-chunk q, then wave, then lane
    int tot = 0;
#pragma unroll
    for (int q = 0; q < kScanRows; ++q) {
      int off = tot;
#pragma unroll
      for (int z = 0; z < kWaves; ++z) {
        off += z < wave ? wcount[q][z] : 0;
        tot += wcount[q][z];
      }
      if (flag[q]) {
        lrow[off + before[q]] = base + q * kPeakThreads + tid;
        lsnr[off + before[q]] = v[q];
        lthr[off + before[q]] = thr[q];
      }
    }
    __syncthreads();
    if (tid == 0) {
      for (int q = 0; q < tot; ++q) {
        const int64_t rr = lrow[q];
        const double fr = nu[rr];
        if (have && nu_prev - fr > sd.gap) {
          emit_peak(a, s, w, best_row, best, best_thr, members);
          have = false;
        }
        if (!have) {
          have = true;
          members = 0;
          best = lsnr[q];
          best_row = rr;
          best_thr = lthr[q];
        } else if (lsnr[q] > best) {  // the first of equal S/N stays
          best = lsnr[q];
          best_row = rr;
          best_thr = lthr[q];
        }
        ++members;
        nu_prev = fr;
      }
    }
    __syncthreads();  // the lists are rewritten by the next chunk
  }
  if (tid == 0 && have) emit_peak(a, s, w, best_row, best, best_thr, members);
}

}  // namespace

hipError_t launch_peak_ctrl(const PeakArgs& a, int32_t max_seg, hipStream_t stream) {
  if (a.nseries <= 0 || a.max_nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_peak_ctrl_wave, dim3(a.nseries * a.max_nseg, a.num_widths), dim3(64), 0,
                     stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || max_seg <= kWaveSortMax) return e;
  hipLaunchKernelGGL(k_peak_ctrl, dim3(a.nseries * a.max_nseg, a.num_widths), dim3(kPeakThreads),
                     0, stream, a);
  return hipGetLastError();
}

hipError_t launch_peak_fit(const PeakArgs& a, hipStream_t stream) {
  if (a.nseries <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_peak_fit, dim3(a.nseries * a.num_widths), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_peak_scan(const PeakArgs& a, hipStream_t stream) {
  if (a.nseries <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_peak_scan, dim3(a.nseries * a.num_widths), dim3(kPeakThreads), 0, stream,
                     a);
  return hipGetLastError();
}

}  // namespace ffa
