// Periodogram peak detection (Sec. 5.5): device records and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffa {

constexpr int kPeakSegMax = 8192;   // most rows of one frequency segment (LDS sort)
constexpr int kPeakWaveSortMax = 1024;  // most rows a segment sorted in registers holds
constexpr int kPeakMaxDegree = 4;   // highest polynomial degree of the threshold
constexpr int kPeakThreads = 256;

// One series of a peak-detection launch.
struct PeakSeriesDev {
  int64_t snr_row0;  // first row of the series in the S/N array
  int64_t rows;      // periodogram rows of the series
  int64_t freq0;     // first row of its plan in the frequency tables
  double gap;        // largest frequency step inside one cluster, Hz
  int32_t seg0;      // first segment of its plan in the segment tables
  int32_t nseg;      // segments of its plan, in row order
};

// Threshold of one (series, width): sum_j c[j] u^j with
// u = (log nu - xbar) * inv_scale; ok = 0 when there are too few control
// points for the degree.
struct PeakFitDev {
  double xbar, inv_scale;
  double c[kPeakMaxDegree + 1];
  int32_t ok, npoints;
};

// One peak as the scan kernel writes it.
struct PeakDev {
  int64_t row;       // row of the brightest member within its series
  double threshold;  // threshold at that row
  float snr;
  int32_t series, width, members, pad;
};

struct PeakArgs {
  const PeakSeriesDev* series;
  int32_t nseries, num_widths, max_nseg, degree, min_points, pad;
  double k_sigma;
  const float* snr;        // S/N array, rows x num_widths, FP32
  const double* nu;        // trial frequency of every plan row
  const double* lognu;     // its natural log
  const int32_t* seg_begin;  // first row (within the series) of every plan segment
  const int32_t* seg_end;    // one past its last row
  const double* seg_x;       // log of the segment's centre frequency
  const int32_t* mid;        // (series, segment) pairs of segments of 1025 .. 2048 rows
  const int32_t* big;        // and of more than 2048 rows
  int32_t nmid, nbig;
  double* ctrl;            // control values, ((series * num_widths) + w) * max_nseg + i
  PeakFitDev* fits;        // series * num_widths + w
  uint64_t* flags;         // rows above the threshold, ((series * num_widths) + w) * nwords words
  int64_t nwords;          // 64-row words per (series, width): rows of the longest series / 64
  PeakDev* peaks;          // capacity records
  int64_t capacity;
  int32_t* count;          // [0]: peaks found; [1 + s]: peaks of series s
};

// Control points of every (series, segment, width), then the least-squares
// threshold of every (series, width), then the selection of the points above
// it (flags) and their clustering. count must hold 1 + nseries zeros.
// Segments above kPeakWaveSortMax rows (the a.nmid pairs of a.mid, up to
// twice that, and the a.nbig pairs of a.big) take further launches.
hipError_t launch_peak_ctrl(const PeakArgs& a, hipStream_t stream);
hipError_t launch_peak_fit(const PeakArgs& a, hipStream_t stream);
hipError_t launch_peak_scan(const PeakArgs& a, hipStream_t stream);

}  // namespace ffa
