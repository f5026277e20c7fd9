// Launchers of the HIP kernels of the FFA search.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ffa.h"
#include "ffa_internal.hpp"

namespace ffa {

// One input series of a launch.
struct SeriesDev {
  const void* ptr;    // raw samples (DEVICE)
  int64_t nsamp;
  int64_t chunk0;     // first downsampling block of this series
  int32_t oct0;       // first octave of this series in the octave table
  int32_t noct;
  int32_t normalise;
  int32_t halo;       // samples past a block needed by its last window
  int32_t block;      // samples per downsampling block
  int32_t pad;
};

// One pseudo-octave of one series: where its downsampled samples go.
struct OctaveDev {
  uint64_t ds_fx;
  int64_t nsamp;      // downsampled samples
  int64_t off;        // element offset in the downsampled buffer
  double rcp;         // 1 / ds_fx: a first estimate of window indices, refined exactly
};

// Normalisation statistics of each series (Sec. 5.2), FP64:
// stats[2i] = mean, stats[2i+1] = population standard deviation.
// norm[kNormFloats i ..] = FP32 mean, 1 / std, the mean's FP32 residual and a
// pad word, for the downsampler.
// partials holds blocks_per_series * nseries * 2 doubles. flag |= 1 when a
// normalised series has zero or non-finite variance.
hipError_t launch_stats(const SeriesDev* series_dev, int32_t nseries, int32_t dtype,
                        int32_t blocks_per_series, double* partials, double* stats, float* norm,
                        int32_t* flag, hipStream_t stream);

// All pseudo-octaves of every series in one pass over the raw samples
// (Sec. 5.3, App. A.4). nblocks = total downsampling blocks of the launch.
// Every series is cut into blocks of its own `block` samples; block_series
// (DEVICE, nblocks entries) names the series of each block, or is null when
// there is one series; lds_floats is the largest
// downsample_lds_floats(block, halo) of the launch.
hipError_t launch_downsample(const SeriesDev* series_dev, const int32_t* block_series,
                             const OctaveDev* oct, const float* norm, int32_t dtype, void* out,
                             int32_t out_dtype, int64_t nblocks, int32_t lds_floats,
                             hipStream_t stream);

// Downsampling block length of a series whose windows reach `halo` samples
// past a block; 0 when the halo is too long for a block's LDS.
int32_t downsample_block_samples(int32_t halo);

// LDS floats a downsampling block of `block` samples and `halo` extra uses.
int32_t downsample_lds_floats(int32_t block, int32_t halo);

// One pass of folding-transform tiles (Sec. 2.2), with the boxcar S/N of
// final rows (Sec. 5.4).
hipError_t launch_pass(const PassArgs& args, hipStream_t stream);

// All passes of a group of transforms in one persistent launch of `grid`
// workgroups; zeroes the ncounters completion counters and the ticket first.
hipError_t launch_persist(const PassArgs& args, int ncounters, int grid, hipStream_t stream);

// LDS bytes a pass launch uses.
int32_t pass_lds_bytes(int32_t rows_cap, int32_t max_p);

// Raises a kernel's dynamic-LDS limit to `bytes` on the current device, once
// per device (done[] holds one flag per device, kMaxDevices of them).
constexpr int kMaxDevices = 64;
inline hipError_t set_lds_limit_once(const void* kernel, int bytes, bool* done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 0 && dev < kMaxDevices && done[dev]) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && dev >= 0 && dev < kMaxDevices) done[dev] = true;
  return e;
}

// Sets a flag word to zero with a kernel (graph-capture friendly).
hipError_t launch_clear_flag(int32_t* flag, hipStream_t stream);

// De-reddening by a running median (Sec. 5.2) of one series of n samples of
// `dtype`: out[i] = x[i] - the median of the `window` (odd) samples centred on
// i, cut at the ends, stored as out_dtype. An internal bound that cannot fail
// for a well-formed launch ORs kMedErrBit into *err.
constexpr int32_t kMedErrBit = 8;
hipError_t launch_running_median(const void* x, int64_t n, int32_t dtype, int32_t window,
                                 void* out, int32_t out_dtype, int32_t* err, hipStream_t stream);

// Bytes of the static device workspace of ffa_search_noalloc (one per device),
// and the offset in it of the status word (the first 256 bytes hold it; the
// rest is laid out per call).
constexpr size_t kNoAllocBytes = FFA_NOALLOC_WORKSPACE_BYTES;
constexpr size_t kNoAllocFlagOffset = 0;
constexpr size_t kNoAllocHeader = 256;

// Device address of that workspace on `device`, which must be the current
// device; looked up once per device and kept.
hipError_t noalloc_setup(int device, void** ptr);

}  // namespace ffa
