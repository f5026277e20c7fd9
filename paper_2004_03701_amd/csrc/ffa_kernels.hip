// HIP kernels of the FFA periodicity search for gfx950 (MI355X).
//
//   k_stats_*      FP64 mean / population std of each series (Sec. 5.2)
//   k_downsample   every pseudo-octave of a series in one read of it
//                  (Sec. 5.3, App. A.4)
//   k_ffa_pass     folding-transform tiles (Sec. 2.2): the bottom merge
//                  levels in registers, the upper ones as paired merges in
//                  LDS, and for the rows of the full transform the boxcar
//                  S/N (Sec. 5.4)
//
// None of the paths is a dense contraction, so nothing here uses MFMA: the
// limits are HBM bandwidth (stats, downsampling) and LDS / VALU throughput
// (the merges and the boxcar widths).
#include <hip/hip_runtime.h>
#include <math.h>
#include <algorithm>
#include <stdint.h>

#include <type_traits>

#include "../../include/ffa.h"
#include "ffa_kernels.hpp"

namespace ffa {
namespace {

// ---------------------------------------------------------------------------
// Sample storage
// ---------------------------------------------------------------------------

__device__ __forceinline__ float load_sample(const void* base, int dtype, int64_t i) {
  if (dtype == FFA_F32) return static_cast<const float*>(base)[i];
  const uint16_t b = static_cast<const uint16_t*>(base)[i];
  if (dtype == FFA_BF16) return __uint_as_float(static_cast<uint32_t>(b) << 16);
  _Float16 h;
  __builtin_memcpy(&h, &b, 2);
  return static_cast<float>(h);
}

// Global-address-space forms with the storage type fixed at compile time:
// straight-line global loads a thread can keep in flight together (a runtime
// type test between loads, or a generic pointer, makes the compiler wait for
// each load in turn).
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
using gptr_w = __attribute__((address_space(1))) T*;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte load

template <int DT>
__device__ __forceinline__ float load_g(const void* base, int64_t i) {
  if (DT == FFA_F32) return ((gptr<float>)base)[i];
  const uint16_t b = ((gptr<uint16_t>)base)[i];
  if (DT == FFA_BF16) return __uint_as_float(static_cast<uint32_t>(b) << 16);
  _Float16 h;
  __builtin_memcpy(&h, &b, 2);
  return static_cast<float>(h);
}

// The stored bits of sample i (FP32 bits, or 16 bits zero-extended), and
// their value: loads kept apart from the conversion, so that loads behind a
// condition stay in flight together.
template <int DT>
__device__ __forceinline__ uint32_t load_bits(const void* base, int64_t i) {
  if (DT == FFA_F32) return __float_as_uint(((gptr<float>)base)[i]);
  return ((gptr<uint16_t>)base)[i];
}

// The same from a uniform row start and a per-lane 32-bit column.
template <int DT>
__device__ __forceinline__ uint32_t load_row_bits(const void* base, int64_t row, uint32_t col) {
  // the row start is the same in every lane and the byte offset an unsigned
  // 32-bit value: a scalar base plus a vector offset
  const uint32_t boff = col * (DT == FFA_F32 ? 4u : 2u);
  if (DT == FFA_F32) {
    gptr<unsigned char> rp = (gptr<unsigned char>)((gptr<float>)base + row);
    return *(gptr<uint32_t>)(rp + boff);
  }
  gptr<unsigned char> rp = (gptr<unsigned char>)((gptr<uint16_t>)base + row);
  return *(gptr<uint16_t>)(rp + boff);
}

template <int DT>
__device__ __forceinline__ float bits_value(uint32_t b) {
  if (DT == FFA_F32) return __uint_as_float(b);
  if (DT == FFA_BF16) return __uint_as_float(b << 16);
  const uint16_t u = (uint16_t)b;
  _Float16 h;
  __builtin_memcpy(&h, &u, 2);
  return static_cast<float>(h);
}

// The 16 bits of v in a 16-bit storage type, rounded to nearest even (the
// hardware conversions).
template <int DT>
__device__ __forceinline__ uint32_t half_bits(float v) {
  uint16_t r;
  if (DT == FFA_BF16) {
    const __bf16 h = static_cast<__bf16>(v);
    __builtin_memcpy(&r, &h, 2);
  } else {
    const _Float16 h = static_cast<_Float16>(v);
    __builtin_memcpy(&r, &h, 2);
  }
  return r;
}

// Two values in a 16-bit storage type, lo in the low half: one packed
// conversion.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
template <int DT>
__device__ __forceinline__ uint32_t pack_half2(float lo, float hi) {
  const f32x2 v = {lo, hi};
  uint32_t r;
  if (DT == FFA_BF16) {
    const bf16x2 h = __builtin_convertvector(v, bf16x2);
    __builtin_memcpy(&r, &h, 4);
  } else {
    const f16x2 h = __builtin_convertvector(v, f16x2);
    __builtin_memcpy(&r, &h, 4);
  }
  return r;
}

__device__ __forceinline__ void store_sample(void* base, int dtype, int64_t i, float v) {
  if (dtype == FFA_F32)
    static_cast<float*>(base)[i] = v;
  else if (dtype == FFA_BF16)
    static_cast<uint16_t*>(base)[i] = (uint16_t)half_bits<FFA_BF16>(v);
  else
    static_cast<uint16_t*>(base)[i] = (uint16_t)half_bits<FFA_F16>(v);
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Inclusive sum over the 64 lanes with DPP row shifts and row broadcasts
// (no LDS traffic): shifts by 1, 2, 4, 8 within each 16-lane row, then
// lane 15 of a row is added to the next row and lane 31 to rows 2 and 3.
__device__ __forceinline__ int wave_scan_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// The same for floats (the DPP moves carry the bits; the adds are FP32).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, kRowMask, 0xf, false));
}

__device__ __forceinline__ float wave_scan_dpp_f32(float v) {
  v += dpp_f32<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f32<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f32<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f32<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f32<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_f32<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Normalisation statistics (Sec. 5.2): mean and population standard deviation
// of the whole raw series, FP64. Sums are taken of x - x[0] so that a large
// offset does not cancel the variance.
// ---------------------------------------------------------------------------

constexpr int kStatsThreads = 256;

__global__ __launch_bounds__(kStatsThreads) void k_stats_partial(const SeriesDev* series,
                                                                 int dtype, double* partials) {
  const SeriesDev sd = series[blockIdx.y];
  const double x0 = (double)load_sample(sd.ptr, dtype, 0);
  double s = 0.0, ss = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kStatsThreads;
  int64_t i = (int64_t)blockIdx.x * kStatsThreads + threadIdx.x;
  if (dtype == FFA_F32 && ((uintptr_t)sd.ptr & 15) == 0) {
    const float4* v4 = static_cast<const float4*>(sd.ptr);
    const int64_t n4 = sd.nsamp / 4;
    for (int64_t k = i; k < n4; k += stride) {
      const float4 v = v4[k];
      const double a = (double)v.x - x0, b = (double)v.y - x0;
      const double c = (double)v.z - x0, d = (double)v.w - x0;
      s += (a + b) + (c + d);
      ss += (a * a + b * b) + (c * c + d * d);
    }
    for (int64_t k = n4 * 4 + i; k < sd.nsamp; k += stride) {
      const double a = (double)load_sample(sd.ptr, dtype, k) - x0;
      s += a;
      ss += a * a;
    }
  } else if (dtype != FFA_F32 && ((uintptr_t)sd.ptr & 15) == 0) {
    // 8 samples of 16 bits per 16-byte load
    const uint4* v8 = static_cast<const uint4*>(sd.ptr);
    const int64_t n8 = sd.nsamp / 8;
    for (int64_t k = i; k < n8; k += stride) {
      const uint4 v = v8[k];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float lo, hi;
        if (dtype == FFA_BF16) {
          lo = __uint_as_float(w[q] << 16);
          hi = __uint_as_float(w[q] & 0xffff0000u);
        } else {
          _Float16 h0, h1;
          const uint16_t u0 = (uint16_t)(w[q] & 0xffffu), u1 = (uint16_t)(w[q] >> 16);
          __builtin_memcpy(&h0, &u0, 2);
          __builtin_memcpy(&h1, &u1, 2);
          lo = (float)h0;
          hi = (float)h1;
        }
        const double d0 = (double)lo - x0, d1 = (double)hi - x0;
        a += d0 + d1;
        b += d0 * d0 + d1 * d1;
      }
      s += a;
      ss += b;
    }
    for (int64_t k = n8 * 8 + i; k < sd.nsamp; k += stride) {
      const double a = (double)load_sample(sd.ptr, dtype, k) - x0;
      s += a;
      ss += a * a;
    }
  } else {
    for (int64_t k = i; k < sd.nsamp; k += stride) {
      const double a = (double)load_sample(sd.ptr, dtype, k) - x0;
      s += a;
      ss += a * a;
    }
  }
  s = wave_sum(s);
  ss = wave_sum(ss);
  __shared__ double red[2][kStatsThreads / 64];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    red[0][wave] = s;
    red[1][wave] = ss;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < kStatsThreads / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    double* out = partials + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
    out[0] = a;
    out[1] = b;
  }
}

__global__ __launch_bounds__(64) void k_stats_final(const SeriesDev* series, int dtype,
                                                    int blocks_per_series,
                                                    const double* partials, double* stats,
                                                    float* norm, int32_t* flag) {
  const SeriesDev sd = series[blockIdx.x];
  const double* pp = partials + (int64_t)blockIdx.x * blocks_per_series * 2;
  double s = 0.0, ss = 0.0;
  for (int b = threadIdx.x; b < blocks_per_series; b += 64) {
    s += pp[2 * b];
    ss += pp[2 * b + 1];
  }
  s = wave_sum(s);
  ss = wave_sum(ss);
  if (threadIdx.x == 0) {
    const double n = (double)sd.nsamp;
    const double x0 = (double)load_sample(sd.ptr, dtype, 0);
    const double mshift = s / n;
    const double var = fmax(ss / n - mshift * mshift, 0.0);
    const double mean = x0 + mshift;
    const double sd_ = sqrt(var);
    stats[2 * blockIdx.x] = mean;
    stats[2 * blockIdx.x + 1] = sd_;
    float* nr = norm + kNormFloats * blockIdx.x;
    nr[0] = (float)mean;
    nr[1] = (float)(1.0 / sd_);
    nr[2] = (float)(mean - (double)(float)mean);
    nr[3] = 0.0f;
    if (sd.normalise && !(sd_ > 0.0 && isfinite(sd_) && isfinite(mean))) atomicOr(flag, 1);
  }
}

__global__ void k_clear_flag(int32_t* flag) { *flag = 0; }

__global__ void k_norm_from_stats(const double* stats, float* norm) {
  norm[0] = (float)stats[0];
  norm[1] = (float)(1.0 / stats[1]);
  norm[2] = (float)(stats[0] - (double)(float)stats[0]);
  norm[3] = 0.0f;
}

// ---------------------------------------------------------------------------
// Downsampling (Sec. 5.3, App. A.4). Output j of octave k integrates the
// normalised series over [j ds, (j+1) ds), ds = ds_fx / 2^32, each input
// sample weighted by its overlap with the window. A block owns `block` input
// samples and emits every output of every octave whose window starts among
// them; it reads those samples plus a halo that the last windows reach into
// and keeps only their exclusive prefix sum P in LDS:
//   y = (1 - fa) x[ia] + (P[ib] - P[ia + 1]) + fb x[ib],  x[i] = P[i + 1] - P[i]
// with a = ia + fa and b = ib + fb the window edges.
//
// The samples of a block are read in rounds of kDsRound: each thread takes 16
// consecutive samples with 16-byte loads, sums them in registers, and one
// block scan of the thread sums places every P; the raw samples never pass
// through LDS. The prefix restarts at every block, which bounds its
// magnitude and with it the FP32 rounding of P.
// ---------------------------------------------------------------------------

constexpr int kDsThreads = 1024;
constexpr int kDsPerThread = 16;                     // samples a thread holds per round
constexpr int kDsRound = kDsThreads * kDsPerThread;  // samples per round

// Smallest j with j * ds_fx >= x_fx (all in 2^-32 samples): a double-precision
// estimate (rcp = 1 / ds_fx), then exact integer fix-ups.
__device__ __forceinline__ int64_t first_window(uint64_t x_fx, uint64_t ds_fx, double rcp) {
  int64_t j = (int64_t)ceil((double)x_fx * rcp);
  if (j < 0) j = 0;
  while (j > 0 && (uint64_t)(j - 1) * ds_fx >= x_fx) --j;
  while ((uint64_t)j * ds_fx < x_fx) ++j;
  return j;
}

constexpr int kDsMaxOctaves = 128;

// The 16 samples [q, q + 16) of a block stretch (relative to the stretch
// start `base`, len samples), minus the mean; samples past len read as 0.
template <int DT>
__device__ __forceinline__ void ds_load16(const void* base, int q, int len, bool vec, float mean,
                                          float (&v)[kDsPerThread]) {
  if (vec && q + kDsPerThread <= len) {
    constexpr int kLoads = DT == FFA_F32 ? 4 : 2;  // 16-byte loads
    gptr<u32x4> src = (gptr<u32x4>)base + (int64_t)q / (DT == FFA_F32 ? 4 : 8);
    u32x4 w[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) w[k] = src[k];
#pragma unroll
    for (int k = 0; k < kLoads; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (DT == FFA_F32) {
          v[4 * k + e] = __uint_as_float(w[k][e]) - mean;
        } else {
          v[8 * k + 2 * e] = bits_value<DT>(w[k][e] & 0xffffu) - mean;
          v[8 * k + 2 * e + 1] = bits_value<DT>(w[k][e] >> 16) - mean;
        }
      }
    return;
  }
  // unaligned series or the ragged end: one load per sample, every load
  // issued (clamped) before any is used
  uint32_t b[kDsPerThread];
#pragma unroll
  for (int k = 0; k < kDsPerThread; ++k) b[k] = load_bits<DT>(base, min(q + k, len - 1));
#pragma unroll
  for (int k = 0; k < kDsPerThread; ++k) v[k] = q + k < len ? bits_value<DT>(b[k]) - mean : 0.0f;
}

template <int DT, int DO>
__global__ __launch_bounds__(kDsThreads) void k_downsample(const SeriesDev* series,
                                                           const int32_t* block_series,
                                                           const OctaveDev* oct,
                                                           const float* norm, void* out) {
  extern __shared__ __align__(16) float ps[];  // P[0 .. rounds * kDsRound + 1]
  __shared__ float s_part[2][kDsThreads / 64];
  __shared__ int64_t s_j0[kDsMaxOctaves], s_j1[kDsMaxOctaves];
  __shared__ uint64_t s_dsfx[kDsMaxOctaves];
  __shared__ int64_t s_off[kDsMaxOctaves];
  __shared__ int s_cum[kDsMaxOctaves + 1];
  __shared__ float s_ncorr[kDsMaxOctaves];
  const int tid = threadIdx.x;
  const int lane = tid % 64, wave = tid / 64;
  const int si = block_series ? block_series[blockIdx.x] : 0;
  const SeriesDev sd = series[si];
  const int64_t c0 = ((int64_t)blockIdx.x - sd.chunk0) * sd.block;
  if (c0 >= sd.nsamp) return;
  const int64_t c1 = min(c0 + (int64_t)sd.block, sd.nsamp);
  const int64_t cend = min(sd.nsamp, c1 + (int64_t)sd.halo);
  const int len = (int)(cend - c0);
  const int rounds = (len + kDsRound - 1) / kDsRound;
  // the samples minus the FP32 mean are summed; the window sums then drop
  // the mean's FP32 residual times the window length (ds), so that a large
  // mean leaves no bias that grows with the window
  const float mean = sd.normalise ? norm[kNormFloats * si] : 0.0f;
  const float inv = sd.normalise ? norm[kNormFloats * si + 1] : 1.0f;
  const float mean_lo = sd.normalise ? norm[kNormFloats * si + 2] : 0.0f;
  const int esize = DT == FFA_F32 ? 4 : 2;
  const void* base = static_cast<const unsigned char*>(sd.ptr) + c0 * esize;
  // block starts are multiples of 8 samples: the 16-byte loads line up when
  // the series itself starts on a 16-byte boundary
  const bool vec = (reinterpret_cast<uintptr_t>(sd.ptr) & 15) == 0;

  // window ranges of every octave, one octave per thread: outputs whose
  // window starts in [c0, c1) are j in [ceil(c0 / ds), ceil(c1 / ds)). They
  // are emitted in groups of kDsGroup consecutive outputs, the groups aligned
  // to multiples of kDsGroup in j (octaves start on such multiples in the
  // output buffer too).
  const uint64_t lo_fx = (uint64_t)c0 << 32, hi_fx = (uint64_t)c1 << 32;
  const int noct = min(sd.noct, kDsMaxOctaves);
  if (tid < noct) {
    const OctaveDev o = oct[sd.oct0 + tid];
    int64_t j0 = 0, j1 = 0;
    if (o.nsamp > 0) {
      j0 = first_window(lo_fx, o.ds_fx, o.rcp);
      j1 = min(first_window(hi_fx, o.ds_fx, o.rcp), o.nsamp);
    }
    s_j0[tid] = j0;
    s_j1[tid] = j1;
    s_dsfx[tid] = o.ds_fx;
    s_off[tid] = o.off;
    s_ncorr[tid] = (float)(-(double)mean_lo * ((double)o.ds_fx * 0x1p-32) * (double)inv);
    // groups, scanned below
    s_cum[tid + 1] = j1 > j0 ? (int)((j1 - 1) / kDsGroup - j0 / kDsGroup + 1) : 0;
  }

  // exclusive prefix sums of the stretch, a round at a time
  float carry = 0.0f;  // sum of the earlier rounds
  for (int r = 0; r < rounds; ++r) {
    const int q = r * kDsRound + tid * kDsPerThread;
    float v[kDsPerThread];
    ds_load16<DT>(base, q, len, vec, mean, v);
    float run = 0.0f;
#pragma unroll
    for (int k = 0; k < kDsPerThread; ++k) {  // v becomes the inclusive prefix
      run += v[k];
      v[k] = run;
    }
    const float incl = wave_scan_dpp_f32(run);
    if (lane == 63) s_part[r & 1][wave] = incl;
    __syncthreads();
    if (r == 0 && wave == 0) {  // output counts of the octaves -> offsets
      int cum = 0;
      for (int b = 0; b < noct; b += 64) {
        const int k = b + lane;
        const int c = k < noct ? s_cum[k + 1] : 0;
        const int ci = wave_inclusive_sum(c, lane);
        wave_lds_sync();
        if (k < noct) s_cum[k + 1] = cum + ci;
        cum += __shfl(ci, 63, 64);
      }
      if (lane == 0) s_cum[0] = 0;
    }
    // the waves' totals scanned across the first 16 lanes (one DPP row):
    // the wave's offset and the round's total are then two lane reads
    static_assert(kDsThreads / 64 == 16, "one DPP row of wave totals");
    float pw = lane < kDsThreads / 64 ? s_part[r & 1][lane] : 0.0f;
    pw += dpp_f32<0x111, 0xf>(pw);  // row_shr:1
    pw += dpp_f32<0x112, 0xf>(pw);  // row_shr:2
    pw += dpp_f32<0x114, 0xf>(pw);  // row_shr:4
    pw += dpp_f32<0x118, 0xf>(pw);  // row_shr:8
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const float total = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pw), kDsThreads / 64 - 1));
    const float woff =
        wv > 0 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pw), wv > 0 ? wv - 1 : 0)) : 0.0f;
    const float p0 = carry + woff + (incl - run);  // P at the thread's first sample
    float4* dst = reinterpret_cast<float4*>(ps + q);
#pragma unroll
    for (int k = 0; k < kDsPerThread / 4; ++k)
      dst[k] = make_float4(p0 + (k ? v[4 * k - 1] : 0.0f), p0 + v[4 * k], p0 + v[4 * k + 1],
                           p0 + v[4 * k + 2]);
    if (r == rounds - 1 && tid == kDsThreads - 1)  // P past the end: the total, twice
      ps[q + kDsPerThread] = ps[q + kDsPerThread + 1] = p0 + run;
    carry += total;
  }
  __syncthreads();

  // all output groups of all octaves, flattened; a group's octave is the
  // last one that starts at or before it (a binary search of the scanned
  // counts, which skips empty octaves). Neighbouring windows share an edge,
  // so a group reads P at kDsGroup + 1 edges.
  const int total = s_cum[noct];
  for (int u = tid; u < total; u += kDsThreads) {
    int k = 0;
#pragma unroll
    for (int step = kDsMaxOctaves / 2; step >= 1; step >>= 1)
      if (k + step < noct && s_cum[k + step] <= u) k += step;
    const uint64_t dsfx = s_dsfx[k];
    const float ncorr = s_ncorr[k];
    const int64_t jlo = s_j0[k], jhi = s_j1[k];
    const int64_t jg = (jlo / kDsGroup + (u - s_cum[k])) * kDsGroup;  // first output of the group
    // edges e = 0..kDsGroup at a = (jg + e) ds, in 2^-32 samples from the
    // stretch start: the integer part is the sample an edge falls in, the
    // fraction how far into it. Outside the block's windows (outputs of the
    // group that belong to a neighbouring block) the reads are clamped into
    // the stretch and the outputs dropped.
    float y[kDsGroup];
    float d_prev = 0.0f, g_prev = 0.0f, p1_prev = 0.0f;
    uint64_t a = (uint64_t)jg * dsfx - ((uint64_t)c0 << 32);
#pragma unroll
    for (int e = 0; e <= kDsGroup; ++e) {
      const int ia = min(max((int)(a >> 32), 0), len);
      const float p0 = ps[ia];
      const float p1 = ps[ia + 1];  // P[len + 1] repeats P[len]
      const float d = p1 - p0;                                          // x of the edge sample
      const float g = (float)(uint32_t)a * 2.3283064365386963e-10f * d;  // its part left of the edge
      // window [a_e-1, a_e): the part of the first sample right of its edge,
      // the whole samples between, and the part of the last sample left of
      // its edge
      if (e > 0) y[e - 1] = fmaf((d_prev - g_prev) + (p0 - p1_prev) + g, inv, ncorr);
      d_prev = d;
      g_prev = g;
      p1_prev = p1;
      a += dsfx;
    }
    const int64_t o0 = s_off[k] + jg;
    if (jg >= jlo && jg + kDsGroup <= jhi) {
      if (DO == FFA_F32) {
        gptr_w<u32x4> dst = (gptr_w<u32x4>)((float*)out + o0);
#pragma unroll
        for (int q = 0; q < kDsGroup / 4; ++q) {
          u32x4 w;
#pragma unroll
          for (int e = 0; e < 4; ++e) w[e] = __float_as_uint(y[4 * q + e]);
          dst[q] = w;
        }
      } else {
        gptr_w<u32x4> dst = (gptr_w<u32x4>)((uint16_t*)out + o0);
#pragma unroll
        for (int q = 0; q < kDsGroup / 8; ++q) {
          u32x4 w;
#pragma unroll
          for (int e = 0; e < 4; ++e) w[e] = pack_half2<DO>(y[8 * q + 2 * e], y[8 * q + 2 * e + 1]);
          dst[q] = w;
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < kDsGroup; ++e)
        if (jg + e >= jlo && jg + e < jhi) store_sample(out, DO, o0 + e, y[e]);
    }
  }
}

// ---------------------------------------------------------------------------
// Folding transform tiles (Sec. 2.2).
//
// The FFA of an m-row block is a binary tree: a block of n >= 2 rows splits
// into a head of m_h = floor(n/2) rows and a tail of m_t = n - m_h rows, and
// row s of its transform is F_s = H_i + (T_j << (s - j)), with
// i = nint((m_h - 1) s / (n - 1)), j = nint((m_t - 1) s / (n - 1)) (ties up).
// A one-row block is its own transform.
//
// A tile computes some rows of one node of that tree inside LDS, level by
// level, every level in place: each thread computes its items into
// registers, the workgroup synchronises, then writes them back.
//   full tile:  a whole subtree, loaded from the input rows;
//   range tile: rows [s0, s1) of a node from the rows L levels below it
//               (read from a scratch buffer written by the previous pass);
//               only the rows that the requested range needs are kept at
//               each level.
// When the node is the root, the rows are final: their boxcar S/N is
// computed and written to the periodogram (or the rows themselves are
// written out, for the raw transform).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void merge_indices(int n, int s, int& i, int& j) {
  // nint(a / c) with ties up is floor((2a + c) / (2c)); a double-precision
  // quotient, then an exact integer fix-up
  const int mh = n >> 1, mt = n - mh;
  const int64_t den = 2 * (int64_t)(n - 1);
  const int64_t ni = 2 * (int64_t)(mh - 1) * s + (n - 1);
  const int64_t nj = 2 * (int64_t)(mt - 1) * s + (n - 1);
  const double rd = 1.0 / (double)den;
  int64_t qi = (int64_t)((double)ni * rd), qj = (int64_t)((double)nj * rd);
  if (qi * den > ni) --qi;
  if ((qi + 1) * den <= ni) ++qi;
  if (qj * den > nj) --qj;
  if ((qj + 1) * den <= nj) ++qj;
  i = (int)qi;
  j = (int)qj;
}

// nint(k s / (n - 1)), ties up, for blocks of at most 32768 rows (k = m_h - 1
// gives i, k = m_t - 1 gives j): an FP32 reciprocal estimate of the quotient
// (off by at most one) and an exact fix-up in 32-bit integers.
__device__ __forceinline__ int merge_index_small(int n, int k, int s) {
  const unsigned den = 2u * (unsigned)(n - 1);
  const unsigned num = 2u * (unsigned)k * (unsigned)s + (unsigned)(n - 1);
  unsigned q = (unsigned)((float)num * __builtin_amdgcn_rcpf((float)den));
  if (q * den > num) --q;
  if ((q + 1) * den <= num) ++q;
  return (int)q;
}

// Both indices; the FP64 form above past 32768 rows.
__device__ __forceinline__ void merge_indices_fast(int n, int s, int& i, int& j) {
  if (n > 32768) {
    merge_indices(n, s, i, j);
    return;
  }
  const int mh = n >> 1, mt = n - mh;
  const unsigned den = 2u * (unsigned)(n - 1);
  const unsigned ni = 2u * (unsigned)(mh - 1) * (unsigned)s + (unsigned)(n - 1);
  const unsigned nj = 2u * (unsigned)(mt - 1) * (unsigned)s + (unsigned)(n - 1);
  const float rd = __builtin_amdgcn_rcpf((float)den);
  unsigned qi = (unsigned)((float)ni * rd), qj = (unsigned)((float)nj * rd);
  if (qi * den > ni) --qi;
  if ((qi + 1) * den <= ni) ++qi;
  if (qj * den > nj) --qj;
  if ((qj + 1) * den <= nj) ++qj;
  i = (int)qi;
  j = (int)qj;
}

__device__ __forceinline__ void node_geometry(int m, int d, int node, int& r0, int& n) {
  int base = 0, size = m;
  for (int b = d - 1; b >= 0; --b) {
    const int mh = size >> 1;
    if ((node >> b) & 1) {
      base += mh;
      size -= mh;
    } else {
      size = mh;
    }
  }
  r0 = base;
  n = size;
}

__device__ __forceinline__ int ceil_log2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Slot <-> (row of the wave, column iteration) mapping shared by the load,
// merge and store phases: slot = r * J + j, row q = wave + WV r, column
// group lane + 64 j. JS = 1 fixes J = 1 at compile time (one column group
// per lane).
template <int JS>
struct Slots {
  int J;
  __device__ __forceinline__ int row(int slot) const { return JS == 1 ? slot : slot / J; }
  __device__ __forceinline__ int iter(int slot) const { return JS == 1 ? 0 : slot - (slot / J) * J; }
};

// The operation of one output row of a merge level, held by lane r of a wave
// for the wave's row r: output <- row h + (row t << rot). Plain copies (and
// one-row blocks, which stay) add the all-zero row.
struct LaneOp {
  int h, t, rot;
};

// One merge level of single rows, in place (the all-LDS form, for rows too
// wide for the register levels and the pair merges), for waves whose rows
// fit in NS slots: a wave takes output rows wave, wave + WV, ...; lane l
// owns the column groups
// l, l + 64, ... of kChunk columns. All reads of a lane are issued first, the
// workgroup synchronises, then the outputs are written back. Groups that
// start past p compute the row's wrapped copy; lanes and slots with nothing
// to write send their values to the junk row, so no step branches.
template <int WV, int JS, int NS>
__device__ __forceinline__ void merge_level_ns(float* rows, int p, int stride, int J,
                                               const LaneOp& op, float* junk, int nrw) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const Slots<JS> sl{J};
  float acc[NS][kChunk];
#pragma unroll
  for (int slot = 0; slot < NS; ++slot) {
    const int r = sl.row(slot);
    const int h = __builtin_amdgcn_readlane(op.h, r);
    const int tl = __builtin_amdgcn_readlane(op.t, r);
    const int rot = __builtin_amdgcn_readlane(op.rot, r);
    const int col0 = (lane + 64 * sl.iter(slot)) * kChunk;
    int t0 = col0 + rot;
    t0 = t0 >= p ? t0 - p : t0;
    if (p < kChunk) t0 %= p;  // rows shorter than the copy
    const float* hr = rows + h * stride + col0;
    const float* trow = rows + tl * stride + t0;
#pragma unroll
    for (int e = 0; e < kChunk; ++e) acc[slot][e] = hr[e] + trow[e];
  }
  __syncthreads();
  const int G = merge_groups(p);
#pragma unroll
  for (int slot = 0; slot < NS; ++slot) {
    const int r = sl.row(slot);
    const int c = lane + 64 * sl.iter(slot);
    float* o = (r < nrw && c < G) ? rows + (wave + WV * r) * stride + c * kChunk : junk;
#pragma unroll
    for (int e = 0; e < kChunk; ++e) o[e] = acc[slot][e];
  }
  __syncthreads();
}

template <int WV, int JS>
__device__ __forceinline__ void merge_level(float* rows, int count, int p, int stride, int J,
                                            const LaneOp& op, float* junk) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nrw = count > wave ? (count - wave + WV - 1) / WV : 0;
  const int need = nrw * J;
  if (need <= 4)
    merge_level_ns<WV, JS, 4>(rows, p, stride, J, op, junk, nrw);
  else if (need <= 8)
    merge_level_ns<WV, JS, 8>(rows, p, stride, J, op, junk, nrw);
  else
    merge_level_ns<WV, JS, kStageMax>(rows, p, stride, J, op, junk, nrw);
}

// ---------------------------------------------------------------------------
// Pair merges. Where two consecutive output rows of a node share their tail
// row (rotations k and k + 1), one lane reads kChunk + 1 bins of the tail
// once and the head row(s), and writes both outputs: 15 LDS instructions and
// about 24 VALU instructions per 10 outputs instead of 18 and 35 for two
// single rows. A single (a row with no partner) has no second output
// (ob = -1). Operation q of a level is held by lane q / WV of wave q % WV
// as LDS byte offsets.
// ---------------------------------------------------------------------------

struct PairOp {
  int ha, hb, t, rot4, oa, ob;
};

template <int WV, int NS>
__device__ __forceinline__ void merge_pairs_ns(unsigned char* base, int p4, int lane20,
                                               const PairOp& op, int nrw) {
  float a[NS][kChunk], b[NS][kChunk];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (r < nrw) {
      const int ha = __builtin_amdgcn_readlane(op.ha, r);
      const int hb = __builtin_amdgcn_readlane(op.hb, r);
      const int tb = __builtin_amdgcn_readlane(op.t, r);
      const int rot4 = __builtin_amdgcn_readlane(op.rot4, r);
      unsigned tc = (unsigned)(lane20 + rot4);
      const unsigned tw = tc - (unsigned)p4;
      tc = tc < tw ? tc : tw;  // wrapped below p
      const float* tr = reinterpret_cast<const float*>(base + tb + tc);
      const float* hr = reinterpret_cast<const float*>(base + ha + lane20);
      float tv[kChunk + 1], hv[kChunk];
#pragma unroll
      for (int e = 0; e <= kChunk; ++e) tv[e] = tr[e];
#pragma unroll
      for (int e = 0; e < kChunk; ++e) hv[e] = hr[e];
#pragma unroll
      for (int e = 0; e < kChunk; ++e) a[r][e] = hv[e] + tv[e];
      if (hb == ha) {
#pragma unroll
        for (int e = 0; e < kChunk; ++e) b[r][e] = hv[e] + tv[e + 1];
      } else {
        const float* hr2 = reinterpret_cast<const float*>(base + hb + lane20);
#pragma unroll
        for (int e = 0; e < kChunk; ++e) b[r][e] = hr2[e] + tv[e + 1];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (r < nrw) {
      const int oa = __builtin_amdgcn_readlane(op.oa, r);
      const int ob = __builtin_amdgcn_readlane(op.ob, r);
      float* wa = reinterpret_cast<float*>(base + oa + lane20);
#pragma unroll
      for (int e = 0; e < kChunk; ++e) wa[e] = a[r][e];
      if (ob >= 0) {  // not a single
        float* wb = reinterpret_cast<float*>(base + ob + lane20);
#pragma unroll
        for (int e = 0; e < kChunk; ++e) wb[e] = b[r][e];
      }
    }
  }
  __syncthreads();
}

template <int WV>
__device__ __forceinline__ void merge_pairs(unsigned char* base, int p4, int lane20, const PairOp& op,
                                            int nops) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nrw = nops > wave ? (nops - wave + WV - 1) / WV : 0;
  const int most = (nops + WV - 1) / WV;  // the same choice in every wave
  if (most <= 2)
    merge_pairs_ns<WV, 2>(base, p4, lane20, op, nrw);
  else if (most <= 3)
    merge_pairs_ns<WV, 3>(base, p4, lane20, op, nrw);
  else if (most <= 5)
    merge_pairs_ns<WV, 5>(base, p4, lane20, op, nrw);
  else
    merge_pairs_ns<WV, 8>(base, p4, lane20, op, nrw);
}

// ---------------------------------------------------------------------------
// Register levels of a full tile. A wave takes a bottom node of at most
// kRegRows rows: lane l holds bins 5l .. 5l + 4 (mod p) of each row, over all
// 64 lanes, and the node's own merges run in registers. A rotation by k <= 5
// bins takes bins e + k < 5 from the lane itself and the rest from lane
// l + 1 (DPP wave shift). The last lane has no right neighbour, so after L
// levels the top L lanes are wrong; they only hold copies past the row's
// kChunk-column groups, which is why the register levels need
// merge_groups(p) + L <= 64.
// ---------------------------------------------------------------------------

__host__ __device__ constexpr int ce_head(int n, int s) {
  return (2 * (n / 2 - 1) * s + (n - 1)) / (2 * (n - 1));
}
__host__ __device__ constexpr int ce_tail(int n, int s) {
  return (2 * ((n - n / 2) - 1) * s + (n - 1)) / (2 * (n - 1));
}

__device__ __forceinline__ float from_next_lane(float v) {
  // wave_shl:1 -- lane l receives lane l + 1; the last lane receives 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__host__ __device__ constexpr int ce_max_rotation(int n) {
  int m = 0;
  for (int s = 0; s < n; ++s) m = (s - ce_tail(n, s)) > m ? (s - ce_tail(n, s)) : m;
  return m;
}

template <int OFF, int N>
struct RegFFA {
  static_assert(ce_max_rotation(N) <= kChunk, "register merges shift by at most one lane");
  static __device__ __forceinline__ void run(float (&v)[kRegRows][kChunk]) {
    constexpr int MH = N / 2, MT = N - MH;
    RegFFA<OFF, MH>::run(v);
    RegFFA<OFF + MH, MT>::run(v);
    float nx[MT][kChunk];
#pragma unroll
    for (int r = 0; r < MT; ++r)
#pragma unroll
      for (int e = 0; e < kChunk; ++e) nx[r][e] = from_next_lane(v[OFF + MH + r][e]);
    float o[N][kChunk];
#pragma unroll
    for (int s = 0; s < N; ++s) {
      const int i = ce_head(N, s), j = ce_tail(N, s), k = s - j;
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int c = e + k;
        o[s][e] = v[OFF + i][e] + (c < kChunk ? v[OFF + MH + j][c] : nx[j][c - kChunk]);
      }
    }
#pragma unroll
    for (int s = 0; s < N; ++s)
#pragma unroll
      for (int e = 0; e < kChunk; ++e) v[OFF + s][e] = o[s][e];
  }
};
template <int OFF>
struct RegFFA<OFF, 1> {
  static __device__ __forceinline__ void run(float (&)[kRegRows][kChunk]) {}
};

// Loads the bottom nodes at depth d_r of an n-row full tile (rows of p bins
// starting at element `base` of the input), folds each in registers and
// writes the rows to LDS with their copied bins.
template <int WV, int DT>
__device__ __forceinline__ void reg_phase(const void* in, int64_t base, int n, int p, int d_r,
                                          float* rows, int stride) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int G = merge_groups(p);
  uint32_t col[kChunk];
#pragma unroll
  for (int e = 0; e < kChunk; ++e) col[e] = (uint32_t)(lane * kChunk + e) % (uint32_t)p;
  const int nodes = 1 << d_r;
  for (int b = wave; b < nodes; b += WV) {
    int r0b, nb;
    node_geometry(n, d_r, b, r0b, nb);
    if (nb == 0) continue;
    uint32_t raw[kRegRows][kChunk];
    const int64_t rb = base + (int64_t)r0b * p;
#pragma unroll
    for (int r = 0; r < kRegRows; ++r)
#pragma unroll
      for (int e = 0; e < kChunk; ++e)
        // unconditional loads, all in flight together with no branch between
        // them: rows past the node re-read its last row (the merges of an
        // nb-row node and the stores below never use rows nb and up); the
        // row start is uniform and the lane's column a 32-bit offset
        raw[r][e] = load_row_bits<DT>(in, rb + (int64_t)(r < nb ? r : nb - 1) * p, col[e]);
    float v[kRegRows][kChunk];
#pragma unroll
    for (int r = 0; r < kRegRows; ++r)
#pragma unroll
      for (int e = 0; e < kChunk; ++e) v[r][e] = bits_value<DT>(raw[r][e]);
    switch (nb) {
      case 2: RegFFA<0, 2>::run(v); break;
      case 3: RegFFA<0, 3>::run(v); break;
      case 4: RegFFA<0, 4>::run(v); break;
      case 5: RegFFA<0, 5>::run(v); break;
      case 6: RegFFA<0, 6>::run(v); break;
      case 7: RegFFA<0, 7>::run(v); break;
      case 8: RegFFA<0, 8>::run(v); break;
      default: break;
    }
    if (lane < G) {
#pragma unroll
      for (int r = 0; r < kRegRows; ++r) {
        if (r < nb) {
          float* o = rows + (r0b + r) * stride + lane * kChunk;
#pragma unroll
          for (int e = 0; e < kChunk; ++e) o[e] = v[r][e];
        }
      }
    }
  }
}

// A full tile of n rows with one column group per lane: register levels up
// to nodes of at most kRegRows rows, then pair merges in LDS with the host's
// pair schedule. Needs merge_groups(p) + kRegLevels <= 64.
template <int WV, int DT>
__device__ __forceinline__ void full_tile_pairs(const PassArgs& a, int64_t base, int n, int p,
                                                int stride, float* rows, int R) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int G = merge_groups(p);
  int d_r = 0;
  while (((n + (1 << d_r) - 1) >> d_r) > kRegRows) ++d_r;
  // the lane's pair operations of every LDS level, fetched before the
  // register levels so that their latency hides behind them
  const int32_t* offs = a.full_pops_off + n * (kMaxFullLevels + 1);
  uint32_t w0[kMaxTileLevels], w1[kMaxTileLevels];
#pragma unroll
  for (int lev = 0; lev < kMaxTileLevels; ++lev) {
    w0[lev] = 0;
    w1[lev] = 1u << 31;  // no operation
    if (lev < d_r) {
      const int o0 = offs[lev], cnt = offs[lev + 1] - o0;
      const int q = wave + WV * lane;
      if (q < cnt) {
        w0[lev] = a.full_pops[2 * (o0 + q)];
        w1[lev] = a.full_pops[2 * (o0 + q) + 1];
      }
    }
  }
  reg_phase<WV, DT>(a.in, base, n, p, d_r, rows, stride);
  if (d_r == 0) {
    __syncthreads();
    return;
  }
  const int stride4 = stride * 4, p4 = p * 4;
  // lanes past the row's column groups repeat a group (same reads, same
  // values written to the same place)
  const int lane20 = (lane < G ? lane : lane % G) * kChunk * 4;
  const int junk4 = (R + 1) * stride4;
  auto decode = [&](uint32_t x0, uint32_t x1) {
    PairOp op{0, 0, 0, 0, junk4, junk4};
    if (!(x1 >> 31)) {
      op.oa = (int)(x0 & 255u) * stride4;
      op.ha = (int)((x0 >> 8) & 255u) * stride4;
      op.hb = (int)((x0 >> 16) & 255u) * stride4;
      op.t = (int)(x0 >> 24) * stride4;
      int rot = (int)(x1 & 0xffffu);
      if (rot >= p) rot %= p;
      op.rot4 = rot * 4;
      op.ob = (x1 >> 16) & 1u ? -1 : op.oa + stride4;
    }
    return op;
  };
  auto fetch = [&](int lev) {
    uint32_t x0 = 0, x1 = 1u << 31;
#pragma unroll
    for (int k = 0; k < kMaxTileLevels; ++k)
      if (k == lev) {
        x0 = w0[k];
        x1 = w1[k];
      }
    return decode(x0, x1);
  };
  int lev = d_r - 1;
  PairOp cur = fetch(lev);
  __syncthreads();  // the register levels' rows are in LDS
  for (; lev >= 0; --lev) {
    const PairOp nxt = fetch(lev - 1);
    merge_pairs<WV>(reinterpret_cast<unsigned char*>(rows), p4, lane20, cur,
                    offs[lev + 1] - offs[lev]);
    cur = nxt;
  }
}

// Loads rows [0, count) into LDS with their wrapped copies; lane r of each
// wave holds in `src` the element offset of the wave's row r. Lanes take
// consecutive columns (coalesced). With one column group per lane (JS = 1,
// rows of at most 316 bins) every load of a lane is issued before its first
// LDS store, so a tile pays one memory round trip; wider rows go four rows at
// a time.
template <int WV, int JS, int DT>
__device__ __forceinline__ void load_rows(float* rows, int count, int p, int stride,
                                          const void* base, int64_t src) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int nrw = count > wave ? (count - wave + WV - 1) / WV : 0;
  const int width = p + kHalo;
  const int lo = (int)(src & 0xffffffff), hi = (int)(src >> 32);
  if (JS == 1) {
    constexpr int KC = 5;  // 5 x 64 columns >= p + kHalo whenever one group per lane suffices
    if (nrw == 0) return;
    // 16-bit types: unconditional loads (rows past the wave's count re-read
    // its first row, columns past the copy wrap), so the conversions are not
    // sunk between them; FP32 keeps the conditions
    uint32_t v[kStageMax][KC];
#pragma unroll
    for (int r = 0; r < kStageMax; ++r) {
      const int rr = (DT == FFA_F32 || r < nrw) ? r : 0;
      const int64_t g = (int64_t)(uint32_t)__builtin_amdgcn_readlane(lo, rr) |
                        ((int64_t)__builtin_amdgcn_readlane(hi, rr) << 32);
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int c = lane + 64 * k;
        int col = c < p ? c : c - p;
        if (col >= p) col %= p;  // rows shorter than the copy
        v[r][k] = DT == FFA_F32 ? ((r < nrw && c < width) ? load_bits<DT>(base, g + col) : 0u)
                                : load_bits<DT>(base, g + col);
      }
    }
#pragma unroll
    for (int r = 0; r < kStageMax; ++r)
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int c = lane + 64 * k;
        if (r < nrw && c < width) rows[(wave + WV * r) * stride + c] = bits_value<DT>(v[r][k]);
      }
    return;
  }
  for (int rb = 0; rb < nrw; rb += 4) {
    int64_t g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      g[u] = (int64_t)(uint32_t)__builtin_amdgcn_readlane(lo, min(rb + u, 63)) |
             ((int64_t)__builtin_amdgcn_readlane(hi, min(rb + u, 63)) << 32);
    for (int c0 = 0; c0 < width; c0 += 128) {
      uint32_t v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int c = c0 + lane + 64 * k;
          int col = c < p ? c : c - p;
          if (col >= p) col %= p;
          v[u][k] = (rb + u < nrw && c < width) ? load_bits<DT>(base, g[u] + col) : 0u;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int c = c0 + lane + 64 * k;
          if (rb + u < nrw && c < width)
            rows[(wave + WV * (rb + u)) * stride + c] = bits_value<DT>(v[u][k]);
        }
    }
  }
}

// load_rows for one column group per lane and FP32 rows, with `work` run
// between the loads and the LDS stores (while the loads are in flight). It
// reads scratch rows, each once, with non-temporal loads.
template <int WV, class F>
__device__ __forceinline__ void load_rows_overlap(float* rows, int count, int p, int stride,
                                                  const float* base, int64_t src, F&& work) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int nrw = count > wave ? (count - wave + WV - 1) / WV : 0;
  const int width = p + kHalo;
  const int lo = (int)(src & 0xffffffff), hi = (int)(src >> 32);
  constexpr int KC = 5;
  // column of copy position c = lane + 64 k (c - p past the row end; shorter
  // rows than half the copy take a remainder, one uniform branch); lanes past
  // the copy repeat its last position, so they read a line the load reads
  // anyway (their values are not stored)
  uint32_t col[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = min(lane + 64 * k, width - 1);
    col[k] = (uint32_t)(c < p ? c : c - p);
  }
  if (2 * p < 64 * KC) {
#pragma unroll
    for (int k = 0; k < KC; ++k) col[k] %= (uint32_t)p;
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) col[k] *= 4u;  // byte offsets: a scalar row start plus a vector offset
  // loads without lane conditions (every address is in the row), the rows
  // past the wave's count skipped by a wave-uniform branch: no use of a
  // loaded value sits between the loads, so they are all in flight together
  float v[kStageMax][KC];
#pragma unroll
  for (int r = 0; r < kStageMax; ++r) {
    if (r < nrw) {
      const int64_t g = (int64_t)(uint32_t)__builtin_amdgcn_readlane(lo, r) |
                        ((int64_t)__builtin_amdgcn_readlane(hi, r) << 32);
      gptr<unsigned char> rp = (gptr<unsigned char>)((gptr<float>)base + g);
#pragma unroll
      for (int k = 0; k < KC; ++k) v[r][k] = __builtin_nontemporal_load((gptr<float>)(rp + col[k]));
    }
  }
  work();
  auto put = [&](auto all) {
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      if (lane + 64 * k < width) {
#pragma unroll
        for (int r = 0; r < kStageMax; ++r)
          if (decltype(all)::value || r < nrw) rows[(wave + WV * r) * stride + lane + 64 * k] = v[r][k];
      }
    }
  };
  if (nrw == kStageMax)
    put(std::true_type{});
  else
    put(std::false_type{});
}

// Writes rows [0, count) of LDS to global rows dst + q * p, coalesced. The
// stores are non-temporal: these rows (scratch between passes, or output
// rows) are read once, by a later launch, and need not displace the
// downsampled series that the transforms of a pseudo-octave share in L2.
// The rows of a wave (row wave + WV r for r < nrw, every r when kAll) with
// one column group per lane: lane l takes columns l + 64 k, those past the
// row end repeating its last column (such lanes read and store the same
// value at the same place, so no lane condition is needed).
template <int WV, bool kAll>
__device__ __forceinline__ void store_rows_g1(const float* rows, int nrw, int p, int stride, float* dst,
                                              int wave, int lane) {
  constexpr int KC = 5;
  uint32_t cc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = lane + 64 * k;
    cc[k] = (uint32_t)(c < p ? c : p - 1);
  }
  float v[kStageMax][KC];
#pragma unroll
  for (int r = 0; r < kStageMax; ++r)
    if (kAll || r < nrw) {
      const float* rw = rows + (wave + WV * r) * stride;
#pragma unroll
      for (int k = 0; k < KC; ++k) v[r][k] = rw[cc[k]];
    }
#pragma unroll
  for (int r = 0; r < kStageMax; ++r)
    if (kAll || r < nrw) {
      // a scalar row start plus a vector byte offset
      gptr_w<unsigned char> rp = (gptr_w<unsigned char>)((gptr_w<float>)dst + (int64_t)(wave + WV * r) * p);
#pragma unroll
      for (int k = 0; k < KC; ++k) __builtin_nontemporal_store(v[r][k], (gptr_w<float>)(rp + 4u * cc[k]));
    }
}

template <int WV, int JS>
__device__ __forceinline__ void store_rows(const float* rows, int count, int p, int stride,
                                           float* dst) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int nrw = count > wave ? (count - wave + WV - 1) / WV : 0;
  if (JS == 1) {
    if (nrw == kStageMax)
      store_rows_g1<WV, true>(rows, nrw, p, stride, dst, wave, lane);
    else if (nrw > 0)
      store_rows_g1<WV, false>(rows, nrw, p, stride, dst, wave, lane);
    return;
  }
  for (int rb = 0; rb < nrw; rb += 4) {
    for (int c0 = 0; c0 < p; c0 += 128) {
      float v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int c = c0 + lane + 64 * k;
          v[u][k] = (rb + u < nrw && c < p) ? rows[(wave + WV * (rb + u)) * stride + c] : 0.0f;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int c = c0 + lane + 64 * k;
          if (rb + u < nrw && c < p)
            __builtin_nontemporal_store(v[u][k], &dst[(int64_t)(wave + WV * (rb + u)) * p + c]);
        }
    }
  }
}

// Range-tile metadata: node h of the tile's subtree (heap order, level l holds
// nodes (1 << l) - 1 ...), fields r0 (first row in the transform), n (rows),
// [lo, hi) rows kept, off (position of row lo in LDS), ooff (first pair
// operation of the node within its level); lops[l] = operations of level l.
struct Meta {
  int* r0;
  int* n;
  int* lo;
  int* hi;
  int* off;
  int* ooff;
  int* lops;
};

// Pair operations of node rows [lo, hi) of an n-row node (n >= 2): rows s and
// s + 1 share their tail row when s is even (n even) or odd (n odd), so a
// leading row of the other parity and a trailing unpaired row are singles.
__device__ __forceinline__ int node_pair_ops(int n, int lo, int hi) {
  if (hi <= lo || n <= 0) return 0;
  if (n == 1) return 1;
  const int lead = ((lo & 1) != (n & 1)) ? 1 : 0;
  const int rem = hi - lo - lead;
  return lead + (rem >> 1) + (rem & 1);
}

// Built by wave 0: lane v handles node v of a level.
__device__ __forceinline__ void build_meta(Meta M, int r0, int n, int s0, int s1, int L) {
  const int lane = threadIdx.x & 63;
  if (lane == 0) {
    M.r0[0] = r0;
    M.n[0] = n;
    M.lo[0] = s0;
    M.hi[0] = s1;
    M.off[0] = 0;
  }
  wave_lds_sync();
  for (int l = 0; l < L; ++l) {
    const int cfirst = (2 << l) - 1;
    if (lane < (1 << l)) {
      const int h = (1 << l) - 1 + lane, hc = cfirst + 2 * lane;
      const int pn = M.n[h], plo = M.lo[h], phi = M.hi[h];
      if (phi <= plo || pn == 0) {
        M.r0[hc] = M.r0[hc + 1] = M.r0[h];
        M.n[hc] = M.n[hc + 1] = 0;
        M.lo[hc] = M.hi[hc] = M.lo[hc + 1] = M.hi[hc + 1] = 0;
      } else if (pn == 1) {
        M.r0[hc] = M.r0[h];
        M.n[hc] = 0;
        M.lo[hc] = M.hi[hc] = 0;
        M.r0[hc + 1] = M.r0[h];
        M.n[hc + 1] = 1;
        M.lo[hc + 1] = 0;
        M.hi[hc + 1] = 1;
      } else {
        const int mh = pn >> 1;
        int i0, j0, i1, j1;
        merge_indices_fast(pn, plo, i0, j0);
        merge_indices_fast(pn, phi - 1, i1, j1);
        M.r0[hc] = M.r0[h];
        M.n[hc] = mh;
        M.lo[hc] = i0;
        M.hi[hc] = i1 + 1;
        M.r0[hc + 1] = M.r0[h] + mh;
        M.n[hc + 1] = pn - mh;
        M.lo[hc + 1] = j0;
        M.hi[hc + 1] = j1 + 1;
      }
    }
    {
      const int ops = lane < (1 << l) ? node_pair_ops(M.n[(1 << l) - 1 + lane], M.lo[(1 << l) - 1 + lane],
                                                      M.hi[(1 << l) - 1 + lane])
                                      : 0;
      const int incl = wave_inclusive_sum(ops, lane);
      if (lane < (1 << l)) M.ooff[(1 << l) - 1 + lane] = incl - ops;
      if (lane == 63) M.lops[l] = incl;
    }
    wave_lds_sync();
    const int len = lane < (2 << l) ? M.hi[cfirst + lane] - M.lo[cfirst + lane] : 0;
    const int incl = wave_inclusive_sum(len, lane);
    if (lane < (2 << l)) M.off[cfirst + lane] = incl - len;
    wave_lds_sync();
  }
}

// The same metadata with every node computed at once: lane h (heap index)
// walks from the tile's node down its path, the row and operation offsets
// are scans within each level. One wave, no LDS round trips between levels.
__device__ __forceinline__ void build_meta_par(Meta M, int r0, int n, int s0, int s1, int L) {
  const int lane = threadIdx.x & 63;
  const int nn = (2 << L) - 1;
  int hr0 = r0, hn = n, hlo = s0, hhi = s1, lev = 0;
  if (lane < nn) {
    lev = 31 - __builtin_clz(lane + 1);
    const int v = lane + 1 - (1 << lev);
    for (int b = lev - 1; b >= 0; --b) {
      const bool right = (v >> b) & 1;
      if (hhi <= hlo || hn == 0) {
        hn = 0;
        hlo = hhi = 0;
      } else if (hn == 1) {  // a one-row block: its tail child is the row
        hn = right ? 1 : 0;
        hlo = 0;
        hhi = right ? 1 : 0;
      } else {
        const int mh = hn >> 1;
        const int k = right ? hn - mh - 1 : mh - 1;  // m_t - 1 or m_h - 1
        int c0, c1;
        if (hn <= 32768) {
          c0 = merge_index_small(hn, k, hlo);
          c1 = merge_index_small(hn, k, hhi - 1);
        } else {
          int i0, j0, i1, j1;
          merge_indices(hn, hlo, i0, j0);
          merge_indices(hn, hhi - 1, i1, j1);
          c0 = right ? j0 : i0;
          c1 = right ? j1 : i1;
        }
        if (right) hr0 += mh;
        hn = right ? hn - mh : mh;
        hlo = c0;
        hhi = c1 + 1;
      }
    }
  }
  // rows (low half) and operations (high half) of the node, scanned together
  const int len = lane < nn ? hhi - hlo : 0;
  const int ops = (lane < nn && lev < L) ? node_pair_ops(hn, hlo, hhi) : 0;
  const int both = len | (ops << 16);
  const int incl = wave_scan_dpp(both);
  // inclusive sums up to the last node of each level above (heap index 2^l - 2)
  int before = 0;
#pragma unroll
  for (int l = 1; l <= kMaxRangeLevels; ++l) {
    const int b = __builtin_amdgcn_readlane(incl, (1 << l) - 2);
    before = lev == l ? b : before;
  }
  const int excl = incl - both - before;
  if (lane < nn) {
    M.r0[lane] = hr0;
    M.n[lane] = hn;
    M.lo[lane] = hlo;
    M.hi[lane] = hhi;
    M.off[lane] = excl & 0xffff;
    M.ooff[lane] = excl >> 16;
    if (lane == (2 << lev) - 2 && lev < L) M.lops[lev] = (incl - before) >> 16;
  }
}

// Node (heap index) of level l holding position q.
__device__ __forceinline__ int find_node(const Meta& M, int l, int q);

// A range tile with one column group per lane: the rows L levels below from
// scratch (the tile's source-row list, made by the host in the order of the
// node metadata), and while their loads are in flight the node metadata
// (wave 0) and every level's pair operations (all threads, LDS byte offsets
// into `ops`, six ints each); then L pair-merge levels. Needs
// merge_groups(p) <= 64.
template <int WV>
__device__ __forceinline__ void range_tile_pairs(const PassArgs& a, const TileDesc& t, const XformDesc& x,
                                                 int r0, int n, int p, int stride, float* rows, int R,
                                                 const Meta& M, int* ops) {
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int L = t.levels;
  const int G = merge_groups(p);
  const int stride4 = stride * 4, p4 = p * 4;
  const int junk4 = (R + 1) * stride4, zero4 = R * stride4;
  constexpr int kThreads = WV * 64;
  const int32_t* srows = a.src_rows + t.rows_off;  // count, then the rows
  const int total = srows[0];
  const float* src = (t.bufs & 1) ? a.scr1 : a.scr0;
  const int q_lane = wave + WV * lane;
  int lbase[kMaxRangeLevels + 1];
  // the source rows' loads are in flight while the metadata and the pair
  // operations of every level are built: kThreads / 8 threads per level (a
  // power of two, at least one per node), an equal share of them per node of
  // the level
  load_rows_overlap<WV>(rows, total, p, stride, src + x.scr_off,
                        q_lane < total ? (int64_t)srows[1 + q_lane] * p : 0, [&]() {
  if (wave == 0) build_meta_par(M, r0, n, t.s0, t.s1, L);
  __syncthreads();
  lbase[0] = 0;
#pragma unroll
  for (int l = 0; l < kMaxRangeLevels; ++l) lbase[l + 1] = lbase[l] + (l < L ? M.lops[l] : 0);
  static_assert(kMaxRangeLevels <= 8 && (kThreads / 8) >> (kMaxRangeLevels - 1) >= 1,
                "thread shares of the pair operations");
  constexpr int kPerLevel = kThreads / 8;
  const int l = tid / kPerLevel;
  if (l < L) {
    const int slots = kPerLevel >> l;
    const int v = (tid % kPerLevel) / slots;
    const int h = (1 << l) - 1 + v, hc = (2 << l) - 1 + 2 * v;
    // the node's and its children's fields, read together
    const int pn = M.n[h], plo = M.lo[h], phi = M.hi[h], hoff = M.off[h], hooff = M.ooff[h];
    const int hc_off = M.off[hc], hc_lo = M.lo[hc], tc_off = M.off[hc + 1], tc_lo = M.lo[hc + 1];
    const int nops = node_pair_ops(pn, plo, phi);
    const int lead = ((plo & 1) != (pn & 1)) ? 1 : 0;
    const int rem = phi - plo - lead;
    for (int kk = tid % slots; kk < nops; kk += slots) {
      int* e = ops + 6 * (lbase[l] + hooff + kk);
      if (pn == 1) {  // a one-row block: its tail child's only row, copied
        e[0] = e[1] = tc_off * stride4;
        e[2] = zero4;
        e[3] = 0;
        e[4] = hoff * stride4;
        e[5] = -1;
        continue;
      }
      int s;
      bool single;
      if (kk < lead) {
        s = plo;
        single = true;
      } else {
        const int q2 = 2 * (kk - lead);
        s = plo + lead + q2;
        single = q2 + 1 >= rem;
      }
      int i, j, hb, j2;
      merge_indices_fast(pn, s, i, j);
      merge_indices_fast(pn, single ? s : s + 1, hb, j2);
      int rot = s - j;
      if (rot >= p) rot %= p;
      const int oa = hoff + (s - plo);
      e[0] = (hc_off + (i - hc_lo)) * stride4;
      e[1] = (hc_off + (hb - hc_lo)) * stride4;
      e[2] = (tc_off + (j - tc_lo)) * stride4;
      e[3] = rot * 4;
      e[4] = oa * stride4;
      e[5] = single ? -1 : (oa + 1) * stride4;
    }
  }
  });
  const int lane20 = (lane < G ? lane : lane % G) * kChunk * 4;
  auto fetch = [&](int l) {
    PairOp op{0, 0, 0, 0, junk4, junk4};
    if (l >= 0) {
      const int q = wave + WV * lane;
      if (q < lbase[l + 1] - lbase[l]) {
        const int* e = ops + 6 * (lbase[l] + q);
        op.ha = e[0];
        op.hb = e[1];
        op.t = e[2];
        op.rot4 = e[3];
        op.oa = e[4];
        op.ob = e[5];
      }
    }
    return op;
  };
  __syncthreads();  // rows loaded, pair operations built
  PairOp cur = fetch(L - 1);
  for (int l = L - 1; l >= 0; --l) {
    const PairOp nxt = fetch(l - 1);
    merge_pairs<WV>(reinterpret_cast<unsigned char*>(rows), p4, lane20, cur, lbase[l + 1] - lbase[l]);
    cur = nxt;
  }
}


__device__ __forceinline__ int find_node(const Meta& M, int l, int q) {
  const int first = (1 << l) - 1;
  int v = 0;
  while (v + 1 < (1 << l) && M.off[first + v + 1] <= q) ++v;
  return first + v;
}

// ---------------------------------------------------------------------------
// Boxcar S/N of final rows (Sec. 5.4). For a profile P of p bins, the boxcar
// of width w starting at bin n sums S[n + w] - S[n], S the exclusive prefix
// sum over two repeats of P; the S/N is the best sum over n times
// 1 / sqrt(m w var) (precomputed in FP64).
//
// Compiled width grids: lane = (row, segment of kSnrSeg window starts). The
// lane reads the kSnrSeg + wmax - 1 bins its windows cover into registers,
// forms their prefix sums there, and takes, per width, the best of kSnrSeg
// differences; every (start, width) pair costs one subtract and half a
// three-input max. All waves of the workgroup take segments, so a tile of 64
// rows keeps 8 waves busy; segment maxima are combined through LDS. Segments
// past bin p repeat windows of the circular profile and change nothing.
// Rows shorter than the register window take the ring form below instead.
// ---------------------------------------------------------------------------

template <int... W>
struct WidthGrid {
  static constexpr int kN = sizeof...(W);
  static constexpr int kW[kN] = {W...};
  static constexpr int kMax = kW[kN - 1];
};
using GridPaper9 = WidthGrid<1, 2, 3, 4, 6, 9, 13, 19, 28>;
using GridDuty9 = WidthGrid<1, 2, 3, 5, 8, 12, 19, 30, 48>;

__device__ __forceinline__ float nan_max(float a, float b) {
  return (a != a || b != b) ? __builtin_nanf("") : fmaxf(a, b);
}

template <class G, bool kCheck>
__device__ __forceinline__ void ring_block(const float* row, int t, int tend, int p, float& S,
                                           float (&ring)[G::kMax + 1], float (&best)[G::kN]) {
  constexpr int NW = G::kN, RS = G::kMax + 1;
  const float* rp = row + t;
#pragma unroll
  for (int u = 0; u < RS; ++u) {
    float v;
    if (kCheck) {
      const int tt = t + u;
      if (tt >= tend) break;
      v = row[tt < p ? tt : tt - p];
    } else {
      v = rp[u];
    }
    S += v;
    ring[(u + 1) % RS] = S;
#pragma unroll
    for (int k = 0; k < NW; ++k) best[k] = fmaxf(best[k], S - ring[(u + 1 + RS - G::kW[k]) % RS]);
  }
}

template <int WV, class G>
__device__ __forceinline__ void snr_grid(const float* rows, int stride, int p, int nvalid, float* part,
                         const float* scale, float* out) {
  constexpr int NW = G::kN, RS = G::kMax + 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ngroups = (nvalid + 63) >> 6;
  const int nseg = ngroups >= 4 ? 1 : (ngroups > 0 ? 4 / ngroups : 1);
  const int rpad = ngroups * 64;
  if (wave < ngroups * nseg) {
    const int g = wave / nseg, sg = wave - g * nseg;
    const int q = g * 64 + lane;
    const int lseg = (p + nseg - 1) / nseg;
    const int n0 = sg * lseg, n1 = min(p, n0 + lseg);
    float best[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) best[k] = -INFINITY;
    float S = 0.0f;
    if (n0 < n1) {
      const int tend = n1 + G::kMax - 1;  // windows starting in [n0, n1)
      const float* row = rows + (q < nvalid ? q : 0) * stride;
      float ring[RS];
      ring[0] = 0.0f;
#pragma unroll
      for (int u = 1; u < RS; ++u) ring[u] = INFINITY;  // before the segment: no window
      int t = n0;
      for (; t + RS <= tend && t + RS <= p; t += RS) ring_block<G, false>(row, t, tend, p, S, ring, best);
      for (; t < tend; t += RS) ring_block<G, true>(row, t, tend, p, S, ring, best);
    }
    if (S != S) {
#pragma unroll
      for (int k = 0; k < NW; ++k) best[k] = S;
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) part[(sg * NW + k) * rpad + q] = best[k];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nvalid * NW; idx += (WV * 64)) {
    const int q = idx / NW, k = idx - q * NW;
    float v = part[k * rpad + q];
    for (int sg = 1; sg < nseg; ++sg) v = nan_max(v, part[(sg * NW + k) * rpad + q]);
    out[idx] = v * scale[k];
  }
}

constexpr int kSnrSeg = 32;

// The register-window form needs the window of a segment that starts below p
// to end, after one wrap, within the row's kHalo copied bins, and the row
// area to hold the partial maxima of one segment per wave.
template <class G>
__device__ __forceinline__ bool snr_seg_fits(int p, int nvalid, int region_floats) {
  constexpr int NV = kSnrSeg + G::kMax - 1;
  return p >= NV - kHalo && region_floats >= G::kN * 64 * ((nvalid + 63) >> 6);
}

template <class G, bool kWrap>
__device__ __forceinline__ void snr_segment(const float* row, int n0, int p, float (&best)[G::kN],
                                            float& total) {
  constexpr int NW = G::kN, NV = kSnrSeg + G::kMax - 1;
  float S[NV + 1];
  S[0] = 0.0f;
  const float* b1 = row + n0;
  const float* b2 = row + n0 - p;
  const int lim = p - n0;  // bins t >= lim of the window wrap to t - p
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    const float v = kWrap ? (t < lim ? b1[t] : b2[t]) : b1[t];
    S[t + 1] = S[t] + v;
  }
  total += S[NV];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    float b = best[k];
    // one chain through b: each pair of starts is one three-input max
#pragma unroll
    for (int u = 0; u + 1 < kSnrSeg; u += 2)
      b = fmaxf(fmaxf(b, S[u + G::kW[k]] - S[u]), S[u + 1 + G::kW[k]] - S[u + 1]);
    best[k] = b;
  }
}

template <int WV, class G>
__device__ __forceinline__ void snr_seg(float* rows, int stride, int p, int nvalid, int region_floats,
                                        const float* scale, float* out) {
  constexpr int NW = G::kN, NV = kSnrSeg + G::kMax - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ngroups = (nvalid + 63) >> 6;
  const int rpad = ngroups * 64;
  int nseg = WV / ngroups;
  const int fit = region_floats / (NW * rpad);
  nseg = nseg < fit ? nseg : fit;
  const int needed = (p + kSnrSeg - 1) / kSnrSeg;
  nseg = nseg < needed ? nseg : needed;
  float best[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) best[k] = -INFINITY;
  float total = 0.0f;
  const bool active = wave < ngroups * nseg;
  const int g = active ? wave / nseg : 0, sg = active ? wave - g * nseg : 0;
  const int q = g * 64 + lane;
  if (active) {
    const float* row = rows + (q < nvalid ? q : nvalid - 1) * stride;
    for (int n0 = sg * kSnrSeg; n0 < p; n0 += nseg * kSnrSeg) {
      if (n0 + NV <= p)
        snr_segment<G, false>(row, n0, p, best, total);
      else
        snr_segment<G, true>(row, n0, p, best, total);
    }
    if (total != total) {
#pragma unroll
      for (int k = 0; k < NW; ++k) best[k] = total;
    }
  }
  __syncthreads();  // every row read: the row area takes the partial maxima
  float* part = rows;
  if (active) {
#pragma unroll
    for (int k = 0; k < NW; ++k) part[(sg * NW + k) * rpad + q] = best[k];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nvalid * NW; idx += (WV * 64)) {
    const int qq = idx / NW, k = idx - qq * NW;
    float v = part[k * rpad + qq];
    for (int s = 1; s < nseg; ++s) v = nan_max(v, part[(s * NW + k) * rpad + qq]);
    out[idx] = v * scale[k];
  }
}

// General widths: one wave per row, lane = contiguous phases; the prefix goes
// to a per-wave LDS array.
template <int WV>
__device__ __forceinline__ void snr_general(const PassArgs& a, const float* rows, int stride, int p, int nvalid,
                            float* snrbuf, const float* scale, float* out) {
  const int wmax = a.wmax, slen = p + wmax + 1;
  int snr_waves = kSnrLdsBytes / (slen * 4);
  snr_waves = snr_waves < WV ? snr_waves : WV;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (wave >= snr_waves) return;
  float* S = snrbuf + wave * slen;
  const int ncol = (p + 63) / 64;
  const int nw = a.num_widths;
  for (int q = wave; q < nvalid; q += snr_waves) {
    const float* row = rows + q * stride;
    float v[kSnrColsMax];
    float run = 0.0f;
#pragma unroll
    for (int e = 0; e < kSnrColsMax; ++e) {
      const int col = lane * ncol + e;
      v[e] = (e < ncol && col < p) ? row[col] : 0.0f;
      run += v[e];
    }
    const float incl_lane = wave_inclusive_sum(run, lane);
    const float total = __shfl(incl_lane, 63, 64);
    float acc = incl_lane - run;
    if (lane == 0) S[0] = 0.0f;
#pragma unroll
    for (int e = 0; e < kSnrColsMax; ++e) {
      const int col = lane * ncol + e;
      acc += v[e];
      if (e < ncol && col < p) {
        S[col + 1] = acc;
        if (col < wmax) S[p + 1 + col] = total + acc;
      }
    }
    wave_lds_sync();
    float res = 0.0f;
    for (int iw = 0; iw < nw; ++iw) {
      const int w = a.widths[iw];
      float best = -INFINITY;
      for (int col = lane; col < p; col += 64) best = fmaxf(best, S[col + w] - S[col]);
      best = wave_max(best);
      if (lane == iw) res = best * scale[iw];
    }
    if (total != total) res = total;  // a NaN anywhere in the profile: NaN S/N
    if (lane < nw) out[q * nw + lane] = res;
    wave_lds_sync();
  }
}

// PO = 2 and 3: a launch whose tiles all take the pair-merge forms and the
// register-window S/N (pairs_only_launch), full tiles only (a first pass) or
// range tiles only (a later pass), compiled without the other forms.
template <int WV, int JS, int DT, int PO>
__device__ __forceinline__ void ffa_tile(const PassArgs& a, const TileDesc& t, const XformDesc& x,
                                         unsigned char* smem) {
  const int p = x.p, stride = lds_stride(p), J = col_iters(p);
  const int R = rows_capacity(p, a.lds_rows_cap, WV);
  float* rows = reinterpret_cast<float*>(smem);
  const int ZR = R;            // all-zero row
  float* junk = rows + (R + 1) * stride;
  int* th = reinterpret_cast<int*>(rows + (R + 2) * stride);
  int* tt = th + R;
  int* tr = tt + R;
  Meta M{tr + R,
         tr + R + kMetaNodes,
         tr + R + 2 * kMetaNodes,
         tr + R + 3 * kMetaNodes,
         tr + R + 4 * kMetaNodes,
         tr + R + 5 * kMetaNodes,
         tr + R + 6 * kMetaNodes};
  // the S/N scratch; range tiles keep their pair operations here until the
  // merges are done
  float* snrbuf = reinterpret_cast<float*>(tr + R + kMetaInts);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  for (int c = tid; c < stride; c += (WV * 64)) rows[ZR * stride + c] = 0.0f;

  int r0, n;
  node_geometry(x.m, t.d_dst, t.node, r0, n);
  int nrows, s_base;
  const int q_lane = wave + WV * lane;  // the wave's row held by this lane

  if (PO != 0) {
    static_assert(PO == 0 || JS == 1, "the pair forms need one column group per lane");
    if (PO == 2) {
      full_tile_pairs<WV, DT>(a, x.in_off + (int64_t)r0 * p, n, p, stride, rows, R);
      nrows = n;
      s_base = 0;
    } else {
      range_tile_pairs<WV>(a, t, x, r0, n, p, stride, rows, R, M, reinterpret_cast<int*>(snrbuf));
      nrows = t.s1 - t.s0;
      s_base = t.s0;
    }
  } else if ((t.flags & kTileFull) && JS == 1 && merge_groups(p) + kRegLevels <= 64) {
    full_tile_pairs<WV, DT>(a, x.in_off + (int64_t)r0 * p, n, p, stride, rows, R);
    nrows = n;
    s_base = 0;
  } else if (t.flags & kTileFull) {
    const int64_t base = x.in_off + (int64_t)r0 * p;
    load_rows<WV, JS, DT>(rows, n, p, stride, a.in, base + (int64_t)q_lane * p);
    if (n >= 2) {
      const int32_t off = a.full_off[n];
      // schedule entries of level `lev` for the lane's row, fetched one level
      // ahead so the loads overlap the previous merge
      auto fetch = [&](int lev) {
        LaneOp op{0, ZR, 0};
        if (lev >= 0 && q_lane < n) {
          const uint32_t ht = a.full_ht[off + lev * n + q_lane];
          int rot = a.full_rot[off + lev * n + q_lane];
          if ((ht >> 16) == 0xffffu) {  // one-row block: stays
            op.h = q_lane;
          } else {
            op.h = (int)(ht & 0xffffu);
            op.t = (int)(ht >> 16);
            op.rot = rot >= p ? rot % p : rot;
          }
        }
        return op;
      };
      int lev = ceil_log2(n) - 1;
      LaneOp cur = fetch(lev);
      __syncthreads();
      for (; lev >= 0; --lev) {
        const LaneOp nxt = fetch(lev - 1);
        merge_level<WV, JS>(rows, n, p, stride, J, cur, junk);
        cur = nxt;
      }
    } else {
      __syncthreads();
    }
    nrows = n;
    s_base = 0;
  } else if (JS == 1 && merge_groups(p) <= 64) {
    range_tile_pairs<WV>(a, t, x, r0, n, p, stride, rows, R, M, reinterpret_cast<int*>(snrbuf));
    nrows = t.s1 - t.s0;
    s_base = t.s0;
  } else {
    const int L = t.levels;
    if (wave == 0) build_meta(M, r0, n, t.s0, t.s1, L);
    __syncthreads();
    const int llast = (2 << L) - 2;
    const int total = M.off[llast] + M.hi[llast] - M.lo[llast];
    for (int q = tid; q < total; q += (WV * 64)) {
      const int h = find_node(M, L, q);
      th[q] = M.r0[h] + M.lo[h] + (q - M.off[h]);
    }
    __syncthreads();
    const float* src = (t.bufs & 1) ? a.scr1 : a.scr0;
    load_rows<WV, JS, FFA_F32>(rows, total, p, stride, src + x.scr_off,
                       q_lane < total ? (int64_t)th[q_lane] * p : 0);
    for (int l = L - 1; l >= 0; --l) {
      const int last = (2 << l) - 2;
      const int cnt = M.off[last] + M.hi[last] - M.lo[last];
      __syncthreads();  // rows loaded / previous tables consumed
      for (int q = tid; q < cnt; q += (WV * 64)) {
        const int h = find_node(M, l, q);
        const int v = h - ((1 << l) - 1);
        const int hc = (2 << l) - 1 + 2 * v;
        const int s = M.lo[h] + (q - M.off[h]);
        if (M.n[h] >= 2) {
          int i, j;
          merge_indices(M.n[h], s, i, j);
          th[q] = M.off[hc] + (i - M.lo[hc]);
          tt[q] = M.off[hc + 1] + (j - M.lo[hc + 1]);
          tr[q] = (s - j) % p;
        } else {
          th[q] = M.off[hc + 1];  // one-row block: its tail child's only row
          tt[q] = ZR;
          tr[q] = 0;
        }
      }
      __syncthreads();
      LaneOp op{0, ZR, 0};
      if (q_lane < cnt) {
        op.h = th[q_lane];
        op.t = tt[q_lane];
        op.rot = tr[q_lane];
      }
      merge_level<WV, JS>(rows, cnt, p, stride, J, op, junk);
    }
    nrows = t.s1 - t.s0;
    s_base = t.s0;
  }

  if (!(t.flags & kTileFinal)) {
    float* dst = (t.bufs & 2) ? a.scr1 : a.scr0;
    store_rows<WV, JS>(rows, nrows, p, stride, dst + x.scr_off + (int64_t)(r0 + s_base) * p);
    return;
  }
  if (t.flags & kTileOutRows) {
    store_rows<WV, JS>(rows, nrows, p, stride, a.out_rows + x.out_row0 + (int64_t)s_base * p);
    return;
  }
  int nvalid = x.keep - s_base;
  nvalid = nvalid < nrows ? nvalid : nrows;
  if (nvalid <= 0) return;
  const float* scale = a.scales + x.scale_off;
  float* out = a.snr + (x.out_row0 + s_base) * a.num_widths;
  const int region = (R + 2) * stride;  // rows, zero row and junk row
  if (PO != 0) {
    if (a.width_set == kWidthsPaper9)
      snr_seg<WV, GridPaper9>(rows, stride, p, nvalid, region, scale, out);
    else
      snr_seg<WV, GridDuty9>(rows, stride, p, nvalid, region, scale, out);
    return;
  }
  if (a.width_set == kWidthsPaper9) {
    if (snr_seg_fits<GridPaper9>(p, nvalid, region))
      snr_seg<WV, GridPaper9>(rows, stride, p, nvalid, region, scale, out);
    else
      snr_grid<WV, GridPaper9>(rows, stride, p, nvalid, snrbuf, scale, out);
  } else if (a.width_set == kWidthsDuty9) {
    if (snr_seg_fits<GridDuty9>(p, nvalid, region))
      snr_seg<WV, GridDuty9>(rows, stride, p, nvalid, region, scale, out);
    else
      snr_grid<WV, GridDuty9>(rows, stride, p, nvalid, snrbuf, scale, out);
  } else
    snr_general<WV>(a, rows, stride, p, nvalid, snrbuf, scale, out);
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup i runs on XCD i mod
// 8), each XCD with its own L2. This maps them so that each XCD takes one
// contiguous eighth of the tile list (neighbouring tiles read neighbouring
// rows of the same octave), a bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int bid, int n) {
  constexpr int kXcds = 8;
  const int q = n / kXcds, r = n % kXcds;
  const int x = bid % kXcds, k = bid / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// One instantiation per (column groups per lane, input storage type): JS = 1
// needs every tile's p <= 316 (one group per lane); JS = 0 serves any p.
template <int WV, int JS, int DT, int PO>
// Four waves per SIMD: two 8-wave workgroups (or one of 16) per CU, 128 VGPRs.
__global__ __launch_bounds__(WV * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_ffa_pass(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const TileDesc t = a.tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const XformDesc x = a.xf[t.xf];
  ffa_tile<WV, JS, DT, PO>(a, t, x, smem);
}

// Persistent form: one workgroup per CU takes tiles in ticket order. A tile of
// a later pass first waits (one thread, bounded polling) until every tile of
// the pass it reads has finished; the tiles it waits for carry smaller
// tickets, so they are held by running workgroups and the wait always ends.
// Finished tiles publish their rows with an agent-scope release before they
// count themselves done.
template <int WV, int JS, int DT>
__global__ __launch_bounds__(WV * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_ffa_persist(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the tile layout leaves the last 64 bytes of the LDS unused (rows_capacity)
  int* s_ticket = reinterpret_cast<int*>(smem + wg_lds_bytes(WV) - 16);
  // the next ticket is fetched while the current tile is processed
  int next = 0;
  if (threadIdx.x == 0) next = atomicAdd(a.ticket, 1);
  for (;;) {
    if (threadIdx.x == 0) *s_ticket = next;
    __syncthreads();
    const int tk = *s_ticket;
    __syncthreads();
    if (tk >= a.ntiles) break;
    if (threadIdx.x == 0) next = atomicAdd(a.ticket, 1);
    const TileDesc t = a.tiles[tk];
    if (t.dep >= 0) {
      if (threadIdx.x == 0) {
        const int need = a.need[t.dep];
        int spins = 0;
        while (__hip_atomic_load(a.counters + t.dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               need) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins > a.spin_limit ||
              (__hip_atomic_load(a.error_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2)) {
            atomicOr(a.error_flag, 2);  // give up: later waits end at once
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // later reads see the rows
      }
      __syncthreads();
    }
    const XformDesc x = a.xf[t.xf];
    ffa_tile<WV, JS, DT, 0>(a, t, x, smem);
    // every wave publishes its own global stores before the tile counts
    // itself done
    if (t.done >= 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0 && t.done >= 0) atomicAdd(a.counters + t.done, 1);
  }
}

__global__ void k_zero_ints(int32_t* p, int n, int32_t* ticket) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (i == 0) *ticket = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_stats(const SeriesDev* series_dev, int32_t nseries, int32_t dtype,
                        int32_t blocks_per_series, double* partials, double* stats, float* norm,
                        int32_t* flag, hipStream_t stream) {
  dim3 grid(blocks_per_series, nseries);
  hipLaunchKernelGGL(k_stats_partial, grid, dim3(kStatsThreads), 0, stream, series_dev, dtype,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_final, dim3(nseries), dim3(64), 0, stream, series_dev, dtype,
                     blocks_per_series, partials, stats, norm, flag);
  return hipGetLastError();
}

constexpr int kDsMaxRounds = 2;  // LDS of a block: kDsMaxRounds * kDsRound floats at most
constexpr int kDsMaxLdsBytes = (kDsMaxRounds * kDsRound + 4) * (int)sizeof(float);

int32_t downsample_lds_floats(int32_t block, int32_t halo) {
  const int32_t rounds = (block + halo + kDsRound - 1) / kDsRound;
  return rounds * kDsRound + 4;
}

int32_t downsample_block_samples(int32_t halo) {
  // a block and its halo fill whole rounds; the block is at least four halos
  // long (at most a fifth of the loads repeat) where LDS allows, and a
  // multiple of 8 samples, so that 16-byte loads stay aligned
  const int32_t pad = (halo + 7) & ~7;
  const int32_t rounds = std::min(kDsMaxRounds, std::max(1, (5 * pad + kDsRound - 1) / kDsRound));
  const int32_t block = rounds * kDsRound - pad;
  return block >= pad ? block : 0;
}

template <int DT, int DO>
hipError_t launch_downsample_t(const SeriesDev* series_dev, const int32_t* block_series,
                               const OctaveDev* oct, const float* norm, void* out, int64_t nblocks,
                               size_t lds, hipStream_t stream) {
  static bool done[kMaxDevices] = {};
  hipError_t e = set_lds_limit_once(reinterpret_cast<const void*>(k_downsample<DT, DO>),
                                    kDsMaxLdsBytes, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_downsample<DT, DO>), dim3((unsigned)nblocks), dim3(kDsThreads), lds,
                     stream, series_dev, block_series, oct, norm, out);
  return hipGetLastError();
}

// Output in the input's type, or FP32 from any input.
hipError_t launch_downsample(const SeriesDev* series_dev, const int32_t* block_series,
                             const OctaveDev* oct, const float* norm, int32_t dtype, void* out,
                             int32_t out_dtype, int64_t nblocks, int32_t lds_floats,
                             hipStream_t stream) {
  const size_t lds = (size_t)lds_floats * sizeof(float);
  if (lds > (size_t)kDsMaxLdsBytes || (out_dtype != dtype && out_dtype != FFA_F32))
    return hipErrorInvalidValue;
  const auto* s = series_dev;
  const auto* b = block_series;
  if (dtype == FFA_BF16)
    return out_dtype == FFA_F32
               ? launch_downsample_t<FFA_BF16, FFA_F32>(s, b, oct, norm, out, nblocks, lds, stream)
               : launch_downsample_t<FFA_BF16, FFA_BF16>(s, b, oct, norm, out, nblocks, lds, stream);
  if (dtype == FFA_F16)
    return out_dtype == FFA_F32
               ? launch_downsample_t<FFA_F16, FFA_F32>(s, b, oct, norm, out, nblocks, lds, stream)
               : launch_downsample_t<FFA_F16, FFA_F16>(s, b, oct, norm, out, nblocks, lds, stream);
  return launch_downsample_t<FFA_F32, FFA_F32>(s, b, oct, norm, out, nblocks, lds, stream);
}

int32_t pass_lds_bytes(int32_t rows_cap, int32_t max_p) {
  (void)rows_cap;
  (void)max_p;
  return kLdsBytes;
}

template <int WV, int JS, int DT>
hipError_t launch_persist_t(const PassArgs& args, int grid, hipStream_t stream) {
  static bool done[kMaxDevices] = {};
  hipError_t e = set_lds_limit_once(reinterpret_cast<const void*>(k_ffa_persist<WV, JS, DT>),
                                    wg_lds_bytes(WV), done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ffa_persist<WV, JS, DT>), dim3(grid), dim3(WV * 64), wg_lds_bytes(WV),
                     stream, args);
  return hipGetLastError();
}

template <int WV, int JS, int DT, int PO>
hipError_t launch_pass_t(const PassArgs& args, hipStream_t stream) {
  static bool done[kMaxDevices] = {};
  hipError_t e = set_lds_limit_once(reinterpret_cast<const void*>(k_ffa_pass<WV, JS, DT, PO>),
                                    wg_lds_bytes(WV), done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ffa_pass<WV, JS, DT, PO>), dim3(args.ntiles), dim3(WV * 64),
                     wg_lds_bytes(WV), stream, args);
  return hipGetLastError();
}

// Instantiation for the launch: workgroup size, column groups per lane (one
// when every p <= 316) and the storage type of the input.
template <bool kPersist>
hipError_t dispatch(const PassArgs& args, int grid, hipStream_t stream) {
  const bool j1 = col_iters(args.max_p) == 1;
  const bool big = args.waves == kWavesLarge;
// The folded (downsampled) series are stored in the input's type. Range
// tiles read only the FP32 scratch rows, so the range-tile kernel is compiled
// once.
#define FFA_LAUNCH(WV, JS, DT)                                                        \
  (kPersist ? launch_persist_t<WV, JS, DT>(args, grid, stream)                        \
   : (JS == 1 && args.pairs_only == 2) ? launch_pass_t<WV, JS, DT, (JS == 1 ? 2 : 0)>(args, stream) \
   : (JS == 1 && args.pairs_only == 3) ? launch_pass_t<WV, JS, FFA_F32, (JS == 1 ? 3 : 0)>(args, stream) \
                                       : launch_pass_t<WV, JS, DT, 0>(args, stream))
#define FFA_BY_DT(WV, JS)                                                  \
  (args.in_dtype == FFA_F32    ? FFA_LAUNCH(WV, JS, FFA_F32)              \
   : args.in_dtype == FFA_BF16 ? FFA_LAUNCH(WV, JS, FFA_BF16)             \
   : args.in_dtype == FFA_F16  ? FFA_LAUNCH(WV, JS, FFA_F16) : hipErrorInvalidValue)
  if (big) return j1 ? FFA_BY_DT(kWavesLarge, 1) : FFA_BY_DT(kWavesLarge, 0);
  return j1 ? FFA_BY_DT(kWavesSmall, 1) : FFA_BY_DT(kWavesSmall, 0);
#undef FFA_BY_DT
#undef FFA_LAUNCH
}

hipError_t launch_persist(const PassArgs& args, int ncounters, int grid, hipStream_t stream) {
  if (args.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((ncounters + 255) / 256), dim3(256), 0, stream,
                     args.counters, ncounters, args.ticket);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return dispatch<true>(args, grid, stream);
}

hipError_t launch_pass(const PassArgs& args, hipStream_t stream) {
  if (args.ntiles <= 0) return hipSuccess;
  return dispatch<false>(args, 0, stream);
}

hipError_t launch_norm_from_stats(const double* stats, float* norm, hipStream_t stream) {
  hipLaunchKernelGGL(k_norm_from_stats, dim3(1), dim3(1), 0, stream, stats, norm);
  return hipGetLastError();
}

hipError_t launch_clear_flag(int32_t* flag, hipStream_t stream) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, stream, flag);
  return hipGetLastError();
}

}  // namespace ffa
