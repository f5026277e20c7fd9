// HIP kernels of the FFA periodicity search for gfx950 (MI355X).
//
//   k_stats_*      FP64 mean / population std of each series (Sec. 5.2)
//   k_downsample   every pseudo-octave of a series in one read of it
//                  (Sec. 5.3, App. A.4)
//   k_ffa_pass     folding-transform tiles in LDS (Sec. 2.2) and, for the
//                  rows of the full transform, the boxcar S/N (Sec. 5.4)
//
// None of the paths is a dense contraction, so nothing here uses MFMA: the
// limits are HBM bandwidth (stats, downsampling) and LDS / VALU throughput
// (the merges and the boxcar widths).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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

__device__ __forceinline__ void store_sample(void* base, int dtype, int64_t i, float v) {
  if (dtype == FFA_F32) {
    static_cast<float*>(base)[i] = v;
  } else if (dtype == FFA_BF16) {
    uint32_t u = __float_as_uint(v);
    uint16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u)
      r = static_cast<uint16_t>((u >> 16) | 0x40u);  // quiet NaN
    else
      r = static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest even
    static_cast<uint16_t*>(base)[i] = r;
  } else {
    _Float16 h = static_cast<_Float16>(v);
    uint16_t r;
    __builtin_memcpy(&r, &h, 2);
    static_cast<uint16_t*>(base)[i] = r;
  }
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
    norm[2 * blockIdx.x] = (float)mean;
    norm[2 * blockIdx.x + 1] = (float)(1.0 / sd_);
    if (sd.normalise && !(sd_ > 0.0 && isfinite(sd_) && isfinite(mean))) atomicOr(flag, 1);
  }
}

__global__ void k_clear_flag(int32_t* flag) { *flag = 0; }

__global__ void k_norm_from_stats(const double* stats, float* norm) {
  norm[0] = (float)stats[0];
  norm[1] = (float)(1.0 / stats[1]);
}

// ---------------------------------------------------------------------------
// Downsampling (Sec. 5.3, App. A.4). Output j of octave k integrates the
// normalised series over [j ds, (j+1) ds), ds = ds_fx / 2^32, each input
// sample weighted by its overlap with the window. A block stages a stretch
// of the raw series in LDS once and emits every output of every octave whose
// window starts in it, using an exclusive prefix sum over the stretch:
//   y = (1 - fa) x[ia] + (P[ib] - P[ia + 1]) + fb x[ib]
// with a = ia + fa and b = ib + fb the window edges.
// ---------------------------------------------------------------------------

constexpr int kDsThreads = 512;

__global__ __launch_bounds__(kDsThreads) void k_downsample(const SeriesDev* series,
                                                           int32_t nseries,
                                                           const OctaveDev* oct,
                                                           const float* norm, int dtype,
                                                           void* out, int out_dtype,
                                                           int32_t block_samples) {
  extern __shared__ float sm[];
  __shared__ int s_series;
  __shared__ float s_part[kDsThreads];
  const int tid = threadIdx.x;
  if (tid == 0) {
    int lo = 0, hi = nseries - 1;  // last series with chunk0 <= blockIdx.x
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (series[mid].chunk0 <= (int64_t)blockIdx.x)
        lo = mid;
      else
        hi = mid - 1;
    }
    s_series = lo;
  }
  __syncthreads();
  const int si = s_series;
  const SeriesDev sd = series[si];
  const int64_t c0 = ((int64_t)blockIdx.x - sd.chunk0) * block_samples;
  if (c0 >= sd.nsamp) return;
  const int64_t c1 = min(c0 + (int64_t)block_samples, sd.nsamp);
  const int64_t cend = min(sd.nsamp, c1 + (int64_t)sd.halo);
  const int len = (int)(cend - c0);
  float* xs = sm;                 // len samples
  float* ps = sm + len + 1;       // len + 1 prefix sums
  const float mean = sd.normalise ? norm[2 * si] : 0.0f;
  const float inv = sd.normalise ? norm[2 * si + 1] : 1.0f;
  for (int q = tid; q < len; q += kDsThreads) xs[q] = load_sample(sd.ptr, dtype, c0 + q) - mean;
  __syncthreads();
  // exclusive prefix: contiguous segments per thread, then a block scan
  const int seg = (len + kDsThreads - 1) / kDsThreads;
  const int q0 = min(tid * seg, len), q1 = min(q0 + seg, len);
  float run = 0.0f;
  for (int q = q0; q < q1; ++q) run += xs[q];
  const int lane = tid % 64, wave = tid / 64;
  float incl = wave_inclusive_sum(run, lane);
  if (lane == 63) s_part[wave] = incl;
  __syncthreads();
  float woff = 0.0f;
  for (int w = 0; w < wave; ++w) woff += s_part[w];
  float acc = woff + incl - run;
  for (int q = q0; q < q1; ++q) {
    ps[q] = acc;
    acc += xs[q];
  }
  if (q1 == len && q0 < q1) ps[len] = acc;
  if (len == 0 && tid == 0) ps[0] = 0.0f;
  __syncthreads();
  const uint64_t lo_fx = (uint64_t)c0 << 32, hi_fx = (uint64_t)c1 << 32;
  for (int k = 0; k < sd.noct; ++k) {
    const OctaveDev o = oct[sd.oct0 + k];
    if (o.nsamp == 0) continue;
    const int64_t j0 = (int64_t)((lo_fx + o.ds_fx - 1) / o.ds_fx);
    const int64_t j1 = min((int64_t)((hi_fx + o.ds_fx - 1) / o.ds_fx), o.nsamp);
    for (int64_t j = j0 + tid; j < j1; j += kDsThreads) {
      const uint64_t a = (uint64_t)j * o.ds_fx, b = a + o.ds_fx;
      const int ia = (int)((int64_t)(a >> 32) - c0), ib = (int)((int64_t)(b >> 32) - c0);
      const float fa = (float)(uint32_t)a * 2.3283064365386963e-10f;
      const float fb = (float)(uint32_t)b * 2.3283064365386963e-10f;
      float y = (1.0f - fa) * xs[ia] + (ps[ib] - ps[ia + 1]);
      if ((uint32_t)b != 0u) y += fb * xs[ib];
      store_sample(out, out_dtype, o.off + j, y * inv);
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
  const int64_t mh = n >> 1, mt = n - mh, den = 2 * (int64_t)(n - 1);
  i = (int)((2 * (mh - 1) * s + (n - 1)) / den);
  j = (int)((2 * (mt - 1) * s + (n - 1)) / den);
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

// Item index -> (row, chunk) with a float reciprocal and an exact fix-up.
__device__ __forceinline__ void split_item(int it, int nch, float rnch, int& q, int& c) {
  q = (int)((float)it * rnch);
  if (q * nch > it) --q;
  if ((q + 1) * nch <= it) ++q;
  c = it - q * nch;
}

// One merge level: output position q takes row th[q] plus row tt[q] rotated
// left by tr[q] (tt[q] == -1: plain copy of row th[q]; -2: nothing to do).
__device__ __forceinline__ void merge_level(float* rows, const int* th, const int* tt,
                                            const int* tr, int count, int p, int stride,
                                            int nch, float rnch) {
  float acc[kItemsMax][kChunk];
  const int items = count * nch;
#pragma unroll
  for (int k = 0; k < kItemsMax; ++k) {
    const int it = threadIdx.x + k * kThreads;
    if (it < items) {
      int q, c;
      split_item(it, nch, rnch, q, c);
      const int tl = tt[q];
      if (tl != -2) {
        const float* hr = rows + th[q] * stride + c * kChunk;
        if (tl < 0) {
#pragma unroll
          for (int e = 0; e < kChunk; ++e) acc[k][e] = hr[e];
        } else {
          int t0 = c * kChunk + tr[q];
          if (t0 >= p) t0 -= p;
          const float* trow = rows + tl * stride + t0;
#pragma unroll
          for (int e = 0; e < kChunk; ++e) acc[k][e] = hr[e] + trow[e];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItemsMax; ++k) {
    const int it = threadIdx.x + k * kThreads;
    if (it < items) {
      int q, c;
      split_item(it, nch, rnch, q, c);
      if (tt[q] != -2) {
        float* o = rows + q * stride;
        const int col0 = c * kChunk;
#pragma unroll
        for (int e = 0; e < kChunk; ++e)
          if (col0 + e < p) o[col0 + e] = acc[k][e];
        if (c == 0) {
#pragma unroll
          for (int e = 0; e < kChunk - 1; ++e) o[p + e] = acc[k][e];
        }
      }
    }
  }
  __syncthreads();
}

// Range-tile metadata: node h of the tile's subtree (heap order, level l holds
// nodes (1 << l) - 1 ...), fields r0 (first row in the transform), n (rows),
// [lo, hi) rows kept, off (position of row lo in LDS).
struct Meta {
  int* r0;
  int* n;
  int* lo;
  int* hi;
  int* off;
};

__device__ void build_meta(Meta M, int r0, int n, int s0, int s1, int L) {
  M.r0[0] = r0;
  M.n[0] = n;
  M.lo[0] = s0;
  M.hi[0] = s1;
  M.off[0] = 0;
  for (int l = 0; l < L; ++l) {
    const int first = (1 << l) - 1, cfirst = (2 << l) - 1;
    int off = 0;
    for (int v = 0; v < (1 << l); ++v) {
      const int h = first + v, hc = cfirst + 2 * v;
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
        merge_indices(pn, plo, i0, j0);
        merge_indices(pn, phi - 1, i1, j1);
        M.r0[hc] = M.r0[h];
        M.n[hc] = mh;
        M.lo[hc] = i0;
        M.hi[hc] = i1 + 1;
        M.r0[hc + 1] = M.r0[h] + mh;
        M.n[hc + 1] = pn - mh;
        M.lo[hc + 1] = j0;
        M.hi[hc + 1] = j1 + 1;
      }
      M.off[hc] = off;
      off += M.hi[hc] - M.lo[hc];
      M.off[hc + 1] = off;
      off += M.hi[hc + 1] - M.lo[hc + 1];
    }
  }
}

// Node (heap index) of level l holding position q.
__device__ __forceinline__ int find_node(const Meta& M, int l, int q) {
  const int first = (1 << l) - 1;
  int v = 0;
  while (v + 1 < (1 << l) && M.off[first + v + 1] <= q) ++v;
  return first + v;
}

__global__ __launch_bounds__(kThreads) void k_ffa_pass(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const TileDesc t = a.tiles[blockIdx.x];
  const XformDesc x = a.xf[t.xf];
  const int p = x.p, stride = lds_stride(p), nch = (p + kChunk - 1) / kChunk;
  const float rnch = 1.0f / (float)nch;
  const int R = rows_capacity(p, a.lds_rows_cap);
  float* rows = reinterpret_cast<float*>(smem);
  int* th = reinterpret_cast<int*>(rows + R * stride);
  int* tt = th + R;
  int* tr = tt + R;
  Meta M{tr + R, tr + R + kMetaNodes, tr + R + 2 * kMetaNodes, tr + R + 3 * kMetaNodes,
         tr + R + 4 * kMetaNodes};
  float* snrbuf = reinterpret_cast<float*>(tr + R + 5 * kMetaNodes);
  const int tid = threadIdx.x;

  int r0, n;
  node_geometry(x.m, t.d_dst, t.node, r0, n);
  int nrows, s_base;

  if (t.flags & kTileFull) {
    // load the node's input rows [r0, r0 + n)
    const int64_t base = x.in_off + (int64_t)r0 * p;
    for (int it = tid; it < n * nch; it += kThreads) {
      int q, c;
      split_item(it, nch, rnch, q, c);
      float* o = rows + q * stride;
      const int col0 = c * kChunk;
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int col = col0 + e;
        if (col < p) {
          const float v = load_sample(a.in, a.in_dtype, base + (int64_t)q * p + col);
          o[col] = v;
          if (col < kChunk - 1) o[p + col] = v;
        }
      }
    }
    __syncthreads();
    // levels from the leaves up; at relative depth lev the block of row q is
    // found by walking down from the tile's node
    for (int lev = ceil_log2(n) - 1; lev >= 0; --lev) {
      for (int q = tid; q < n; q += kThreads) {
        int b0 = 0, sz = n;
        for (int k = 0; k < lev; ++k) {
          const int mh = sz >> 1;
          if (q - b0 < mh) {
            sz = mh;
          } else {
            b0 += mh;
            sz -= mh;
          }
        }
        if (sz < 2) {
          tt[q] = -2;  // a one-row block stays as it is
        } else {
          const int s = q - b0, mh = sz >> 1;
          int i, j;
          merge_indices(sz, s, i, j);
          th[q] = b0 + i;
          tt[q] = b0 + mh + j;
          tr[q] = (s - j) % p;
        }
      }
      __syncthreads();
      merge_level(rows, th, tt, tr, n, p, stride, nch, rnch);
    }
    nrows = n;
    s_base = 0;
  } else {
    const int L = t.levels;
    if (tid == 0) build_meta(M, r0, n, t.s0, t.s1, L);
    __syncthreads();
    const int lfirst = (1 << L) - 1, llast = (2 << L) - 2;
    const int total = M.off[llast] + M.hi[llast] - M.lo[llast];
    // source rows of the bottom level, from the previous pass's scratch
    for (int q = tid; q < total; q += kThreads) {
      const int h = find_node(M, L, q);
      th[q] = M.r0[h] + M.lo[h] + (q - M.off[h]);
    }
    __syncthreads();
    const float* src = (t.bufs & 1) ? a.scr1 : a.scr0;
    for (int it = tid; it < total * nch; it += kThreads) {
      int q, c;
      split_item(it, nch, rnch, q, c);
      const float* g = src + x.scr_off + (int64_t)th[q] * p;
      float* o = rows + q * stride;
      const int col0 = c * kChunk;
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int col = col0 + e;
        if (col < p) {
          const float v = g[col];
          o[col] = v;
          if (col < kChunk - 1) o[p + col] = v;
        }
      }
    }
    __syncthreads();
    (void)lfirst;
    for (int l = L - 1; l >= 0; --l) {
      const int last = (2 << l) - 2;
      const int cnt = M.off[last] + M.hi[last] - M.lo[last];
      for (int q = tid; q < cnt; q += kThreads) {
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
          tt[q] = -1;
        }
      }
      __syncthreads();
      merge_level(rows, th, tt, tr, cnt, p, stride, nch, rnch);
    }
    nrows = t.s1 - t.s0;
    s_base = t.s0;
  }

  if (!(t.flags & kTileFinal)) {
    // intermediate rows of node (r0, n) -> scratch, rows r0 + s_base + q
    float* dst = (t.bufs & 2) ? a.scr1 : a.scr0;
    float* g = dst + x.scr_off + (int64_t)(r0 + s_base) * p;
    for (int it = tid; it < nrows * nch; it += kThreads) {
      int q, c;
      split_item(it, nch, rnch, q, c);
      const float* o = rows + q * stride;
      const int col0 = c * kChunk;
#pragma unroll
      for (int e = 0; e < kChunk; ++e)
        if (col0 + e < p) g[(int64_t)q * p + col0 + e] = o[col0 + e];
    }
    return;
  }
  if (t.flags & kTileOutRows) {
    float* g = a.out_rows + x.out_row0 + (int64_t)s_base * p;
    for (int it = tid; it < nrows * nch; it += kThreads) {
      int q, c;
      split_item(it, nch, rnch, q, c);
      const float* o = rows + q * stride;
      const int col0 = c * kChunk;
#pragma unroll
      for (int e = 0; e < kChunk; ++e)
        if (col0 + e < p) g[(int64_t)q * p + col0 + e] = o[col0 + e];
    }
    return;
  }

  // Boxcar S/N of the final rows (Sec. 5.4): each wave takes whole rows. The
  // exclusive prefix S over two repeats of the profile goes to a per-wave LDS
  // array, S[t] for t <= p + wmax; the boxcar of width w starting at bin n
  // sums S[n + w] - S[n]; the best over n, times 1 / sqrt(m w var), is the
  // S/N (the scale is precomputed in FP64).
  const int wmax = a.wmax, slen = p + wmax + 1;
  int snr_waves = kSnrLdsBytes / (slen * 4);
  snr_waves = snr_waves < kWaves ? snr_waves : kWaves;
  const int wave = tid / 64, lane = tid % 64;
  if (wave >= snr_waves) return;
  float* S = snrbuf + wave * slen;
  const int ncol = (p + 63) / 64;  // contiguous phases per lane for the scan
  const int nw = a.num_widths;
  const float* scale = a.scales + x.scale_off;
  for (int q = wave; q < nrows; q += snr_waves) {
    const int s = s_base + q;
    if (s >= x.keep) break;
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
        S[col + 1] = acc;                          // S[col + 1] = sum of bins 0..col
        if (col < wmax) S[p + 1 + col] = total + acc;  // second repeat
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
    if (total != total) res = total;  // a NaN anywhere in the profile: NaN S/N (fmaxf drops NaNs)
    if (lane < nw) a.snr[(x.out_row0 + s) * nw + lane] = res;
    wave_lds_sync();
  }
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

int32_t downsample_block_samples(int32_t max_halo) {
  int32_t b = 8192;
  while (b < 4 * max_halo) b *= 2;
  return b;
}

hipError_t launch_downsample(const SeriesDev* series_dev, int32_t nseries, const OctaveDev* oct,
                             const float* norm, int32_t dtype, void* out, int32_t out_dtype,
                             int64_t nblocks, int32_t block_samples, int32_t max_halo,
                             hipStream_t stream) {
  const size_t lds = (size_t)(2 * (block_samples + max_halo) + 2) * sizeof(float);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_downsample),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kLdsBytes - 4096);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > (size_t)(kLdsBytes - 4096)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_downsample, dim3((unsigned)nblocks), dim3(kDsThreads), lds, stream,
                     series_dev, nseries, oct, norm, dtype, out, out_dtype, block_samples);
  return hipGetLastError();
}

int32_t pass_lds_bytes(int32_t rows_cap, int32_t max_p) {
  (void)rows_cap;
  (void)max_p;
  return kLdsBytes;
}

hipError_t launch_pass(const PassArgs& args, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ffa_pass),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (args.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ffa_pass, dim3(args.ntiles), dim3(kThreads), kLdsBytes, stream, args);
  return hipGetLastError();
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
