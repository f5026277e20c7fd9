// De-reddening by a running median (Sec. 5.2): out[i] = x[i] - med[i], med[i]
// the median of the window of 2h + 1 samples centred on i, cut at the ends
// of the series; the median of n samples is their k-th smallest value,
// k = (n - 1) / 2 (at the ends, for even n, the lower middle value). The
// result is exact: the median is one of the samples and the difference is
// one FP32 subtraction.
//
// One workgroup takes a block of B consecutive outputs (B <= (min(n, h + 1)
// + 1) / 2). Their windows all contain the core C = [s(i1 - 1), e(i0)), and
// each window adds at most B - 1 samples to it, so the k-th smallest of a
// window lies between the (k - extra)-th and the k-th smallest of C. The
// workgroup
//   1. finds the two bounding values lo and hi of C by one radix selection
//      for both on order-preserving 32-bit keys (digits of 11, 11, 10 bits);
//      when, after the first digit, the keys between the two bounds' digits
//      are few enough, it instead gathers them (with the union's) and finds
//      both bounds in their sorted order, which step 2 sorts anyway;
//   2. keeps every sample of the union of the windows whose key lies strictly
//      between them as a candidate (at most 4 B of them whatever the ties:
//      samples equal to a bound are only counted) and sorts the candidates
//      by (key, index) in LDS;
//   3. lets each of 512 threads slide a sub-block of outputs: the counts
//      of window samples below lo, equal to lo and strictly between the
//      bounds change by at most two per output, and the position of the
//      median among the sorted candidates moves by a few places; a thread's
//      first position comes from one walk over the candidates that lie
//      outside C (the others are in every window).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ffa.h"
#include "ffa_kernels.hpp"

namespace ffa {
namespace {

constexpr int kMedThreads = 1024;
constexpr int kMedBlockMax = 2048;          // outputs per workgroup
constexpr int kMedCap = 4 * kMedBlockMax;   // candidates (a power of two)
constexpr int kMedLanes = 512;              // threads sliding the outputs, a sub-block each

template <class T>
using gptr = const __attribute__((address_space(1))) T*;

template <int DT>
__device__ __forceinline__ float load_value(const void* base, int64_t i) {
  if (DT == FFA_F32) return ((gptr<float>)base)[i];
  const uint16_t b = ((gptr<uint16_t>)base)[i];
  if (DT == FFA_BF16) return __uint_as_float(static_cast<uint32_t>(b) << 16);
  _Float16 h;
  __builtin_memcpy(&h, &b, 2);
  return static_cast<float>(h);
}

// Order-preserving key of a value (-0 taken as +0, so equal values have equal
// keys), and back.
__device__ __forceinline__ uint32_t key_of(float v) {
  uint32_t u = __float_as_uint(v);
  if (u == 0x80000000u) u = 0;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float value_of(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

template <int DT>
__device__ __forceinline__ uint32_t key_at(const void* x, int64_t i) {
  return key_of(load_value<DT>(x, i));
}

// Calls f(i, key) for every sample i of x[a, b), each thread a share; the
// aligned middle is read 16 bytes at a time (when x is 16-byte aligned).
template <int DT, class F>
__device__ __forceinline__ void for_each_key(const void* x, int64_t a, int64_t b, F&& f) {
  constexpr int kPer = DT == FFA_F32 ? 4 : 8;  // samples per 16-byte load
  int64_t va = (a + kPer - 1) / kPer * kPer, vb = b / kPer * kPer;
  if (va > vb || (reinterpret_cast<uintptr_t>(x) & 15) != 0) va = vb = b;
  for (int64_t i = a + threadIdx.x; i < va; i += kMedThreads) f(i, key_at<DT>(x, i));
  for (int64_t i = vb + threadIdx.x; i < b; i += kMedThreads) f(i, key_at<DT>(x, i));
  for (int64_t v = va / kPer + threadIdx.x; v < vb / kPer; v += kMedThreads) {
    const uint4 w = reinterpret_cast<const uint4*>(x)[v];
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      float val;
      if (DT == FFA_F32) {
        val = __uint_as_float(u[q]);
      } else {
        const uint16_t h16 = (uint16_t)(u[q / 2] >> (16 * (q % 2)));
        if (DT == FFA_BF16) {
          val = __uint_as_float((uint32_t)h16 << 16);
        } else {
          _Float16 hv;
          __builtin_memcpy(&hv, &h16, 2);
          val = (float)hv;
        }
      }
      f(v * kPer + q, key_of(val));
    }
  }
}

constexpr int kDigitBits[3] = {11, 11, 10};  // digits from the top of the key

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
constexpr int kBins = 2048;

// The keys of ranks r0 and r1 (0-based) among the keys of x[c0, c1), by one
// radix selection for both: three digit passes, each counting the keys that
// share the prefix found so far of either rank. All threads return them.
//
// After the first pass it may stop early: when the keys of x[c0, c1) whose
// top digit lies between the two ranks' digits, plus `extra` more, fit
// kMedCap, it returns true with that key range [*range_lo, *range_hi] and
// the count of keys below it (*below) instead of the two keys; the caller then
// gathers the range and finds both keys by sorting it.
template <int DT>
__device__ bool select_two(const void* x, int64_t c0, int64_t c1, int64_t r0, int64_t r1,
                           int64_t extra, int* hist /* 2 * kBins */, uint32_t* k0, uint32_t* k1,
                           uint32_t* range_lo, uint32_t* range_hi, int64_t* below) {
  __shared__ uint32_t s_prefix[2];
  __shared__ int64_t s_rank[2];
  __shared__ int64_t s_inrange;
  if (threadIdx.x == 0) {
    s_prefix[0] = s_prefix[1] = 0;
    s_rank[0] = r0;
    s_rank[1] = r1;
  }
  int shift = 32;
  for (int pass = 0; pass < 3; ++pass) {
    const int bits = kDigitBits[pass];
    const uint32_t mask = shift == 32 ? 0u : (0xffffffffu << shift);
    shift -= bits;
    for (int q = threadIdx.x; q < 2 * kBins; q += kMedThreads) hist[q] = 0;
    __syncthreads();
    const uint32_t p0 = s_prefix[0], p1 = s_prefix[1];
    const uint32_t dmask = (1u << bits) - 1u;
    const int sh = shift;
    // while both ranks share their prefix (always in the first pass) one
    // histogram serves both
    const bool shared = p0 == p1;
    for_each_key<DT>(x, c0, c1, [&](int64_t, uint32_t k) {
      const uint32_t d = (k >> sh) & dmask;
      if ((k & mask) == p0) atomicAdd(&hist[d], 1);
      if (!shared && (k & mask) == p1) atomicAdd(&hist[kBins + d], 1);
    });
    __syncthreads();
    // wave w < 2 finds the digit of rank w: lane l holds bins 32 l .. 32 l + 31
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (w < 2) {
      const int* hh = hist + (shared ? 0 : w * kBins);
      int tot = 0;
      for (int q = 0; q < kBins / 64; ++q) tot += hh[(kBins / 64) * l + q];
      int incl = tot;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d, 64);
        if (l >= d) incl += u;
      }
      const int64_t r = s_rank[w];
      int64_t before = incl - tot;
      if (before <= r && r < incl) {
        for (int q = 0; q < kBins / 64; ++q) {
          const int c = hh[(kBins / 64) * l + q];
          if (before <= r && r < before + c) {
            s_prefix[w] = (w == 0 ? p0 : p1) | ((uint32_t)((kBins / 64) * l + q) << sh);
            s_rank[w] = r - before;
          }
          before += c;
        }
      }
    }
    __syncthreads();
    if (pass == 0) {  // one histogram serves both ranks here
      const uint32_t d0 = s_prefix[0] >> sh, d1 = s_prefix[1] >> sh;
      if (threadIdx.x < 64) {
        int64_t c = 0;
        for (uint32_t d = d0 + threadIdx.x; d <= d1; d += 64) c += hist[d];
        c = wave_sum64(c);
        if (threadIdx.x == 0) s_inrange = c;
      }
      __syncthreads();
      if (s_inrange + extra <= kMedCap) {
        *range_lo = d0 << sh;
        *range_hi = (d1 << sh) | ((1u << sh) - 1u);
        *below = r0 - s_rank[0];
        __syncthreads();  // every thread has read them before a later call resets them
        return true;
      }
    }
  }
  *k0 = s_prefix[0];
  *k1 = s_prefix[1];
  __syncthreads();  // every thread has read them before a later call resets them
  return false;
}

template <int DT>
__global__ __launch_bounds__(kMedThreads) void k_running_median(const void* x, int64_t n,
                                                                int32_t h, int32_t B, void* out,
                                                                int32_t out_dtype, int32_t* err) {
  __shared__ unsigned long long cand[kMedCap];  // (key << 32) | index - us, sorted
  __shared__ int edge_pos[2 * kMedBlockMax];     // sorted positions of candidates outside C
  __shared__ uint32_t lk[kMedBlockMax];          // keys of the samples that leave
  __shared__ uint32_t ek[kMedBlockMax];          // keys of the samples that enter
  __shared__ float ybuf[kMedBlockMax];
  __shared__ int hist[2 * kBins];
  __shared__ int s_lane[kMedLanes][3];  // counts of each sliding lane's first window
  __shared__ int s_cnt, s_nedge, s_lo_rank, s_hi_rank;
  __shared__ int s_cb, s_clo, s_cs;

  const int64_t i0 = (int64_t)blockIdx.x * B;
  const int64_t i1 = i0 + B < n ? i0 + B : n;
  const int nb = (int)(i1 - i0);
  auto ws = [&](int64_t i) { return i - h > 0 ? i - h : (int64_t)0; };
  auto we = [&](int64_t i) { return i + h + 1 < n ? i + h + 1 : n; };
  const int64_t cs = ws(i1 - 1), ce = we(i0);  // core
  const int64_t us = ws(i0), ue = we(i1 - 1);  // union
  const int64_t cn = ce - cs;

  // 1. ranks of the bounds within C
  if (threadIdx.x == 0) {
    s_lo_rank = 0x7fffffff;
    s_hi_rank = -1;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nb; j += kMedThreads) {
    const int64_t i = i0 + j;
    const int64_t cnt = we(i) - ws(i);
    const int64_t k = (cnt - 1) / 2;
    atomicMin(&s_lo_rank, (int)(k - (cnt - cn)));
    atomicMax(&s_hi_rank, (int)k);
  }
  __syncthreads();
  const int lo_rank = s_lo_rank, hi_rank = s_hi_rank;
  if (lo_rank < 0 || hi_rank >= cn) {  // the block is too long for its windows
    if (threadIdx.x == 0) atomicOr(err, kMedErrBit);
    return;
  }
  uint32_t lo = 0, hi = 0, range_lo = 0, range_hi = 0;
  int64_t below = 0;
  const bool early = select_two<DT>(x, cs, ce, lo_rank, hi_rank, (cs - us) + (ue - ce), hist, &lo,
                                    &hi, &range_lo, &range_hi, &below);

  // 2. candidates (lo < key < hi) of the union, and the counts of window i0;
  // after an early stop of the selection, every key of the union in the
  // range that holds both bounds (sorted below, where the bounds are found)
  if (threadIdx.x == 0) {
    s_cnt = 0;
    s_cb = s_clo = s_cs = 0;
  }
  __syncthreads();
  if (early) {
    int cb = 0;
    const int64_t w0 = ws(i0), w1 = we(i0);
    for_each_key<DT>(x, us, ue, [&](int64_t i, uint32_t k) {
      if (k < range_lo) {
        cb += i >= w0 && i < w1;
      } else if (k <= range_hi) {
        const int slot = atomicAdd(&s_cnt, 1);
        if (slot < kMedCap) cand[slot] = ((unsigned long long)k << 32) | (uint32_t)(i - us);
      }
    });
    atomicAdd(&s_cb, cb);
  } else {
    int cb = 0, clo = 0, csn = 0;
    const int64_t w0 = ws(i0), w1 = we(i0);
    for_each_key<DT>(x, us, ue, [&](int64_t i, uint32_t k) {
      const bool in0 = i >= w0 && i < w1;
      if (k < lo) {
        cb += in0;
      } else if (k == lo) {
        clo += in0;
      } else if (k < hi) {
        csn += in0;
        const int slot = atomicAdd(&s_cnt, 1);
        if (slot < kMedCap) cand[slot] = ((unsigned long long)k << 32) | (uint32_t)(i - us);
      }
    });
    atomicAdd(&s_cb, cb);
    atomicAdd(&s_clo, clo);
    atomicAdd(&s_cs, csn);
  }
  // keys of the samples that leave and enter the windows of the block
  const int64_t l0 = ws(i0), e0 = we(i0);
  const int nl = (int)(ws(i1 - 1) - l0), ne = (int)(we(i1 - 1) - e0);
  for (int j = threadIdx.x; j < nl; j += kMedThreads) lk[j] = key_at<DT>(x, l0 + j);
  for (int j = threadIdx.x; j < ne; j += kMedThreads) ek[j] = key_at<DT>(x, e0 + j);
  __syncthreads();
  int ncand = s_cnt;
  if (ncand > kMedCap) {  // cannot happen: at most 2 B from C and 2 B outside it
    if (threadIdx.x == 0) atomicOr(err, kMedErrBit);
    return;
  }
  int np2 = 1;
  while (np2 < ncand) np2 <<= 1;
  for (int j = ncand + threadIdx.x; j < np2; j += kMedThreads) cand[j] = ~0ull;
  __syncthreads();
  // bitonic sort of the candidates by (key, index); two stages per pass
  // over LDS where the stride allows: a thread takes the four elements that
  // the two stages of strides s and s / 2 mix among themselves
  for (int size = 2; size <= np2; size <<= 1) {
    int stride = size >> 1;
    while (stride > 0) {
      if (stride >= 2) {
        const int half = stride >> 1;
        const int lh = __builtin_ctz(half);
        for (int g = threadIdx.x; g < (np2 >> 2); g += kMedThreads) {
          const int base = ((g >> lh) << (lh + 2)) | (g & (half - 1));
          const bool up = (base & size) == 0;
          unsigned long long v0 = cand[base], v1 = cand[base + half];
          unsigned long long v2 = cand[base + stride], v3 = cand[base + stride + half];
          auto cx = [up](unsigned long long& a, unsigned long long& b) {
            if ((a > b) == up) {
              const unsigned long long t = a;
              a = b;
              b = t;
            }
          };
          cx(v0, v2);
          cx(v1, v3);
          cx(v0, v1);
          cx(v2, v3);
          cand[base] = v0;
          cand[base + half] = v1;
          cand[base + stride] = v2;
          cand[base + stride + half] = v3;
        }
        stride >>= 2;
      } else {
        for (int t = threadIdx.x; t < (np2 >> 1); t += kMedThreads) {
          const int a = 2 * t;
          const bool up = (a & size) == 0;
          const unsigned long long va = cand[a], vb = cand[a + 1];
          if ((va > vb) == up) {
            cand[a] = vb;
            cand[a + 1] = va;
          }
        }
        stride = 0;
      }
      __syncthreads();
    }
  }
  if (early) {
    // the bounds are the C members of ranks lo_rank - below and
    // hi_rank - below in the sorted range; then the run strictly between
    // them moves to the front, and the counts of window i0 are completed
    constexpr int kEach = kMedCap / kMedThreads;
    __shared__ int s_wc[kMedThreads / 64];
    __shared__ uint32_t s_lo_key, s_hi_key;
    __shared__ int s_pa, s_pb;
    const int t = threadIdx.x, a0 = kEach * t, lane = t & 63, wave = t >> 6;
    auto in_core = [&](int j) {
      const int64_t idx = us + (int64_t)(uint32_t)cand[j];
      return idx >= cs && idx < ce;
    };
    int own = 0;
#pragma unroll
    for (int e = 0; e < kEach; ++e) own += (a0 + e < ncand && in_core(a0 + e)) ? 1 : 0;
    int incl = own;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(incl, d, 64);
      if (lane >= d) incl += u;
    }
    if (lane == 63) s_wc[wave] = incl;
    if (t == 0) s_pa = s_pb = 0;
    __syncthreads();
    int rank = incl - own;
    for (int w = 0; w < wave; ++w) rank += s_wc[w];
    const int64_t rlo = lo_rank - below, rhi = hi_rank - below;
#pragma unroll
    for (int e = 0; e < kEach; ++e) {
      if (a0 + e < ncand && in_core(a0 + e)) {
        if (rank == rlo) s_lo_key = (uint32_t)(cand[a0 + e] >> 32);
        if (rank == rhi) s_hi_key = (uint32_t)(cand[a0 + e] >> 32);
        ++rank;
      }
    }
    __syncthreads();
    lo = s_lo_key;
    hi = s_hi_key;
    int le = 0, lt = 0, cb = 0, clo = 0, csn = 0;
    const int64_t w0 = ws(i0), w1 = we(i0);
#pragma unroll
    for (int e = 0; e < kEach; ++e) {
      if (a0 + e < ncand) {
        const uint32_t k = (uint32_t)(cand[a0 + e] >> 32);
        const int64_t idx = us + (int64_t)(uint32_t)cand[a0 + e];
        const bool in0 = idx >= w0 && idx < w1;
        le += k <= lo;
        lt += k < hi;
        cb += in0 && k < lo;
        clo += in0 && k == lo;
        csn += in0 && k > lo && k < hi;
      }
    }
    atomicAdd(&s_pa, le);
    atomicAdd(&s_pb, lt);
    atomicAdd(&s_cb, cb);
    atomicAdd(&s_clo, clo);
    atomicAdd(&s_cs, csn);
    __syncthreads();
    const int pa = s_pa, pb = s_pb;
    unsigned long long keep[kEach];
#pragma unroll
    for (int e = 0; e < kEach; ++e) keep[e] = pa + a0 + e < pb ? cand[pa + a0 + e] : 0ull;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kEach; ++e)
      if (pa + a0 + e < pb) cand[a0 + e] = keep[e];
    __syncthreads();
    ncand = pb > pa ? pb - pa : 0;
  }
  // sorted positions of the candidates outside C, ascending
  if (threadIdx.x == 0) s_nedge = 0;
  __syncthreads();
  if (threadIdx.x < 64) {
    int base = 0;
    for (int j0 = 0; j0 < ncand; j0 += 64) {
      const int j = j0 + (int)threadIdx.x;
      bool outside = false;
      if (j < ncand) {
        const int64_t idx = us + (int64_t)(uint32_t)cand[j];
        outside = idx < cs || idx >= ce;
      }
      const unsigned long long bal = __ballot(outside);
      const int before = __popcll(bal & ((1ull << threadIdx.x) - 1ull));
      if (outside) edge_pos[base + before] = j;
      base += __popcll(bal);
    }
    if (threadIdx.x == 0) s_nedge = base;
  }
  // counts of each sliding lane's first window: window i0 minus the samples
  // that left, plus those that entered. The three counts of a key (below lo,
  // equal to lo, strictly between) sit in 16-bit fields of one 64-bit word;
  // an exclusive scan over the leaving and over the entering keys (two per
  // thread, held per thread in the histogram's LDS, free by now) gives every
  // lane its counts with two reads.
  {
    __shared__ unsigned long long s_wtot[2][kMedThreads / 64];
    unsigned long long* pre = reinterpret_cast<unsigned long long*>(hist);  // [2][kMedThreads]
    auto cls = [&](uint32_t k) -> unsigned long long {
      return k < lo ? 1ull : k == lo ? (1ull << 16) : k < hi ? (1ull << 32) : 0ull;
    };
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    unsigned long long own[2], incl[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const uint32_t* keys = side ? ek : lk;
      const int cnt = side ? ne : nl;
      own[side] = (2 * t < cnt ? cls(keys[2 * t]) : 0ull) + (2 * t + 1 < cnt ? cls(keys[2 * t + 1]) : 0ull);
      unsigned long long v = own[side];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
      }
      incl[side] = v;
      if (lane == 63) s_wtot[side][wave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      unsigned long long off = 0;
      for (int w = 0; w < wave; ++w) off += s_wtot[side][w];
      pre[side * kMedThreads + t] = off + incl[side] - own[side];
    }
    __syncthreads();
    if (t < kMedLanes) {
      const int sb = (nb + kMedLanes - 1) / kMedLanes;
      const int64_t ia = i0 + (int64_t)t * sb;
      if (t * sb < nb) {
        auto prefix = [&](int side, int p) {  // the fields summed over keys [0, p)
          const uint32_t* keys = side ? ek : lk;
          unsigned long long v = pre[side * kMedThreads + p / 2];
          if (p & 1) v += cls(keys[p - 1]);
          return v;
        };
        const unsigned long long gone = prefix(0, (int)(ws(ia) - l0));
        const unsigned long long come = prefix(1, (int)(we(ia) - e0));
        s_lane[t][0] = (int)(come & 0xffff) - (int)(gone & 0xffff);
        s_lane[t][1] = (int)((come >> 16) & 0xffff) - (int)((gone >> 16) & 0xffff);
        s_lane[t][2] = (int)((come >> 32) & 0xffff) - (int)((gone >> 32) & 0xffff);
      }
    }
  }
  __syncthreads();
  const int nedge = s_nedge;

  // 3. kMedLanes threads slide the outputs, each a sub-block
  if (threadIdx.x < kMedLanes) {
    const int lane = threadIdx.x;
    const int sb = (nb + kMedLanes - 1) / kMedLanes;
    const int j0 = lane * sb, j1 = min(nb, j0 + sb);
    if (j0 < j1) {
      const int64_t ia = i0 + j0;
      int cb = s_cb + s_lane[lane][0], clo = s_clo + s_lane[lane][1], csn = s_cs + s_lane[lane][2];
      int64_t s = ws(ia), e = we(ia);
      auto member = [&](int pos) {
        const int64_t idx = us + (int64_t)(uint32_t)cand[pos];
        return idx >= s && idx < e;
      };
      // first position: walk the candidates outside C in sorted order; the
      // candidates between two non-members are all members
      int m = ncand, r = 0;
      int64_t t0 = (e - s - 1) / 2 - cb - clo;
      if (t0 >= 0 && t0 < csn) {
        int prev = 0, below = 0;
        m = -1;
        for (int q = 0; q < nedge; ++q) {
          const int pq = edge_pos[q];
          if (member(pq)) continue;
          if (below + (pq - prev) > t0) {
            m = prev + (int)(t0 - below);
            break;
          }
          below += pq - prev;
          prev = pq + 1;
        }
        if (m < 0) m = prev + (int)(t0 - below);
        r = (int)t0;
      } else {
        m = 0;  // the answer is a bound; r counts members below m = 0
        r = 0;
      }
      for (int j = j0; j < j1; ++j) {
        const int64_t i = i0 + j;
        if (j > j0) {
          const int64_t s2 = ws(i), e2 = we(i);
          const unsigned long long cm = m < ncand ? cand[m] : ~0ull;
          if (s2 > s) {  // sample s leaves
            const uint32_t k = lk[s - l0];
            if (k < lo) {
              --cb;
            } else if (k == lo) {
              --clo;
            } else if (k < hi) {
              --csn;
              const unsigned long long ck = ((unsigned long long)k << 32) | (uint32_t)(s - us);
              if (ck < cm) --r;
            }
          }
          if (e2 > e) {  // sample e enters
            const uint32_t k = ek[e - e0];
            if (k < lo) {
              ++cb;
            } else if (k == lo) {
              ++clo;
            } else if (k < hi) {
              ++csn;
              const unsigned long long ck = ((unsigned long long)k << 32) | (uint32_t)(e - us);
              if (ck < cm) ++r;
            }
          }
          s = s2;
          e = e2;
        }
        const int64_t k = (e - s - 1) / 2;
        uint32_t mk;
        if (k < cb) {  // cannot happen: lo bounds the median from below
          atomicOr(err, kMedErrBit);
          mk = lo;
        } else if (k < cb + clo) {
          mk = lo;
        } else if (k - cb - clo >= csn) {
          mk = hi;
        } else {
          const int t = (int)(k - cb - clo);
          // move to the member with t members before it (r counts the
          // members before position m)
          for (;;) {
            if (r > t) {
              --m;
              if (member(m)) --r;
              continue;
            }
            if (m < ncand && member(m)) {
              if (r == t) break;
              ++r;
            }
            ++m;
          }
          mk = (uint32_t)(cand[m] >> 32);
        }
        const float xi = load_value<DT>(x, i);
        ybuf[j] = xi - value_of(mk);
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nb; j += kMedThreads) {
    const float v = ybuf[j];
    if (out_dtype == FFA_F32) {
      static_cast<float*>(out)[i0 + j] = v;
    } else if (out_dtype == FFA_BF16) {
      uint32_t u = __float_as_uint(v);
      uint16_t b;
      if ((u & 0x7fffffffu) > 0x7f800000u)
        b = static_cast<uint16_t>((u >> 16) | 0x40u);
      else
        b = static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
      static_cast<uint16_t*>(out)[i0 + j] = b;
    } else {
      _Float16 hv = static_cast<_Float16>(v);
      uint16_t b;
      __builtin_memcpy(&b, &hv, 2);
      static_cast<uint16_t*>(out)[i0 + j] = b;
    }
  }
}

}  // namespace

int32_t median_block(int64_t n, int32_t window) {
  const int64_t h = window / 2;
  int64_t b = ((n < h + 1 ? n : h + 1) + 1) / 2;
  if (b > kMedBlockMax) b = kMedBlockMax;
  return b < 1 ? 1 : (int32_t)b;
}

hipError_t launch_running_median(const void* x, int64_t n, int32_t dtype, int32_t window,
                                 void* out, int32_t out_dtype, int32_t* err, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int32_t B = median_block(n, window);
  const int64_t blocks = (n + B - 1) / B;
  const int32_t h = window / 2;
  if (dtype == FFA_BF16)
    hipLaunchKernelGGL(k_running_median<FFA_BF16>, dim3((unsigned)blocks), dim3(kMedThreads), 0,
                       stream, x, n, h, B, out, out_dtype, err);
  else if (dtype == FFA_F16)
    hipLaunchKernelGGL(k_running_median<FFA_F16>, dim3((unsigned)blocks), dim3(kMedThreads), 0,
                       stream, x, n, h, B, out, out_dtype, err);
  else
    hipLaunchKernelGGL(k_running_median<FFA_F32>, dim3((unsigned)blocks), dim3(kMedThreads), 0,
                       stream, x, n, h, B, out, out_dtype, err);
  return hipGetLastError();
}

}  // namespace ffa
