// dev_kernels.h -- device building blocks of the CCWSIM hot path:
// separable Haar lifting (forward, per level), inverse reconstruction of a
// pattern window, wavefront-level sorting and the block-wide top-K.
#pragma once

#include "ccwsim_common.h"

namespace ccw {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;   // every kernel here runs 4 wavefronts of 64
constexpr int kTopMax = 16;     // largest K handled by block_topk

// ---------------------------------------------------------------------------
// Forward Haar DWT, one level (Sec. 3.1 filter-and-decimate steps done as a
// separable two-point lifting per axis).  One thread per level-j cell: it
// gathers the 2^ND children of level j-1 (the TI itself, edge-replicated,
// when j = 1), applies the butterfly (e, o) -> (e + o, e - o) along x, then
// y, then z, and writes the approximation and the 2^ND - 1 detail sub-bands
// (sub-band index = bitmask of the axes that took the high-pass).
// ---------------------------------------------------------------------------
template <int ND>
__global__ __launch_bounds__(kThreads) void k_dwt_level(const int8_t* __restrict__ ti,
                                                        const int32_t* __restrict__ src,
                                                        int32_t* __restrict__ dst,
                                                        _Float16* __restrict__ dst_h,
                                                        int32_t* __restrict__ det, Geom g, int j) {
  const int* Gd = g.Gj[j];
  const long long cells = (long long)Gd[0] * Gd[1] * Gd[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cells) return;
  const int x = (int)(id % Gd[0]);
  const int y = (int)((id / Gd[0]) % Gd[1]);
  const int z = (int)(id / ((long long)Gd[0] * Gd[1]));
  constexpr int NC = 1 << ND;
  int v[NC];
#pragma unroll
  for (int d = 0; d < NC; ++d) {
    int cx = 2 * x + (d & 1), cy = 2 * y + ((d >> 1) & 1);
    int cz = (ND == 3) ? 2 * z + ((d >> 2) & 1) : z;
    if (j == 1) {
      cx = cx < g.ti[0] ? cx : g.ti[0] - 1;
      cy = cy < g.ti[1] ? cy : g.ti[1] - 1;
      cz = cz < g.ti[2] ? cz : g.ti[2] - 1;
      v[d] = ti[idx3(cx, cy, cz, g.ti)];
    } else {
      v[d] = src[idx3(cx, cy, cz, g.Gj[j - 1])];
    }
  }
#pragma unroll
  for (int a = 0; a < ND; ++a) {
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      if (!(d & (1 << a))) {
        const int e = v[d], o = v[d | (1 << a)];
        v[d] = e + o;
        v[d | (1 << a)] = e - o;
      }
    }
  }
  dst[id] = v[0];
  if (dst_h) dst_h[id] = (_Float16)(float)v[0];
#pragma unroll
  for (int s = 1; s < NC; ++s) det[g.det_off[j] + (long long)(s - 1) * cells + id] = v[s];
}

// Level 0 "transform": the approximation is the image itself.
__global__ void k_level0(const int8_t* __restrict__ ti, int32_t* __restrict__ dst,
                         _Float16* __restrict__ dst_h, long long cells) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cells) return;
  const int v = ti[id];
  dst[id] = v;
  if (dst_h) dst_h[id] = (_Float16)(float)v;
}

// ---------------------------------------------------------------------------
// Inverse transform of one template window (Sec. 3.1 bijective filters;
// Algorithm 1 Inv-DWT).  Starts from the level-J approximation over the
// block range [c0, c0 + tc) and, level by level, combines each coefficient
// with its detail sub-bands into its 2^ND children:
//   child(delta) = 2^-ND * sum_s (-1)^popcount(s & delta) * coef_s
// (exact: the numerator is a non-negative multiple of 2^ND).  The last level
// writes the cells inside the template extent T into P.  All threads of the
// block take part; bufA/bufB hold at least the level-1 region.
// ---------------------------------------------------------------------------
template <int ND>
__device__ void idwt_window(const int32_t* __restrict__ approx, const int32_t* __restrict__ det,
                            const Geom& g, int c0x, int c0y, int c0z, int32_t* bufA,
                            int32_t* bufB, int8_t* P) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int J = g.level;
  if (J == 0) {
    for (long long u = tid; u < g.wcells; u += nth) {
      const int ux = (int)(u % g.T[0]);
      const int uy = (int)((u / g.T[0]) % g.T[1]);
      const int uz = (int)(u / ((long long)g.T[0] * g.T[1]));
      P[u] = (int8_t)approx[idx3(c0x + ux, c0y + uy, c0z + uz, g.G)];
    }
    __syncthreads();
    return;
  }
  int e[3] = {g.tc[0], g.tc[1], g.tc[2]};
  int o[3] = {c0x, c0y, c0z};
  {
    const long long n = (long long)e[0] * e[1] * e[2];
    for (long long i = tid; i < n; i += nth) {
      const int x = (int)(i % e[0]), y = (int)((i / e[0]) % e[1]), z = (int)(i / ((long long)e[0] * e[1]));
      bufA[i] = approx[idx3(o[0] + x, o[1] + y, o[2] + z, g.G)];
    }
  }
  __syncthreads();
  int32_t* cur = bufA;
  int32_t* nxt = bufB;
  constexpr int NC = 1 << ND;
  for (int j = J; j >= 1; --j) {
    const int* Gd = g.Gj[j];
    const long long gcells = (long long)Gd[0] * Gd[1] * Gd[2];
    const long long rc = (long long)e[0] * e[1] * e[2];
    const int en[3] = {e[0] * 2, e[1] * 2, ND == 3 ? e[2] * 2 : 1};
    for (long long i = tid; i < rc; i += nth) {
      const int x = (int)(i % e[0]), y = (int)((i / e[0]) % e[1]), z = (int)(i / ((long long)e[0] * e[1]));
      int c[NC];
      c[0] = cur[i];
      const long long gi = idx3(o[0] + x, o[1] + y, o[2] + z, Gd);
#pragma unroll
      for (int s = 1; s < NC; ++s) c[s] = det[g.det_off[j] + (long long)(s - 1) * gcells + gi];
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        int acc = 0;
#pragma unroll
        for (int s = 0; s < NC; ++s) acc += (__popc(s & d) & 1) ? -c[s] : c[s];
        const int val = acc >> ND;
        const int fx = 2 * x + (d & 1), fy = 2 * y + ((d >> 1) & 1);
        const int fz = ND == 3 ? 2 * z + ((d >> 2) & 1) : 0;
        if (j > 1) {
          nxt[idx3(fx, fy, fz, en)] = val;
        } else if (fx < g.T[0] && fy < g.T[1] && fz < g.T[2]) {
          P[idx3(fx, fy, fz, g.T)] = (int8_t)val;
        }
      }
    }
    __syncthreads();
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    for (int a = 0; a < ND; ++a) {
      e[a] *= 2;
      o[a] *= 2;
    }
  }
}

// ---------------------------------------------------------------------------
// Wavefront-wide helpers on 64-bit keys.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m, 64);
  hi = __shfl_xor(hi, m, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// Bitonic sort of one value per lane; on return lane i holds the i-th
// smallest of the 64 inputs.
__device__ __forceinline__ uint64_t wave_sort_asc(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t other = shfl_xor64(v, stride);
      const bool asc = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const uint64_t mn = v < other ? v : other;
      const uint64_t mx = v < other ? other : v;
      v = (lower == asc) ? mn : mx;
    }
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint64_t o = shfl_xor64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

struct TopkShared {
  uint64_t small[64];
  uint64_t top[kTopMax];
  uint64_t thr;
  unsigned cnt;
};

// ---------------------------------------------------------------------------
// Block-wide K smallest of n distinct keys key_at(0..n-1), 1 <= k <= 16,
// k <= n, blockDim = 256.  Pass 1 takes each thread's minimum; the k-th
// smallest of those minima bounds the k-th smallest key from above.  Pass 2
// collects every key under the bound; if they fit one wavefront they are
// sorted there, otherwise k rounds of block minima finish the job.  On
// return sh.top[0..k-1] holds the k smallest keys in ascending order.
// ---------------------------------------------------------------------------
template <class KeyFn>
__device__ void block_topk(long long n, int k, KeyFn key_at, TopkShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t m = ~0ull;
  for (long long i = tid; i < n; i += kThreads) {
    const uint64_t key = key_at(i);
    m = key < m ? key : m;
  }
  const uint64_t srt = wave_sort_asc(m);
  if (tid < 64) sh.small[tid] = ~0ull;
  if (tid == 0) sh.cnt = 0;
  __syncthreads();
  if (lane < k) sh.small[wave * 16 + lane] = srt;
  __syncthreads();
  if (wave == 0) {
    const uint64_t v = wave_sort_asc(sh.small[lane]);
    if (lane == k - 1) sh.thr = v;
  }
  __syncthreads();
  const uint64_t thr = sh.thr;
  if (tid < 64) sh.small[tid] = ~0ull;
  __syncthreads();
  for (long long i = tid; i < n; i += kThreads) {
    const uint64_t key = key_at(i);
    if (key <= thr) {
      const unsigned p = atomicAdd(&sh.cnt, 1u);
      if (p < 64) sh.small[p] = key;
    }
  }
  __syncthreads();
  const unsigned cnt = sh.cnt;
  if (cnt <= 64) {
    if (wave == 0) {
      const uint64_t v = wave_sort_asc(sh.small[lane]);
      if (lane < k) sh.top[lane] = v;
    }
    __syncthreads();
    return;
  }
  // rare path: k rounds of "smallest key above the previous one"
  uint64_t prev = 0;
  for (int r = 0; r < k; ++r) {
    uint64_t mm = ~0ull;
    for (long long i = tid; i < n; i += kThreads) {
      const uint64_t key = key_at(i);
      if ((r == 0 || key > prev) && key < mm) mm = key;
    }
    mm = wave_min64(mm);
    __syncthreads();
    if (lane == 0) sh.small[wave] = mm;
    __syncthreads();
    uint64_t best = sh.small[0];
    for (int w = 1; w < kThreads / 64; ++w) best = sh.small[w] < best ? sh.small[w] : best;
    prev = best;
    if (tid == 0) sh.top[r] = best;
  }
  __syncthreads();
}

}  // namespace ccw
