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
constexpr int kShortMax = 32;   // longest shortlist rescored exactly

// Coordinates of the cells start, start + step, start + 2 step, ... of an
// e0 x e1 x (..) box in x-fastest order, advanced with adds and compares
// instead of a division per cell (the step is split once).
struct BoxWalk {
  int x, y, z, dx, dy, dz, e0, e1;
  __device__ __forceinline__ BoxWalk(int start, int step, int e0_, int e1_) : e0(e0_), e1(e1_) {
    split3(start, e0, e1, x, y, z);
    split3(step, e0, e1, dx, dy, dz);
  }
  __device__ __forceinline__ void next() {
    x += dx;
    y += dy;
    z += dz;
    if (x >= e0) { x -= e0; ++y; }
    if (y >= e1) { y -= e1; ++z; }
  }
};

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
    for (int u = tid; u < (int)g.wcells; u += nth) {
      int ux, uy, uz;
      split3(u, g.T[0], g.T[1], ux, uy, uz);
      P[u] = (int8_t)approx[idx3(c0x + ux, c0y + uy, c0z + uz, g.G)];
    }
    __syncthreads();
    return;
  }
  int e[3] = {g.tc[0], g.tc[1], g.tc[2]};
  int o[3] = {c0x, c0y, c0z};
  {
    const int n = e[0] * e[1] * e[2];
    for (int i = tid; i < n; i += nth) {
      int x, y, z;
      split3(i, e[0], e[1], x, y, z);
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
    const int rc = e[0] * e[1] * e[2];
    const int en[3] = {e[0] * 2, e[1] * 2, ND == 3 ? e[2] * 2 : 1};
    for (int i = tid; i < rc; i += nth) {
      int x, y, z;
      split3(i, e[0], e[1], x, y, z);
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
// Block-subtree layout of the Haar pyramid.  The transform of one level-J
// block touches nothing outside it, so its 2^(ND*J) coefficients can be
// stored together: [approximation][level-J details][level-(J-1) details of
// the 2^ND children] ... [level-1 details], each level's nodes x-fastest,
// 2^ND - 1 sub-bands per node.  It is a permutation of the planar layout
// (the transform is orthogonal), and rebuilding a block needs one
// contiguous read and no cooperation between threads.
// ---------------------------------------------------------------------------
template <int ND, int J>
struct HaarTree {
  static constexpr int NC = 1 << ND;
  static constexpr int B = 1 << (ND * J);
  // offset of the level-j details (1 <= j <= J)
  static constexpr int off(int j) {
    int o = 1, n = 1;
    for (int jj = J; jj > j; --jj) {
      o += (NC - 1) * n;
      n *= NC;
    }
    return o;
  }
  // node index of child delta of node (x, y, z) on a grid of nj nodes per axis
  static constexpr int child(int x, int y, int z, int delta, int nj) {
    const int cx = 2 * x + (delta & 1), cy = 2 * y + ((delta >> 1) & 1);
    const int cz = ND == 3 ? 2 * z + ((delta >> 2) & 1) : 0;
    return cx + 2 * nj * (cy + 2 * nj * cz);
  }
};

// Forward transform of one level-J block: v holds the B fine cells (x
// fastest), out receives the block-subtree layout.
template <int ND, int J, int BB = (1 << (ND * J))>
__device__ __forceinline__ void haar_tree_forward(const int (&v)[BB], int (&out)[BB]) {
  using T = HaarTree<ND, J>;
  constexpr int NC = T::NC;
  int cur[T::B];
#pragma unroll
  for (int i = 0; i < T::B; ++i) cur[i] = v[i];
#pragma unroll
  for (int j = 1; j <= J; ++j) {
    const int nj = 1 << (J - j);                 // nodes per axis at level j
    const int nn = ND == 3 ? nj * nj * nj : nj * nj;
    int nxt[T::B];
#pragma unroll
    for (int n = 0; n < nn; ++n) {
      const int x = n % nj, y = (n / nj) % nj, z = ND == 3 ? n / (nj * nj) : 0;
      int c[NC];
#pragma unroll
      for (int d = 0; d < NC; ++d) c[d] = cur[T::child(x, y, z, d, nj)];
#pragma unroll
      for (int a = 0; a < ND; ++a) {
#pragma unroll
        for (int d = 0; d < NC; ++d) {
          if (!(d & (1 << a))) {
            const int e = c[d], o = c[d | (1 << a)];
            c[d] = e + o;
            c[d | (1 << a)] = e - o;
          }
        }
      }
      nxt[n] = c[0];
#pragma unroll
      for (int q = 1; q < NC; ++q) out[T::off(j) + n * (NC - 1) + q - 1] = c[q];
    }
#pragma unroll
    for (int n = 0; n < nn; ++n) cur[n] = nxt[n];
  }
  out[0] = cur[0];
}

// Inverse of haar_tree_forward: rebuilds the B fine cells of one block.
template <int ND, int J, int BB = (1 << (ND * J))>
__device__ __forceinline__ void haar_tree_inverse(const int (&t)[BB], int (&v)[BB]) {
  using T = HaarTree<ND, J>;
  constexpr int NC = T::NC;
  int cur[T::B];
  cur[0] = t[0];
#pragma unroll
  for (int j = J; j >= 1; --j) {
    const int nj = 1 << (J - j);
    const int nn = ND == 3 ? nj * nj * nj : nj * nj;
    int nxt[T::B];
#pragma unroll
    for (int n = 0; n < nn; ++n) {
      const int x = n % nj, y = (n / nj) % nj, z = ND == 3 ? n / (nj * nj) : 0;
      int c[NC];
      c[0] = cur[n];
#pragma unroll
      for (int q = 1; q < NC; ++q) c[q] = t[T::off(j) + n * (NC - 1) + q - 1];
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        int acc = 0;
#pragma unroll
        for (int q = 0; q < NC; ++q) acc += (__popc(q & d) & 1) ? -c[q] : c[q];
        nxt[T::child(x, y, z, d, nj)] = acc >> ND;
      }
    }
#pragma unroll
    for (int i = 0; i < nn * NC; ++i) cur[i] = nxt[i];
  }
#pragma unroll
  for (int i = 0; i < T::B; ++i) v[i] = cur[i];
}

// One thread per level-J block: fine cells (edge-replicated) -> subtree
// layout, plus the approximation in int32 and fp16.
template <int ND, int J>
__global__ __launch_bounds__(kThreads) void k_dwt_tree(const int8_t* __restrict__ ti, int32_t* __restrict__ tree,
                                                       int32_t* __restrict__ approx, _Float16* __restrict__ approx_h,
                                                       Geom g) {
  using T = HaarTree<ND, J>;
  const long long cells = (long long)g.G[0] * g.G[1] * g.G[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cells) return;
  int bx, by, bz;
  split3((int)id, g.G[0], g.G[1], bx, by, bz);
  constexpr int b = 1 << J;
  int v[T::B], out[T::B];
#pragma unroll
  for (int i = 0; i < T::B; ++i) {
    const int lx = i % b, ly = (i / b) % b, lz = ND == 3 ? i / (b * b) : 0;
    const int x = min(b * bx + lx, g.ti[0] - 1), y = min(b * by + ly, g.ti[1] - 1);
    const int z = ND == 3 ? min(b * bz + lz, g.ti[2] - 1) : 0;
    v[i] = ti[idx3(x, y, z, g.ti)];
  }
  haar_tree_forward<ND, J>(v, out);
  int4* dst = (int4*)(tree + id * T::B);
#pragma unroll
  for (int i = 0; i < T::B / 4; ++i) dst[i] = make_int4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
  approx[id] = out[0];
  approx_h[id] = (_Float16)(float)out[0];
}

// Level J >= 3 in 2D: one thread per level-2 node of each level-J block.
// The thread walks from the block's approximation down to its node (one
// inverse step per level, three details each), gathers the node's level-2
// and level-1 details into the level-2 subtree layout and rebuilds its 4 x 4
// cells with haar_tree_inverse<2, 2>.
template <int J>
__device__ __forceinline__ void idwt_window_tree_split(const int32_t* __restrict__ tree, const Geom& g, int c0x,
                                                       int c0y, int8_t* P) {
  using T = HaarTree<2, J>;
  constexpr int b = 1 << J;
  constexpr int nq = 1 << (J - 2);          // level-2 nodes per axis in a block
  const int nblk = g.tc[0] * g.tc[1];
  for (int t = threadIdx.x; t < nblk * nq * nq; t += kThreads) {
    const int blk = t / (nq * nq), q = t - blk * (nq * nq);
    const int bx = blk % g.tc[0], by = blk / g.tc[0];
    const int qx = q % nq, qy = q / nq;      // the level-2 node within the block
    const int32_t* src = tree + idx3(c0x + bx, c0y + by, 0, g.G) * T::B;
    // approximation of the node: from the root down, one level at a time
    int a = src[0];
    for (int j = J; j > 2; --j) {
      const int nj = 1 << (J - j);           // nodes per axis at level j
      const int sh = j - 3;                  // path bit of level j
      const int x = qx >> (sh + 1), y = qy >> (sh + 1);
      const int d = ((qx >> sh) & 1) | (((qy >> sh) & 1) << 1);
      const int* dt = src + T::off(j) + (x + nj * y) * 3;
      const int c1 = dt[0], c2 = dt[1], c3 = dt[2];
      // inverse of e + o / e - o on both axes, child d (bit 0: x, bit 1: y)
      const int s1 = (d & 1) ? -c1 : c1, s2 = (d & 2) ? -c2 : c2, s3 = (d == 1 || d == 2) ? -c3 : c3;
      a = (a + s1 + s2 + s3) >> 2;
    }
    // the node's level-2 details and its children's level-1 details
    int tv[16], v[16];
    tv[0] = a;
    const int n2 = qx + nq * qy;
#pragma unroll
    for (int i = 0; i < 3; ++i) tv[1 + i] = src[T::off(2) + n2 * 3 + i];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int n1 = (2 * qx + (e & 1)) + 2 * nq * (2 * qy + (e >> 1));
#pragma unroll
      for (int i = 0; i < 3; ++i) tv[4 + e * 3 + i] = src[T::off(1) + n1 * 3 + i];
    }
    haar_tree_inverse<2, 2>(tv, v);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int ux = b * bx + 4 * qx + (i & 3), uy = b * by + 4 * qy + (i >> 2);
      if (ux < g.T[0] && uy < g.T[1]) P[idx3(ux, uy, 0, g.T)] = (int8_t)v[i];
    }
  }
  __syncthreads();
}

// Rebuild the template window at block origin c0 from the subtree layout:
// one thread per level-J block of the window.
template <int ND, int J>
__device__ __forceinline__ void idwt_window_tree(const int32_t* __restrict__ tree, const Geom& g, int c0x, int c0y,
                                                 int c0z, int8_t* P) {
  if constexpr (J >= 3) {
    static_assert(ND == 2, "the subtree layout above level 2 is built in 2D only");
    idwt_window_tree_split<J>(tree, g, c0x, c0y, P);
    return;
  }
  using T = HaarTree<ND, J>;
  constexpr int b = 1 << J;
  const int nblk = g.tc[0] * g.tc[1] * g.tc[2];
  for (int t = threadIdx.x; t < nblk; t += kThreads) {
    int bx, by, bz;
    split3(t, g.tc[0], g.tc[1], bx, by, bz);
    const long long gb = idx3(c0x + bx, c0y + by, c0z + bz, g.G);
    const int4* src = (const int4*)(tree + gb * T::B);
    int tv[T::B], v[T::B];
#pragma unroll
    for (int i = 0; i < T::B / 4; ++i) {
      const int4 q = src[i];
      tv[4 * i] = q.x;
      tv[4 * i + 1] = q.y;
      tv[4 * i + 2] = q.z;
      tv[4 * i + 3] = q.w;
    }
    haar_tree_inverse<ND, J>(tv, v);
    // a block inside the window whose rows start on 4-byte boundaries
    // writes each row of four cells as one 32-bit store; others cell by cell
    const bool whole = b == 4 && (g.T[0] & 3) == 0 && b * bx + b <= g.T[0] && b * by + b <= g.T[1] &&
                       (ND < 3 || b * bz + b <= g.T[2]);
    if (whole) {
#pragma unroll
      for (int r = 0; r < T::B / b; ++r) {   // row r = (ly, lz)
        const int ly = r % b, lz = ND == 3 ? r / b : 0;
        const uint32_t w = (uint32_t)(v[b * r] & 0xFF) | ((uint32_t)(v[b * r + 1] & 0xFF) << 8) |
                           ((uint32_t)(v[b * r + 2] & 0xFF) << 16) | ((uint32_t)(v[b * r + 3] & 0xFF) << 24);
        *(uint32_t*)(P + idx3i(b * bx, b * by + ly, ND == 3 ? b * bz + lz : 0, g.T)) = w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < T::B; ++i) {
        const int lx = i % b, ly = (i / b) % b, lz = ND == 3 ? i / (b * b) : 0;
        const int ux = b * bx + lx, uy = b * by + ly, uz = ND == 3 ? b * bz + lz : 0;
        if (ux < g.T[0] && uy < g.T[1] && uz < g.T[2]) P[idx3i(ux, uy, uz, g.T)] = (int8_t)v[i];
      }
    }
  }
  __syncthreads();
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

// Workgroup barrier that orders LDS only: the fences cover the local
// address space, so outstanding global loads (prefetches) and stores are
// not waited for, as __syncthreads would.  For kernels whose workgroups
// share data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint64_t o = shfl_xor64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

// k smallest of n distinct keys held in LDS, by rank: each key counts the
// keys below it and, if its rank is under k, writes itself to out[rank].
// Cost n^2 / 256 comparisons per thread, so only for short lists.  When the
// list is short enough, P adjacent lanes (P a power of two, P * n <= the
// workgroup) share one key's comparisons, each taking every P-th key, and
// add their counts with lane shuffles: a workgroup runs alone on its CU
// here, so the length of each thread's chain of LDS reads is the cost.
__device__ __forceinline__ void block_rank_select(const uint64_t* v, int n, int k, uint64_t* out) {
  int lp = 0;   // log2 P
  while (lp < 3 && (n << (lp + 1)) <= kThreads) ++lp;
  const int P = 1 << lp;
  for (int t = threadIdx.x; t < (n << lp); t += kThreads) {
    const int i = t >> lp, part = t & (P - 1);
    const uint64_t x = v[i];
    int rank = 0;
    int j = part;
    for (; j + 7 * P < n; j += 8 * P) {   // eight reads in flight per wait
      uint64_t y[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) y[e] = v[j + e * P];
#pragma unroll
      for (int e = 0; e < 8; ++e) rank += y[e] < x ? 1 : 0;
    }
    for (; j < n; j += P) rank += v[j] < x ? 1 : 0;
    // the P lanes of a key are adjacent and active together
    for (int m = 1; m < P; m <<= 1) rank += __shfl_xor(rank, m, 64);
    if (part == 0 && rank < k) out[rank] = x;
  }
  __syncthreads();
}

// Number of coefficients idwt_window_lds stages: the level-J block range and
// the detail sub-bands of every level over the same window.
__host__ __device__ inline long long idwt_coef_count(const Geom& g) {
  long long e = 1;
  for (int a = 0; a < g.ndim; ++a) e *= g.tc[a];
  const long long nsub = (1 << g.ndim) - 1;
  long long total = e;  // level-J approximation
  for (int j = g.level; j >= 1; --j) {
    total += nsub * e;
    e <<= g.ndim;
  }
  return total;
}

// Same reconstruction as idwt_window, but every coefficient the window needs
// is first loaded into `coef` (LDS) with all loads in flight at once, so the
// whole pyramid costs one memory round trip.
template <int ND>
__device__ void idwt_window_lds(const int32_t* __restrict__ approx, const int32_t* __restrict__ det,
                                const Geom& g, int c0x, int c0y, int c0z, int32_t* coef, int32_t* bufA,
                                int32_t* bufB, int8_t* P) {
  const int tid = threadIdx.x;
  const int J = g.level;
  constexpr int NC = 1 << ND;
  // segment table: level-J approximation, then details of level J, J-1, .., 1
  {
    constexpr int U = 8;
    const int total = (int)idwt_coef_count(g);
    for (int base = tid; base < total; base += kThreads * U) {
      int32_t v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        int i = base + q * kThreads;
        v[q] = 0;
        if (i >= total) continue;
        int e[3] = {g.tc[0], g.tc[1], g.tc[2]};
        int o[3] = {c0x, c0y, c0z};
        int cells = e[0] * e[1] * e[2];
        if (i < cells) {
          int x, y, z;
          split3(i, e[0], e[1], x, y, z);
          v[q] = approx[idx3(o[0] + x, o[1] + y, o[2] + z, g.G)];
          continue;
        }
        i -= cells;
        for (int j = J; j >= 1; --j) {
          if (i < (NC - 1) * cells) {
            const int s = i / cells + 1;
            const int r = i - (s - 1) * cells;
            int x, y, z;
            split3(r, e[0], e[1], x, y, z);
            const int* Gd = g.Gj[j];
            const long long gcells = (long long)Gd[0] * Gd[1] * Gd[2];
            v[q] = det[g.det_off[j] + (long long)(s - 1) * gcells + idx3(o[0] + x, o[1] + y, o[2] + z, Gd)];
            break;
          }
          i -= (NC - 1) * cells;
          for (int a = 0; a < ND; ++a) {
            e[a] *= 2;
            o[a] *= 2;
          }
          cells <<= ND;
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        if (i < total) coef[i] = v[q];
      }
    }
  }
  __syncthreads();
  int e[3] = {g.tc[0], g.tc[1], g.tc[2]};
  const int32_t* cur = coef;
  int doff = e[0] * e[1] * e[2];   // details of level J start here
  int32_t* nxt = bufA;
  for (int j = J; j >= 1; --j) {
    const int rc = e[0] * e[1] * e[2];
    const int en[3] = {e[0] * 2, e[1] * 2, ND == 3 ? e[2] * 2 : 1};
    for (int i = tid; i < rc; i += kThreads) {
      int x, y, z;
      split3(i, e[0], e[1], x, y, z);
      int c[NC];
      c[0] = cur[i];
#pragma unroll
      for (int s = 1; s < NC; ++s) c[s] = coef[doff + (s - 1) * rc + i];
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
    doff += (NC - 1) * rc;
    cur = nxt;
    nxt = (nxt == bufA) ? bufB : bufA;
    for (int a = 0; a < ND; ++a) e[a] *= 2;
  }
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
