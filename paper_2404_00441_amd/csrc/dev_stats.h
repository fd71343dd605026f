// dev_stats.h -- statistics of categorical images used to validate
// realizations against the training image: facies counts and the ensemble
// map (Sec. 5.2, Fig. 7b; Sec. 5.8, Fig. 16b), indicator variograms along a
// cardinal axis and the probability of connection (Sec. 5.3, Fig. 9).
//
// Images are int8 codes, [image][z][y][x] with x fastest.  A facies f is
// handled through its bit plane: per image and row (y, z) the codes == f
// packed into nwx = ceil(nx / 32) words plus one zero word, so lag-h pairs
// along x are a funnel shift and a popcount, and pairs along y or z are two
// rows' words.  Connected components of f (cells sharing a face) come from a
// union-find over cell indices: every cell starts at the first cell of its
// run along x, runs are joined where they overlap a run of the next row or
// slice, and every link points to a smaller index, so every find and every
// union ends.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccwsim_common.h"
#include "dev_kernels.h"

namespace ccw {

struct StatShape {
  int n[3];          // x, y, z extents
  int nwx, nwp;      // words of a row's bits, and with the zero word
  int rows;          // ny * nz
  long long cells;   // nx * ny * nz
};

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// per_cell[f][c] = images holding f at cell c (int32), one thread per cell,
// eight facies per pass over the images.
__global__ __launch_bounds__(kThreads) void k_st_hist_cells(const int8_t* __restrict__ codes, long long cells,
                                                            int n_img, int nf, int32_t* __restrict__ per_cell) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  for (int f0 = 0; f0 < nf; f0 += 8) {
    int cnt[8] = {};
#pragma unroll 4
    for (int i = 0; i < n_img; ++i) {
      const int v = codes[(long long)i * cells + c] - f0;
#pragma unroll
      for (int q = 0; q < 8; ++q) cnt[q] += v == q ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (f0 + q < nf) per_cell[(long long)(f0 + q) * cells + c] = cnt[q];
  }
}

// per_image[i][f] += cells of image i (blockIdx.y) holding f in this
// block's share of the cells (int64 counters, cleared by the caller).
__global__ __launch_bounds__(kThreads) void k_st_hist_images(const int8_t* __restrict__ codes, long long cells,
                                                             int nf, unsigned long long* __restrict__ per_image) {
  __shared__ int s_part[kThreads / 64][8];
  const int img = blockIdx.y, tid = threadIdx.x;
  const int8_t* im = codes + (long long)img * cells;
  for (int f0 = 0; f0 < nf; f0 += 8) {
    int cnt[8] = {};
    for (long long c = (long long)blockIdx.x * kThreads + tid; c < cells; c += (long long)gridDim.x * kThreads) {
      const int v = im[c] - f0;
#pragma unroll
      for (int q = 0; q < 8; ++q) cnt[q] += v == q ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int s = wave_sum(cnt[q]);
      if ((tid & 63) == 0) s_part[tid >> 6][q] = s;
    }
    __syncthreads();
    if (tid < 8 && f0 + tid < nf) {
      unsigned long long s = 0;
      for (int w = 0; w < kThreads / 64; ++w) s += (unsigned)s_part[w][tid];
      if (s) atomicAdd(per_image + (long long)img * nf + f0 + tid, s);
    }
    __syncthreads();
  }
}

// Bit planes of facies f: bits[img][row][w], one thread per word.
__global__ __launch_bounds__(kThreads) void k_st_pack(const int8_t* __restrict__ codes, StatShape s, int n_img,
                                                      int f, uint32_t* __restrict__ bits) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)n_img * s.rows * s.nwp;
  if (id >= total) return;
  const int w = (int)(id % s.nwp);
  const long long t = id / s.nwp;
  const int row = (int)(t % s.rows);
  const long long img = t / s.rows;
  uint32_t m = 0;
  if (w < s.nwx) {
    const int8_t* rp = codes + img * s.cells + (long long)row * s.n[0];
    const int x0 = 32 * w;
#pragma unroll 8
    for (int b = 0; b < 32; ++b) {
      const int x = x0 + b;
      if (x < s.n[0] && rp[x] == f) m |= 1u << b;
    }
  }
  bits[id] = m;
}

// Pairs at lags 1..H along `axis` whose indicators of f differ, counted from
// the bit planes.  Grid (row blocks of rb rows, images); out[img * out_stride + h-1]
// += the block's count.  Dynamic LDS: H 32-bit counters.
__global__ __launch_bounds__(kThreads) void k_st_pairs(const uint32_t* __restrict__ bits, StatShape s, int axis,
                                                       int H, int rb, unsigned long long* __restrict__ out,
                                                       long long out_stride) {
  extern __shared__ uint32_t s_acc[];
  const int tid = threadIdx.x, img = blockIdx.y;
  for (int h = tid; h < H; h += kThreads) s_acc[h] = 0;
  __syncthreads();
  const uint32_t* P = bits + (long long)img * s.rows * s.nwp;
  const int r0 = blockIdx.x * rb, r1 = min(s.rows, r0 + rb);
  const int nx = s.n[0], ny = s.n[1];
  const long long total = (long long)H * s.nwx;
  for (long long idx = tid; idx < total; idx += kThreads) {
    const int h = (int)(idx / s.nwx) + 1, w = (int)(idx - (long long)(h - 1) * s.nwx);
    uint32_t acc = 0;
    if (axis == 0) {
      // bit b of word w pairs cell 32w + b with cell 32w + b + h of the row
      const int lim = nx - h - 32 * w;
      if (lim <= 0) continue;
      const uint32_t vm = lim >= 32 ? ~0u : ((1u << lim) - 1u);
      const int q = h >> 5;
      const uint32_t sh = (uint32_t)(h & 31);
      for (int r = r0; r < r1; ++r) {
        const uint32_t* R = P + (long long)r * s.nwp;
        const uint32_t a = R[w];
        const uint32_t b = __builtin_amdgcn_alignbit(R[w + q + 1], R[w + q], sh);
        acc += __popc((a ^ b) & vm);
      }
    } else {
      // row r = z * ny + y pairs with r + h (y) or r + h * ny (z)
      const long long step = axis == 1 ? 1 : ny;
      const int na = s.n[axis];
      for (int r = r0; r < r1; ++r) {
        const int coord = axis == 1 ? r % ny : r / ny;
        if (coord + h >= na) continue;
        const uint32_t a = P[(long long)r * s.nwp + w];
        const uint32_t b = P[((long long)r + h * step) * s.nwp + w];
        acc += __popc(a ^ b);
      }
    }
    if (acc) atomicAdd(&s_acc[h - 1], acc);
  }
  __syncthreads();
  for (int h = tid; h < H; h += kThreads)
    if (s_acc[h]) atomicAdd(out + (long long)img * out_stride + h, (unsigned long long)s_acc[h]);
}

// ---- connected components of facies f (one int32 label per cell, image-local
// cell index of the parent; -1 outside f) ----
__device__ __forceinline__ int st_find(int32_t* L, int x) {
  while (true) {
    const int p = __hip_atomic_load(L + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    x = p;   // parents are smaller indices
  }
}

__device__ __forceinline__ void st_union(int32_t* L, int a, int b) {
  while (true) {
    a = st_find(L, a);
    b = st_find(L, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(L + b, b, a);   // hang the larger root below the smaller
    if (old == b) return;
    b = old;   // b gained a parent meanwhile: retry from there (old < b)
  }
}

// Every cell of f points at the first cell of its run along x.
__global__ __launch_bounds__(kThreads) void k_st_ccl_init(const uint32_t* __restrict__ bits, StatShape s, int n_img,
                                                          int32_t* __restrict__ L) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n_img * s.cells) return;
  const long long img = id / s.cells;
  const int c = (int)(id - img * s.cells);
  const int nx = s.n[0];
  const int row = c / nx, x = c - row * nx;
  const uint32_t* R = bits + (img * s.rows + row) * s.nwp;
  const int w = x >> 5, b = x & 31;
  const uint32_t M = R[w];
  if (!((M >> b) & 1u)) {
    L[id] = -1;
    return;
  }
  const uint32_t z = ~M & ((1u << b) - 1u);   // cells not in f below x in this word
  int start = 0;
  if (z) {
    start = 32 * w + (32 - __clz(z));
  } else {
    for (int ww = w - 1; ww >= 0; --ww) {     // words before w are full rows of 32 cells
      const uint32_t zz = ~R[ww];
      if (zz) {
        start = 32 * ww + (32 - __clz(zz));
        break;
      }
    }
  }
  L[id] = row * nx + start;
}

// Runs of row r joined to the runs of row r + 1 (y) and of row r + ny (z)
// that they overlap: one union at the first cell of every overlap segment.
// One thread per (image, row, word).
__global__ __launch_bounds__(kThreads) void k_st_ccl_merge(const uint32_t* __restrict__ bits, StatShape s, int n_img,
                                                           int32_t* __restrict__ L) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n_img * s.rows * s.nwx) return;
  const int w = (int)(id % s.nwx);
  const long long t = id / s.nwx;
  const int row = (int)(t % s.rows);
  const long long img = t / s.rows;
  const int nx = s.n[0], ny = s.n[1], nz = s.n[2];
  const int y = row % ny, z = row / ny;
  const uint32_t* R = bits + (img * s.rows + row) * s.nwp;
  int32_t* Li = L + img * s.cells;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const bool ok = d == 0 ? y + 1 < ny : z + 1 < nz;
    if (!ok) continue;
    const int nrow = d == 0 ? row + 1 : row + ny;
    const uint32_t* Q = bits + (img * s.rows + nrow) * s.nwp;
    const uint32_t ov = R[w] & Q[w];
    const uint32_t carry = w > 0 ? ((R[w - 1] & Q[w - 1]) >> 31) : 0u;
    uint32_t starts = ov & ~((ov << 1) | carry);
    while (starts) {
      const int b = __ffs(starts) - 1;
      starts &= starts - 1;
      const int x = 32 * w + b;
      st_union(Li, row * nx + x, nrow * nx + x);
    }
  }
}

// Every label replaced by its root, in two passes.  Only the first cell of
// a run ever changes its parent during the merge (the others keep pointing
// at it), so the first pass resolves the run starts and the second copies
// each start's root to the rest of its run.
template <bool STARTS>
__global__ __launch_bounds__(kThreads) void k_st_ccl_flatten(StatShape s, int n_img, int32_t* __restrict__ L) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n_img * s.cells) return;
  const long long img = id / s.cells;
  const int c = (int)(id - img * s.cells);
  int32_t* Li = L + img * s.cells;
  const int p = Li[c];
  if (p < 0) return;
  const bool start = c % s.n[0] == 0 || Li[c - 1] < 0;   // membership of f never changes
  if (STARTS) {
    if (start) Li[c] = st_find(Li, c);
  } else if (!start) {
    Li[c] = Li[p];   // p is the run's start, resolved by the first pass
  }
}

// Pairs at lags 1..H along `axis` whose cells both hold f, and those whose
// cells share a component.  Grid (blocks, images); each block takes a
// strided share of the cells, counts per lag with wave ballots into LDS and
// adds its totals to both / conn [img * out_stride + h-1].  Dynamic LDS: 2H
// 32-bit counters.
__global__ __launch_bounds__(kThreads) void k_st_conn(const int32_t* __restrict__ L, StatShape s, int axis, int H,
                                                      unsigned long long* __restrict__ both,
                                                      unsigned long long* __restrict__ conn, long long out_stride) {
  extern __shared__ uint32_t s_acc[];
  uint32_t* s_both = s_acc;
  uint32_t* s_conn = s_acc + H;
  const int tid = threadIdx.x, lane = tid & 63, img = blockIdx.y;
  for (int h = tid; h < 2 * H; h += kThreads) s_acc[h] = 0;
  __syncthreads();
  const int32_t* Li = L + (long long)img * s.cells;
  const int nx = s.n[0], ny = s.n[1];
  const long long step = axis == 0 ? 1 : axis == 1 ? nx : (long long)nx * ny;
  const long long stride = (long long)gridDim.x * kThreads;
  // every lane of a wavefront runs the same number of iterations
  const long long cbase = (long long)blockIdx.x * kThreads + (tid & ~63);
  for (long long c0 = cbase; c0 < s.cells; c0 += stride) {
    const long long c = c0 + lane;
    const bool in = c < s.cells;
    const int la = in ? Li[c] : -1;
    if (__ballot(la >= 0) == 0) continue;
    int coord = 0;
    if (in) {
      const int x = (int)(c % nx);
      const long long yz = c / nx;
      coord = axis == 0 ? x : axis == 1 ? (int)(yz % ny) : (int)(yz / ny);
    }
    const int lim = s.n[axis] - 1 - coord;   // lags that stay inside the image
    for (int h = 1; h <= H; ++h) {
      const bool v = la >= 0 && h <= lim;
      const int lb = v ? Li[c + h * step] : -1;
      const unsigned long long mb = __ballot(v && lb >= 0);
      if (mb == 0) {
        if (__ballot(la >= 0 && h < lim) == 0) break;   // no lane has a longer lag left
        continue;
      }
      const unsigned long long mc = __ballot(v && lb == la);
      if (lane == 0) {
        atomicAdd(&s_both[h - 1], (uint32_t)__popcll(mb));
        if (mc) atomicAdd(&s_conn[h - 1], (uint32_t)__popcll(mc));
      }
    }
  }
  __syncthreads();
  for (int h = tid; h < H; h += kThreads) {
    if (s_both[h]) atomicAdd(both + (long long)img * out_stride + h, (unsigned long long)s_both[h]);
    if (s_conn[h]) atomicAdd(conn + (long long)img * out_stride + h, (unsigned long long)s_conn[h]);
  }
}

// The same counts along x with one lag per thread: a block stages each of
// its rows' labels in LDS (padded by -1) and every thread walks the row for
// its lag, four cells per step (one broadcast 16-byte read of the cells,
// four reads of their partners, which differ between lanes by one word).
// Grid (row blocks of rb rows, images); dynamic LDS (nx + 4) labels.
__global__ __launch_bounds__(kThreads) void k_st_conn_x(const int32_t* __restrict__ L, StatShape s, int H, int rb,
                                                        unsigned long long* __restrict__ both,
                                                        unsigned long long* __restrict__ conn, long long out_stride) {
  extern __shared__ __align__(16) int32_t s_row[];
  const int tid = threadIdx.x, img = blockIdx.y;
  const int nx = s.n[0];
  const int r0 = blockIdx.x * rb, r1 = min(s.rows, r0 + rb);
  const int32_t* Li = L + (long long)img * s.cells;
  constexpr int kLagsPerThread = 16;   // H <= 4096 = 16 * 256
  uint32_t nb[kLagsPerThread], nc[kLagsPerThread];
#pragma unroll
  for (int k = 0; k < kLagsPerThread; ++k) nb[k] = nc[k] = 0;
  if (tid < 4) s_row[nx + tid] = -1;
  for (int r = r0; r < r1; ++r) {
    __syncthreads();
    for (int x = tid; x < nx; x += kThreads) s_row[x] = Li[(long long)r * nx + x];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kLagsPerThread; ++k) {
      const int h = 1 + tid + k * kThreads;
      if (k * kThreads >= H) break;
      if (h > H) continue;
      uint32_t b = 0, c = 0;
      for (int x = 0; x < nx - h; x += 4) {
        const int4 a = *(const int4*)(s_row + x);
        const int p0 = s_row[x + h], p1 = s_row[x + h + 1], p2 = s_row[x + h + 2], p3 = s_row[x + h + 3];
        b += (a.x >= 0 && p0 >= 0) + (a.y >= 0 && p1 >= 0) + (a.z >= 0 && p2 >= 0) + (a.w >= 0 && p3 >= 0);
        c += (a.x >= 0 && a.x == p0) + (a.y >= 0 && a.y == p1) + (a.z >= 0 && a.z == p2) + (a.w >= 0 && a.w == p3);
      }
      nb[k] += b;
      nc[k] += c;
    }
  }
#pragma unroll
  for (int k = 0; k < kLagsPerThread; ++k) {
    const int h = 1 + tid + k * kThreads;
    if (h > H) break;
    if (nb[k]) atomicAdd(both + (long long)img * out_stride + h - 1, (unsigned long long)nb[k]);
    if (nc[k]) atomicAdd(conn + (long long)img * out_stride + h - 1, (unsigned long long)nc[k]);
  }
}

// The same counts along y or z, eight lags per thread: a thread owns one
// column x of one line (fixed z for y, fixed y for z) and lags
// 8 g + 1 .. 8 g + 8 (g = blockIdx.y).  It walks the line once, keeping the
// labels at the eight partner positions in a sliding window of registers
// (two loads per position), and its 16 counters are summed over the block
// at the end.  Grid (x blocks x lines, lag groups, images).
__global__ __launch_bounds__(kThreads) void k_st_conn_col(const int32_t* __restrict__ L, StatShape s, int axis, int H,
                                                          unsigned long long* __restrict__ both,
                                                          unsigned long long* __restrict__ conn, long long out_stride) {
  __shared__ uint32_t s_red[kThreads / 64][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, img = blockIdx.z;
  const int nx = s.n[0], ny = s.n[1];
  const int nxb = (nx + kThreads - 1) / kThreads;
  const int line = blockIdx.x / nxb, x = (blockIdx.x - line * nxb) * kThreads + tid;
  const int na = s.n[axis];
  const long long step = axis == 1 ? nx : (long long)nx * ny;
  // cell of position 0 of this thread's line
  const long long base = axis == 1 ? (long long)line * ny * nx + x : (long long)line * nx + x;
  const int32_t* Li = L + (long long)img * s.cells;
  const int h0 = 8 * blockIdx.y + 1;   // lags h0 .. h0 + 7
  uint32_t nb[8], nc[8];
  int w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    nb[q] = nc[q] = 0;
    w[q] = (x < nx && h0 + q < na) ? Li[base + (h0 + q) * step] : -1;
  }
  if (x < nx) {
    for (int p = 0; p + h0 < na; ++p) {
      const int av = Li[base + p * step];
      const int nxt = p + 1 + h0 + 7 < na ? Li[base + (p + 1 + h0 + 7) * step] : -1;
      if (av >= 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          nb[q] += w[q] >= 0 ? 1u : 0u;
          nc[q] += w[q] == av ? 1u : 0u;
        }
      }
#pragma unroll
      for (int q = 0; q < 7; ++q) w[q] = w[q + 1];
      w[7] = nxt;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int sb = wave_sum((int)nb[q]), sc = wave_sum((int)nc[q]);
    if (lane == 0) {
      s_red[wv][q] = (uint32_t)sb;
      s_red[wv][8 + q] = (uint32_t)sc;
    }
  }
  __syncthreads();
  if (tid < 16) {
    const int q = tid & 7;
    if (h0 + q <= H) {
      unsigned long long t = 0;
      for (int k = 0; k < kThreads / 64; ++k) t += s_red[k][tid];
      if (t) atomicAdd((tid < 8 ? both : conn) + (long long)img * out_stride + h0 + q - 1, t);
    }
  }
}

__global__ void k_st_fill_u64(unsigned long long* __restrict__ p, long long n) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = 0ull;
}

}  // namespace ccw
