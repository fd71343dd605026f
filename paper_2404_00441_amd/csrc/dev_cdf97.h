// CDF 9/7 wavelet path in floating point: the lifting transform and its
// inverse, and the candidate scores over the level-J approximation with a
// precision split (an fp16 / bf16 MFMA bulk ranks every candidate, fp32
// rescoring decides among the best of them).
//
// Sec. 4.2 makes the Haar wavelet one choice of mother wavelet.  The
// Cohen-Daubechies-Feauveau 9/7 biorthogonal wavelet is taken here in the
// lifting factorisation of Daubechies and Sweldens: predict with alpha,
// update with beta, predict with gamma, update with delta, then the low band
// times zeta and the high band over zeta (gain sqrt 2 at DC).  Lines use
// whole-sample symmetric extension, evaluated as lifting on the mirrored
// line itself: every output reads the nine mirrored samples around it.
//
// Scores (Sec. 4.3, over the approximation): a data event is a known-block
// mask n (0/1) and the event's approximation A; candidate c scores
// S(c) = sum over blocks b with n_b = 1 of (K[c + b] - A_b)^2.
#pragma once

#include "dev_kernels.h"

namespace ccw {

constexpr float kC97Alpha = -1.586134342059924f;
constexpr float kC97Beta = -0.052980118572961f;
constexpr float kC97Gamma = 0.882911075530934f;
constexpr float kC97Delta = 0.443506852043971f;
constexpr float kC97Zeta = 1.149604398860241f;
constexpr int kC97BlocksMax = 256;    // template blocks of a 9/7 event
constexpr int kC97ShortMax = 128;     // candidates rescored per event
constexpr int kC97Seg = 256;          // candidates of a row per bulk workgroup, at most

// Index i of a line of n samples under whole-sample symmetric extension
// (period 2(n - 1); parity is kept).
__device__ __forceinline__ int c97_mirror(int i, int n) {
  if (n == 1) return 0;
  const int p = 2 * (n - 1);
  i %= p;
  i = i < 0 ? i + p : i;
  return i >= n ? p - i : i;
}

// The TI edge-replicated to the padded extent, float.
__global__ void k_c97_pad(const int8_t* __restrict__ ti, float* __restrict__ out, Geom g) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)g.np[0] * g.np[1] * g.np[2];
  if (id >= n) return;
  const int x = (int)(id % g.np[0]), y = (int)((id / g.np[0]) % g.np[1]), z = (int)(id / ((long long)g.np[0] * g.np[1]));
  out[id] = (float)ti[idx3(min(x, g.ti[0] - 1), min(y, g.ti[1] - 1), min(z, g.ti[2] - 1), g.ti)];
}

// One analysis pass along `axis` over nb stacked bands of extent e: band q
// becomes q (low half) and q + nb (high half).  One thread per output k.
__global__ __launch_bounds__(kThreads) void k_c97_fwd(const float* __restrict__ src, float* __restrict__ dst, int e0,
                                                      int e1, int e2, int axis, int nb) {
  const int e[3] = {e0, e1, e2};
  int eo[3] = {e0, e1, e2};
  eo[axis] >>= 1;
  const long long half = (long long)eo[0] * eo[1] * eo[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= half * nb) return;
  const int q = (int)(id / half);
  const long long r = id - q * half;
  int u[3] = {(int)(r % eo[0]), (int)((r / eo[0]) % eo[1]), (int)(r / ((long long)eo[0] * eo[1]))};
  const int k = u[axis], n = e[axis];
  const long long st = axis == 0 ? 1 : axis == 1 ? e0 : (long long)e0 * e1;
  u[axis] = 0;
  const float* line = src + q * ((long long)e0 * e1 * e2) + (u[0] + (long long)e0 * (u[1] + (long long)e1 * u[2]));
  float x[9];   // x[2k - 4 .. 2k + 4]
#pragma unroll
  for (int i = 0; i < 9; ++i) x[i] = line[st * c97_mirror(2 * k - 4 + i, n)];
  // d1[k-2..k+1] at x[1], x[3], x[5], x[7]; s1[k-1..k+1] at x[2], x[4], x[6]
  float d1[4], s1[3], d2[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) d1[i] = x[2 * i + 1] + kC97Alpha * (x[2 * i] + x[2 * i + 2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) s1[i] = x[2 * i + 2] + kC97Beta * (d1[i] + d1[i + 1]);
#pragma unroll
  for (int i = 0; i < 2; ++i) d2[i] = d1[i + 1] + kC97Gamma * (s1[i] + s1[i + 1]);   // d2[k-1], d2[k]
  const float s2 = s1[1] + kC97Delta * (d2[0] + d2[1]);
  u[axis] = k;
  const long long o = u[0] + (long long)eo[0] * (u[1] + (long long)eo[1] * u[2]);
  dst[q * half + o] = s2 * kC97Zeta;
  dst[(q + nb) * half + o] = d2[1] / kC97Zeta;
}

// One synthesis pass along `axis`: bands q and q + nb (extent with the axis
// halved) of src become band q of dst (extent eo).  One thread per output
// pair x[2k], x[2k+1]; the bands are read under the symmetric extension
// their samples inherit from the line (the same mirror on line positions).
__global__ __launch_bounds__(kThreads) void k_c97_inv(const float* __restrict__ src, float* __restrict__ dst, int eo0,
                                                      int eo1, int eo2, int axis, int nb) {
  int ei[3] = {eo0, eo1, eo2};
  ei[axis] >>= 1;
  const long long half = (long long)ei[0] * ei[1] * ei[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= half * nb) return;
  const int q = (int)(id / half);
  const long long r = id - q * half;
  int u[3] = {(int)(r % ei[0]), (int)((r / ei[0]) % ei[1]), (int)(r / ((long long)ei[0] * ei[1]))};
  const int k = u[axis], n = 2 * ei[axis];
  const long long st = axis == 0 ? 1 : axis == 1 ? ei[0] : (long long)ei[0] * ei[1];
  u[axis] = 0;
  const long long base = u[0] + (long long)ei[0] * (u[1] + (long long)ei[1] * u[2]);
  const float* S = src + q * half + base;
  const float* D = src + (q + nb) * half + base;
  auto s_at = [&](int i) { return S[st * (c97_mirror(2 * i, n) >> 1)] / kC97Zeta; };
  auto d_at = [&](int i) { return D[st * (c97_mirror(2 * i + 1, n) >> 1)] * kC97Zeta; };
  float d2[5], s1[4], d1[3], s0[2];
#pragma unroll
  for (int i = 0; i < 5; ++i) d2[i] = d_at(k - 2 + i);                                    // d2[k-2..k+2]
#pragma unroll
  for (int i = 0; i < 4; ++i) s1[i] = s_at(k - 1 + i) - kC97Delta * (d2[i] + d2[i + 1]);   // s1[k-1..k+2]
#pragma unroll
  for (int i = 0; i < 3; ++i) d1[i] = d2[i + 1] - kC97Gamma * (s1[i] + s1[i + 1]);        // d1[k-1..k+1]
#pragma unroll
  for (int i = 0; i < 2; ++i) s0[i] = s1[i + 1] - kC97Beta * (d1[i] + d1[i + 1]);         // s0[k], s0[k+1]
  const float d0 = d1[1] - kC97Alpha * (s0[0] + s0[1]);
  const long long so = axis == 0 ? 1 : axis == 1 ? eo0 : (long long)eo0 * eo1;
  u[axis] = 2 * k;
  const long long o = u[0] + (long long)eo0 * (u[1] + (long long)eo1 * u[2]);
  dst[q * (half * 2) + o] = s0[0];
  dst[q * (half * 2) + o + so] = d0;
}

// ---------------------------------------------------------------------------
// Scores
// ---------------------------------------------------------------------------

// Offset of template block b from a candidate's base cell in a box of
// row length e0 and e1 rows per plane.
__device__ __forceinline__ int c97_block_off(int b, const Geom& g, int e0, int e1) {
  const int bx = b % g.tc[0], by = (b / g.tc[0]) % g.tc[1], bz = b / (g.tc[0] * g.tc[1]);
  return bx + e0 * (by + e1 * bz);
}

// Per event: its known blocks in template order as (block index b, offset
// of the block in the score map's LDS strip of row length wmap, A_b), and
// their count.  One wavefront per event; blocks are compacted 64 at a
// time by ballot.
__global__ __launch_bounds__(kThreads) void k_c97_pack(const int32_t* __restrict__ or_n, const float* __restrict__ or_m,
                                                       int n_filters, Geom g, int wmap, int32_t* __restrict__ cnt,
                                                       int32_t* __restrict__ off, int32_t* __restrict__ soff,
                                                       float* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int f = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (f >= n_filters) return;
  int c = 0;
  for (int b0 = 0; b0 < (int)g.tcells; b0 += 64) {
    const int b = b0 + lane;
    const bool known = b < (int)g.tcells && or_n[(long long)f * g.tcells + b] != 0;
    const uint64_t m = __ballot(known);
    if (known) {
      const int pos = c + __popcll(m & ((1ull << lane) - 1ull));
      off[(long long)f * kC97BlocksMax + pos] = b;
      soff[(long long)f * kC97BlocksMax + pos] = c97_block_off(b, g, wmap, g.tc[1]);
      val[(long long)f * kC97BlocksMax + pos] = or_m[(long long)f * g.tcells + b];
    }
    c += __popcll(m);
  }
  if (lane == 0) cnt[f] = c;
}

// Cell of candidate c in the K grid.
__device__ __forceinline__ int c97_base(int c, const Geom& g) {
  const int cx = c % g.cand[0], cy = (c / g.cand[0]) % g.cand[1], cz = c / (g.cand[0] * g.cand[1]);
  return idx3i(cx, cy, cz, g.G);
}

// S(c) in fp32, in the event's block order: the one routine behind the score
// map and the rescoring, so both give the same value for a candidate (K
// read from the grid or from an LDS copy of it).
template <typename OffP, typename ValP>
__device__ __forceinline__ float c97_score(const float* K, int base, OffP off, ValP A, int nk) {
  float s = 0.f;
  for (int i = 0; i < nk; ++i) {
    const float d = K[base + off[i]] - A[i];
    s = fmaf(d, d, s);
  }
  return s;
}

// Selection key of a score (S >= 0, so its bits order like its value): the
// score above a keyed bijection of the candidate index (ties are broken by
// the same permutation as the exact paths).
__device__ __forceinline__ uint64_t c97_key(float S, int c, uint64_t tkey) {
  return ((uint64_t)__float_as_uint(S) << 20) | tie_perm((uint32_t)c, tkey);
}

// Order-preserving 32-bit key of a float: ascending with the value.
__device__ __forceinline__ uint32_t c97_asc(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Candidates are taken in chunks of 32 consecutive x positions of one
// candidate row: chunk q = row * nchr + x / 32, nchr = ceil(C_x / 32), so the
// chunks ascend with the candidate index.  The score map and the bulk pass
// leave each chunk's best value (smallest score, largest bulk value) for
// the selections below.

// Stage the K values a candidate row segment reaches: strip entry i =
// (x, r) of W x (T_c,y T_c,z) holds K[x0 + x, cy + by, cz + bz] with r = by
// + T_c,y bz (0 past the grid's x end), passed to store(i, x, value).
// Every load of a thread goes out before its stores.
template <class Store>
__device__ __forceinline__ void c97_stage(const float* __restrict__ K, const Geom& g, int x0, int cy, int cz, int W,
                                          Store store) {
  constexpr int U = 8;
  const int n = g.tc[1] * g.tc[2] * W;
  BoxWalk w(threadIdx.x, kThreads, W, g.tc[1]);
  for (int i0 = threadIdx.x; i0 < n; i0 += U * kThreads) {
    float v[U];
    int xs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // positions past the strip read a clamped cell and are not stored
      const int x = x0 + w.x;
      const int y = min(cy + w.y, g.G[1] - 1), z = min(cz + w.z, g.G[2] - 1);
      v[u] = K[idx3i(min(x, g.G[0] - 1), y, z, g.G)];
      v[u] = x < g.G[0] ? v[u] : 0.f;
      xs[u] = w.x;
      w.next();
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * kThreads < n) store(i0 + u * kThreads, xs[u], v[u]);
  }
}

// The score map.  Workgroup: one segment of sw candidates of a candidate
// row (grid x = row * segments + segment) against up to kC97MapEvents
// events (grid y).  The K values the segment reaches (T_c,y x T_c,z grid
// rows of Wc = sw + T_c,x cells, rounded up to even) are staged once in LDS
// in two copies, K[x] and K[x + 1], so that a thread reads the values of
// its two adjacent candidates for a block with one aligned 8-byte load
// (copy 0 for an even block offset, copy 1 for an odd one).  The two halves
// of the workgroup take alternate events; the event lists are read with
// scalar loads.  Optionally the smallest score of each chunk.
constexpr int kC97MapEvents = 8;
constexpr int kC97MapLds = 64 * 1024;
__host__ __device__ inline int c97_map_wc(int sw, const Geom& g) { return (sw + g.tc[0] + 1) & ~1; }
inline size_t c97_map_lds(int sw, const Geom& g) { return (size_t)8 * g.tc[1] * g.tc[2] * c97_map_wc(sw, g); }
// Segment width: the widest multiple of 32 (<= 256) whose strips fit
// kC97MapLds; 0 when not even 32 does (very tall, narrow templates).
inline int c97_map_width(const Geom& g) {
  for (int sw = 256; sw >= 32; sw -= 32)
    if (c97_map_lds(sw, g) <= kC97MapLds) return sw;
  return 0;
}
__global__ __launch_bounds__(kThreads) void k_c97_map(const float* __restrict__ K, Geom g, int sw,
                                                      const int32_t* __restrict__ cnt, const int32_t* __restrict__ soff,
                                                      const float* __restrict__ val, int n_filters,
                                                      float* __restrict__ out, float* __restrict__ cmin) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nseg = (g.cand[0] + sw - 1) / sw;
  const int row = blockIdx.x / nseg, seg = blockIdx.x - row * nseg, tid = threadIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int Wc = c97_map_wc(sw, g), nrows = g.tc[1] * g.tc[2];
  float* k0 = (float*)smem;          // K[x0 + i]
  float* k1 = k0 + nrows * Wc;       // K[x0 + i + 1]
  const int x0 = seg * sw;
  c97_stage(K, g, x0, cy, cz, Wc, [&](int i, int xi, float v) {
    k0[i] = v;
    if (xi > 0) k1[i - 1] = v;
  });
  __syncthreads();
  const int half = tid >> 7, tl = tid & 127;
  const int xa = x0 + 2 * tl;                     // this thread's candidates xa, xa + 1
  const bool ok0 = 2 * tl < sw && xa < g.cand[0], ok1 = 2 * tl + 1 < sw && xa + 1 < g.cand[0];
  const int ca = row * g.cand[0] + xa;
  const int nchr = (g.cand[0] + 31) / 32;
  const long long nchk = (long long)g.cand[1] * g.cand[2] * nchr;
  const int f1 = min(n_filters, (int)(blockIdx.y + 1) * kC97MapEvents);
  for (int f = (int)blockIdx.y * kC97MapEvents + half; f < f1; f += 2) {
    const int fu = __builtin_amdgcn_readfirstlane(f);   // one event per wavefront
    const int nk = cnt[fu];
    const int32_t* so = soff + (long long)fu * kC97BlocksMax;
    const float* av = val + (long long)fu * kC97BlocksMax;
    // per candidate the same operations in the same order as c97_score
    float s0 = 0.f, s1 = 0.f;
    for (int i = 0; i < (2 * tl < sw ? nk : 0); ++i) {   // threads past the segment read nothing
      const int o = so[i];
      const float a = av[i];
      const float2 kv = *(const float2*)(((o & 1) ? k1 + (o - 1) : k0 + o) + 2 * tl);
      const float d0 = kv.x - a, d1 = kv.y - a;
      s0 = fmaf(d0, d0, s0);
      s1 = fmaf(d1, d1, s1);
    }
    if (ok0) out[(long long)fu * g.ncand + ca] = s0;
    if (ok1) out[(long long)fu * g.ncand + ca + 1] = s1;
    if (cmin) {
      float m = fminf(ok0 ? s0 : INFINITY, ok1 ? s1 : INFINITY);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) m = fminf(m, __shfl_xor(m, o));
      if ((tl & 15) == 0 && ok0) cmin[fu * nchk + (long long)row * nchr + (xa >> 5)] = m;
    }
  }
}

// Largest |K| over the grid: one partial maximum per workgroup (64 of them).
constexpr int kC97MaxParts = 64;
__global__ __launch_bounds__(kThreads) void k_c97_absmax(const float* __restrict__ K, long long n, float* __restrict__ part) {
  __shared__ float s_m[kThreads / 64];
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    m = fmaxf(m, fabsf(K[i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = s_m[0];
    for (int w = 1; w < kThreads / 64; ++w) r = fmaxf(r, s_m[w]);
    part[blockIdx.x] = r;
  }
}

// Workgroup-wide inclusive prefix sum of one value per thread (threads in
// order); s_w holds kThreads / 64 + 1 entries.  Every thread must call it.
__device__ __forceinline__ unsigned c97_incl_scan(unsigned v, unsigned* s_w, unsigned& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == 63) s_w[wave] = v;
  __syncthreads();
  unsigned base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    base += w < wave ? s_w[w] : 0u;
    tot += s_w[w];
  }
  __syncthreads();
  total = tot;
  return base + v;
}

struct C97Sel {
  unsigned hist[2048];
  unsigned w[kThreads / 64 + 1];
  uint32_t key, need;
};

// The k-th smallest of n 32-bit keys key_at(i) (1 <= k <= n): its value,
// and how many keys equal to it the k smallest take.  Three histogram
// passes of 11, 11 and 10 bits; each pass finds its bin with a prefix sum
// over the workgroup (thread t owns bins 8t .. 8t + 7).
template <class KeyFn>
__device__ void c97_kth_smallest(int n, int k, KeyFn key_at, C97Sel& sh) {
  const int tid = threadIdx.x;
  uint32_t prefix = 0, need = (uint32_t)k;
  const int shifts[3] = {21, 10, 0}, bits[3] = {11, 11, 10};
  for (int pass = 0; pass < 3; ++pass) {
    for (int i = tid; i < 2048; i += kThreads) sh.hist[i] = 0;
    __syncthreads();
    const int shf = shifts[pass];
    const uint32_t hmask = pass == 0 ? 0u : ~((1u << (shf + bits[pass])) - 1u);
    const uint32_t dmask = (1u << bits[pass]) - 1u;
    for (int i = tid; i < n; i += kThreads) {
      const uint32_t key = key_at(i);
      if ((key & hmask) == (prefix & hmask)) atomicAdd(&sh.hist[(key >> shf) & dmask], 1u);
    }
    __syncthreads();
    unsigned loc[8], sum = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      loc[j] = sh.hist[8 * tid + j];
      sum += loc[j];
    }
    unsigned total;
    const unsigned incl = c97_incl_scan(sum, sh.w, total);
    unsigned acc = incl - sum;
    if (acc < need && incl >= need) {
      int j = 0;
      while (acc + loc[j] < need) acc += loc[j++];
      sh.key = prefix | ((uint32_t)(8 * tid + j) << shf);
      sh.need = need - acc;
    }
    __syncthreads();
    prefix = sh.key;
    need = sh.need;
    __syncthreads();
  }
  if (tid == 0) {
    sh.key = prefix;
    sh.need = need;
  }
  __syncthreads();
}

// Ordered compaction: of n items with 32-bit keys keyf(i), every key below
// tk and, in index order, the first lim keys equal to tk; emit(i, pos) for
// each in index order (pos = 0, 1, ...).  Rounds of 8 consecutive items per
// thread, two workgroup prefix sums per round.  Returns how many were taken.
// Every thread must call it; LDS that emit writes is visible to the whole
// workgroup on return (closing barrier).
template <class KeyF, class Emit>
__device__ unsigned c97_take_ordered(int n, uint32_t tk, unsigned lim, KeyF keyf, Emit emit, unsigned* s_w) {
  unsigned base = 0, eqb = 0;
  for (int r0 = 0; r0 < n; r0 += 8 * kThreads) {
    const int i0 = r0 + 8 * (int)threadIdx.x;
    uint32_t key[8];
    unsigned neq = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      key[e] = i0 + e < n ? keyf(i0 + e) : 0u;
      neq += (i0 + e < n && key[e] == tk) ? 1u : 0u;
    }
    unsigned eq_tot;
    unsigned er = eqb + c97_incl_scan(neq, s_w, eq_tot) - neq;
    bool take[8];
    unsigned nt = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const bool in = i0 + e < n, at = in && key[e] == tk;
      take[e] = in && (key[e] < tk || (at && er < lim));
      er += at ? 1u : 0u;
      nt += take[e] ? 1u : 0u;
    }
    unsigned tot;
    unsigned pos = base + c97_incl_scan(nt, s_w, tot) - nt;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (take[e]) emit(i0 + e, pos++);
    base += tot;
    eqb += eq_tot;
  }
  __syncthreads();
  return base;
}

constexpr int kC97ListMax = 256;   // chunks a selection gathers into LDS

// Shortlist of the bulk pass: the R largest bulk values of an event (ties
// to the smaller index), R <= 128, as ascending candidate indices.  The
// R-th largest chunk maximum tau bounds the R-th largest value from below,
// so every member lies in a chunk whose maximum is >= tau: all chunks above
// tau (fewer than R) and, in index order, at most R chunks at tau (they hold
// the smallest-index candidates at tau).  Those chunks (< 2R) go to LDS and
// the selection finishes there.  One workgroup per event.
__global__ __launch_bounds__(kThreads) void k_c97_short(const float* __restrict__ bulk, const float* __restrict__ cmax,
                                                        Geom g, int R, int32_t* __restrict__ out) {
  __shared__ C97Sel sh;
  __shared__ int s_list[kC97ListMax];
  __shared__ float s_v[kC97ListMax * 32];
  const int f = blockIdx.x, tid = threadIdx.x;
  const int nchr = (g.cand[0] + 31) / 32;
  const int nchk = g.cand[1] * g.cand[2] * nchr;
  const float* cm = cmax + (long long)f * nchk;
  const float* bv = bulk + (long long)f * g.ncand;
  // tau as a descending key: the R-th smallest of ~asc(max)
  uint32_t tk = 0xFFFFFFFFu;
  if (nchk > R) {
    c97_kth_smallest(nchk, R, [&](int i) { return ~c97_asc(cm[i]); }, sh);
    tk = sh.key;
  }
  // ordered compaction of the chunks above tau and the first R at tau (all
  // of them when there are no more than R)
  const unsigned base = c97_take_ordered(nchk, tk, (unsigned)R, [&](int q) { return ~c97_asc(cm[q]); },
                                         [&](int q, unsigned pos) {
                                           if (pos < kC97ListMax) s_list[pos] = q;
                                         },
                                         sh.w);
  const int nl = (int)min(base, (unsigned)kC97ListMax);
  for (int i = tid; i < nl * 32; i += kThreads) {
    const int q = s_list[i >> 5], x = (q % nchr) * 32 + (i & 31);
    s_v[i] = x < g.cand[0] ? bv[(long long)(q / nchr) * g.cand[0] + x] : -INFINITY;
  }
  __syncthreads();
  c97_kth_smallest(nl * 32, R, [&](int i) { return ~c97_asc(s_v[i]); }, sh);
  const uint32_t pk = sh.key, pneed = sh.need;
  // every value above the R-th and, in index order, pneed of those equal
  c97_take_ordered(nl * 32, pk, pneed, [&](int i) { return ~c97_asc(s_v[i]); },
                   [&](int i, unsigned pos) {
                     if (pos < (unsigned)R) {
                       const int q = s_list[i >> 5];
                       out[(long long)f * R + pos] = (q / nchr) * g.cand[0] + (q % nchr) * 32 + (i & 31);
                     }
                   },
                   sh.w);
}

// The K best keys of every candidate from the score map and its chunk
// minima: tau = the K-th smallest chunk minimum bounds the K-th smallest
// score from above, so the K best lie in chunks whose minimum is <= tau.
// Their keys go to LDS when they fit (at most kC97ListMax chunks), else the
// whole row of the map is searched.  One workgroup per event; keys ascending.
__global__ __launch_bounds__(kThreads) void k_c97_best(const float* __restrict__ map, const float* __restrict__ cmin,
                                                       Geom g, int k, uint64_t seed, const int32_t* __restrict__ real,
                                                       const int64_t* __restrict__ steps, uint64_t* __restrict__ out) {
  __shared__ C97Sel sh;
  __shared__ TopkShared tsh;
  __shared__ int s_list[kC97ListMax];
  const int f = blockIdx.x, tid = threadIdx.x;
  const uint64_t tkey = draw64(seed, kStreamTiebreak, (uint64_t)real[f], (uint64_t)steps[f]);
  const int nchr = (g.cand[0] + 31) / 32;
  const int nchk = g.cand[1] * g.cand[2] * nchr;
  const float* cm = cmin + (long long)f * nchk;
  const float* m = map + (long long)f * g.ncand;
  uint32_t tk = 0xFFFFFFFFu;
  if (nchk > k) {
    c97_kth_smallest(nchk, k, [&](int i) { return c97_asc(cm[i]); }, sh);
    tk = sh.key;
  }
  const unsigned base = c97_take_ordered(nchk, tk, 0xFFFFFFFFu, [&](int q) { return c97_asc(cm[q]); },
                                         [&](int q, unsigned pos) {
                                           if (pos < kC97ListMax) s_list[pos] = q;
                                         },
                                         sh.w);
  if (base <= (unsigned)kC97ListMax) {
    const int n = (int)base * 32;
    block_topk(n, k, [&](long long i) {
      const int q = s_list[i >> 5], x = (q % nchr) * 32 + (int)(i & 31);
      const int c = (q / nchr) * g.cand[0] + x;
      // past the row's end: a key above every real one
      return x < g.cand[0] ? c97_key(m[c], c, tkey) : (~0ull - (uint64_t)i);
    }, tsh);
  } else {
    block_topk(g.ncand, k, [&](long long c) { return c97_key(m[c], (int)c, tkey); }, tsh);
  }
  if (tid < k) out[(long long)f * k + tid] = tsh.top[tid];
}

template <typename OT>
struct C97Op;
template <>
struct C97Op<_Float16> {
  typedef _Float16 vec8 __attribute__((ext_vector_type(8)));
  static constexpr float kMax = 65504.f;
  static __device__ __forceinline__ float16_t mma(vec8 a, vec8 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  // K^2 scaled by 2^-q stays below 2^15
  static __device__ __forceinline__ int q_of(float kmax) {
    const float m2 = kmax * kmax;
    return m2 >= 1.f ? min(max(0, ilogbf(m2) - 14), 60) : 0;
  }
};
template <>
struct C97Op<__bf16> {
  typedef __bf16 vec8 __attribute__((ext_vector_type(8)));
  static constexpr float kMax = 3.0e38f;
  static __device__ __forceinline__ float16_t mma(vec8 a, vec8 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int q_of(float) { return 0; }
};

template <typename OT>
__device__ __forceinline__ OT c97_op(float v) {
  return (OT)fminf(fmaxf(v, -C97Op<OT>::kMax), C97Op<OT>::kMax);
}

struct C97BulkArgs {
  Geom g;
  const float* K;            // level-J grid
  const int32_t* cnt;        // [event] known blocks
  const int32_t* blk;        // [event][kC97BlocksMax] their template block indices
  const float* val;          // [event][kC97BlocksMax] their A values
  const float* kmax;         // kC97MaxParts partial maxima of |K| (device)
  int n_filters;
  int kpad;                  // 2 T_c cells, padded to 16
  int seg;                   // candidates of a row per workgroup (a multiple of 32, <= kC97Seg)
  int W;                     // strip width: seg + T_c,x - 1
  float* bulk;               // [event][candidates]: sum n A K - n K^2 / 2
  float* cmax;               // [event][chunks]: largest bulk value of each chunk
};

// LDS of a bulk workgroup: both strips (16-byte aligned end), the block
// offsets, and 32 event rows of kpad + 8 operands (16-byte aligned rows).
__host__ __device__ inline size_t c97_strip_bytes(int nrows, int W) { return ((size_t)4 * nrows * W + 15) & ~(size_t)15; }
inline size_t c97_bulk_lds(int nrows, int W, int kpad) {
  return c97_strip_bytes(nrows, W) + (size_t)kpad * 4 + (size_t)32 * (kpad + 8) * 2;
}

// Bulk ranking value of every (event, candidate): B = sum_b n_b (A_b K -
// K^2 / 2) at K = K[c + b], i.e. -(S - sum n A^2) / 2, so the best
// candidates have the largest B.  One contraction over 2 T_c cells per
// candidate: the first half pairs n A with K, the second -n 2^q / 2 with
// K^2 2^-q, operands in OT (fp16 / bf16), fp32 accumulation.  Workgroup:
// seg candidates of one row (grid z) against 32 events (grid y); each
// wavefront takes 32-candidate chunks.  The MFMA takes the events as A and the K strip as B, so lane l
// holds candidate l % 32 of 16 events and the stores are contiguous runs.
template <typename OT>
__global__ __launch_bounds__(kThreads) void k_c97_bulk(C97BulkArgs a) {
  typedef typename C97Op<OT>::vec8 vec8;
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = blockIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int f0 = blockIdx.y * 32, x0 = blockIdx.z * a.seg;
  const int W = a.W, kpad = a.kpad;
  const int nrows = g.tc[1] * g.tc[2];
  const int tcells = (int)g.tcells;
  float kmax = 0.f;
  for (int i = 0; i < kC97MaxParts; ++i) kmax = fmaxf(kmax, a.kmax[i]);
  const int q = C97Op<OT>::q_of(kmax);
  const float down = ldexpf(1.f, -q), tap = -0.5f * ldexpf(1.f, q);
  OT* s_k = (OT*)smem;                       // [nrows][W] K, then [nrows][W] K^2 2^-q
  int* s_off = (int*)(smem + c97_strip_bytes(nrows, W));
  OT* s_b = (OT*)(smem + c97_strip_bytes(nrows, W) + (size_t)kpad * 4);
  const int bstride = kpad + 8;
  c97_stage(a.K, g, x0, cy, cz, W, [&](int i, int, float v) {
    s_k[i] = c97_op<OT>(v);
    s_k[nrows * W + i] = c97_op<OT>(v * v * down);
  });
  // the blocks known to any of the tile's events, ascending: the
  // contraction runs over those only (2 nu taps, padded to 16)
  __shared__ int s_u[kC97BlocksMax], s_bl[kC97BlocksMax], s_cnt[32];
  __shared__ int s_nu, s_mc;
  for (int b = tid; b < tcells; b += kThreads) s_u[b] = 0;
  if (tid < 64) {
    const int c = tid < 32 && f0 + tid < a.n_filters ? a.cnt[f0 + tid] : 0;
    if (tid < 32) s_cnt[tid] = c;
    int m = c;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) m = max(m, __shfl_xor(m, o));
    if (tid == 0) s_mc = m;
  }
  __syncthreads();
  // slots (event jf, list entry e) of the tile, e < the tile's longest list
  const int fl = a.n_filters - 1, mc = max(s_mc, 1), nslot = 32 * mc;
  constexpr int U = 8;
  for (int i0 = tid; i0 < nslot; i0 += U * kThreads) {
    int bb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(i0 + u * kThreads, nslot - 1), jf = i / mc;
      bb[u] = a.blk[(long long)min(f0 + jf, fl) * kC97BlocksMax + (i - jf * mc)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kThreads, jf = i / mc;
      if (i < nslot && i - jf * mc < s_cnt[jf]) s_u[bb[u]] = 1;
    }
  }
  __syncthreads();
  if (wave == 0) {
    int c = 0;
    for (int b0 = 0; b0 < tcells; b0 += 64) {
      const int b = b0 + lane;
      const bool u = b < tcells && s_u[b] != 0;
      const uint64_t m = __ballot(u);
      if (u) {
        const int pos = c + __popcll(m & ((1ull << lane) - 1ull));
        s_bl[pos] = b;
        s_u[b] = pos;   // from here on: the block's position in the list
      }
      c += __popcll(m);
    }
    if (lane == 0) s_nu = c;
  }
  __syncthreads();
  const int nu = s_nu, kp = (2 * nu + 15) / 16 * 16;
  for (int k = tid; k < kp; k += kThreads) {
    int o = 0;
    if (k < 2 * nu) {
      const int b = s_bl[k < nu ? k : k - nu];
      const int bx = b % g.tc[0], by = (b / g.tc[0]) % g.tc[1], bz = b / (g.tc[0] * g.tc[1]);
      o = (bz * g.tc[1] + by) * W + bx + (k < nu ? 0 : nrows * W);
    }
    s_off[k] = o;
  }
  for (int i = tid; i < 32 * kp; i += kThreads) {
    const int jf = i / kp;
    s_b[jf * bstride + (i - jf * kp)] = (OT)0.0f;
  }
  __syncthreads();
  const OT tap_op = c97_op<OT>(tap);
  for (int i0 = tid; i0 < nslot; i0 += U * kThreads) {
    int bb[U];
    float vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(i0 + u * kThreads, nslot - 1), jf = i / mc;
      const long long o = (long long)min(f0 + jf, fl) * kC97BlocksMax + (i - jf * mc);
      bb[u] = a.blk[o];
      vv[u] = a.val[o];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kThreads, jf = i / mc;
      if (i < nslot && i - jf * mc < s_cnt[jf]) {
        const int pos = s_u[bb[u]];
        s_b[jf * bstride + pos] = c97_op<OT>(vv[u]);
        s_b[jf * bstride + nu + pos] = tap_op;
      }
    }
  }
  __syncthreads();
  const int nchunks = min(a.seg, g.cand[0] - x0 + 31) / 32;
  const int j = lane & 31, g8 = (lane >> 5) * 8;
  const OT* erow = s_b + j * bstride + g8;
  const long long rowbase = (long long)g.cand[0] * row + x0;
  for (int ch = wave; ch < nchunks; ch += kThreads / 64) {
    const int cb = ch * 32 + j;
    float16_t acc = {};
    for (int kc = 0; kc < kp; kc += 16) {
      vec8 kv;
#pragma unroll
      for (int e = 0; e < 8; ++e) kv[e] = s_k[s_off[kc + g8 + e] + cb];
      acc = C97Op<OT>::mma(*(const vec8*)(erow + kc), kv, acc);
    }
    const bool ok = x0 + cb < g.cand[0];
    if (ok) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int f = f0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (f < a.n_filters) a.bulk[(long long)f * g.ncand + rowbase + cb] = acc[v];
      }
    }
    // each event's largest value over the chunk's 32 candidates (the lanes
    // of a half wavefront)
    const int nchr = (g.cand[0] + 31) / 32;
    const long long nchk = (long long)g.cand[1] * g.cand[2] * nchr;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float m = ok ? acc[v] : -INFINITY;
#pragma unroll
      for (int o = 1; o < 32; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
      const int f = f0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (j == 0 && f < a.n_filters) a.cmax[f * nchk + (long long)row * nchr + (x0 >> 5) + ch] = m;
    }
  }
}

// fp32 rescoring of each event's shortlist (R ascending candidate indices)
// and the K best of it: one workgroup per event, keys ascending.
__global__ __launch_bounds__(kThreads) void k_c97_rescore(const float* __restrict__ K, Geom g,
                                                          const int32_t* __restrict__ cnt,
                                                          const int32_t* __restrict__ off, const float* __restrict__ val,
                                                          const int32_t* __restrict__ shortlist, int R, int k,
                                                          uint64_t seed, const int32_t* __restrict__ real,
                                                          const int64_t* __restrict__ steps,
                                                          uint64_t* __restrict__ out) {
  __shared__ int s_off[kC97BlocksMax];
  __shared__ float s_val[kC97BlocksMax];
  __shared__ uint64_t s_key[kC97ShortMax];
  __shared__ TopkShared sh;
  const int f = blockIdx.x, tid = threadIdx.x;
  const int nk = cnt[f];
  for (int i = tid; i < nk; i += kThreads) {
    s_off[i] = c97_block_off(off[(long long)f * kC97BlocksMax + i], g, g.G[0], g.G[1]);
    s_val[i] = val[(long long)f * kC97BlocksMax + i];
  }
  __syncthreads();
  const uint64_t tkey = draw64(seed, kStreamTiebreak, (uint64_t)real[f], (uint64_t)steps[f]);
  for (int t = tid; t < R; t += kThreads) {
    const int c = shortlist[(long long)f * R + t];
    s_key[t] = c97_key(c97_score(K, c97_base(c, g), s_off, s_val, nk), c, tkey);
  }
  __syncthreads();
  block_topk(R, k, [&](long long t) { return s_key[t]; }, sh);
  if (tid < k) out[(long long)f * k + tid] = sh.top[tid];
}

}  // namespace ccw
