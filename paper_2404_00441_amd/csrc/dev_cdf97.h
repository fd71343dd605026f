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
constexpr int kC97ShortMax = 256;     // candidates rescored per event
constexpr int kC97Seg = 256;          // candidates of a row per bulk workgroup

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

// Per event: its known blocks in template order as (offset of block b from a
// candidate's base cell in the K grid, A_b), and their count.
__global__ void k_c97_pack(const int32_t* __restrict__ or_n, const float* __restrict__ or_m, int n_filters, Geom g,
                           int32_t* __restrict__ cnt, int32_t* __restrict__ off, float* __restrict__ val) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_filters) return;
  int c = 0;
  for (int b = 0; b < (int)g.tcells; ++b) {
    if (or_n[(long long)f * g.tcells + b] == 0) continue;
    const int bx = b % g.tc[0], by = (b / g.tc[0]) % g.tc[1], bz = b / (g.tc[0] * g.tc[1]);
    off[(long long)f * kC97BlocksMax + c] = idx3i(bx, by, bz, g.G);
    val[(long long)f * kC97BlocksMax + c] = or_m[(long long)f * g.tcells + b];
    ++c;
  }
  cnt[f] = c;
}

// Cell of candidate c in the K grid.
__device__ __forceinline__ int c97_base(int c, const Geom& g) {
  const int cx = c % g.cand[0], cy = (c / g.cand[0]) % g.cand[1], cz = c / (g.cand[0] * g.cand[1]);
  return idx3i(cx, cy, cz, g.G);
}

// S(c) in fp32, in the event's block order: the one routine behind the score
// map and the rescoring, so both give the same value for a candidate.
__device__ __forceinline__ float c97_score(const float* __restrict__ K, int base, const int* off, const float* A,
                                           int nk) {
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

// The score map: grid (candidate blocks of 256, events).
__global__ __launch_bounds__(kThreads) void k_c97_map(const float* __restrict__ K, Geom g, const int32_t* __restrict__ cnt,
                                                      const int32_t* __restrict__ off, const float* __restrict__ val,
                                                      float* __restrict__ out) {
  __shared__ int s_off[kC97BlocksMax];
  __shared__ float s_val[kC97BlocksMax];
  const int f = blockIdx.y, tid = threadIdx.x;
  const int nk = cnt[f];
  for (int i = tid; i < nk; i += kThreads) {
    s_off[i] = off[(long long)f * kC97BlocksMax + i];
    s_val[i] = val[(long long)f * kC97BlocksMax + i];
  }
  __syncthreads();
  const int c = blockIdx.x * kThreads + tid;
  if (c >= g.ncand) return;
  out[(long long)f * g.ncand + c] = c97_score(K, c97_base(c, g), s_off, s_val, nk);
}

// The K best of every candidate (from the score map): one workgroup per
// event, keys ascending.
__global__ __launch_bounds__(kThreads) void k_c97_topk_all(const float* __restrict__ map, Geom g, int k, uint64_t seed,
                                                           const int32_t* __restrict__ real,
                                                           const int64_t* __restrict__ steps, uint64_t* __restrict__ out) {
  __shared__ TopkShared sh;
  const int f = blockIdx.x;
  const uint64_t tkey = draw64(seed, kStreamTiebreak, (uint64_t)real[f], (uint64_t)steps[f]);
  const float* m = map + (long long)f * g.ncand;
  block_topk(g.ncand, k, [&](long long c) { return c97_key(m[c], (int)c, tkey); }, sh);
  if ((int)threadIdx.x < k) out[(long long)f * k + threadIdx.x] = sh.top[threadIdx.x];
}

// Largest |K| over the grid (one workgroup); it sets the fp16 operands'
// power-of-two scaling of K^2.
__global__ __launch_bounds__(kThreads) void k_c97_absmax(const float* __restrict__ K, long long n, float* __restrict__ out) {
  __shared__ float s_m[kThreads / 64];
  float m = 0.f;
  for (long long i = threadIdx.x; i < n; i += kThreads) m = fmaxf(m, fabsf(K[i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = s_m[0];
    for (int w = 1; w < kThreads / 64; ++w) r = fmaxf(r, s_m[w]);
    *out = r;
  }
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
  const int32_t* or_n;       // [event][T_c cells]
  const float* or_m;         // [event][T_c cells]
  const float* kmax;         // largest |K| (device)
  int n_filters;
  int kpad;                  // 2 T_c cells, padded to 16
  int W;                     // strip width: kC97Seg + T_c,x - 1
  float* bulk;               // [event][candidates]: sum n A K - n K^2 / 2
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
// kC97Seg candidates of one row (grid z) against 32 events (grid y); each
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
  const int f0 = blockIdx.y * 32, x0 = blockIdx.z * kC97Seg;
  const int W = a.W, kpad = a.kpad;
  const int nrows = g.tc[1] * g.tc[2];
  const int tcells = (int)g.tcells;
  const int q = C97Op<OT>::q_of(*a.kmax);
  const float down = ldexpf(1.f, -q), tap = -0.5f * ldexpf(1.f, q);
  OT* s_k = (OT*)smem;                       // [nrows][W] K, then [nrows][W] K^2 2^-q
  int* s_off = (int*)(smem + c97_strip_bytes(nrows, W));
  OT* s_b = (OT*)(smem + c97_strip_bytes(nrows, W) + (size_t)kpad * 4);
  const int bstride = kpad + 8;
  for (int i = tid; i < nrows * W; i += kThreads) {
    const int x = x0 + i % W, r = i / W;
    const int by = r % g.tc[1], bz = r / g.tc[1];
    float v = 0.f;
    if (x < g.G[0]) v = a.K[idx3i(x, cy + by, cz + bz, g.G)];
    s_k[i] = c97_op<OT>(v);
    s_k[nrows * W + i] = c97_op<OT>(v * v * down);
  }
  for (int k = tid; k < kpad; k += kThreads) {
    const int b = k < tcells ? k : k - tcells;
    int o = 0;
    if (k < 2 * tcells) {
      const int bx = b % g.tc[0], by = (b / g.tc[0]) % g.tc[1], bz = b / (g.tc[0] * g.tc[1]);
      o = (bz * g.tc[1] + by) * W + bx + (k < tcells ? 0 : nrows * W);
    }
    s_off[k] = o;
  }
  for (int i = tid; i < 32 * kpad; i += kThreads) {
    const int jf = i / kpad, k = i - jf * kpad, f = f0 + jf;
    float v = 0.f;
    if (f < a.n_filters && k < 2 * tcells) {
      const int b = k < tcells ? k : k - tcells;
      const bool known = a.or_n[(long long)f * tcells + b] != 0;
      v = !known ? 0.f : k < tcells ? a.or_m[(long long)f * tcells + b] : tap;
    }
    s_b[jf * bstride + k] = c97_op<OT>(v);
  }
  __syncthreads();
  const int nchunks = min(kC97Seg, g.cand[0] - x0 + 31) / 32;
  const int j = lane & 31, g8 = (lane >> 5) * 8;
  const OT* erow = s_b + j * bstride + g8;
  const long long rowbase = (long long)g.cand[0] * row + x0;
  for (int ch = wave; ch < nchunks; ch += kThreads / 64) {
    const int cb = ch * 32 + j;
    float16_t acc = {};
    for (int kc = 0; kc < kpad; kc += 16) {
      vec8 kv;
#pragma unroll
      for (int e = 0; e < 8; ++e) kv[e] = s_k[s_off[kc + g8 + e] + cb];
      acc = C97Op<OT>::mma(*(const vec8*)(erow + kc), kv, acc);
    }
    if (x0 + cb < g.cand[0]) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int f = f0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (f < a.n_filters) a.bulk[(long long)f * g.ncand + rowbase + cb] = acc[v];
      }
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
    s_off[i] = off[(long long)f * kC97BlocksMax + i];
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
