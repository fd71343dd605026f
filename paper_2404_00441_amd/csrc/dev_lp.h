// dev_lp.h -- the learned candidate proposer: two small convolutional
// encoders over level-J approximation coefficients (Sec. 3.1, Sec. 4.3: the
// search runs on the approximation), trained to rank candidate positions by
// their agreement with a data event, so that only a shortlist of positions
// needs the exact CCW score (Sec. 4.4 keeps the K best of those).
//
// Key encoder over the TI's approximation grid K / |beta| (one channel),
// query encoder over a data event (two channels: m / |beta| and
// n / |beta| over the T_c template blocks, zero off the overlap).  Both are
// 4 layers: 3x3 convolutions with dilations 1, 2, 4 (32 channels, ReLU)
// and a 1x1 convolution to 64 channels.  The key of candidate c is the key
// map at c + (tc / 2) (the centre of its template window, which the
// 15-block receptive field covers); the query is the query map at the same
// offset of the event window.  The proposer's score of c is q . k_c.
//
// Everything is fp32 on the vector units: the networks are small and the
// training step is dominated by memory traffic, not arithmetic.
#pragma once

#include "dev_kernels.h"
#include "dev_scan.h"

namespace ccw {

constexpr int kLpC = 32;      // hidden channels
constexpr int kLpD = 64;      // embedding dimension
constexpr int kLpLayers = 4;

// Layer l of an encoder with `cin0` input channels: input channels, output
// channels, taps (9 or 1) and dilation.
struct LpLayer {
  int cin, cout, taps, dil;
};
__host__ __device__ inline LpLayer lp_layer(int l, int cin0) {
  if (l == 0) return {cin0, kLpC, 9, 1};
  if (l == 1) return {kLpC, kLpC, 9, 2};
  if (l == 2) return {kLpC, kLpC, 9, 4};
  return {kLpC, kLpD, 1, 1};
}
// Floats of layer l (weights [cout][cin][taps], then biases [cout]).
__host__ __device__ inline long long lp_layer_size(int l, int cin0) {
  const LpLayer L = lp_layer(l, cin0);
  return (long long)L.cout * L.cin * L.taps + L.cout;
}
// Offset of layer l of encoder e (0 key, cin 1; 1 query, cin 2) in the
// weight buffer, and the total size.
__host__ __device__ inline long long lp_offset(int e, int l) {
  long long o = 0;
  for (int ee = 0; ee <= e; ++ee)
    for (int ll = 0; ll < kLpLayers; ++ll) {
      if (ee == e && ll == l) return o;
      o += lp_layer_size(ll, ee == 0 ? 1 : 2);
    }
  return o;
}
__host__ __device__ inline long long lp_weights_total() { return lp_offset(1, kLpLayers); }

// out[n][co][y][x] = b[co] + sum_ci sum_t W[co][ci][t] in[n][ci][y + dil dy_t][x + dil dx_t],
// zero outside the image, optionally ReLU.  One thread per output value.
__global__ __launch_bounds__(kThreads) void k_lp_conv_fwd(const float* __restrict__ in, const float* __restrict__ Wb,
                                                          float* __restrict__ out, int N, int cin, int cout, int H,
                                                          int Wd, int taps, int dil, int relu) {
  const long long hw = (long long)H * Wd;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)N * cout * hw) return;
  const int n = (int)(id / (cout * hw));
  const long long r = id - (long long)n * cout * hw;
  const int co = (int)(r / hw);
  const long long p = r - (long long)co * hw;
  const int y = (int)(p / Wd), x = (int)(p - (long long)y * Wd);
  const float* W = Wb + (long long)co * cin * taps;
  float s = Wb[(long long)cout * cin * taps + co];
  for (int ci = 0; ci < cin; ++ci) {
    const float* src = in + ((long long)n * cin + ci) * hw;
    for (int t = 0; t < taps; ++t) {
      const int yy = taps == 9 ? y + dil * (t / 3 - 1) : y;
      const int xx = taps == 9 ? x + dil * (t % 3 - 1) : x;
      if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) s += W[ci * taps + t] * src[(long long)yy * Wd + xx];
    }
  }
  out[id] = relu ? fmaxf(s, 0.f) : s;
}

// dpre = dout * [out > 0] (ReLU layers) in place.
__global__ void k_lp_relu_bwd(float* __restrict__ d, const float* __restrict__ out, long long n) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n && !(out[id] > 0.f)) d[id] = 0.f;
}

// din[n][ci][y][x] = sum_co sum_t W[co][ci][t] dpre[n][co][y - dil dy_t][x - dil dx_t].
__global__ __launch_bounds__(kThreads) void k_lp_conv_bwd_in(const float* __restrict__ dpre,
                                                             const float* __restrict__ Wb, float* __restrict__ din,
                                                             int N, int cin, int cout, int H, int Wd, int taps,
                                                             int dil) {
  const long long hw = (long long)H * Wd;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)N * cin * hw) return;
  const int n = (int)(id / (cin * hw));
  const long long r = id - (long long)n * cin * hw;
  const int ci = (int)(r / hw);
  const long long p = r - (long long)ci * hw;
  const int y = (int)(p / Wd), x = (int)(p - (long long)y * Wd);
  float s = 0.f;
  for (int co = 0; co < cout; ++co) {
    const float* src = dpre + ((long long)n * cout + co) * hw;
    const float* W = Wb + ((long long)co * cin + ci) * taps;
    for (int t = 0; t < taps; ++t) {
      const int yy = taps == 9 ? y - dil * (t / 3 - 1) : y;
      const int xx = taps == 9 ? x - dil * (t % 3 - 1) : x;
      if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) s += W[t] * src[(long long)yy * Wd + xx];
    }
  }
  din[id] = s;
}

// Gradients of one layer's weights: one workgroup per (co, ci) pair sums
// dW[co][ci][t] over every image and position (and db[co] when ci = 0),
// in a fixed order (block tree reduction), so results are reproducible.
__global__ __launch_bounds__(kThreads) void k_lp_conv_bwd_w(const float* __restrict__ in,
                                                            const float* __restrict__ dpre, float* __restrict__ gWb,
                                                            int N, int cin, int cout, int H, int Wd, int taps,
                                                            int dil) {
  __shared__ float red[10][kThreads];
  const int co = blockIdx.x / cin, ci = blockIdx.x - (blockIdx.x / cin) * cin;
  const long long hw = (long long)H * Wd;
  float acc[10] = {};
  for (int n = 0; n < N; ++n) {
    const float* d = dpre + ((long long)n * cout + co) * hw;
    const float* s = in + ((long long)n * cin + ci) * hw;
    for (long long p = threadIdx.x; p < hw; p += kThreads) {
      const int y = (int)(p / Wd), x = (int)(p - (long long)y * Wd);
      const float g = d[p];
      if (g == 0.f) continue;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        if (t >= taps) break;
        const int yy = taps == 9 ? y + dil * (t / 3 - 1) : y;
        const int xx = taps == 9 ? x + dil * (t % 3 - 1) : x;
        if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) acc[t] += g * s[(long long)yy * Wd + xx];
      }
      acc[9] += g;
    }
  }
  for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)taps) gWb[((long long)co * cin + ci) * taps + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 0 && ci == 0) gWb[(long long)cout * cin * taps + co] = red[9][0];
}

// Geometry of the proposer on one TI: candidate c = (cx, cy[, cz]) reads
// the key map at (c + half) with half = tc / 2 per axis.
struct LpGeom {
  int G[3];      // key map extent (the level-J grid)
  int cand[3];   // candidates per axis
  int half[3];   // key offset of a candidate (tc / 2)
  int tc[3];     // template blocks (event window)
  long long ncand;
};

__device__ __forceinline__ long long lp_key_pos(const LpGeom& q, long long c) {
  const int cx = (int)(c % q.cand[0]), cy = (int)((c / q.cand[0]) % q.cand[1]);
  const int cz = (int)(c / ((long long)q.cand[0] * q.cand[1]));
  return (long long)(cx + q.half[0]) + (long long)q.G[0] * ((cy + q.half[1]) + (long long)q.G[1] * (cz + q.half[2]));
}

// Keys of every candidate, [c][64], from the key map [64][G].
__global__ void k_lp_gather_keys(const float* __restrict__ kmap, LpGeom q, float* __restrict__ keys) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= q.ncand * kLpD) return;
  const long long c = id / kLpD;
  const int d = (int)(id - c * kLpD);
  const long long gc = (long long)q.G[0] * q.G[1] * q.G[2];
  keys[id] = kmap[d * gc + lp_key_pos(q, c)];
}

// Queries [b][64] from the query maps [b][64][tc] (the centre block).
__global__ void k_lp_gather_queries(const float* __restrict__ qmap, LpGeom q, int B, float* __restrict__ qv) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= B * kLpD) return;
  const int b = id / kLpD, d = id - b * kLpD;
  const long long wc = (long long)q.tc[0] * q.tc[1] * q.tc[2];
  const long long o = q.half[0] + (long long)q.tc[0] * (q.half[1] + (long long)q.tc[1] * q.half[2]);
  qv[id] = qmap[((long long)b * kLpD + d) * wc + o];
}

// Proposer scores S[b][c] = q_b . k_c; one thread per (b, c).
__global__ void k_lp_scores(const float* __restrict__ qv, const float* __restrict__ keys, long long ncand, int B,
                            float* __restrict__ S) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ncand * B) return;
  const int b = (int)(id / ncand);
  const long long c = id - (long long)b * ncand;
  const float4* qq = (const float4*)(qv + (long long)b * kLpD);
  const float4* kk = (const float4*)(keys + c * kLpD);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kLpD / 4; ++i) {
    const float4 a = qq[i], k = kk[i];
    s += a.x * k.x + a.y * k.y + a.z * k.z + a.w * k.w;
  }
  S[id] = s;
}

// Cross-entropy of the softmax over candidates against a set T of L
// positions (distinct; L = 1: the best position), per example:
// loss = log sum_c exp S_c - log sum_{c in T} exp S_c, and in place of S
// its gradient for the batch mean, dS_c = (p_c - [c in T] exp S_c / sum_T exp S) / B.
// One workgroup per example, fixed-order reductions.
constexpr int kLpPosMax = 32;
__global__ __launch_bounds__(kThreads) void k_lp_ce(float* __restrict__ S, const int32_t* __restrict__ label,
                                                    int L, long long ncand, int B, float* __restrict__ loss) {
  __shared__ float red[kThreads];
  __shared__ float s_lv[kLpPosMax];
  const int b = blockIdx.x;
  float* s = S + (long long)b * ncand;
  float m = -3.4e38f;
  for (long long c = threadIdx.x; c < ncand; c += kThreads) m = fmaxf(m, s[c]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  m = red[0];
  __syncthreads();
  float z = 0.f;
  for (long long c = threadIdx.x; c < ncand; c += kThreads) z += expf(s[c] - m);
  red[threadIdx.x] = z;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  z = red[0];
  const int32_t* lb = label + (long long)b * L;
  if ((int)threadIdx.x < L) s_lv[threadIdx.x] = expf(s[lb[threadIdx.x]] - m);
  __syncthreads();
  float zt = 0.f;
  for (int j = 0; j < L; ++j) zt += s_lv[j];
  if (threadIdx.x == 0) loss[b] = logf(z) - logf(zt);
  const float inv = 1.f / (z * (float)B);
  for (long long c = threadIdx.x; c < ncand; c += kThreads) s[c] = expf(s[c] - m) * inv;
  __syncthreads();
  if ((int)threadIdx.x < L) s[lb[threadIdx.x]] -= s_lv[threadIdx.x] / (zt * (float)B);
}

// dq[b][d] = sum_c dS[b][c] k_c[d]; one workgroup per example, 4 threads
// per dimension summing interleaved candidates, then a fixed-order sum.
__global__ __launch_bounds__(kThreads) void k_lp_grad_q(const float* __restrict__ dS, const float* __restrict__ keys,
                                                        long long ncand, float* __restrict__ dq) {
  __shared__ float red[kThreads];
  const int b = blockIdx.x;
  const int d = threadIdx.x % kLpD, part = threadIdx.x / kLpD;
  const float* g = dS + (long long)b * ncand;
  float s = 0.f;
  for (long long c = part; c < ncand; c += kThreads / kLpD) s += g[c] * keys[c * kLpD + d];
  red[threadIdx.x] = s;
  __syncthreads();
  if (part == 0) {
    float t = 0.f;
    for (int k = 0; k < kThreads / kLpD; ++k) t += red[k * kLpD + d];
    dq[(long long)b * kLpD + d] = t;
  }
}

// dkeymap[d][key position of c] = sum_b dS[b][c] q_b[d]; every other
// position of the map is zero (cleared first).
__global__ void k_lp_grad_k(const float* __restrict__ dS, const float* __restrict__ qv, LpGeom q, int B,
                            float* __restrict__ dkmap) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= q.ncand * kLpD) return;
  const long long c = id / kLpD;
  const int d = (int)(id - c * kLpD);
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dS[(long long)b * q.ncand + c] * qv[(long long)b * kLpD + d];
  const long long gc = (long long)q.G[0] * q.G[1] * q.G[2];
  dkmap[d * gc + lp_key_pos(q, c)] = s;
}

// dqmap: the query gradient at the centre block, zero elsewhere.
__global__ void k_lp_scatter_dq(const float* __restrict__ dq, LpGeom q, int B, float* __restrict__ dqmap) {
  const long long wc = (long long)q.tc[0] * q.tc[1] * q.tc[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)B * kLpD * wc) return;
  const long long bd = id / wc, p = id - bd * wc;
  const long long o = q.half[0] + (long long)q.tc[0] * (q.half[1] + (long long)q.tc[1] * q.half[2]);
  dqmap[id] = p == o ? dq[bd] : 0.f;
}

// Adam (Kingma and Ba, 2015) with bias correction; t >= 1.
__global__ void k_lp_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, int t) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const float gi = g[id];
  const float mi = b1 * m[id] + (1.f - b1) * gi;
  const float vi = b2 * v[id] + (1.f - b2) * gi * gi;
  m[id] = mi;
  v[id] = vi;
  const float mh = mi / (1.f - powf(b1, (float)t)), vh = vi / (1.f - powf(b2, (float)t));
  w[id] -= lr * mh / (sqrtf(vh) + eps);
}

// He-uniform initialisation from the counter-based generator: weight i of
// a layer with fan-in F is (2u - 1) sqrt(6 / F), u uniform in [0, 1);
// biases zero.
__global__ void k_lp_init(float* __restrict__ w, uint64_t seed) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= lp_weights_total()) return;
  for (int e = 0; e < 2; ++e)
    for (int l = 0; l < kLpLayers; ++l) {
      const long long o = lp_offset(e, l);
      const LpLayer L = lp_layer(l, e == 0 ? 1 : 2);
      const long long nw = (long long)L.cout * L.cin * L.taps;
      if (id >= o && id < o + nw) {
        const double u = (double)(draw64(seed, 11, (uint64_t)e * 16 + l, (uint64_t)(id - o)) >> 11) * (1.0 / 9007199254740992.0);
        w[id] = (float)((2.0 * u - 1.0) * sqrt(6.0 / (double)(L.cin * L.taps)));
        return;
      }
      if (id >= o + nw && id < o + nw + L.cout) {
        w[id] = 0.f;
        return;
      }
    }
}

// Query encoder input from data events given per template block as
// or_n (known cells) and or_m (sum of their codes): m / |beta| and
// n / |beta| as two channels.
__global__ void k_lp_events(const int32_t* __restrict__ or_n, const int32_t* __restrict__ or_m, int B, long long wc,
                            float inv_beta, float* __restrict__ out) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)B * wc) return;
  const long long b = id / wc, p = id - b * wc;
  out[(b * 2) * wc + p] = (float)or_m[id] * inv_beta;
  out[(b * 2 + 1) * wc + p] = (float)or_n[id] * inv_beta;
}

// The TI's approximation as the key encoder's input: K / |beta|.
__global__ void k_lp_kin(const int32_t* __restrict__ K, long long n, float inv_beta, float* __restrict__ out) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) out[id] = (float)K[id] * inv_beta;
}

// The k largest scores of each example (k <= 256), ties to the smaller
// index: a radix select over order-preserving 32-bit keys of the floats
// (three passes of 11, 11 and 10 bits with LDS histograms), then every
// candidate strictly above the threshold and, in index order, as many
// candidates at the threshold as the k still need.  One workgroup per
// example; the k indices come out in ascending order.
__device__ __forceinline__ uint32_t lp_desc_key(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // ascending with f
  return ~asc;                                                          // ascending with -f
}
// The same order for exact integer scores: the k smallest first.
__device__ __forceinline__ uint32_t lp_desc_key(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lp_topk(const T* __restrict__ S, long long ncand, int k,
                                                      int32_t* __restrict__ out) {
  __shared__ unsigned hist[2048];
  __shared__ unsigned s_pref, s_need, s_cnt, s_tie[kThreads + 1];
  __shared__ int32_t s_out[256];
  const T* s = S + (long long)blockIdx.x * ncand;
  const int tid = threadIdx.x;
  uint32_t prefix = 0, need = (uint32_t)k;
  const int shifts[3] = {21, 10, 0}, bits[3] = {11, 11, 10};
  for (int pass = 0; pass < 3; ++pass) {
    for (int i = tid; i < 2048; i += kThreads) hist[i] = 0;
    __syncthreads();
    const int sh = shifts[pass];
    const uint32_t hmask = pass == 0 ? 0u : ~((1u << (sh + bits[pass])) - 1u);
    const uint32_t dmask = (1u << bits[pass]) - 1u;
    for (long long c = tid; c < ncand; c += kThreads) {
      const uint32_t key = lp_desc_key(s[c]);
      if ((key & hmask) == (prefix & hmask)) atomicAdd(&hist[(key >> sh) & dmask], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      unsigned acc = 0, b = 0;
      for (; b < (1u << bits[pass]); ++b) {
        if (acc + hist[b] >= need) break;
        acc += hist[b];
      }
      s_pref = prefix | (b << sh);
      s_need = need - acc;
    }
    __syncthreads();
    prefix = s_pref;
    need = s_need;
    __syncthreads();
  }
  // prefix is the k-th smallest key; `need` of the candidates equal to it
  // are taken, in index order
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  const long long per = (ncand + kThreads - 1) / kThreads;
  const long long c0 = tid * per, c1 = min(ncand, c0 + per);
  unsigned ties = 0;
  for (long long c = c0; c < c1; ++c) {
    const uint32_t key = lp_desc_key(s[c]);
    if (key < prefix) s_out[atomicAdd(&s_cnt, 1u)] = (int32_t)c;
    else if (key == prefix) ++ties;
  }
  s_tie[tid] = ties;
  __syncthreads();
  if (tid == 0) {
    unsigned acc = 0;
    for (int i = 0; i < kThreads; ++i) {
      const unsigned v = s_tie[i];
      s_tie[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  unsigned before = s_tie[tid];
  const unsigned base = s_cnt;   // every candidate above the threshold is placed
  __syncthreads();
  for (long long c = c0; c < c1 && before < need; ++c) {
    if (lp_desc_key(s[c]) == prefix) {
      s_out[base + before] = (int32_t)c;
      ++before;
    }
  }
  __syncthreads();
  // in ascending index order (distinct indices: the rank is the position),
  // so the output does not depend on the order of the atomics above
  for (int i = tid; i < k; i += kThreads) {
    const int32_t v = s_out[i];
    int r = 0;
    for (int j = 0; j < k; ++j) r += s_out[j] < v ? 1 : 0;
    out[(long long)blockIdx.x * k + r] = v;
  }
}

// ---------------------------------------------------------------------------
// Inverted lists over the keys, built once per TI and weights: Lloyd's
// k-means in the 64-d key space puts every candidate in the list of its
// nearest centroid.  A data event's query ranks the centroids by inner
// product; only the members of the best lists are scored exactly.
// ---------------------------------------------------------------------------
constexpr int32_t kLpMagic = 0x4C504958;
constexpr int kLpListsMax = 1024;   // lists of an index
constexpr int kLpProbeMax = 16;     // lists probed per data event
constexpr int kLpCandMax = 1792;    // candidates scored exactly per data event

struct LpIndexHeader {
  int32_t magic, n_lists, level, ndim;
  int32_t G[3], cand[3], tc[3], pad0;
  int64_t ncand;
  int64_t off_w;      // bytes from the index base: the query encoder's weights (float)
  int64_t off_cent;   // centroids [n_lists][64] (float), then the same values as
                      // [16][n_lists][4] at off_cent + lp_cent_bytes(n_lists), so
                      // that a thread per list reads its 16-byte words coalesced
  int64_t off_list;   // list offsets [n_lists + 1] (int32)
  int64_t off_mem;    // members [ncand] (int32), by list, ascending within a list
  int64_t bytes;
};
__host__ __device__ inline long long lp_query_floats() { return lp_weights_total() - lp_offset(1, 0); }
__host__ __device__ inline long long lp_cent_bytes(int n_lists) {
  return ((long long)n_lists * kLpD * 4 + 255) & ~255ll;
}

// The centroids' second copy: word d4 (4 floats) of list j at d4 * n_lists + j.
__global__ void k_km_transpose(const float* __restrict__ cent, int nl, float* __restrict__ ct) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nl * (kLpD / 4)) return;
  const int j = id % nl, d4 = id / nl;
  ((float4*)ct)[id] = ((const float4*)cent)[(long long)j * (kLpD / 4) + d4];
}

// Starting centroids: keys at evenly spaced candidate indices.
__global__ void k_km_init(const float* __restrict__ keys, long long ncand, int nl, float* __restrict__ cent) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nl * kLpD) return;
  const int j = id / kLpD, d = id - j * kLpD;
  cent[id] = keys[((long long)j * ncand / nl) * kLpD + d];
}

// Nearest centroid of every key by squared distance (ties to the smaller
// list); the centroids pass through LDS 64 at a time.
__global__ __launch_bounds__(kThreads) void k_km_assign(const float* __restrict__ keys, long long ncand,
                                                        const float* __restrict__ cent, int nl,
                                                        int32_t* __restrict__ assign) {
  __shared__ float s_c[64][kLpD + 1];
  __shared__ float s_nrm[64];
  const int tid = threadIdx.x;
  const long long c = (long long)blockIdx.x * kThreads + tid;
  float k[kLpD];
#pragma unroll
  for (int d = 0; d < kLpD; ++d) k[d] = c < ncand ? keys[c * kLpD + d] : 0.f;
  float best = 3.4e38f;
  int bj = 0;
  for (int j0 = 0; j0 < nl; j0 += 64) {
    __syncthreads();
    for (int i = tid; i < 64 * kLpD; i += kThreads) {
      const int jj = i / kLpD, d = i - jj * kLpD;
      s_c[jj][d] = j0 + jj < nl ? cent[(long long)(j0 + jj) * kLpD + d] : 0.f;
    }
    __syncthreads();
    if (tid < 64) {
      float n = 0.f;
      for (int d = 0; d < kLpD; ++d) n += s_c[tid][d] * s_c[tid][d];
      s_nrm[tid] = n;
    }
    __syncthreads();
    const int nj = min(64, nl - j0);
    for (int jj = 0; jj < nj; ++jj) {
      float dot = 0.f;
#pragma unroll
      for (int d = 0; d < kLpD; ++d) dot += k[d] * s_c[jj][d];
      const float dist = s_nrm[jj] - 2.f * dot;
      if (dist < best) {
        best = dist;
        bj = j0 + jj;
      }
    }
  }
  if (c < ncand) assign[c] = bj;
}

// Members of list j (one workgroup per list) in ascending candidate order:
// with off == null only their number goes to cnt[j]; otherwise they are
// written from off[j] on.
__global__ __launch_bounds__(kThreads) void k_km_lists(const int32_t* __restrict__ assign, long long ncand,
                                                       const int32_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ int s_w[kThreads / 64];
  __shared__ int s_run;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = blockIdx.x;
  if (tid == 0) s_run = 0;
  __syncthreads();
  for (long long b = 0; b < ncand; b += kThreads) {
    const long long c = b + tid;
    const bool hit = c < ncand && assign[c] == j;
    const unsigned long long bal = __ballot(hit);
    if (lane == 0) s_w[wave] = __popcll(bal);
    __syncthreads();
    int before = s_run;
    for (int w = 0; w < wave; ++w) before += s_w[w];
    before += __popcll(bal & ((1ull << lane) - 1ull));
    if (hit && off) out[off[j] + before] = (int32_t)c;
    __syncthreads();
    if (tid == 0) s_run += s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
  }
  if (!off && tid == 0) out[j] = s_run;
}

// Exclusive prefix sums of the list sizes, off[0..nl] (one thread: nl <= 1024).
__global__ void k_km_offsets(const int32_t* __restrict__ cnt, int nl, int32_t* __restrict__ off) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int run = 0;
  for (int j = 0; j < nl; ++j) {
    off[j] = run;
    run += cnt[j];
  }
  off[nl] = run;
}

// Centroid j = mean of its members' keys, summed in a fixed order; an
// empty list keeps its centroid.
__global__ __launch_bounds__(kThreads) void k_km_update(const float* __restrict__ keys,
                                                        const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ mem, float* __restrict__ cent) {
  __shared__ float s_p[kThreads / kLpD][kLpD];
  const int j = blockIdx.x, tid = threadIdx.x;
  const int d = tid % kLpD, part = tid / kLpD;
  const int lo = off[j], n = off[j + 1] - lo;
  float s = 0.f;
  for (int i = part; i < n; i += kThreads / kLpD) s += keys[(long long)mem[lo + i] * kLpD + d];
  s_p[part][d] = s;
  __syncthreads();
  if (tid < kLpD && n > 0) {
    float t = 0.f;
    for (int q = 0; q < kThreads / kLpD; ++q) t += s_p[q][tid];
    cent[(long long)j * kLpD + tid] = t / (float)n;
  }
}

// ---------------------------------------------------------------------------
// The query of one data event, evaluated only where the query encoder's
// output at the window's centre block h depends on it: layer 2 (dilation
// 4) at h, layer 1 (dilation 2) at h + 4 d, layer 0 at h + 4 d + 2 e for
// d, e in {-1, 0, 1}^2 (a 7 x 7 lattice of step 2), each position outside
// the window being zero (the maps' zero padding).  Equal to the full
// encoder's output at h.  All threads of the workgroup take part.
//   ev: [2][tc1 + 2][tc0 + 2] input channels with a zero border; a0: [49][32];
//   a1: [9][32]; a2: [32];
//   q: [64] output.  W: the query encoder's weights.
// ---------------------------------------------------------------------------
__device__ void lp_query_sparse(const float* __restrict__ W, const float* ev, int tc0, int tc1, float* a0, float* a1,
                                float* a2, float* q) {
  const int tid = threadIdx.x;
  const int h0 = tc0 / 2, h1 = tc1 / 2;
  const long long o0 = 0, o1 = lp_layer_size(0, 2), o2 = o1 + lp_layer_size(1, 2), o3 = o2 + lp_layer_size(2, 2);
  // every weight this thread uses is loaded once, up front, in 16-byte
  // words (W is 256-byte aligned and every block below starts on a 16-byte
  // boundary): layer 0 by co = tid % 32 (8-byte words), layers 1 and 2 by
  // (co = tid / 8, input channels 4 (tid % 8) .. + 3), whose 36 weights are
  // consecutive, layer 3 by (d = tid / 4, input channels 8 (tid % 4) .. + 7)
  const int c1 = tid >> 3, p1 = tid & 7;
  float w1[36], w2[36], w3[8];
  {
    const float4* s1 = (const float4*)(W + o1 + (long long)(c1 * kLpC + p1 * 4) * 9);
    const float4* s2 = (const float4*)(W + o2 + (long long)(c1 * kLpC + p1 * 4) * 9);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      const float4 x = s1[v], y = s2[v];
      w1[4 * v] = x.x, w1[4 * v + 1] = x.y, w1[4 * v + 2] = x.z, w1[4 * v + 3] = x.w;
      w2[4 * v] = y.x, w2[4 * v + 1] = y.y, w2[4 * v + 2] = y.z, w2[4 * v + 3] = y.w;
    }
  }
  const float b1 = W[o1 + kLpC * kLpC * 9 + c1], b2 = W[o2 + kLpC * kLpC * 9 + c1];
  const int d3 = tid >> 2, p3 = tid & 3;
  {
    const float4* s3 = (const float4*)(W + o3 + (long long)d3 * kLpC + p3 * 8);
    const float4 x = s3[0], y = s3[1];
    w3[0] = x.x, w3[1] = x.y, w3[2] = x.z, w3[3] = x.w, w3[4] = y.x, w3[5] = y.y, w3[6] = y.z, w3[7] = y.w;
  }
  const float b3 = W[o3 + kLpD * kLpC + d3];
  // layer 0: 2 -> 32 channels, dilation 1.  Thread (co, group) takes every
  // eighth lattice position.
  {
    const int co = tid & (kLpC - 1), grp = tid >> 5;
    float w0[18];
    const float2* s0 = (const float2*)(W + o0 + co * 18);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      const float2 x = s0[v];
      w0[2 * v] = x.x, w0[2 * v + 1] = x.y;
    }
    const float b0 = W[o0 + kLpC * 2 * 9 + co];
    const int ew = tc0 + 2, eh = tc1 + 2;
    for (int pos = grp; pos < 49; pos += kThreads / kLpC) {
      const int py = h1 + 2 * (pos / 7) - 6, px = h0 + 2 * (pos % 7) - 6;
      float s = 0.f;
      if (py >= 0 && py < tc1 && px >= 0 && px < tc0) {
        // the 3 x 3 neighbourhood lies in the bordered canvas
        const float* e0 = ev + py * ew + px;
        float sc[2] = {b0, 0.f};   // one chain per input channel
#pragma unroll
        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
          for (int t = 0; t < 9; ++t) sc[ci] += w0[ci * 9 + t] * e0[ci * eh * ew + (t / 3) * ew + (t % 3)];
        s = fmaxf(sc[0] + sc[1], 0.f);
      }
      a0[pos * kLpC + co] = s;
    }
  }
  __syncthreads();
  // layer 1: 32 -> 32, dilation 2, at the 9 points h + 4 d.  Thread
  // (co, part) sums its 4 input channels (one 16-byte LDS read per tap) for
  // all 9 points; the 8 parts of an output are added with lane shuffles.
#pragma unroll 3
  for (int pos = 0; pos < 9; ++pos) {
    const int dy = pos / 3 - 1, dx = pos % 3 - 1;
    const int py = h1 + 4 * dy, px = h0 + 4 * dx;
    const bool in = py >= 0 && py < tc1 && px >= 0 && px < tc0;   // uniform
    float sc[4] = {0.f, 0.f, 0.f, 0.f};   // one chain per input channel
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      // layer-0 lattice point h + 4 d + 2 e with e = tap offset
      const int ly = 2 * (dy + 1) + (t / 3), lx = 2 * (dx + 1) + (t % 3);
      const float4 x = *(const float4*)(a0 + (ly * 7 + lx) * kLpC + p1 * 4);
      sc[0] += w1[t] * x.x;
      sc[1] += w1[9 + t] * x.y;
      sc[2] += w1[18 + t] * x.z;
      sc[3] += w1[27 + t] * x.w;
    }
    float s = (sc[0] + sc[1]) + (sc[2] + sc[3]);
    s += __shfl_xor(s, 1, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 4, 8);
    if (p1 == 0) a1[pos * kLpC + c1] = in ? fmaxf(s + b1, 0.f) : 0.f;
  }
  __syncthreads();
  // layer 2: 32 -> 32, dilation 4, at h only; 8 lanes per output
  {
    float sc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const float4 x = *(const float4*)(a1 + t * kLpC + p1 * 4);
      sc[0] += w2[t] * x.x;
      sc[1] += w2[9 + t] * x.y;
      sc[2] += w2[18 + t] * x.z;
      sc[3] += w2[27 + t] * x.w;
    }
    float s = (sc[0] + sc[1]) + (sc[2] + sc[3]);
    s += __shfl_xor(s, 1, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 4, 8);
    if (p1 == 0) a2[c1] = fmaxf(s + b2, 0.f);
  }
  __syncthreads();
  // layer 3: 1x1, 32 -> 64; 4 lanes per output
  {
    const float4 x = *(const float4*)(a2 + p3 * 8), y = *(const float4*)(a2 + p3 * 8 + 4);
    float s = w3[0] * x.x + w3[1] * x.y + w3[2] * x.z + w3[3] * x.w + w3[4] * y.x + w3[5] * y.y + w3[6] * y.z +
              w3[7] * y.w;
    s += __shfl_xor(s, 1, 4);
    s += __shfl_xor(s, 2, 4);
    if (p3 == 0) q[d3] = s + b3;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Proposal for one data event per workgroup: the query, the probed lists,
// the exact score of every member (Sec. 4.3 score in integers, from the
// level-J grid staged in LDS), the K best keys among them and the gate.
// A patch falls back to the full scan when its overlap is empty, when hard
// data lie in its virtual template, when fewer than K candidates were
// scored, or when the best match error exceeds the gate.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The step's patches that fall back, packed into scan tiles of one
// orientation each (in slot order), with their records and data events;
// map[slot] = the packed slot, or -1 where the proposal stands.  Run by one
// workgroup (the step's last proposal); the packed tiles never outnumber
// the step's tiles.  A packed tile's records name their patches, whose
// data events the scan reads in place.
// ---------------------------------------------------------------------------
struct LpCompactArgs {
  const TileDev* tiles;   // the step's tiles
  const ScanRec* recs;    // [tile][kFiltersPerTile]
  int ntiles, nf, n_orient, fbegin;
  const int32_t* ok;      // [slot], written by the step's other workgroups
  TileDev* dtiles;
  ScanRec* drecs;
  int32_t* map;           // [slot]
  int32_t* dcount;        // packed tiles
};

__device__ void lp_compact(const LpCompactArgs& a, unsigned char* smem) {
  int* s_or = (int*)smem;          // [nf] orientation, -1: proposal stands
  int* s_ri = s_or + a.nf;         // [nf] record index
  int* s_zm = s_ri + a.nf;         // [nf] zmask bit
  int* s_map = s_zm + a.nf;        // [nf]
  uint32_t* s_dz = (uint32_t*)(s_map + a.nf);   // [256] zmask of each packed tile
  __shared__ int s_w[kThreads / 64];
  __shared__ int s_cnt[8], s_bslot[8], s_btile[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < a.nf; i += kThreads) s_or[i] = -1;
  for (int i = tid; i < 256; i += kThreads) s_dz[i] = 0u;
  __syncthreads();
  for (int i = tid; i < a.ntiles * kFiltersPerTile; i += kThreads) {
    const int t = i / kFiltersPerTile, j = i - t * kFiltersPerTile;
    const TileDev td = a.tiles[t];
    if (j < td.count) {
      const int slot = td.first + j;
      const int okv = __hip_atomic_load(&a.ok[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool fb = a.recs[i].gidx >= 0 && okv == 0;
      s_or[slot] = fb ? td.orient : -1;
      s_ri[slot] = i;
      s_zm[slot] = (int)((td.zmask >> j) & 1u);
    }
  }
  __syncthreads();
  // per orientation: the packed position of each of its patches, in slot order
  for (int o = 0; o < a.n_orient; ++o) {
    int run = 0;
    for (int b = 0; b < a.nf; b += kThreads) {
      const int slot = b + tid;
      const bool hit = slot < a.nf && s_or[slot] == o;
      const unsigned long long bal = __ballot(hit);
      if (lane == 0) s_w[wave] = __popcll(bal);
      __syncthreads();
      int before = run;
      for (int w = 0; w < wave; ++w) before += s_w[w];
      before += __popcll(bal & ((1ull << lane) - 1ull));
      if (hit) s_map[slot] = before;   // position within the orientation for now
      run += s_w[0] + s_w[1] + s_w[2] + s_w[3];
      __syncthreads();
    }
    if (tid == 0) s_cnt[o] = run;
  }
  __syncthreads();
  if (tid == 0) {
    int bs = 0, bt = 0;
    for (int o = 0; o < a.n_orient; ++o) {
      s_bslot[o] = bs;
      s_btile[o] = bt;
      bs += s_cnt[o];
      bt += (s_cnt[o] + kFiltersPerTile - 1) / kFiltersPerTile;
    }
    *a.dcount = bt;
  }
  __syncthreads();
  for (int slot = tid; slot < a.nf; slot += kThreads) {
    const int o = s_or[slot];
    int cs = -1;
    if (o >= 0) {
      const int pos = s_map[slot];
      cs = s_bslot[o] + pos;
      const int t = s_btile[o] + pos / kFiltersPerTile, j = pos % kFiltersPerTile;
      a.drecs[t * kFiltersPerTile + j] = a.recs[s_ri[slot]];
      if (s_zm[slot]) atomicOr(&s_dz[t], 1u << j);
    }
    s_map[slot] = cs;
    a.map[slot] = cs;
  }
  __syncthreads();
  for (int o = 0; o < a.n_orient; ++o) {
    const int nt = (s_cnt[o] + kFiltersPerTile - 1) / kFiltersPerTile;
    for (int i = tid; i < nt * kFiltersPerTile; i += kThreads) {
      const int tt = i / kFiltersPerTile, j = i - tt * kFiltersPerTile;
      const int t = s_btile[o] + tt;
      const int count = min(kFiltersPerTile, s_cnt[o] - tt * kFiltersPerTile);
      if (j == 0) {
        TileDev d;
        d.first = s_bslot[o] + tt * kFiltersPerTile;
        d.count = count;
        d.orient = o;
        d.zmask = s_dz[t];
        a.dtiles[t] = d;
      }
      if (j >= count) {
        ScanRec r = {};
        r.gidx = -1;
        a.drecs[t * kFiltersPerTile + j] = r;
      }
    }
  }
}

struct LpPropArgs {
  Geom g;
  const unsigned char* index;   // LpIndexHeader and its arrays
  const void* grid;             // level-J grid, KT [G1][G0], 16-byte padded
  int probe, cap, top_k, kpad;
  float gate;                   // largest accepted match error (< 0: always fall back)
  uint64_t seed;
  int standalone;
  // simulation: the step's patches
  const FilterDev* filters;
  int fbegin;
  const int32_t* kbeta;         // [orient][kKMax] block lists
  const int32_t* nbt;           // [shape][tcells] known cells per block
  const int32_t* mbuf;          // [patch][kKMax] data events
  const int32_t* hd_off;        // [patch + 1] hard data per virtual template, or null
  uint64_t* sel;                // [slot][top_k] the K best keys
  int32_t* ok;                  // [slot] 1: the proposal stands, 0: the full scan decides
  unsigned long long* report;
  int32_t* ticket;              // proposals of the step done (the last packs; reset to 0 after)
  LpCompactArgs cmp;
  // standalone: events as for the scan
  const int32_t* or_n;
  const int32_t* or_m;
  const int32_t* fil_real;
  const int64_t* fil_step;
  uint64_t* keys_out;           // [f][top_k]
  int32_t* list_out;            // [f][cap] candidates scored, or null
  int32_t* nlist_out;           // [f], or null
  float* q_out;                 // [f][64], or null
  float* err_out;               // [f] best match error, or null
};

// LDS of k_lp_propose: the grid, then one area used in turn by the
// encoder's scratch, the list scores, and the members with their keys; the
// event's block list after it.
__host__ __device__ inline long long lp_prop_grid_bytes(const Geom& g, int kt_bytes) {
  return ((long long)g.G[0] * g.G[1] * kt_bytes + 15) & ~15ll;
}
__host__ __device__ inline long long lp_prop_alias_bytes(const Geom& g, int cap) {
  long long v = (2ll * (g.tc[0] + 2) * (g.tc[1] + 2) + 49 * kLpC + 9 * kLpC + kLpC) * 4;   // encoder scratch
  const long long ck = (((long long)cap * 4 + 15) & ~15ll) + (long long)cap * 4;         // members, scores
  if (ck > v) v = ck;
  if (4ll * kLpListsMax > v) v = 4ll * kLpListsMax;                                       // list scores
  return (v + 15) & ~15ll;
}
__host__ __device__ inline long long lp_prop_lds(const Geom& g, int kt_bytes, int cap, int list_len) {
  return lp_prop_grid_bytes(g, kt_bytes) + lp_prop_alias_bytes(g, cap) + 20ll * list_len;
}

// Two workgroups per CU (LDS for two grid copies; at most 256 registers).
template <typename KT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_lp_propose(LpPropArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ TopkShared sh;
  __shared__ int s_probe[kLpProbeMax], s_lo[kLpProbeMax], s_len[kLpProbeMax], s_pos[kLpProbeMax];
  __shared__ int s_nk, s_M, s_np, s_force;
  __shared__ float s_q[kLpD];
  __shared__ double s_rt[kThreads / 64], s_rn[kThreads / 64];
  const Geom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int slot = blockIdx.x;
  const LpIndexHeader* H = (const LpIndexHeader*)a.index;
  const int G0 = g.G[0];
  const int tcells = (int)g.tcells;
  KT* s_K = (KT*)smem;
  unsigned char* alias = smem + lp_prop_grid_bytes(g, (int)sizeof(KT));
  int* s_cand = (int*)alias;   // members, after the list scores
  int32_t* s_sc = (int32_t*)(alias + (((long long)a.cap * 4 + 15) & ~15ll));   // exact scores of the members
  float* s_a0 = (float*)alias;
  float* s_a1 = s_a0 + 49 * kLpC;
  float* s_a2 = s_a1 + 9 * kLpC;
  float* s_ev = s_a2 + kLpC;
  float* s_cs = (float*)alias;   // list scores, after the encoder
  const int L = a.standalone ? tcells : a.kpad;   // block list capacity
  int4* s_ent = (int4*)(alias + lp_prop_alias_bytes(g, a.cap));   // (grid offset, m, n, 0) per listed block
  int* s_beta = (int*)(s_ent + L);

  // the grid goes to LDS by direct loads (global to LDS, no registers),
  // issued first and waited for only before the exact scores: wavefront w
  // moves 1 KiB chunks w, w + 4, ..., lane l the chunk's 16 bytes at 16 l
  {
    const int nv = (int)(lp_prop_grid_bytes(g, (int)sizeof(KT)) / 16);
    const unsigned char* src = (const unsigned char*)a.grid;
    for (int c = wave; c * 64 < nv; c += kThreads / 64) {
      if (c * 64 + lane < nv)
        __builtin_amdgcn_global_load_lds(
            (const void __attribute__((address_space(1)))*)(src + (long long)(c * 64 + lane) * 16),
            (void __attribute__((address_space(3)))*)((unsigned char*)s_K + c * 1024), 16, 0, 0);
    }
  }
  // an index built for another geometry sends every patch to the scan
  const bool hdr_ok = H->magic == kLpMagic && H->n_lists >= 1 && H->n_lists <= kLpListsMax && H->ncand == g.ncand &&
                      H->G[0] == g.G[0] && H->G[1] == g.G[1] && H->cand[0] == g.cand[0] &&
                      H->cand[1] == g.cand[1] && H->tc[0] == g.tc[0] && H->tc[1] == g.tc[1];
  const int ew = g.tc[0] + 2, eh = g.tc[1] + 2;   // the encoder's input with a zero border
  for (int i = tid; i < 2 * ew * eh; i += kThreads) s_ev[i] = 0.f;
  uint64_t tkey = 0;
  if (tid == 0) {
    s_nk = 0;
    s_force = hdr_ok ? 0 : 1;
  }
  __syncthreads();
  // the event's block list: (block, offset in the grid, m, n)
  if (!a.standalone) {
    const FilterDev f = a.filters[slot];
    tkey = draw64(a.seed, kStreamTiebreak, (uint64_t)f.r, (uint64_t)f.step);
    if (tid < a.kpad) {
      const int beta = a.kbeta[f.orient * kKMax + tid];
      int m = 0, n = 0, off = 0;
      if (beta >= 0 && f.bandmask) {
        m = a.mbuf[(long long)(a.fbegin + slot) * kKMax + tid];
        n = a.nbt[(long long)f.shape * tcells + beta];
        int bx, by, bz;
        split3(beta, g.tc[0], g.tc[1], bx, by, bz);
        off = by * G0 + bx;
      }
      s_beta[tid] = n > 0 ? beta : -1;
      s_ent[tid] = make_int4(off, m, n, 0);
    }
    if (tid == 0) {
      s_nk = a.kpad;
      const bool hd = a.hd_off && a.hd_off[a.fbegin + slot + 1] > a.hd_off[a.fbegin + slot];
      if (f.bandmask == 0 || hd) s_force = 1;
    }
  } else {
    if (a.fil_real) tkey = draw64(a.seed, kStreamTiebreak, (uint64_t)a.fil_real[slot], (uint64_t)a.fil_step[slot]);
    for (int b = tid; b < tcells; b += kThreads) {
      const int n = a.or_n[(long long)slot * tcells + b];
      if (n > 0) {
        const int i = atomicAdd(&s_nk, 1);   // list order does not change integer sums
        int bx, by, bz;
        split3(b, g.tc[0], g.tc[1], bx, by, bz);
        s_beta[i] = b;
        s_ent[i] = make_int4(by * G0 + bx, a.or_m[(long long)slot * tcells + b], n, 0);
      }
    }
  }
  __syncthreads();
  const int nk = s_nk;
  // the encoder's input, and the match error's constant term
  // sum |beta|^2 m^2 / n and the known cells sum n
  const double B = (double)(1 << (g.shift - 1));
  double ct = 0.0, cn = 0.0;
  for (int i = tid; i < nk; i += kThreads) {
    const int4 e = s_ent[i];
    if (e.z > 0) {
      const float inv = 1.f / (float)g.beta;
      const int by = s_beta[i] / g.tc[0], bx = s_beta[i] - by * g.tc[0];
      s_ev[(by + 1) * ew + bx + 1] = (float)e.y * inv;
      s_ev[eh * ew + (by + 1) * ew + bx + 1] = (float)e.z * inv;
      ct += B * B * (double)e.y * (double)e.y / (double)e.z;
      cn += (double)e.z;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    ct += __shfl_xor(ct, m, 64);
    cn += __shfl_xor(cn, m, 64);
  }
  if (lane == 0) {
    s_rt[wave] = ct;
    s_rn[wave] = cn;
  }
  __syncthreads();
  if (!hdr_ok) {   // nothing of the index is read
    if (tid == 0) {
      s_M = 0;
      s_np = 0;
    }
    for (int i = tid; i < kLpD; i += kThreads) s_q[i] = 0.f;
    __syncthreads();
  } else {
  lp_query_sparse((const float*)(a.index + H->off_w), s_ev, g.tc[0], g.tc[1], s_a0, s_a1, s_a2, s_q);
  if (a.q_out && tid < kLpD) a.q_out[(long long)slot * kLpD + tid] = s_q[tid];
  // the lists by the inner product of the query with their centroid
  const int nl = hdr_ok ? H->n_lists : 1;
  const float4* ct = (const float4*)(a.index + H->off_cent + lp_cent_bytes(nl));
  for (int j = tid; j < nl; j += kThreads) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < kLpD / 4; ++d) {
      const float4 c = ct[(long long)d * nl + j];   // coalesced across the lists
      s += s_q[4 * d] * c.x + s_q[4 * d + 1] * c.y + s_q[4 * d + 2] * c.z + s_q[4 * d + 3] * c.w;
    }
    s_cs[j] = s == s ? s : -INFINITY;   // a total order for the ranks below
  }
  __syncthreads();
  // the P best lists: the P smallest keys (descending score, then index)
  const int P = min(a.probe, nl);
  block_topk(nl, P, [&](long long j) {
    const uint32_t u = __float_as_uint(s_cs[j]);
    const uint32_t up = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // ascending with the score
    return ((uint64_t)(~up) << 32) | (uint64_t)j;
  }, sh);
  if (tid < P) s_probe[tid] = (int)(sh.top[tid] & 0xFFFFFFFFull);
  __syncthreads();
  const int32_t* loff = (const int32_t*)(a.index + H->off_list);
  const int32_t* mem = (const int32_t*)(a.index + H->off_mem);
  if (tid < P) {   // the probed lists' extents, loaded together
    const int j = s_probe[tid];
    const int lo = loff[j];
    s_lo[tid] = lo;
    s_len[tid] = loff[j + 1] - lo;
  }
  __syncthreads();
  if (tid == 0) {
    int M = 0, np = 0;
    for (int r = 0; r < P; ++r) {
      int len = s_len[r];
      if (M + len > a.cap) {
        if (r > 0) break;
        len = a.cap;
        s_len[r] = len;
      }
      s_pos[np] = M;
      M += len;
      ++np;
    }
    s_M = M;
    s_np = np;
    if (M < min(a.top_k, (int)g.ncand)) s_force = 1;
  }
  __syncthreads();
  {
    // every member load of a thread issued at once: list r of entry i by
    // a search of the (few) list starts
    const int np = s_np, Mt = s_M;
    for (int i = tid; i < Mt; i += kThreads) {
      int r = 0;
      while (r + 1 < np && s_pos[r + 1] <= i) ++r;
      s_cand[i] = mem[s_lo[r] + (i - s_pos[r])];
    }
  }
  __syncthreads();
  }
  const int M = s_M;
  const int k = min(a.top_k, (int)g.ncand);
  const bool force = s_force != 0;
  // the grid's direct loads of this wavefront, then everyone's
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (!force || a.standalone) {
    // exact keys of the members (mismatch 0: patches with hard data fall
    // back), four members per thread so that each list entry read serves four
    const int C0 = g.cand[0];
    const int shift = g.shift;
    for (int i0 = tid; i0 < M; i0 += 4 * kThreads) {
      const KT* kb[4];
      int cc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = min(i0 + u * kThreads, M - 1);
        const int c = min(max(s_cand[i], 0), (int)g.ncand - 1);
        const int cy = c / C0, cx = c - cy * C0;
        kb[u] = s_K + cy * G0 + cx;
        cc[u] = c;
      }
      int E[4] = {0, 0, 0, 0}, C[4] = {0, 0, 0, 0};
#pragma unroll 2
      for (int q = 0; q < nk; ++q) {
        const int4 e = s_ent[q];   // one broadcast read
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kv = (int)kb[u][e.x];
          E[u] += e.z * kv * kv;
          C[u] += e.y * kv;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * kThreads < M) s_sc[i0 + u * kThreads] = E[u] - (C[u] << shift);
    }
    __syncthreads();
    // keys rebuilt from (score, member) where they are compared
    if (M >= k)
      block_topk(M, k, [&](long long i) {
        const int c = min(max(s_cand[i], 0), (int)g.ncand - 1);
        return make_key(0u, s_sc[i], tie_perm((uint32_t)c, tkey));
      }, sh);
  }
  if (tid == 0) {
    double err = -1.0;
    const double tsum = s_rt[0] + s_rt[1] + s_rt[2] + s_rt[3], nsum = s_rn[0] + s_rn[1] + s_rn[2] + s_rn[3];
    if (M >= k && nsum > 0.0 && (!force || a.standalone)) {
      const int32_t S = (int32_t)((uint32_t)((sh.top[0] >> 20) & 0xFFFFFFFFull) ^ 0x80000000u);
      err = ((double)S + tsum) / (B * B * nsum);
    }
    const bool fb = force || a.gate < 0.f || err > (double)a.gate;
    if (!a.standalone) {
      a.ok[slot] = fb ? 0 : 1;
      atomicAdd(&a.report[fb ? 6 : 4], 1ull);
      if (!force) atomicAdd(&a.report[5], (unsigned long long)M);
    } else {
      if (a.nlist_out) a.nlist_out[slot] = M;
      if (a.err_out) a.err_out[slot] = (float)err;
    }
  }
  if (!a.standalone) {
    if (tid < k && !force) a.sel[(long long)slot * a.top_k + tid] = sh.top[tid];
    // the step's last proposal packs the patches the gate sends to the scan
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const int t = __hip_atomic_fetch_add(a.ticket, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      s_last = t == (int)gridDim.x - 1 ? 1 : 0;
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      lp_compact(a.cmp, smem);
      if (tid == 0) __hip_atomic_store(a.ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else {
    if (tid < k) a.keys_out[(long long)slot * a.top_k + tid] = M >= k ? sh.top[tid] : ~0ull;
    if (a.list_out)
      for (int i = tid; i < M; i += kThreads) a.list_out[(long long)slot * a.cap + i] = s_cand[i];
  }
}

// The level-J grid narrowed for the proposal's LDS copy (every value fits).
template <typename KT>
__global__ void k_lp_narrow(const int32_t* __restrict__ Ki, long long n, long long npad, KT* __restrict__ out) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < npad) out[id] = id < n ? (KT)Ki[id] : (KT)0;
}

}  // namespace ccw
