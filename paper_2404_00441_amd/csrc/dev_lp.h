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

// Cross-entropy of the softmax over candidates against the best position,
// per example; dS = (softmax - onehot) / B in place of S.  One workgroup
// per example, fixed-order reductions.
__global__ __launch_bounds__(kThreads) void k_lp_ce(float* __restrict__ S, const int32_t* __restrict__ label,
                                                    long long ncand, int B, float* __restrict__ loss) {
  __shared__ float red[kThreads];
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
  const int lb = label[b];
  const float sl = s[lb];
  __syncthreads();
  if (threadIdx.x == 0) loss[b] = logf(z) + m - sl;
  const float inv = 1.f / (z * (float)B);
  for (long long c = threadIdx.x; c < ncand; c += kThreads)
    s[c] = expf(s[c] - m) * inv - (c == lb ? 1.f / (float)B : 0.f);
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
// example; the output order is not significant.
__device__ __forceinline__ uint32_t lp_desc_key(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // ascending with f
  return ~asc;                                                          // ascending with -f
}
__global__ __launch_bounds__(kThreads) void k_lp_topk(const float* __restrict__ S, long long ncand, int k,
                                                      int32_t* __restrict__ out) {
  __shared__ unsigned hist[2048];
  __shared__ unsigned s_pref, s_need, s_cnt, s_tie[kThreads + 1];
  const float* s = S + (long long)blockIdx.x * ncand;
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
    if (key < prefix) out[(long long)blockIdx.x * k + atomicAdd(&s_cnt, 1u)] = (int32_t)c;
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
      out[(long long)blockIdx.x * k + base + before] = (int32_t)c;
      ++before;
    }
  }
}

}  // namespace ccw
