// dev_learn.h -- the learned candidate proposer.
//
// The key encoder is a D-dimensional principal-component basis P of the
// candidates' level-J windows x_c (every block of the template footprint,
// read from the approximation grid), fitted on the device from the TI:
// partial moments per workgroup, a fixed-order reduction, then subspace
// iteration with Gram-Schmidt in one workgroup.  Every candidate gets an
// embedding e_c = P (x_c - mu) and the norm r_c of what the basis leaves
// out.  A patch's data event m (block sums of its known overlap cells) is
// encoded as q = P m, a = mu . m and |m|.
//
// Since m . x_c = a + q . e_c + m . (x_c - mu - P^T e_c), the squared-
// difference score S(c) = E(c) - 2|beta| m . x_c is bounded from below by
//   E(c) - 2|beta| (a + q . e_c) - 2|beta| |m| r_c  (minus a rounding margin).
// The proxy scan writes, per patch and candidate row, the smallest such
// bound (with the exact hard-data mismatch); the selection then computes
// exact keys row by row in order of these bounds until the K best exact
// keys lie below every bound left, so the result equals the full scan's.
// The basis only decides how many rows that takes.
#pragma once

#include "dev_kernels.h"
#include "dev_scan.h"

namespace ccw {

constexpr int kPcaParts = 64;       // workgroups of the moments pass
constexpr int kPcaMaxCells = 192;   // template blocks the proposer supports
constexpr int kPcaMaxDim = 32;
constexpr int kPcaIters = 12;       // subspace iterations (any count is exact downstream)
constexpr int kPcaBatch = 16;       // candidates staged per moments round

// Offset of template block beta from a candidate's corner in the level-J
// grid (x fastest over the footprint), one entry per block.
__device__ __forceinline__ void pca_window_offsets(const Geom& g, int* s_off) {
  for (int beta = threadIdx.x; beta < (int)g.tcells; beta += kThreads) {
    int bx, by, bz;
    split3(beta, g.tc[0], g.tc[1], bx, by, bz);
    s_off[beta] = idx3i(bx, by, bz, g.G);
  }
}

// Partial sums of x and x x^T over part b's share of the candidates (fp32;
// thread t owns matrix entries t, t + 256, ...).
template <int R>   // R = ceil(n^2 / 256) entries per thread
__global__ __launch_bounds__(kThreads) void k_pca_moments(const int32_t* __restrict__ K, Geom g,
                                                          float* __restrict__ part) {
  __shared__ float s_x[kPcaBatch][kPcaMaxCells];
  __shared__ int s_off[kPcaMaxCells];
  const int n = (int)g.tcells, nn = n * n;
  pca_window_offsets(g, s_off);
  const int nc = (int)g.ncand;
  const int per = (nc + gridDim.x - 1) / gridDim.x;
  const int c0 = blockIdx.x * per, c1 = min(nc, c0 + per);
  float acc[R];
  float sx = 0.f;
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.f;
  for (int cb = c0; cb < c1; cb += kPcaBatch) {
    const int nb = min(kPcaBatch, c1 - cb);
    __syncthreads();
    for (int i = threadIdx.x; i < kPcaBatch * n; i += kThreads) {
      const int q = i / n, beta = i - q * n;
      float v = 0.f;
      if (q < nb) {
        int cx, cy, cz;
        split3(cb + q, g.cand[0], g.cand[1], cx, cy, cz);
        v = (float)K[idx3i(cx, cy, cz, g.G) + s_off[beta]];
      }
      s_x[q][beta] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = threadIdx.x + r * kThreads;
      if (e < nn) {
        const int i = e / n, j = e - i * n;
        float s = 0.f;
        for (int q = 0; q < nb; ++q) s += s_x[q][i] * s_x[q][j];
        acc[r] += s;
      }
    }
    if (threadIdx.x < n)
      for (int q = 0; q < nb; ++q) sx += s_x[q][threadIdx.x];
  }
  float* out = part + (long long)blockIdx.x * (nn + n);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = threadIdx.x + r * kThreads;
    if (e < nn) out[e] = acc[r];
  }
  if (threadIdx.x < n) out[nn + threadIdx.x] = sx;
}

// Covariance from the parts (fixed summation order): cov[i][j], mu[i].
__global__ void k_pca_reduce(const float* __restrict__ part, int nparts, Geom g, float* __restrict__ cov,
                             float* __restrict__ mu) {
  const int n = (int)g.tcells, nn = n * n;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn + n) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += (double)part[(long long)b * (nn + n) + e];
  const double N = (double)g.ncand;
  if (e >= nn) {
    mu[e - nn] = (float)(s / N);
    return;
  }
  // mean of x_i x_j; the centring needs mu, done by the fit
  cov[e] = (float)(s / N);
}

// Top-D subspace of the covariance by subspace iteration (one workgroup).
// Output: P [D][n] with orthonormal rows.
__global__ __launch_bounds__(kThreads) void k_pca_fit(const float* __restrict__ exx, const float* __restrict__ mu_g,
                                                      Geom g, int D, float* __restrict__ P) {
  __shared__ float s_X[kPcaMaxCells * kPcaMaxDim];
  __shared__ float s_Y[kPcaMaxCells * kPcaMaxDim];
  __shared__ float s_mu[kPcaMaxCells];
  __shared__ float s_red[kThreads / 64];
  const int n = (int)g.tcells;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n; i += kThreads) s_mu[i] = mu_g[i];
  // deterministic start: columns of a fixed pseudo-random matrix
  for (int e = tid; e < n * D; e += kThreads) {
    const uint64_t h = mix64((uint64_t)e * 0x9E3779B97F4A7C15ull + 12345u);
    s_X[e] = (float)((int)(h & 0xFFFF) - 32768) / 32768.f;
  }
  __syncthreads();
  auto block_sum = [&](float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) s_red[wave] = v;
    __syncthreads();
    float t = 0.f;
    for (int w = 0; w < kThreads / 64; ++w) t += s_red[w];
    __syncthreads();
    return t;
  };
  for (int it = 0; it <= kPcaIters; ++it) {
    // orthonormalise the columns of X (modified Gram-Schmidt)
    for (int d = 0; d < D; ++d) {
      for (int e = 0; e < d; ++e) {
        float pv = 0.f;
        for (int i = tid; i < n; i += kThreads) pv += s_X[i * D + d] * s_X[i * D + e];
        const float dot = block_sum(pv);
        for (int i = tid; i < n; i += kThreads) s_X[i * D + d] -= dot * s_X[i * D + e];
        __syncthreads();
      }
      float pv = 0.f;
      for (int i = tid; i < n; i += kThreads) pv += s_X[i * D + d] * s_X[i * D + d];
      const float nrm = sqrtf(block_sum(pv));
      const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
      for (int i = tid; i < n; i += kThreads) s_X[i * D + d] *= inv;
      __syncthreads();
    }
    if (it == kPcaIters) break;
    // Y = C X with C = E[x x^T] - mu mu^T
    for (int e = tid; e < n * D; e += kThreads) {
      const int i = e / D, d = e - i * D;
      float s = 0.f, mx = 0.f;
      for (int j = 0; j < n; ++j) {
        s += exx[i * n + j] * s_X[j * D + d];
        mx += s_mu[j] * s_X[j * D + d];
      }
      s_Y[e] = s - s_mu[i] * mx;
    }
    __syncthreads();
    for (int e = tid; e < n * D; e += kThreads) s_X[e] = s_Y[e];
    __syncthreads();
  }
  for (int e = tid; e < n * D; e += kThreads) {
    const int i = e / D, d = e - i * D;
    P[d * n + i] = s_X[e];
  }
}

// Test hook: row d >= 1 of the basis gets s times row 0 added and row 0 is
// scaled by 1 + s, so the rows are neither orthogonal nor of unit length
// (the bound must not depend on either).
__global__ void k_pca_skew(float* __restrict__ P, int D, int n, float s) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const float p0 = P[b];
  for (int d = 1; d < D; ++d) P[d * n + b] += s * p0;
  P[b] = p0 * (1.f + s);
}

// Embedding e_c = P (x_c - mu), residual bound r_c and |e_c| per candidate.
__global__ __launch_bounds__(kThreads) void k_pca_embed(const int32_t* __restrict__ K, Geom g, int D,
                                                        const float* __restrict__ mu_g, const float* __restrict__ P_g,
                                                        float* __restrict__ emb, float2* __restrict__ rn) {
  __shared__ float s_P[kPcaMaxDim * kPcaMaxCells];
  __shared__ float s_mu[kPcaMaxCells];
  __shared__ int s_off[kPcaMaxCells];
  const int n = (int)g.tcells;
  for (int i = threadIdx.x; i < D * n; i += kThreads) s_P[i] = P_g[i];
  for (int i = threadIdx.x; i < n; i += kThreads) s_mu[i] = mu_g[i];
  pca_window_offsets(g, s_off);
  __syncthreads();
  const int c = min((int)(blockIdx.x * kThreads + threadIdx.x), (int)g.ncand - 1);
  int cx, cy, cz;
  split3(c, g.cand[0], g.cand[1], cx, cy, cz);
  const int32_t* Kc = K + idx3i(cx, cy, cz, g.G);
  float e[kPcaMaxDim];
#pragma unroll
  for (int d = 0; d < kPcaMaxDim; ++d) e[d] = 0.f;
  float xx = 0.f;
  for (int b0 = 0; b0 < n; b0 += 8) {   // eight reads in flight per round
    int xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = Kc[s_off[min(b0 + q, n - 1)]];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (b0 + q >= n) break;
      const float xb = (float)xv[q] - s_mu[b0 + q];
      xx += xb * xb;
#pragma unroll
      for (int d = 0; d < kPcaMaxDim; ++d)
        if (d < D) e[d] += s_P[d * n + b0 + q] * xb;
    }
  }
  (void)xx;
  // The residual r = x - mu - P^T e of the stored (fp32) e, computed
  // directly in fp64, so that m . x = mu . m + (P m) . e + m . r holds for
  // any basis P, orthonormal or not.  Every product below (fp32 by fp32 or
  // by an integer) is exact in fp64; each sum of at most D + 2 terms is off
  // by under (D + 2) 2^-53 of its absolute terms (< 1e-14 relative); the
  // norm is then rounded up to the next fp32 value above it, plus a 1e-9
  // relative margin that dominates those errors by five orders of magnitude.
  double rr = 0.0;
  for (int b = 0; b < n; ++b) {
    double rb = (double)Kc[s_off[b]] - (double)s_mu[b];
#pragma unroll
    for (int d = 0; d < kPcaMaxDim; ++d)
      if (d < D) rb -= (double)s_P[d * n + b] * (double)e[d];
    rr += rb * rb;
  }
  if ((int)(blockIdx.x * kThreads + threadIdx.x) >= (int)g.ncand) return;
  float ee = 0.f;
#pragma unroll
  for (int d = 0; d < kPcaMaxDim; ++d)
    if (d < D) {
      ee += e[d] * e[d];
      emb[(long long)c * D + d] = e[d];
    }
  const double rd = sqrt(rr) * (1.0 + 1e-9);
  float rf = (float)rd;
  if ((double)rf < rd) rf = nextafterf(rf, INFINITY);
  rn[c] = make_float2(rf, sqrtf(ee));
}

// Query of one data event (block sums m over the template blocks, in LDS):
// out = [q = P m (D), a = mu . m, |m|, unused], in fp64 (products of fp32
// values and integers are exact; the sums' rounding is covered by the
// proxy's margin).  Called by a whole workgroup.
__device__ __forceinline__ void pca_query(const int* s_m, int n, int D, const float* __restrict__ P_g,
                                          const float* __restrict__ mu_g, double* __restrict__ out) {
  const int tid = threadIdx.x;
  if (tid < D) {
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += (double)P_g[tid * n + b] * (double)s_m[b];
    out[tid] = s;
  } else if (tid == D) {
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += (double)mu_g[b] * (double)s_m[b];
    out[D] = s;
  } else if (tid == D + 1) {
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += (double)s_m[b] * (double)s_m[b];
    out[D + 1] = sqrt(s) * (1.0 + 1e-15);
  }
}

struct ProxyArgs {
  Geom g;
  const TileDev* tiles;        // tiles of this step
  const ScanRec* recs;         // [tile][kFiltersPerTile]
  const double* qbuf;          // [patch][D + 4]
  const float* emb;            // [candidate][D]
  const float2* rn;            // [candidate] (residual bound, |e|)
  const int32_t* energy;       // [shape][ncand]
  const HdEnt* hd_ent;
  const int8_t* ti;
  uint64_t* rowmin;            // [slot][candidate rows]
  int fbegin;
  int D;
  int has_hd;
};

// Lower bounds of every candidate of one candidate row against one tile of
// patches; only each patch's smallest bound key per row is written.  A
// patch without overlap (the first of a realization) has S = 0 exactly, so
// its keys are exact (with the tie-break) instead of bounds.
__global__ __launch_bounds__(kThreads) void k_proxy(ProxyArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom& g = a.g;
  const int D = a.D;
  const int tid = threadIdx.x, j = tid & 31, grp = tid >> 5;   // 8 groups of 32 patch lanes
  const int row = blockIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int C0 = g.cand[0];
  const TileDev t = a.tiles[blockIdx.y];
  const ScanRec rec = a.recs[blockIdx.y * kFiltersPerTile + j];
  float* s_emb = (float*)smem;                       // [C0][D]
  float2* s_rn = (float2*)(s_emb + C0 * D);          // [C0]
  __shared__ unsigned long long s_min[kFiltersPerTile];
  if (tid < kFiltersPerTile) s_min[tid] = ~0ull;
  const long long rowbase = (long long)C0 * row;
  for (int i = tid; i < C0 * D; i += kThreads) s_emb[i] = a.emb[rowbase * D + i];
  for (int i = tid; i < C0; i += kThreads) s_rn[i] = a.rn[rowbase + i];
  const bool fvalid = rec.gidx >= 0;
  const bool exact = fvalid && ((t.zmask >> j) & 1u);   // no overlap: S = 0 for every candidate
  double q[kPcaMaxDim];
  double qa = 0.0, qm = 0.0;
  if (fvalid) {
    const double* qb = a.qbuf + (long long)(a.fbegin + t.first + j) * (D + 4);
#pragma unroll
    for (int d = 0; d < kPcaMaxDim; ++d) q[d] = d < D ? qb[d] : 0.0;
    qa = qb[D];
    qm = qb[D + 1];
  }
  const int32_t* erow = a.energy + (long long)rec.shape * g.ncand + rowbase;
  const int two_beta = 2 * g.beta;
  const int J = g.level, Jz = g.ndim == 3 ? J : 0;
  __syncthreads();
  uint64_t best = ~0ull;
  if (fvalid) {
    for (int cx = grp; cx < C0; cx += kThreads / 32) {
      // hard-data mismatch of this candidate, exact
      unsigned mis = 0;
      for (int h = 0; h < rec.nhd; ++h) {
        const HdEnt e = a.hd_ent[rec.hd0 + h];
        const int fx = (cx << J) + e.u[0], fy = (cy << J) + e.u[1], fz = (cz << Jz) + e.u[2];
        if (fx >= 0 && fy >= 0 && fz >= 0 && fx < g.ti[0] && fy < g.ti[1] && fz < g.ti[2])
          mis += a.ti[(fz * g.ti[1] + fy) * g.ti[0] + fx] != e.v ? 1u : 0u;
      }
      uint64_t key;
      if (exact) {
        key = make_key(mis, 0, tie_perm((uint32_t)(rowbase + cx), rec.tkey));
      } else {
        // m . x = a + q . e + m . r <= a + q . e + |m| |r| (Cauchy-Schwarz),
        // in fp64 with a 1e-9 margin over the absolute terms (the sums'
        // rounding is under 1e-14 of them)
        double dot = 0.0, dabs = 0.0;
#pragma unroll
        for (int d = 0; d < kPcaMaxDim; ++d)
          if (d < D) {
            const double t = q[d] * (double)s_emb[cx * D + d];
            dot += t;
            dabs += fabs(t);
          }
        const double mr = qm * (double)s_rn[cx].x;
        const double lin = qa + dot + mr;
        const double slack = 1e-9 * (fabs(qa) + dabs + mr) + 1e-9;
        const double lb = (double)erow[cx] - (double)two_beta * (lin + slack);
        const int lbi = lb <= -2147483648.0 ? (int)0x80000000 : lb >= 2147483647.0 ? 0x7FFFFFFF : (int)floor(lb);
        key = make_key(mis, lbi, 0);
      }
      best = key < best ? key : best;
    }
  }
  if (fvalid) atomicMin(&s_min[j], (unsigned long long)best);
  __syncthreads();
  if (tid < t.count) a.rowmin[(long long)(t.first + tid) * (g.cand[1] * g.cand[2]) + row] = s_min[tid];
}

}  // namespace ccw
