// ccwsim.hip -- CCWSIM hot path on MI355X: C ABI, simulation plan and the
// per-step kernels (data-event extraction, selection + reconstruction + cut +
// paste).  The scan itself is in dev_scan.h, the transform and top-K
// building blocks in dev_kernels.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "ccwsim.h"
#include "dev_scan.h"
#include "dev_learn.h"
#include "dev_lp.h"
#include "dev_stats.h"
#include "dev_cdf97.h"

using namespace ccw;

constexpr int kSeamRowsMax = 64;   // longest seam of the register dynamic programme
constexpr int kMaxSucc = 64;       // overlapping successors of one patch
constexpr int kFinInline = 64;     // patch records passed by value to a finalize launch

// ===========================================================================
// errors
// ===========================================================================
namespace {
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(x)                                                                 \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) return fail(CCWSIM_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

#define CCW_TRY(x)        \
  do {                    \
    int s_ = (x);         \
    if (s_) return s_;    \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline unsigned nblocks(long long n, int per = kThreads) { return (unsigned)((n + per - 1) / per); }
inline long long align256(long long x) { return (x + 255) & ~255ll; }

// ===========================================================================
// geometry
// ===========================================================================
int geom_ti(Geom& g, const ccwsim_shape& s, int level) {
  memset(&g, 0, sizeof g);
  if (s.ndim < 2 || s.ndim > 3) return fail(CCWSIM_ERR_SHAPE, "ndim must be 2 or 3 (got %d)", s.ndim);
  if (level < 0 || level > kMaxLevel) return fail(CCWSIM_ERR_SHAPE, "level must be in [0, %d]", kMaxLevel);
  g.ndim = s.ndim;
  g.level = level;
  for (int a = 0; a < 3; ++a) {
    const bool used = a < s.ndim;
    const int n = s.n[a];
    if (!used && n != 1) return fail(CCWSIM_ERR_SHAPE, "extent of unused axis %d must be 1", a);
    if (n < 1) return fail(CCWSIM_ERR_SHAPE, "extent %d on axis %d", n, a);
    g.ti[a] = n;
    g.b[a] = used ? (1 << level) : 1;
    g.np[a] = (n + g.b[a] - 1) / g.b[a] * g.b[a];
    g.G[a] = g.np[a] / g.b[a];
  }
  // kernels index the (padded) TI and its grids with 32-bit offsets
  if ((long long)g.np[0] * g.np[1] * g.np[2] > 0x7FFFFFFFll)
    return fail(CCWSIM_ERR_SHAPE, "padded TI exceeds 2^31 - 1 cells");
  g.beta = g.b[0] * g.b[1] * g.b[2];
  g.log2beta = level * s.ndim;
  g.shift = g.log2beta + 1;
  for (int j = 0; j <= level; ++j)
    for (int a = 0; a < 3; ++a) g.Gj[j][a] = a < s.ndim ? (g.np[a] >> j) : 1;
  g.det_off[1] = 0;
  for (int j = 1; j <= level; ++j) {
    const long long cells = (long long)g.Gj[j][0] * g.Gj[j][1] * g.Gj[j][2];
    g.det_off[j + 1] = g.det_off[j] + (long long)((1 << s.ndim) - 1) * cells;
  }
  g.det_total = level > 0 ? g.det_off[level + 1] : 0;
  return CCWSIM_OK;
}

int geom_tmpl(Geom& g, const int32_t T[3]) {
  long long nc = 1;
  for (int a = 0; a < 3; ++a) {
    const bool used = a < g.ndim;
    const int t = used ? T[a] : 1;
    if (used && (t < 1 || t > g.ti[a]))
      return fail(CCWSIM_ERR_SHAPE, "template %d on axis %d must be in [1, TI extent %d]", t, a, g.ti[a]);
    g.T[a] = t;
    g.tc[a] = (t + g.b[a] - 1) / g.b[a];
    g.cand[a] = (g.ti[a] - t) / g.b[a] + 1;
    nc *= g.cand[a];
  }
  if (nc > (1 << 20)) return fail(CCWSIM_ERR_UNSUPPORTED, "%lld candidates exceed 2^20", nc);
  g.ncand = (int)nc;
  g.tcells = (long long)g.tc[0] * g.tc[1] * g.tc[2];
  g.wcells = (long long)g.T[0] * g.T[1] * g.T[2];
  return CCWSIM_OK;
}

int geom_grid(Geom& g, const ccwsim_shape& grid, const int32_t OV[3], const int32_t margin[3]) {
  if (grid.ndim != g.ndim) return fail(CCWSIM_ERR_SHAPE, "grid and TI must have the same ndim");
  for (int a = 0; a < 3; ++a) {
    const bool used = a < g.ndim;
    const int n = grid.n[a];
    if (!used && n != 1) return fail(CCWSIM_ERR_SHAPE, "grid extent of unused axis %d must be 1", a);
    if (n < 1) return fail(CCWSIM_ERR_SHAPE, "grid extent %d on axis %d", n, a);
    g.sg[a] = n;
    g.OV[a] = used ? OV[a] : 0;
    if (used && !(g.T[a] > g.OV[a] && g.OV[a] >= 1))
      return fail(CCWSIM_ERR_SHAPE, "need T > OV >= 1 on axis %d (T=%d, OV=%d)", a, g.T[a], g.OV[a]);
    g.margin[a] = used ? (margin[a] < 0 ? OV[a] : margin[a]) : 0;
    if (g.margin[a] > 4096) return fail(CCWSIM_ERR_SHAPE, "margin too large");
    g.stride[a] = used ? g.T[a] - g.OV[a] : 1;
    const int l = used ? (n - g.OV[a] + g.stride[a] - 1) / g.stride[a] : 1;
    g.lat[a] = l < 1 ? 1 : l;
    g.pad[a] = used ? g.lat[a] * g.stride[a] + g.OV[a] : 1;
  }
  g.pcells = (long long)g.pad[0] * g.pad[1] * g.pad[2];
  // kernels address a realization's padded grid with 32-bit offsets
  if (g.pcells > 0x7FFFFFFFll) return fail(CCWSIM_ERR_SHAPE, "padded grid of %lld cells exceeds 2^31 - 1", g.pcells);
  return CCWSIM_OK;
}

// Bounds under which fp16 inputs and fp32 accumulation are exact and the
// int32 score cannot overflow.  maxc = largest code, ovcells = largest number
// of known overlap cells of a data event.
long long floor_div(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

int check_exact(const Geom& g, long long maxc, long long ovcells) {
  const long long kmax = maxc * g.beta;
  if (kmax > 2048) return fail(CCWSIM_ERR_UNSUPPORTED, "block sums up to %lld are not exact in fp16", kmax);
  const long long cmax = maxc * maxc * g.beta * ovcells;  // bound on any partial cross sum
  if (cmax >= (1ll << 24))
    return fail(CCWSIM_ERR_UNSUPPORTED, "cross sums up to %lld are not exact in fp32", cmax);
  const long long smax = 3ll * ovcells * kmax * kmax;
  if (smax >= (1ll << 31)) return fail(CCWSIM_ERR_UNSUPPORTED, "scores up to %lld overflow int32", smax);
  return CCWSIM_OK;
}

// Groups per lane of the fused-selection scan: the fewest (2^gbits) that give
// every patch at least ksel groups holding a candidate (each such group's
// minimum is a distinct candidate, so the ksel-th smallest bounds the
// ksel-th best).  Lane (wave w, half h) holds, for value v of chunk ch (ch = w
// mod 4), candidate 32 ch + 8 (v / 4) + 4 h + v % 4; its group is v mod 2^gbits.
int sel_group_bits(int C0, int nchunks, int ksel) {
  const int nwv = std::min(kThreads / 64, nchunks);
  for (int gb = 0; gb <= 4; ++gb) {
    const int NG = 1 << gb;
    int valid = 0;
    for (int w = 0; w < nwv; ++w)
      for (int hh = 0; hh < 2; ++hh)
        for (int gi = 0; gi < NG; ++gi) {
          bool any = false;
          for (int ch = w; ch < nchunks && !any; ch += kThreads / 64)
            for (int v = gi; v < 16 && !any; v += NG) any = ch * 32 + 8 * (v >> 2) + 4 * hh + (v & 3) < C0;
          valid += any ? 1 : 0;
        }
    if (valid >= ksel) return gb;
  }
  return 4;   // fewer candidates than ksel in a row: every candidate survives
}

__global__ void k_fill_f32(float* __restrict__ p, long long n, float v) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = v;
}

// ---- launch profiler (events around each kernel launch) -------------------
struct ProfRec {
  int kind;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_scan_g_force = 0;   // 0: tuned choice; else tiles per scan workgroup (testing)
float g_pca_skew = 0.f;    // test hook: rows of the certified proposer's basis skewed (not orthonormal)
int g_sel_force = 0;      // 0: tuned choice; 1: stored keys; 2: row minima + exact rescoring
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Scope object: records an event before and after the launches in its scope.
struct ProfScope {
  hipStream_t st;
  int kind;
  hipEvent_t a = nullptr;
  ProfScope(int k, hipStream_t s) : st(s), kind(k) {
    if (!g_prof_on || k < 0) return;
    a = prof_event();
    if (a) (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event();
    if (!b) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_recs.push_back({kind, a, b});
  }
};

// Events for one kernel launch, recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so the interval is the kernel's own run and not
// the gaps around it; both null when profiling is off.
struct ProfKernel {
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  explicit ProfKernel(int k) : kind(k) {
    if (!g_prof_on || k < 0) return;
    a = prof_event();
    b = a ? prof_event() : nullptr;
    if (!b && a) {
      g_prof_pool.push_back(a);
      a = nullptr;
    }
  }
  ~ProfKernel() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_recs.push_back({kind, a, b});
  }
};

}  // namespace

// ===========================================================================
// status
// ===========================================================================
extern "C" const char* ccwsim_status_string(int status) {
  switch (status) {
    case CCWSIM_OK: return "ok";
    case CCWSIM_ERR_INVALID_ARG: return "invalid argument";
    case CCWSIM_ERR_SHAPE: return "invalid shape";
    case CCWSIM_ERR_WORKSPACE: return "workspace missing or too small";
    case CCWSIM_ERR_HIP: return "HIP runtime error";
    case CCWSIM_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

extern "C" const char* ccwsim_last_error(void) { return g_err.c_str(); }

// ===========================================================================
// A1: DWT
// ===========================================================================
namespace {

// Runs the J level kernels.  tmp must hold 2 * |level-1 grid| int32 when J >= 2.
int launch_dwt(const Geom& g, const int8_t* x, int32_t* approx, _Float16* approx_h, int32_t* det,
               int32_t* tmp, hipStream_t st) {
  const int J = g.level;
  if (J == 0) {
    const long long cells = (long long)g.ti[0] * g.ti[1] * g.ti[2];
    k_level0<<<nblocks(cells), kThreads, 0, st>>>(x, approx, approx_h, cells);
    HIP_TRY(hipGetLastError());
    return CCWSIM_OK;
  }
  const long long c1 = (long long)g.Gj[1][0] * g.Gj[1][1] * g.Gj[1][2];
  for (int j = 1; j <= J; ++j) {
    const long long cells = (long long)g.Gj[j][0] * g.Gj[j][1] * g.Gj[j][2];
    const int32_t* src = j >= 2 ? tmp + ((j - 1) & 1) * c1 : nullptr;
    int32_t* dst = j == J ? approx : tmp + (j & 1) * c1;
    _Float16* dh = j == J ? approx_h : nullptr;
    if (g.ndim == 2)
      k_dwt_level<2><<<nblocks(cells), kThreads, 0, st>>>(x, src, dst, dh, det, g, j);
    else
      k_dwt_level<3><<<nblocks(cells), kThreads, 0, st>>>(x, src, dst, dh, det, g, j);
    HIP_TRY(hipGetLastError());
  }
  return CCWSIM_OK;
}

}  // namespace

// ---- LeGall 5/3 transform with every sub-band (Sec. 4.2: the mother
// wavelet is a choice).  Integer lifting on even-length lines with
// whole-sample symmetric extension: d[k] = x[2k+1] - floor((x[2k] +
// x[2k+2]) / 2), s[k] = x[2k] + floor((d[k-1] + d[k] + 2) / 4), with the
// mirrored x[n] = x[n-2] and d[-1] = d[0].  Per level the lines run along
// x, then y, then z.  Bands live stacked in one buffer ([band][z][y][x]); a
// pass along axis a turns bands q < 2^a into q (low half) and q + 2^a (high
// half), so after the level's last pass band q has bit a set when axis a
// took the high-pass, the layout of the detail sub-bands.
namespace {

// The TI edge-replicated to the padded extent, int32.
__global__ void k_pad_ti(const int8_t* __restrict__ ti, int32_t* __restrict__ out, Geom g) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)g.np[0] * g.np[1] * g.np[2];
  if (id >= n) return;
  const int x = (int)(id % g.np[0]), y = (int)((id / g.np[0]) % g.np[1]), z = (int)(id / ((long long)g.np[0] * g.np[1]));
  out[id] = ti[idx3(min(x, g.ti[0] - 1), min(y, g.ti[1] - 1), min(z, g.ti[2] - 1), g.ti)];
}

// One forward pass along `axis` over nb stacked bands of extent e; one
// thread per output position (k, and the other coordinates) of one band.
__global__ void k_lift53_fwd(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int e0, int e1, int e2,
                             int axis, int nb) {
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
  const long long full = (long long)e0 * e1 * e2;
  const int32_t* line = src + q * full;
  const long long st = axis == 0 ? 1 : axis == 1 ? e0 : (long long)e0 * e1;
  u[axis] = 0;
  const long long base = u[0] + (long long)e0 * (u[1] + (long long)e1 * u[2]);
  auto X = [&](int i) {   // mirrored sample
    i = i < 0 ? -i : i;
    i = i >= n ? 2 * (n - 1) - i : i;
    return line[base + st * i];
  };
  const int x0 = X(2 * k), x1 = X(2 * k + 1), x2 = X(2 * k + 2);
  const int dk = x1 - ((x0 + x2) >> 1);
  const int dl = k == 0 ? dk : X(2 * k - 1) - ((X(2 * k - 2) + x0) >> 1);
  const int sk = x0 + ((dl + dk + 2) >> 2);
  u[axis] = k;
  const long long o = u[0] + (long long)eo[0] * (u[1] + (long long)eo[1] * u[2]);
  dst[q * half + o] = sk;
  dst[(q + nb) * half + o] = dk;
}

// One inverse pass along `axis`: bands q and q + nb (extent with axis
// halved) of src become band q of dst (extent eo); one thread per output
// pair x[2k], x[2k+1].
__global__ void k_lift53_inv(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int eo0, int eo1, int eo2,
                             int axis, int nb) {
  int ei[3] = {eo0, eo1, eo2};
  ei[axis] >>= 1;
  const long long half = (long long)ei[0] * ei[1] * ei[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= half * nb) return;
  const int q = (int)(id / half);
  const long long r = id - q * half;
  int u[3] = {(int)(r % ei[0]), (int)((r / ei[0]) % ei[1]), (int)(r / ((long long)ei[0] * ei[1]))};
  const int k = u[axis], h = ei[axis];
  const long long st = axis == 0 ? 1 : axis == 1 ? ei[0] : (long long)ei[0] * ei[1];
  u[axis] = 0;
  const long long base = u[0] + (long long)ei[0] * (u[1] + (long long)ei[1] * u[2]);
  const int32_t* S = src + q * half + base;
  const int32_t* D = src + (q + nb) * half + base;
  const int dk = D[st * k];
  const int dl = k == 0 ? dk : D[st * (k - 1)];
  const int xe = S[st * k] - ((dl + dk + 2) >> 2);
  int xn = xe;   // x[2k + 2], mirrored to x[2k] past the end
  if (k + 1 < h) xn = S[st * (k + 1)] - ((dk + D[st * (k + 1)] + 2) >> 2);
  const int xo = dk + ((xe + xn) >> 1);
  const long long so = axis == 0 ? 1 : axis == 1 ? eo0 : (long long)eo0 * eo1;
  u[axis] = 2 * k;
  const long long o = u[0] + (long long)eo0 * (u[1] + (long long)eo1 * u[2]);
  dst[q * (half * 2) + o] = xe;
  dst[q * (half * 2) + o + so] = xo;
}

// Workspace of the 5/3 transforms: three buffers of the padded TI (int32).
long long lift53_ws_bytes(const Geom& g) { return 3 * align256((long long)g.np[0] * g.np[1] * g.np[2] * 4); }

// Level-J 5/3 DWT of the TI into approx and the detail layout of the Haar
// path.
int launch_dwt53(const Geom& g, const int8_t* x, int32_t* approx, int32_t* details, unsigned char* ws, hipStream_t st) {
  const long long npc = (long long)g.np[0] * g.np[1] * g.np[2];
  int32_t* C = (int32_t*)ws;
  int32_t* A = (int32_t*)(ws + align256(npc * 4));
  int32_t* B = (int32_t*)(ws + 2 * align256(npc * 4));
  k_pad_ti<<<nblocks(npc), kThreads, 0, st>>>(x, C, g);
  int e[3] = {g.np[0], g.np[1], g.np[2]};
  const int nd = g.ndim;
  if (g.level == 0) {
    HIP_TRY(hipMemcpyAsync(approx, C, npc * 4, hipMemcpyDeviceToDevice, st));
    return CCWSIM_OK;
  }
  for (int j = 1; j <= g.level; ++j) {
    const int32_t* src = C;
    int32_t* bufs[2] = {A, B};
    int32_t* dst = nullptr;
    for (int a = 0; a < nd; ++a) {
      dst = bufs[a & 1];
      const long long outc = (long long)e[0] * e[1] * e[2] / 2 * (1 << a);
      k_lift53_fwd<<<nblocks(outc), kThreads, 0, st>>>(src, dst, e[0], e[1], e[2], a, 1 << a);
      e[a] >>= 1;
      src = dst;
    }
    const long long band = (long long)e[0] * e[1] * e[2];
    HIP_TRY(hipMemcpyAsync(details + g.det_off[j], dst + band, band * ((1 << nd) - 1) * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(j == g.level ? approx : C, dst, band * 4, hipMemcpyDeviceToDevice, st));
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// Full-image 5/3 inverse from approx and details into the workspace's first
// buffer (the padded TI), then the patterns as crops of it.
__global__ void k_crop_patterns(const int32_t* __restrict__ img, Geom g, const int32_t* __restrict__ origins,
                                int n, int8_t* __restrict__ out) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n * g.wcells) return;
  const int p = (int)(id / g.wcells);
  const int u = (int)(id - (long long)p * g.wcells);
  const int c0[3] = {origins[3 * p], origins[3 * p + 1], origins[3 * p + 2]};
  bool ok = true;
  for (int d = 0; d < 3; ++d) ok = ok && c0[d] >= 0 && c0[d] + g.tc[d] <= g.G[d];
  if (!ok) {
    out[id] = -1;
    return;
  }
  const int ux = u % g.T[0], uy = (u / g.T[0]) % g.T[1], uz = u / (g.T[0] * g.T[1]);
  out[id] = (int8_t)img[idx3(c0[0] * g.b[0] + ux, c0[1] * g.b[1] + uy, c0[2] * g.b[2] + uz, g.np)];
}

int launch_idwt53(const Geom& g, const int32_t* approx, const int32_t* details, unsigned char* ws, hipStream_t st) {
  const long long npc = (long long)g.np[0] * g.np[1] * g.np[2];
  int32_t* C = (int32_t*)ws;
  int32_t* A = (int32_t*)(ws + align256(npc * 4));
  int32_t* B = (int32_t*)(ws + 2 * align256(npc * 4));
  const int nd = g.ndim;
  int e[3] = {g.G[0], g.G[1], g.G[2]};
  if (g.level == 0) {
    HIP_TRY(hipMemcpyAsync(C, approx, npc * 4, hipMemcpyDeviceToDevice, st));
    return CCWSIM_OK;
  }
  const int32_t* cur = approx;
  for (int j = g.level; j >= 1; --j) {
    const long long band = (long long)e[0] * e[1] * e[2];
    int32_t* bufs[2] = {A, B};
    // stack the bands: the approximation of level j, then the details
    HIP_TRY(hipMemcpyAsync(A, cur, band * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(A + band, details + g.det_off[j], band * ((1 << nd) - 1) * 4, hipMemcpyDeviceToDevice, st));
    const int32_t* src = A;
    int32_t* dst = nullptr;
    for (int a = nd - 1, i = 1; a >= 0; --a, ++i) {
      dst = (a == 0) ? C : bufs[i & 1];
      e[a] <<= 1;
      const long long pairs = (long long)e[0] * e[1] * e[2] / 2 * (1 << a);
      k_lift53_inv<<<nblocks(pairs), kThreads, 0, st>>>(src, dst, e[0], e[1], e[2], a, 1 << a);
      src = dst;
    }
    cur = C;
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

}  // namespace

extern "C" int ccwsim_dwt_sizes(ccwsim_shape s, int32_t level, int32_t wavelet, int64_t* n_approx, int64_t* n_details,
                                int64_t* workspace_bytes) {
  Geom g;
  CCW_TRY(geom_ti(g, s, level));
  if (wavelet != 0 && wavelet != 1) return fail(CCWSIM_ERR_INVALID_ARG, "wavelet must be 0 (Haar) or 1 (LeGall 5/3)");
  if (n_approx) *n_approx = (int64_t)g.G[0] * g.G[1] * g.G[2];
  if (n_details) *n_details = g.det_total;
  if (workspace_bytes) {
    const long long c1 = level >= 2 ? (long long)g.Gj[1][0] * g.Gj[1][1] * g.Gj[1][2] : 0;
    *workspace_bytes = wavelet == 1 ? lift53_ws_bytes(g) : align256(2 * c1 * 4);
  }
  return CCWSIM_OK;
}

extern "C" int ccwsim_dwt(const int8_t* x, ccwsim_shape s, int32_t level, int32_t wavelet, int32_t* approx,
                          int32_t* details, void* workspace, int64_t workspace_bytes, void* stream) {
  Geom g;
  CCW_TRY(geom_ti(g, s, level));
  if (wavelet != 0 && wavelet != 1) return fail(CCWSIM_ERR_INVALID_ARG, "wavelet must be 0 (Haar) or 1 (LeGall 5/3)");
  if (!x || !approx || (level > 0 && !details)) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  int64_t need = 0;
  CCW_TRY(ccwsim_dwt_sizes(s, level, wavelet, nullptr, nullptr, &need));
  if (need > 0 && (!workspace || workspace_bytes < need))
    return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", (long long)need);
  if (need > 0 && ((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  if (wavelet == 1) return launch_dwt53(g, x, approx, details, (unsigned char*)workspace, st);
  return launch_dwt(g, x, approx, nullptr, details, level >= 2 ? (int32_t*)workspace : nullptr, st);
}

// ===========================================================================
// A3: standalone scan
// ===========================================================================
namespace {

__global__ void k_to_half(const int32_t* __restrict__ src, _Float16* __restrict__ dst, long long n) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) dst[id] = (_Float16)(float)src[id];
}

__global__ void k_to_bf16(const int32_t* __restrict__ src, __bf16* __restrict__ dst, long long n) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) dst[id] = (__bf16)(float)src[id];
}

// Standalone data events: or_m[f][beta] -> mbuf[f][k = beta], zero pad.
__global__ void k_events_to_mbuf(const int32_t* __restrict__ or_m, int32_t* __restrict__ mbuf,
                                 int n_filters, long long tcells) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n_filters * kKMax) return;
  const long long f = id / kKMax, k = id - f * kKMax;
  mbuf[id] = k < tcells ? or_m[f * tcells + k] : 0;
}

// Standalone data events in the fused scan's tap order: tap t of a filter
// is block (row t / (8 spr), x t % (8 spr)) of the template window, spr =
// ceil(T_c,x / 8) segments of 8 blocks per block row; taps past the row are 0.
__global__ void k_events_to_taps(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n_filters, Geom g,
                                 int kk) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n_filters * kKMax) return;
  const long long f = id / kKMax;
  const int t = (int)(id - f * kKMax);
  const int wr = ((g.tc[0] + 7) / 8) * 8;
  const int r = t / wr, bx = t - r * wr;
  const int nrows = g.tc[1] * g.tc[2];
  dst[id] = (t < kk && r < nrows && bx < g.tc[0]) ? src[f * g.tcells + (long long)r * g.tc[0] + bx] : 0;
}

// Scan variants: 1, 2, 4, 8 = candidate-major output with up to that many
// tiles per workgroup; kScanFilterMajor = filter-major output, one tile.
constexpr int kScanFilterMajor = -1;

// Launch scan variant V over `ngroups` workgroup columns.
void launch_scan(int precision, int V, unsigned rows, int ngroups, size_t lds, hipStream_t st, const ScanArgs& sa,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const dim3 grid(rows, (unsigned)ngroups), block(kThreads);
  const uint32_t sh = (uint32_t)lds;
#define CCW_SCAN(OT)                                                                                  \
  do {                                                                                                \
    if (V == kScanFilterMajor) hipExtLaunchKernelGGL((k_scan_fm<OT>), grid, block, sh, st, e0, e1, 0, sa); \
    else if (V == 8) hipExtLaunchKernelGGL((k_scan<OT, 8>), grid, block, sh, st, e0, e1, 0, sa);     \
    else if (V == 4) hipExtLaunchKernelGGL((k_scan<OT, 4>), grid, block, sh, st, e0, e1, 0, sa);     \
    else if (V == 2) hipExtLaunchKernelGGL((k_scan<OT, 2>), grid, block, sh, st, e0, e1, 0, sa);     \
    else hipExtLaunchKernelGGL((k_scan<OT, 1>), grid, block, sh, st, e0, e1, 0, sa);                 \
  } while (0)
  if (precision == 1) CCW_SCAN(__bf16);
  else CCW_SCAN(_Float16);
#undef CCW_SCAN
}

// Launch the fused-selection scan over `ntiles` tiles of 32 filters.
void launch_scan_sel(int precision, bool hd, int en, unsigned rows, int ntiles, size_t lds, hipStream_t st,
                     const ScanArgs& sa, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const dim3 grid(rows, (unsigned)ntiles), block(kThreads);
  const uint32_t sh = (uint32_t)lds;
#define CCW_SEL(OT)                                                                                       \
  do {                                                                                                    \
    if (hd) hipExtLaunchKernelGGL((k_scan_sel<OT, true, kEnStage>), grid, block, sh, st, e0, e1, 0, sa);    \
    else if (en == kEnFold) hipExtLaunchKernelGGL((k_scan_sel<OT, false, kEnFold>), grid, block, sh, st, e0, e1, 0, sa); \
    else if (en == kEnMem) hipExtLaunchKernelGGL((k_scan_sel<OT, false, kEnMem>), grid, block, sh, st, e0, e1, 0, sa);   \
    else hipExtLaunchKernelGGL((k_scan_sel<OT, false, kEnStage>), grid, block, sh, st, e0, e1, 0, sa);  \
  } while (0)
  if (precision == 1) CCW_SEL(__bf16);
  else CCW_SEL(_Float16);
#undef CCW_SEL
}

int scan_strip_width(const Geom& g) {
  return ((g.cand[0] + 31) / 32) * 32 + g.tc[0] - 1 + 1;  // +1 keeps an even length
}

}  // namespace

namespace {
// K best keys of each filter from the fused scan's per-row survivors: the
// K rows with the smallest minima hold them (a row holding one of the K
// best keys has its minimum among them), and within each such row they are
// among its survivors.  One workgroup per filter.
__global__ __launch_bounds__(kThreads) void k_topk_rows(const uint64_t* __restrict__ keys,
                                                        const uint64_t* __restrict__ rowmin,
                                                        const int32_t* __restrict__ rowcnt, Geom g, int k,
                                                        uint64_t seed, const int32_t* __restrict__ real,
                                                        const int64_t* __restrict__ steps,
                                                        uint64_t* __restrict__ out) {
  __shared__ TopkShared sh;
  __shared__ int s_row[kTopMax], s_pre[kTopMax + 1];
  const int f = blockIdx.x, tid = threadIdx.x;
  const int nrows = g.cand[1] * g.cand[2], C0 = g.cand[0];
  const uint64_t tkey = draw64(seed, kStreamTiebreak, (uint64_t)real[f], (uint64_t)steps[f]);
  const uint64_t* rm = rowmin + (long long)f * nrows;
  const int kr = min(k, nrows);
  block_topk(nrows, kr, [&](long long i) { return rm[i]; }, sh);
  if (tid == 0) {
    int pre = 0;
    for (int b = 0; b < kr; ++b) {
      const int id = (int)tie_perm_inv((uint32_t)(sh.top[b] & kMask20), tkey);
      const int row = min(max(id / C0, 0), nrows - 1);
      s_row[b] = row;
      s_pre[b] = pre;
      pre += rowcnt[(long long)f * nrows + row];
    }
    s_pre[kr] = pre;
  }
  __syncthreads();
  const uint64_t* kf = keys + (long long)f * g.ncand;
  const int total = s_pre[kr];
  block_topk(total, k, [&](long long i) {
    int b = 0;
    while (b + 1 < kr && s_pre[b + 1] <= i) ++b;
    return kf[(long long)s_row[b] * C0 + (i - s_pre[b])];
  }, sh);
  if (tid < k) out[(long long)f * k + tid] = sh.top[tid];
}

// Coefficient bound of the level-J LeGall 5/3 approximation of codes in
// [0, max_code]: an interval carried through the J * ndim lifting passes
// (prediction, then the rounded update).
long long lift53_bound(int max_code, int passes) {
  long long lo = 0, hi = max_code > 0 ? max_code : 1;
  for (int k = 0; k < passes; ++k) {
    const long long dlo = lo - hi, dhi = hi - lo;
    const long long nlo = lo + floor_div(2 * dlo + 2, 4), nhi = hi + floor_div(2 * dhi + 2, 4);
    lo = nlo;
    hi = nhi;
  }
  return std::max(-lo, hi);
}

// Everything the standalone scan needs besides its inputs and outputs.
struct ScanPlan {
  Geom g;
  int kpad = 0, W = 0, en = kEnStage, gbits = 0, sel_kk = 0, sel_W = 0;
  bool fused = false, full = false;
  long long ws_kh = 0, ws_mbuf = 0, ws_nbuf = 0, ws_tbuf = 0, ws_energy = 0, ws_keys = 0, ws_rowmin = 0, ws_rowcnt = 0,
            ws_total = 0;
  size_t sel_lds = 0;
};

int scan_plan(ccwsim_shape ti, int32_t level, int32_t wavelet, int32_t max_code, int32_t precision,
              const int32_t tmpl[3], int32_t n_filters, int32_t score_mode, int32_t top_k, bool want_scores,
              bool want_keys, ScanPlan& sp) {
  Geom& g = sp.g;
  CCW_TRY(geom_ti(g, ti, level));
  if (!tmpl) return fail(CCWSIM_ERR_INVALID_ARG, "null template");
  CCW_TRY(geom_tmpl(g, tmpl));
  if (n_filters < 1) return fail(CCWSIM_ERR_INVALID_ARG, "n_filters must be >= 1");
  if (score_mode != 0 && score_mode != 1) return fail(CCWSIM_ERR_INVALID_ARG, "score_mode");
  if (wavelet != 0 && wavelet != 1) return fail(CCWSIM_ERR_INVALID_ARG, "wavelet must be 0 (Haar) or 1 (LeGall 5/3)");
  if (precision != 0 && precision != 1) return fail(CCWSIM_ERR_INVALID_ARG, "precision must be 0 (fp16) or 1 (bf16)");
  if (max_code < 1 || max_code > 126) return fail(CCWSIM_ERR_INVALID_ARG, "max_code must be in [1, 126]");
  if (!want_scores && !want_keys) return fail(CCWSIM_ERR_INVALID_ARG, "neither scores nor top-K keys requested");
  if (want_keys && (top_k < 1 || top_k > kTopMax))
    return fail(CCWSIM_ERR_UNSUPPORTED, "top_k must be in [1, %d]", kTopMax);
  sp.kpad = (int)((g.tcells + 15) / 16 * 16);
  if (sp.kpad > kKMax) return fail(CCWSIM_ERR_UNSUPPORTED, "template has %lld blocks (> %d)", g.tcells, kKMax);
  // operand range: block sums (Haar) or 5/3 coefficients
  long long kmax;
  if (wavelet == 0) {
    CCW_TRY(check_exact(g, max_code, g.wcells));
    kmax = (long long)max_code * g.beta;
  } else {
    g.wavelet = 1;
    g.shift = 1;
    kmax = lift53_bound(max_code, g.level * g.ndim);
    const long long cmax = g.tcells * kmax * kmax;
    if (kmax > 2048) return fail(CCWSIM_ERR_UNSUPPORTED, "5/3 coefficients up to %lld are not exact in fp16", kmax);
    if (cmax >= (1ll << 24)) return fail(CCWSIM_ERR_UNSUPPORTED, "cross sums up to %lld are not exact in fp32", cmax);
    if (3 * cmax >= (1ll << 31)) return fail(CCWSIM_ERR_UNSUPPORTED, "scores up to %lld overflow int32", 3 * cmax);
  }
  if (precision == 1 && kmax > 256)
    return fail(CCWSIM_ERR_UNSUPPORTED, "approximation values up to %lld are not exact in bf16", kmax);
  sp.W = scan_strip_width(g);
  const int nrows = g.tc[1] * g.tc[2];
  if (scan_group_lds(nrows, sp.W, sp.kpad, 1) > 64 * 1024)
    return fail(CCWSIM_ERR_UNSUPPORTED, "scan strip needs %zu bytes of LDS", scan_group_lds(nrows, sp.W, sp.kpad, 1));
  sp.full = want_scores;
  sp.fused = want_keys;
  const int ksel = std::min<long long>(top_k, g.ncand);
  if (sp.fused) {
    if (g.cand[0] > 4096) return fail(CCWSIM_ERR_UNSUPPORTED, "fused selection supports <= 4096 candidates per row");
    // the energy in the contraction when K^2 and the sums stay exact
    const long long klim = precision == 1 ? 256 : 2048;
    sp.en = (score_mode == 0 && kmax * kmax <= klim && g.tcells * g.beta * kmax * kmax < (1ll << 24))
                ? kEnFold : kEnMem;
    const int nchunks = (g.cand[0] + 31) / 32;
    sp.gbits = sel_group_bits(g.cand[0], nchunks, ksel);
    // segments of 8 blocks over every block row of the template
    const int nseg = nrows * ((g.tc[0] + 7) / 8);
    if (nseg > kSegMax)
      return fail(CCWSIM_ERR_UNSUPPORTED, "fused selection supports templates of <= %d 8-block row segments", kSegMax);
    const int ks = ((nseg + 1) / 2 + 3) / 4 * 4;   // K-slices, a multiple of 4
    sp.sel_kk = 16 * ks;
    sp.sel_W = scan_sel_width(nchunks * 32, g.tc[0]);
    sp.sel_lds = scan_sel_lds(nrows, sp.sel_W, sp.sel_kk, 16, sp.en, 1, nchunks * 32, sp.gbits, false);
    if (sp.sel_lds > 64 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "fused scan needs %zu bytes of LDS", sp.sel_lds);
  }
  const long long gcells = (long long)g.G[0] * g.G[1] * g.G[2];
  const long long rows = (long long)g.cand[1] * g.cand[2];
  long long o = 0;
  sp.ws_kh = o;      o += align256(gcells * 2);
  sp.ws_mbuf = o;    o += align256((long long)n_filters * kKMax * 4);
  if (sp.fused) {
    sp.ws_tbuf = o;    o += align256((long long)n_filters * kKMax * 4);
    if (sp.en == kEnFold) {
      sp.ws_nbuf = o;  o += align256((long long)n_filters * kKMax * 4);
    } else if (score_mode == 0) {
      sp.ws_energy = o; o += align256((long long)n_filters * g.ncand * 4);
    }
    sp.ws_keys = o;    o += align256((long long)n_filters * g.ncand * 8);
    sp.ws_rowmin = o;  o += align256((long long)n_filters * rows * 8);
    sp.ws_rowcnt = o;  o += align256((long long)n_filters * rows * 4);
  }
  sp.ws_total = o;
  return CCWSIM_OK;
}

int enqueue_scan(const ScanPlan& sp, int32_t precision, int32_t score_mode, const int32_t* approx,
                 const int32_t* or_n, const int32_t* or_m, int32_t n_filters, int32_t* scores, int32_t top_k,
                 uint64_t seed, const int32_t* realization, const int64_t* step, uint64_t* topk_keys,
                 unsigned char* ws, hipStream_t st, bool profile = true) {
  // the profiler's events are created on demand, so a caller that must not
  // allocate runs without them
  const int kEn = profile ? CCWSIM_KIND_ENERGY : -1, kSc = profile ? CCWSIM_KIND_SCAN : -1;
  const Geom& g = sp.g;
  const long long gcells = (long long)g.G[0] * g.G[1] * g.G[2];
  void* Kh = ws + sp.ws_kh;
  int32_t* mbuf = (int32_t*)(ws + sp.ws_mbuf);
  if (precision == 1) k_to_bf16<<<nblocks(gcells), kThreads, 0, st>>>(approx, (__bf16*)Kh, gcells);
  else k_to_half<<<nblocks(gcells), kThreads, 0, st>>>(approx, (_Float16*)Kh, gcells);
  k_events_to_mbuf<<<nblocks((long long)n_filters * kKMax), kThreads, 0, st>>>(or_m, mbuf, n_filters, g.tcells);
  const int ntiles = (n_filters + kFiltersPerTile - 1) / kFiltersPerTile;
  const long long crow = (long long)g.cand[1] * g.cand[2];
  const int nrows = g.tc[1] * g.tc[2];
  ScanArgs a = {};
  a.g = g;
  a.Kop = Kh;
  a.mbuf = mbuf;
  a.kpad = sp.kpad;
  a.W = sp.W;
  a.score_mode = score_mode;
  a.standalone = 1;
  a.n_filters = n_filters;
  a.ntiles = ntiles;
  if (sp.full) {
    // the whole score map: energies written first, the scan completes them
    if (score_mode == 0) {
      ProfScope ps(kEn, st);
      k_energy<<<nblocks((long long)n_filters * g.ncand), kThreads, 0, st>>>(approx, or_n, n_filters, scores, g);
    }
    int G = 1;
    auto group_ok = [&](int c) {
      return sp.kpad <= kScanGroupKMax && scan_group_lds(nrows, sp.W, sp.kpad, c) <= 64 * 1024;
    };
    for (int c : {2, 4, 8})
      if (c <= ntiles && crow * ((ntiles + c - 1) / c) >= 512 && group_ok(c)) G = c;
    if (g_scan_g_force > 0) {
      G = 1;
      for (int c : {2, 4, 8})
        if (c <= g_scan_g_force && group_ok(c)) G = c;
    } else if (g_scan_g_force == kScanFilterMajor) {
      G = kScanFilterMajor;
    }
    a.scores = scores;
    ProfKernel pk(kSc);
    const int Gt = G == kScanFilterMajor ? 1 : G;
    launch_scan(precision, G, (unsigned)crow, (ntiles + Gt - 1) / Gt, scan_group_lds(nrows, sp.W, sp.kpad, Gt), st,
                a, pk.a, pk.b);
  }
  if (sp.fused) {
    int32_t* energy = nullptr;
    int32_t* tbuf = (int32_t*)(ws + sp.ws_tbuf);
    k_events_to_taps<<<nblocks((long long)n_filters * kKMax), kThreads, 0, st>>>(or_m, tbuf, n_filters, g, sp.sel_kk);
    a.mbuf = tbuf;
    if (sp.en == kEnFold) {
      int32_t* nbuf = (int32_t*)(ws + sp.ws_nbuf);
      k_events_to_taps<<<nblocks((long long)n_filters * kKMax), kThreads, 0, st>>>(or_n, nbuf, n_filters, g, sp.sel_kk);
      a.nbuf = nbuf;
    } else if (score_mode == 0) {
      energy = (int32_t*)(ws + sp.ws_energy);
      ProfScope ps(kEn, st);
      k_energy<<<nblocks((long long)n_filters * g.ncand), kThreads, 0, st>>>(approx, or_n, n_filters, energy, g);
    }
    uint64_t* keys = (uint64_t*)(ws + sp.ws_keys);
    uint64_t* rowmin = (uint64_t*)(ws + sp.ws_rowmin);
    int32_t* rowcnt = (int32_t*)(ws + sp.ws_rowcnt);
    const int k = (int)std::min<long long>(top_k, g.ncand);
    a.scores = nullptr;
    a.energy = energy;
    a.keys = keys;
    a.rowmin = rowmin;
    a.rowcnt = rowcnt;
    a.seed = seed;
    a.fil_real = realization;
    a.fil_step = step;
    a.ksel = k;
    a.gbits = sp.gbits;
    a.n_bm = 1;
    a.kpad = sp.sel_kk;
    a.W = sp.sel_W;
    {
      ProfKernel pk(kSc);
      launch_scan_sel(precision, false, sp.en, (unsigned)crow, ntiles, sp.sel_lds, st, a, pk.a, pk.b);
    }
    k_topk_rows<<<(unsigned)n_filters, kThreads, 0, st>>>(keys, rowmin, rowcnt, g, k, seed, realization, step,
                                                          topk_keys);
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}
}  // namespace

extern "C" int64_t ccwsim_ccf_scan_workspace_size(ccwsim_shape ti, int32_t level, int32_t wavelet,
                                                  int32_t max_code, int32_t precision, const int32_t tmpl[3],
                                                  int32_t n_filters, int32_t score_mode, int32_t top_k,
                                                  int32_t want_scores, int32_t want_keys) {
  ScanPlan sp;
  if (scan_plan(ti, level, wavelet, max_code, precision, tmpl, n_filters, score_mode, top_k, want_scores != 0,
                want_keys != 0, sp))
    return -1;
  return sp.ws_total;
}

extern "C" int ccwsim_ccf_scan(ccwsim_shape ti, int32_t level, int32_t wavelet, int32_t max_code, int32_t precision,
                               const int32_t* approx, const int32_t tmpl[3], const int32_t* or_n,
                               const int32_t* or_m, int32_t n_filters, int32_t score_mode, int32_t* scores,
                               int32_t top_k, uint64_t seed, const int32_t* realization, const int64_t* step,
                               uint64_t* topk_keys, void* workspace, int64_t workspace_bytes, void* stream) {
  ScanPlan sp;
  CCW_TRY(scan_plan(ti, level, wavelet, max_code, precision, tmpl, n_filters, score_mode, top_k, scores != nullptr,
                    topk_keys != nullptr, sp));
  if (!approx || !or_m || (score_mode == 0 && !or_n)) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (topk_keys && (!realization || !step)) return fail(CCWSIM_ERR_INVALID_ARG, "top-K keys need realization and step");
  if (!workspace || workspace_bytes < sp.ws_total)
    return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", sp.ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return enqueue_scan(sp, precision, score_mode, approx, or_n, or_m, n_filters, scores, top_k, seed, realization,
                      step, topk_keys, (unsigned char*)workspace, as_stream(stream));
}

// ---- the scan without a workspace: temporaries in a static device array ----
namespace {
constexpr size_t kScratchBytes = 64ull << 20;
// One copy per device, held from module load until the process ends.  In
// host code its name is only a stand-in: kernels receive the device address
// that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;   // device -> address of its scratch

int scratch_of_current_device(unsigned char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CCWSIM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, (unsigned char*)ptr).first;
  }
  *out = it->second;
  return CCWSIM_OK;
}
}  // namespace

extern "C" int64_t ccwsim_ccf_scan_noalloc_capacity(void) { return (int64_t)kScratchBytes; }

extern "C" int ccwsim_ccf_scan_noalloc(ccwsim_shape ti, int32_t level, int32_t wavelet, int32_t max_code,
                                       int32_t precision, const int32_t* approx, const int32_t tmpl[3],
                                       const int32_t* or_n, const int32_t* or_m, int32_t n_filters,
                                       int32_t score_mode, int32_t* scores, int32_t top_k, uint64_t seed,
                                       const int32_t* realization, const int64_t* step, uint64_t* topk_keys,
                                       void* stream) {
  ScanPlan sp;
  CCW_TRY(scan_plan(ti, level, wavelet, max_code, precision, tmpl, n_filters, score_mode, top_k, scores != nullptr,
                    topk_keys != nullptr, sp));
  if (!approx || !or_m || (score_mode == 0 && !or_n)) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (topk_keys && (!realization || !step)) return fail(CCWSIM_ERR_INVALID_ARG, "top-K keys need realization and step");
  if ((size_t)sp.ws_total > kScratchBytes)
    return fail(CCWSIM_ERR_UNSUPPORTED, "this scan needs %lld bytes of temporaries; the static scratch holds %zu",
                (long long)sp.ws_total, kScratchBytes);
  unsigned char* ptr = nullptr;
  CCW_TRY(scratch_of_current_device(&ptr));
  return enqueue_scan(sp, precision, score_mode, approx, or_n, or_m, n_filters, scores, top_k, seed, realization,
                      step, topk_keys, ptr, as_stream(stream), false);
}

// ===========================================================================
// A9 learned proposer: training and encoding (Sec. 4.3-4.4 search on the
// approximation; the proposer ranks positions, the exact score judges them)
// ===========================================================================
namespace {

struct LpPlan {
  LpGeom q;
  Geom g;
  int B = 0;
  long long gc = 0, wc = 0;
  long long o_kin = 0, o_ka = 0, o_kmap = 0, o_keys = 0, o_qin = 0, o_qa = 0, o_qmap = 0, o_qv = 0, o_S = 0, o_gW = 0,
            o_dkmap = 0, o_dk = 0, o_dqmap = 0, o_dq = 0, o_dqa = 0, total = 0;
};

int lp_plan(ccwsim_shape ti, int32_t level, const int32_t tmpl[3], int32_t batch, LpPlan& L) {
  CCW_TRY(geom_ti(L.g, ti, level));
  if (!tmpl) return fail(CCWSIM_ERR_INVALID_ARG, "null template");
  CCW_TRY(geom_tmpl(L.g, tmpl));
  if (L.g.ndim != 2) return fail(CCWSIM_ERR_UNSUPPORTED, "the learned proposer runs on 2D training images");
  if (batch < 0 || batch > 4096) return fail(CCWSIM_ERR_INVALID_ARG, "batch must be in [0, 4096]");
  const Geom& g = L.g;
  for (int a = 0; a < 3; ++a) {
    L.q.G[a] = g.G[a];
    L.q.cand[a] = g.cand[a];
    L.q.tc[a] = g.tc[a];
    L.q.half[a] = a < g.ndim ? g.tc[a] / 2 : 0;
  }
  L.q.ncand = g.ncand;
  L.B = batch;
  L.gc = (long long)g.G[0] * g.G[1] * g.G[2];
  L.wc = g.tcells;
  const long long B = std::max(batch, 1);
  long long o = 0;
  auto take = [&](long long floats) {
    const long long at = o;
    o += align256(floats * 4);
    return at;
  };
  L.o_kin = take(L.gc);
  L.o_ka = take(3 * kLpC * L.gc);
  L.o_kmap = take(kLpD * L.gc);
  L.o_keys = take(g.ncand * kLpD);
  L.o_qin = take(B * 2 * L.wc);
  L.o_qa = take(3 * B * kLpC * L.wc);
  L.o_qmap = take(B * kLpD * L.wc);
  L.o_qv = take(B * kLpD);
  L.o_S = take(B * g.ncand);
  L.o_gW = take(lp_weights_total());
  L.o_dkmap = take(kLpD * L.gc);
  L.o_dk = take(2 * kLpC * L.gc);
  L.o_dqmap = take(B * kLpD * L.wc);
  L.o_dq = take(B * kLpD);
  L.o_dqa = take(2 * B * kLpC * L.wc);
  L.total = o;
  return CCWSIM_OK;
}

void lp_conv(const float* in, const float* Wb, float* out, int N, int l, int cin0, int H, int Wd, bool relu,
             hipStream_t st) {
  const LpLayer Ly = lp_layer(l, cin0);
  const long long n = (long long)N * Ly.cout * H * Wd;
  k_lp_conv_fwd<<<nblocks(n), kThreads, 0, st>>>(in, Wb, out, N, Ly.cin, Ly.cout, H, Wd, Ly.taps, Ly.dil, relu ? 1 : 0);
}

// Forward of one encoder: acts[0..2] (32 channels), out (64 channels).
void lp_encoder_fwd(const float* W, int e, const float* in, float* acts, float* out, int N, int H, int Wd,
                    hipStream_t st) {
  const int cin0 = e == 0 ? 1 : 2;
  const long long a = (long long)N * kLpC * H * Wd;
  const float* src = in;
  for (int l = 0; l < kLpLayers; ++l) {
    float* dst = l < 3 ? acts + l * a : out;
    lp_conv(src, W + lp_offset(e, l), dst, N, l, cin0, H, Wd, l < 3, st);
    src = dst;
  }
}

// Backward of one encoder from the gradient of its output (dout, 64
// channels): weight gradients into gW, input gradient not needed.
void lp_encoder_bwd(const float* W, float* gW, int e, const float* in, const float* acts, float* dout, float* dbuf,
                    int N, int H, int Wd, hipStream_t st) {
  const int cin0 = e == 0 ? 1 : 2;
  const long long a = (long long)N * kLpC * H * Wd;
  float* d = dout;   // gradient at the current layer's output (pre-activation once masked)
  for (int l = kLpLayers - 1; l >= 0; --l) {
    const LpLayer Ly = lp_layer(l, cin0);
    const float* lin = l == 0 ? in : acts + (l - 1) * a;
    k_lp_conv_bwd_w<<<(unsigned)(Ly.cout * Ly.cin), kThreads, 0, st>>>(lin, d, gW + lp_offset(e, l), N, Ly.cin,
                                                                     Ly.cout, H, Wd, Ly.taps, Ly.dil);
    if (l == 0) break;
    float* dn = dbuf + (l & 1) * a;
    const long long n = (long long)N * Ly.cin * H * Wd;
    k_lp_conv_bwd_in<<<nblocks(n), kThreads, 0, st>>>(d, W + lp_offset(e, l), dn, N, Ly.cin, Ly.cout, H, Wd, Ly.taps,
                                                     Ly.dil);
    k_lp_relu_bwd<<<nblocks(n), kThreads, 0, st>>>(dn, lin, n);   // layer l-1 ends in a ReLU
    d = dn;
  }
}

// Forward through the scores; returns nothing, fills keys, queries, S.
void lp_forward(const LpPlan& L, const float* W, const int32_t* approx, const int32_t* or_n, const int32_t* or_m,
                unsigned char* ws, bool want_keys, hipStream_t st) {
  const Geom& g = L.g;
  float* kin = (float*)(ws + L.o_kin);
  float* ka = (float*)(ws + L.o_ka);
  float* kmap = (float*)(ws + L.o_kmap);
  float* keys = (float*)(ws + L.o_keys);
  if (want_keys) {
    k_lp_kin<<<nblocks(L.gc), kThreads, 0, st>>>(approx, L.gc, 1.f / (float)g.beta, kin);
    lp_encoder_fwd(W, 0, kin, ka, kmap, 1, g.G[1], g.G[0], st);
    k_lp_gather_keys<<<nblocks(g.ncand * kLpD), kThreads, 0, st>>>(kmap, L.q, keys);
  }
  if (L.B > 0 && or_n && or_m) {
    float* events = (float*)(ws + L.o_qin);
    k_lp_events<<<nblocks((long long)L.B * L.wc), kThreads, 0, st>>>(or_n, or_m, L.B, L.wc, 1.f / (float)g.beta, events);
    float* qa = (float*)(ws + L.o_qa);
    float* qmap = (float*)(ws + L.o_qmap);
    float* qv = (float*)(ws + L.o_qv);
    float* S = (float*)(ws + L.o_S);
    lp_encoder_fwd(W, 1, events, qa, qmap, L.B, g.tc[1], g.tc[0], st);
    k_lp_gather_queries<<<nblocks((long long)L.B * kLpD), kThreads, 0, st>>>(qmap, L.q, L.B, qv);
    k_lp_scores<<<nblocks(g.ncand * L.B), kThreads, 0, st>>>(qv, keys, g.ncand, L.B, S);
  }
}
}  // namespace

extern "C" int ccwsim_lp_sizes(ccwsim_shape ti, int32_t level, const int32_t tmpl[3], int32_t batch,
                               int64_t* n_weights, int64_t* workspace_bytes, int64_t* n_cand) {
  LpPlan L;
  CCW_TRY(lp_plan(ti, level, tmpl, batch, L));
  if (n_weights) *n_weights = lp_weights_total();
  if (workspace_bytes) *workspace_bytes = L.total;
  if (n_cand) *n_cand = L.g.ncand;
  return CCWSIM_OK;
}

extern "C" int ccwsim_lp_init(float* weights, uint64_t seed, void* stream) {
  if (!weights) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  k_lp_init<<<nblocks(lp_weights_total()), kThreads, 0, as_stream(stream)>>>(weights, seed);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int ccwsim_lp_encode(const float* weights, const int32_t* approx, ccwsim_shape ti, int32_t level,
                                const int32_t tmpl[3], const int32_t* or_n, const int32_t* or_m, int32_t batch,
                                float* keys_out,
                                float* queries_out, float* scores_out, void* workspace, int64_t workspace_bytes,
                                void* stream) {
  LpPlan L;
  CCW_TRY(lp_plan(ti, level, tmpl, batch, L));
  if (!weights || !approx || (batch > 0 && (!or_n || !or_m))) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (!workspace || workspace_bytes < L.total) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", L.total);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  unsigned char* ws = (unsigned char*)workspace;
  lp_forward(L, weights, approx, or_n, or_m, ws, true, st);
  const Geom& g = L.g;
  if (keys_out)
    HIP_TRY(hipMemcpyAsync(keys_out, ws + L.o_keys, g.ncand * kLpD * 4, hipMemcpyDeviceToDevice, st));
  if (queries_out && batch > 0)
    HIP_TRY(hipMemcpyAsync(queries_out, ws + L.o_qv, (size_t)batch * kLpD * 4, hipMemcpyDeviceToDevice, st));
  if (scores_out && batch > 0)
    HIP_TRY(hipMemcpyAsync(scores_out, ws + L.o_S, (size_t)batch * g.ncand * 4, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int ccwsim_lp_train_step(float* weights, float* adam_m, float* adam_v, int32_t step, float lr,
                                    const int32_t* approx, ccwsim_shape ti, int32_t level, const int32_t tmpl[3],
                                    const int32_t* or_n, const int32_t* or_m, const int32_t* labels, int32_t n_pos,
                                    int32_t batch, float* loss,
                                    float* grad_out, void* workspace, int64_t workspace_bytes, void* stream) {
  LpPlan L;
  CCW_TRY(lp_plan(ti, level, tmpl, batch, L));
  if (!weights || !adam_m || !adam_v || !approx || !or_n || !or_m || !labels || !loss)
    return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (batch < 1) return fail(CCWSIM_ERR_INVALID_ARG, "batch must be >= 1");
  if (n_pos < 1 || n_pos > kLpPosMax || n_pos > L.g.ncand)
    return fail(CCWSIM_ERR_INVALID_ARG, "n_pos must be in [1, min(%d, candidates)]", kLpPosMax);
  if (step < 1) return fail(CCWSIM_ERR_INVALID_ARG, "Adam steps count from 1");
  if (!workspace || workspace_bytes < L.total) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", L.total);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  unsigned char* ws = (unsigned char*)workspace;
  const Geom& g = L.g;
  lp_forward(L, weights, approx, or_n, or_m, ws, true, st);
  float* S = (float*)(ws + L.o_S);
  k_lp_ce<<<(unsigned)batch, kThreads, 0, st>>>(S, labels, n_pos, g.ncand, batch, loss);   // S becomes dS
  float* gW = (float*)(ws + L.o_gW);
  float* dq = (float*)(ws + L.o_dq);
  float* dkmap = (float*)(ws + L.o_dkmap);
  k_lp_grad_q<<<(unsigned)batch, kThreads, 0, st>>>(S, (const float*)(ws + L.o_keys), g.ncand, dq);
  k_fill_f32<<<nblocks(kLpD * L.gc), kThreads, 0, st>>>(dkmap, kLpD * L.gc, 0.f);
  k_lp_grad_k<<<nblocks(g.ncand * kLpD), kThreads, 0, st>>>(S, (const float*)(ws + L.o_qv), L.q, batch, dkmap);
  // query encoder
  float* dqmap = (float*)(ws + L.o_dqmap);
  k_lp_scatter_dq<<<nblocks((long long)batch * kLpD * L.wc), kThreads, 0, st>>>(dq, L.q, batch, dqmap);
  lp_encoder_bwd(weights, gW, 1, (const float*)(ws + L.o_qin), (const float*)(ws + L.o_qa), dqmap, (float*)(ws + L.o_dqa), batch, g.tc[1],
                 g.tc[0], st);
  // key encoder
  lp_encoder_bwd(weights, gW, 0, (const float*)(ws + L.o_kin), (const float*)(ws + L.o_ka), dkmap,
                 (float*)(ws + L.o_dk), 1, g.G[1], g.G[0], st);
  if (grad_out) HIP_TRY(hipMemcpyAsync(grad_out, gW, lp_weights_total() * 4, hipMemcpyDeviceToDevice, st));
  k_lp_adam<<<nblocks(lp_weights_total()), kThreads, 0, st>>>(weights, gW, adam_m, adam_v, lp_weights_total(), lr,
                                                              0.9f, 0.999f, 1e-8f, step);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int ccwsim_lp_shortlist(const float* scores, int32_t batch, int64_t n_cand, int32_t k, int32_t* idx_out,
                                   void* stream) {
  if (!scores || !idx_out) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (batch < 0 || n_cand < 1 || n_cand > (1 << 20)) return fail(CCWSIM_ERR_INVALID_ARG, "sizes");
  if (k < 1 || k > 256 || k > n_cand) return fail(CCWSIM_ERR_INVALID_ARG, "k must be in [1, min(256, n_cand)]");
  if (batch == 0) return CCWSIM_OK;
  k_lp_topk<float><<<(unsigned)batch, kThreads, 0, as_stream(stream)>>>(scores, n_cand, k, idx_out);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int ccwsim_lp_labels(const int32_t* scores, int32_t batch, int64_t n_cand, int32_t k, int32_t* idx_out,
                                void* stream) {
  if (!scores || !idx_out) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (batch < 0 || n_cand < 1 || n_cand > (1 << 20)) return fail(CCWSIM_ERR_INVALID_ARG, "sizes");
  if (k < 1 || k > 256 || k > n_cand) return fail(CCWSIM_ERR_INVALID_ARG, "k must be in [1, min(256, n_cand)]");
  if (batch == 0) return CCWSIM_OK;
  k_lp_topk<int32_t><<<(unsigned)batch, kThreads, 0, as_stream(stream)>>>(scores, n_cand, k, idx_out);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// ---- inverted lists over the keys, and the proposal on its own ----------
namespace {
__global__ void k_lp_header(LpIndexHeader h, LpIndexHeader* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = h;
}

int lp_index_layout(const LpPlan& L, int n_lists, LpIndexHeader& h) {
  const Geom& g = L.g;
  if (n_lists < 1 || n_lists > kLpListsMax || n_lists > g.ncand)
    return fail(CCWSIM_ERR_INVALID_ARG, "n_lists must be in [1, min(%d, candidates)]", kLpListsMax);
  memset(&h, 0, sizeof h);
  h.magic = kLpMagic;
  h.n_lists = n_lists;
  h.level = g.level;
  h.ndim = g.ndim;
  for (int a = 0; a < 3; ++a) {
    h.G[a] = g.G[a];
    h.cand[a] = g.cand[a];
    h.tc[a] = g.tc[a];
  }
  h.ncand = g.ncand;
  long long o = align256(sizeof h);
  h.off_w = o;
  o += align256(lp_query_floats() * 4);
  h.off_cent = o;
  o += 2 * lp_cent_bytes(n_lists);   // [n_lists][64], then [16][n_lists][4]
  h.off_list = o;
  o += align256((long long)(n_lists + 1) * 4);
  h.off_mem = o;
  o += align256(g.ncand * 4);
  h.bytes = o;
  return CCWSIM_OK;
}

// Dynamic LDS beyond 64 KiB for the proposal kernel (once per size).
int lp_lds_allow(int kt, size_t bytes) {
  if (bytes <= 64 * 1024) return CCWSIM_OK;
  int dev = 0, lim = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if ((size_t)lim < bytes)
    return fail(CCWSIM_ERR_UNSUPPORTED, "the proposal needs %zu B of LDS, the device allows %d", bytes, lim);
  if (kt == 1)
    HIP_TRY(hipFuncSetAttribute((const void*)k_lp_propose<int8_t>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  else
    HIP_TRY(hipFuncSetAttribute((const void*)k_lp_propose<int16_t>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return CCWSIM_OK;
}

// The index header, checked against the geometry (a synchronous read).
int lp_index_check(const void* index, const Geom& g, hipStream_t st, LpIndexHeader* out) {
  LpIndexHeader h;
  HIP_TRY(hipMemcpyAsync(&h, index, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h.magic != kLpMagic) return fail(CCWSIM_ERR_INVALID_ARG, "the proposer pointer holds no index");
  if (h.n_lists < 1 || h.n_lists > kLpListsMax || h.ncand != g.ncand || h.level != g.level || h.G[0] != g.G[0] ||
      h.G[1] != g.G[1] || h.cand[0] != g.cand[0] || h.cand[1] != g.cand[1] || h.tc[0] != g.tc[0] ||
      h.tc[1] != g.tc[1])
    return fail(CCWSIM_ERR_INVALID_ARG, "the proposer index was built for another TI, level or template");
  if (out) *out = h;
  return CCWSIM_OK;
}
}  // namespace

extern "C" int ccwsim_lp_index_size(ccwsim_shape ti, int32_t level, const int32_t tmpl[3], int32_t n_lists,
                                    int64_t* index_bytes, int64_t* workspace_bytes) {
  LpPlan L;
  CCW_TRY(lp_plan(ti, level, tmpl, 0, L));
  LpIndexHeader h;
  CCW_TRY(lp_index_layout(L, n_lists, h));
  if (index_bytes) *index_bytes = h.bytes;
  if (workspace_bytes) *workspace_bytes = L.total + align256(L.g.ncand * 4) + align256((long long)n_lists * 4);
  return CCWSIM_OK;
}

extern "C" int ccwsim_lp_build_index(const float* weights, const int32_t* approx, ccwsim_shape ti, int32_t level,
                                     const int32_t tmpl[3], int32_t n_lists, int32_t iters, void* index,
                                     int64_t index_bytes, void* workspace, int64_t workspace_bytes, void* stream) {
  LpPlan L;
  CCW_TRY(lp_plan(ti, level, tmpl, 0, L));
  LpIndexHeader h;
  CCW_TRY(lp_index_layout(L, n_lists, h));
  if (!weights || !approx || !index) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (iters < 1 || iters > 100) return fail(CCWSIM_ERR_INVALID_ARG, "iters must be in [1, 100]");
  if (index_bytes < h.bytes) return fail(CCWSIM_ERR_INVALID_ARG, "index of %lld bytes needed", (long long)h.bytes);
  const long long need = L.total + align256(L.g.ncand * 4) + align256((long long)n_lists * 4);
  if (!workspace || workspace_bytes < need) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", need);
  if ((((uintptr_t)workspace | (uintptr_t)index) & 255) != 0)
    return fail(CCWSIM_ERR_WORKSPACE, "workspace and index must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  unsigned char* ws = (unsigned char*)workspace;
  unsigned char* ix = (unsigned char*)index;
  const Geom& g = L.g;
  lp_forward(L, weights, approx, nullptr, nullptr, ws, true, st);
  const float* keys = (const float*)(ws + L.o_keys);
  int32_t* assign = (int32_t*)(ws + L.total);
  int32_t* cnt = (int32_t*)(ws + L.total + align256(g.ncand * 4));
  float* cent = (float*)(ix + h.off_cent);
  int32_t* off = (int32_t*)(ix + h.off_list);
  int32_t* mem = (int32_t*)(ix + h.off_mem);
  k_lp_header<<<1, 64, 0, st>>>(h, (LpIndexHeader*)ix);
  HIP_TRY(hipMemcpyAsync(ix + h.off_w, weights + lp_offset(1, 0), lp_query_floats() * 4, hipMemcpyDeviceToDevice, st));
  k_km_init<<<nblocks((long long)n_lists * kLpD), kThreads, 0, st>>>(keys, g.ncand, n_lists, cent);
  const unsigned nb = (unsigned)((g.ncand + kThreads - 1) / kThreads);
  for (int it = 0; it < iters; ++it) {
    k_km_assign<<<nb, kThreads, 0, st>>>(keys, g.ncand, cent, n_lists, assign);
    k_km_lists<<<(unsigned)n_lists, kThreads, 0, st>>>(assign, g.ncand, nullptr, cnt);
    k_km_offsets<<<1, 64, 0, st>>>(cnt, n_lists, off);
    k_km_lists<<<(unsigned)n_lists, kThreads, 0, st>>>(assign, g.ncand, off, mem);
    k_km_update<<<(unsigned)n_lists, kThreads, 0, st>>>(keys, off, mem, cent);
  }
  k_km_transpose<<<nblocks((long long)n_lists * (kLpD / 4)), kThreads, 0, st>>>(
      cent, n_lists, (float*)(ix + h.off_cent + lp_cent_bytes(n_lists)));
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int64_t ccwsim_lp_propose_workspace_size(ccwsim_shape ti, int32_t level, int32_t max_code,
                                                    const int32_t tmpl[3]) {
  Geom g;
  if (geom_ti(g, ti, level) != CCWSIM_OK || !tmpl || geom_tmpl(g, tmpl) != CCWSIM_OK) return -1;
  if (max_code < 1 || max_code > 126) {
    fail(CCWSIM_ERR_INVALID_ARG, "max_code must be in [1, 126]");
    return -1;
  }
  return align256(lp_prop_grid_bytes(g, 2));
}

extern "C" int ccwsim_lp_propose(const void* index, const int32_t* approx, ccwsim_shape ti, int32_t level,
                                 int32_t max_code, const int32_t tmpl[3], const int32_t* or_n, const int32_t* or_m,
                                 int32_t n_filters, int32_t probe, int32_t top_k, uint64_t seed,
                                 const int32_t* realization, const int64_t* step, uint64_t* topk_keys,
                                 int32_t* members, int32_t* n_members, float* queries, float* best_error,
                                 void* workspace, int64_t workspace_bytes, void* stream) {
  Geom g;
  CCW_TRY(geom_ti(g, ti, level));
  if (!tmpl) return fail(CCWSIM_ERR_INVALID_ARG, "null template");
  CCW_TRY(geom_tmpl(g, tmpl));
  if (g.ndim != 2) return fail(CCWSIM_ERR_UNSUPPORTED, "the learned proposer runs on 2D training images");
  if (!index || !approx || !topk_keys || (n_filters > 0 && (!or_n || !or_m)))
    return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (max_code < 1 || max_code > 126) return fail(CCWSIM_ERR_INVALID_ARG, "max_code must be in [1, 126]");
  if ((long long)max_code * g.beta > 32767) return fail(CCWSIM_ERR_UNSUPPORTED, "block sums exceed int16");
  if (probe < 1 || probe > kLpProbeMax) return fail(CCWSIM_ERR_INVALID_ARG, "probe must be in [1, %d]", kLpProbeMax);
  if (top_k < 1 || top_k > kTopMax) return fail(CCWSIM_ERR_INVALID_ARG, "top_k must be in [1, %d]", kTopMax);
  if ((realization == nullptr) != (step == nullptr))
    return fail(CCWSIM_ERR_INVALID_ARG, "realization and step go together");
  if (n_filters < 0) return fail(CCWSIM_ERR_INVALID_ARG, "n_filters");
  const long long need = align256(lp_prop_grid_bytes(g, 2));
  if (!workspace || workspace_bytes < need) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", need);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const int kt = (long long)max_code * g.beta <= 127 ? 1 : 2;   // the grid's LDS copy as int8 or int16
  const size_t lds = (size_t)lp_prop_lds(g, kt, kLpCandMax, (int)g.tcells);
  if (lds > 160 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "the proposal needs %zu B of LDS", lds);
  hipStream_t st = as_stream(stream);
  CCW_TRY(lp_index_check(index, g, st, nullptr));
  CCW_TRY(lp_lds_allow(kt, lds));
  if (n_filters == 0) return CCWSIM_OK;
  const long long gc = (long long)g.G[0] * g.G[1];
  const long long npad = lp_prop_grid_bytes(g, kt) / kt;
  if (kt == 1) k_lp_narrow<int8_t><<<nblocks(npad), kThreads, 0, st>>>(approx, gc, npad, (int8_t*)workspace);
  else k_lp_narrow<int16_t><<<nblocks(npad), kThreads, 0, st>>>(approx, gc, npad, (int16_t*)workspace);
  LpPropArgs la = {};
  la.g = g;
  la.index = (const unsigned char*)index;
  la.grid = workspace;
  la.probe = probe;
  la.cap = kLpCandMax;
  la.top_k = top_k;
  la.gate = -1.f;
  la.seed = seed;
  la.standalone = 1;
  la.or_n = or_n;
  la.or_m = or_m;
  la.fil_real = realization;
  la.fil_step = step;
  la.keys_out = topk_keys;
  la.list_out = members;
  la.nlist_out = n_members;
  la.q_out = queries;
  la.err_out = best_error;
  if (kt == 1) k_lp_propose<int8_t><<<(unsigned)n_filters, kThreads, lds, st>>>(la);
  else k_lp_propose<int16_t><<<(unsigned)n_filters, kThreads, lds, st>>>(la);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// ===========================================================================
// A6: standalone select
// ===========================================================================
namespace {

__global__ __launch_bounds__(kThreads) void k_select(const int32_t* __restrict__ scores,
                                                     const uint16_t* __restrict__ mism, long long n,
                                                     int k, uint64_t seed, const int32_t* __restrict__ real,
                                                     const int64_t* __restrict__ steps,
                                                     int32_t* __restrict__ chosen, uint64_t* __restrict__ topk) {
  __shared__ TopkShared sh;
  const int f = blockIdx.x;
  const uint64_t r = (uint64_t)real[f], s = (uint64_t)steps[f];
  const uint64_t tkey = draw64(seed, kStreamTiebreak, r, s);
  const int32_t* sc = scores + (long long)f * n;
  const uint16_t* mm = mism ? mism + (long long)f * n : nullptr;
  block_topk(n, k, [&](long long i) {
    return make_key(mm ? mm[i] : 0u, sc[i], tie_perm((uint32_t)i, tkey));
  }, sh);
  if (threadIdx.x == 0) {
    const uint64_t u = draw64(seed, kStreamDraw, r, s) >> 32;
    const int jpick = (int)((u * (uint64_t)k) >> 32);
    chosen[f] = (int32_t)tie_perm_inv((uint32_t)(sh.top[jpick] & kMask20), tkey);
  }
  if (topk && threadIdx.x < k) topk[(long long)f * k + threadIdx.x] = sh.top[threadIdx.x];
}

}  // namespace

extern "C" int ccwsim_select(const int32_t* scores, const uint16_t* mismatch, int64_t n_cand,
                             int32_t n_filters, int32_t top_k, uint64_t seed, const int32_t* realization,
                             const int64_t* step, int32_t* chosen, uint64_t* topk_keys, void* stream) {
  if (!scores || !realization || !step || !chosen) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (n_cand < 1 || n_cand > (1 << 20)) return fail(CCWSIM_ERR_INVALID_ARG, "n_cand must be in [1, 2^20]");
  if (n_filters < 1) return fail(CCWSIM_ERR_INVALID_ARG, "n_filters must be >= 1");
  if (top_k < 1 || top_k > kTopMax) return fail(CCWSIM_ERR_UNSUPPORTED, "top_k must be in [1, %d]", kTopMax);
  const int k = (int)std::min<int64_t>(top_k, n_cand);
  hipStream_t st = as_stream(stream);
  k_select<<<(unsigned)n_filters, kThreads, 0, st>>>(scores, mismatch, n_cand, k, seed, realization, step,
                                                     chosen, topk_keys);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// ===========================================================================
// A7: standalone inverse transform of patterns
// ===========================================================================
namespace {

long long idwt_buf_cells(const Geom& g) {
  if (g.level == 0) return 0;
  long long c = 1;
  for (int a = 0; a < 3; ++a) c *= a < g.ndim ? (long long)g.tc[a] << (g.level - 1) : 1;
  return c;
}

template <int ND>
__global__ __launch_bounds__(kThreads) void k_idwt(const int32_t* __restrict__ approx,
                                                   const int32_t* __restrict__ det, Geom g,
                                                   const int32_t* __restrict__ origins,
                                                   int8_t* __restrict__ out, long long buf_cells) {
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t* bufA = (int32_t*)smem;
  int32_t* bufB = bufA + buf_cells;
  int8_t* P = (int8_t*)(bufB + buf_cells);
  const int p = blockIdx.x;
  const int c0x = origins[3 * p], c0y = origins[3 * p + 1], c0z = origins[3 * p + 2];
  const int c0[3] = {c0x, c0y, c0z};
  bool ok = true;
  for (int d = 0; d < 3; ++d) ok = ok && c0[d] >= 0 && c0[d] + g.tc[d] <= g.G[d];
  if (!ok) {  // origin outside the approximation grid: mark the pattern invalid
    for (int u = threadIdx.x; u < (int)g.wcells; u += kThreads) out[(long long)p * g.wcells + u] = -1;
    return;
  }
  idwt_window<ND>(approx, det, g, c0x, c0y, c0z, bufA, bufB, P);
  __syncthreads();
  for (int u = threadIdx.x; u < (int)g.wcells; u += kThreads) out[(long long)p * g.wcells + u] = P[u];
}

}  // namespace

extern "C" int64_t ccwsim_idwt_workspace_size(ccwsim_shape ti, int32_t level, int32_t wavelet) {
  Geom g;
  if (geom_ti(g, ti, level)) return -1;
  if (wavelet != 0 && wavelet != 1) {
    fail(CCWSIM_ERR_INVALID_ARG, "wavelet must be 0 (Haar) or 1 (LeGall 5/3)");
    return -1;
  }
  return wavelet == 1 ? lift53_ws_bytes(g) : 0;
}

extern "C" int ccwsim_idwt(const int32_t* approx, const int32_t* details, ccwsim_shape ti, int32_t level,
                           int32_t wavelet, const int32_t* block_origins, int32_t n, const int32_t patch[3],
                           int8_t* patches, void* workspace, int64_t workspace_bytes, void* stream) {
  Geom g;
  CCW_TRY(geom_ti(g, ti, level));
  if (wavelet != 0 && wavelet != 1) return fail(CCWSIM_ERR_INVALID_ARG, "wavelet must be 0 (Haar) or 1 (LeGall 5/3)");
  if (!approx || !block_origins || !patches || !patch || (level > 0 && !details))
    return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (n < 0) return fail(CCWSIM_ERR_INVALID_ARG, "n must be >= 0");
  for (int a = 0; a < 3; ++a) {
    const int t = a < g.ndim ? patch[a] : 1;
    if (t < 1 || t > 64) return fail(CCWSIM_ERR_UNSUPPORTED, "patch extent %d on axis %d", t, a);
    g.T[a] = t;
    g.tc[a] = (t + g.b[a] - 1) / g.b[a];
    if (g.tc[a] > g.G[a]) return fail(CCWSIM_ERR_SHAPE, "patch larger than the TI on axis %d", a);
  }
  g.tcells = (long long)g.tc[0] * g.tc[1] * g.tc[2];
  g.wcells = (long long)g.T[0] * g.T[1] * g.T[2];
  if (g.wcells > 16384) return fail(CCWSIM_ERR_UNSUPPORTED, "patch has more than 16384 cells");
  if (wavelet == 1) {
    const long long need = lift53_ws_bytes(g);
    if (!workspace || workspace_bytes < need) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", need);
    if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  }
  if (n == 0) return CCWSIM_OK;
  hipStream_t st53 = as_stream(stream);
  if (wavelet == 1) {
    // the whole padded image by the inverse lifting, then crops of it
    CCW_TRY(launch_idwt53(g, approx, details, (unsigned char*)workspace, st53));
    k_crop_patterns<<<nblocks((long long)n * g.wcells), kThreads, 0, st53>>>((const int32_t*)workspace, g, block_origins,
                                                                            n, patches);
    HIP_TRY(hipGetLastError());
    return CCWSIM_OK;
  }
  const long long bc = idwt_buf_cells(g);
  const size_t lds = (size_t)bc * 8 + (size_t)g.wcells;
  if (lds > 64 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "pattern needs %zu bytes of LDS", lds);
  hipStream_t st = as_stream(stream);
  if (g.ndim == 2)
    k_idwt<2><<<(unsigned)n, kThreads, lds, st>>>(approx, details, g, block_origins, patches, bc);
  else
    k_idwt<3><<<(unsigned)n, kThreads, lds, st>>>(approx, details, g, block_origins, patches, bc);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// ===========================================================================
// whole hot path
// ===========================================================================
namespace {

struct StepRange {
  int fbegin, fcount;  // filters of this wavefront step (consecutive)
  int tbegin, tcount;  // tiles of this step
  int gbegin[4], gcount[4];   // scan workgroups of 1, 2, 4, 8 tiles of one orientation
};

struct DpDesc {        // one boundary-cut dynamic programme
  int axis;            // band axis a
  int rowaxis;         // axis along which the seam runs
  int sliceaxis;       // remaining axis (3D) or -1
  int slice;           // fixed coordinate on sliceaxis
};

struct Plan {
  Geom g;
  int n_orient = 0, n_shapes = 0, kpad = 0, W = 0;
  int scan_g_max = 1;                 // most tiles one scan workgroup may take (LDS)
  int learn = 0;                      // proposer dimension (0: plain scan)
  long long ws_pca_part = 0, ws_pca_cov = 0, ws_pca_mu = 0, ws_pca_P = 0, ws_emb = 0, ws_rn = 0, ws_qbuf = 0;
  long long learn_off = 0;            // finalize LDS offset of the row-rescoring area
  int learn_kbr = 0, learn_w = 0;
  size_t proxy_lds = 0;
  bool lp = false;                    // learned convolutional proposer (proposer_dim 64)
  int lp_kt = 1;                      // bytes per value of its LDS copy of the grid
  int lp_cap = 0;                     // candidates scored exactly per data event
  int lp_tmax = 0;                    // most scan tiles in one step
  size_t lp_lds = 0, lp_cmp_lds = 0;
  const void* lp_checked = nullptr;   // the index whose header was last read back
  long long ws_lp_grid = 0, ws_lp_sel = 0, ws_lp_ok = 0, ws_lp_map = 0, ws_lp_dtiles = 0, ws_lp_drecs = 0,
            ws_lp_dcount = 0;
  long long ws_err = 0;               // every patch's drawn candidate (for the match errors)
  int scan_g = 1;                     // tiles per scan workgroup (tuned)
  bool rows_ok = false;               // the row-minima selection fits this plan
  bool ev_delta = false;              // additive Haar data events (see k_event_init)
  bool sel_rows = false;              // row-minima selection chosen (tuned)
  bool sel_fused_ok = false;          // the scan may select per row itself (k_scan_sel)
  bool sel_fused = false;             // fused selection chosen (tuned)
  int sel_gbits = 0, sel_n_bm = 1;    // k_scan_sel: 2^gbits groups of a lane's values; band masks
  int sel_kk = 0, sel_W = 0;          // k_scan_sel: taps (16 per K-slice) and strip row length
  size_t sel_lds_nohd = 0, sel_lds_hd = 0;
  bool tuned = false;
  int max_slots = 0, nsteps_raster = 0;
  long long patches = 0, or_blocks = 0, band_cells = 0, succ_links = 0;
  long long hd_cap = 0;               // hard-data entries of all virtual templates
  bool hdm = false;                   // hard-data mismatches from the bit table
  HdmGeom hm = {};
  int nfilters = 0;
  std::vector<StepRange> steps;
  // host tables, uploaded on every call: built in pageable memory (so that
  // sizes and statistics need no device), copied to pinned memory the first
  // time a call uploads them
  size_t tbl_bytes = 0;
  std::vector<unsigned char> tbl_host;   // kbeta | nbt | filters | tiles | recs | npred | succ_off | succ
  unsigned char* tbl = nullptr;          // pinned copy of tbl_host, or null
  size_t off_segoff = 0, off_taps = 0;   // k_scan_sel segment tables, [orient][kSegMax] / [orient][kSegMax * 8]
  size_t off_kbeta = 0, off_nbt = 0, off_filters = 0, off_tiles = 0, off_recs = 0, off_groups = 0, off_npred = 0,
         off_succoff = 0, off_succ = 0;
  long long nrecs = 0;
  // workspace carve-up (bytes from the workspace base)
  long long ws_kh = 0, ws_ki = 0, ws_det = 0, ws_tmp = 0, ws_energy = 0, ws_tbl = 0, ws_sg = 0,
            ws_hdmap = 0, ws_mbuf = 0, ws_predcnt = 0, ws_report = 0, ws_hdoff = 0, ws_hdent = 0, ws_keys = 0, ws_rowmin = 0,
            ws_hdmask = 0, ws_hdbits = 0, ws_lift = 0, ws_rowcnt = 0,
            ws_total = 0;
  size_t scan_lds = 0, fin_lds = 0;
  long long buf_cells = 0, cand_cap = 0, coef_lds = 0;
  int tree_level = 0;   // 1, 2 (or 3 in 2D): block-subtree coefficients; 0: planar details
  int dp_stride = 0, dp_batch = 0, rows_max = 0, dp_wave = 0, dp_evs = 0;
  ~Plan() {
    if (tbl) (void)hipHostFree(tbl);
  }
};

// Plans are cached per parameter set (the seed included: it fixes the
// paths and tie-break keys baked into the tables), least recently used
// dropped first beyond kMaxPlans together with the graphs captured on them.
// A call keeps its plan alive through shared ownership.
std::mutex g_plan_mu;
struct PlanEntry {
  std::string key;
  std::shared_ptr<Plan> plan;
};
std::vector<PlanEntry> g_plans;   // most recent last
constexpr size_t kMaxPlans = 16;
void drop_graphs_of(const std::string& plan_key);   // defined with the graph cache

// path of realization r: perm[k] = lattice axis at path depth k (0 fastest),
// flip[a] = 1 when axis a is walked from its high end
void path_of(const ccwsim_params& p, int r, int perm[3], int flip[3]) {
  for (int a = 0; a < 3; ++a) {
    perm[a] = a;
    flip[a] = 0;
  }
  if (p.path_mode == 1) {
    const uint64_t u = draw64(p.seed, kStreamPath, (uint64_t)r, 0);
    for (int a = 0; a < p.ti.ndim; ++a) flip[a] = (int)((u >> a) & 1u);
    if (p.ti.ndim == 2 && ((u >> 3) & 1u)) {
      perm[0] = 1;
      perm[1] = 0;
    }
  }
}

// cell u of the window is in a band of (orient, bandmask)
bool in_band(const Geom& g, int orient, int bandmask, const int u[3]) {
  for (int a = 0; a < g.ndim; ++a) {
    if (!((bandmask >> a) & 1)) continue;
    const int w = ((orient >> a) & 1) ? g.T[a] - 1 - u[a] : u[a];
    if (w < g.OV[a]) return true;
  }
  return false;
}

int build_plan(const ccwsim_params& p, Plan& P) {
  Geom& g = P.g;
  CCW_TRY(geom_ti(g, p.ti, p.level));
  CCW_TRY(geom_tmpl(g, p.tmpl));
  CCW_TRY(geom_grid(g, p.grid, p.overlap, p.nc_margin));
  if (p.top_k < 1 || p.top_k > kTopMax) return fail(CCWSIM_ERR_UNSUPPORTED, "top_k must be in [1, %d]", kTopMax);
  if (p.n_real < 1) return fail(CCWSIM_ERR_INVALID_ARG, "n_real must be >= 1");
  if (p.n_facies < 1 || p.n_facies > 127) return fail(CCWSIM_ERR_INVALID_ARG, "n_facies must be in [1, 127]");
  if (p.path_mode != 0 && p.path_mode != 1) return fail(CCWSIM_ERR_INVALID_ARG, "path_mode");
  if (p.score_mode != 0 && p.score_mode != 1) return fail(CCWSIM_ERR_INVALID_ARG, "score_mode");
  if (p.cut != 0 && p.cut != 1) return fail(CCWSIM_ERR_INVALID_ARG, "cut");
  if (p.precision != 0 && p.precision != 1) return fail(CCWSIM_ERR_UNSUPPORTED, "precision %d", p.precision);
  if (p.shortlist != 0 && (p.shortlist < p.top_k || p.shortlist > kShortMax))
    return fail(CCWSIM_ERR_INVALID_ARG, "shortlist must be 0 or in [top_k, %d]", kShortMax);
  if (p.hd_direct != 0 && p.hd_direct != 1) return fail(CCWSIM_ERR_INVALID_ARG, "hd_direct must be 0 or 1");
  if (p.wavelet != 0 && p.wavelet != 1) return fail(CCWSIM_ERR_INVALID_ARG, "wavelet must be 0 (Haar) or 1 (5/3)");
  if (p.wavelet == 1 && (p.shortlist != 0 || p.proposer_dim != 0))
    return fail(CCWSIM_ERR_INVALID_ARG, "the 5/3 wavelet needs shortlist 0 and proposer_dim 0");
  if (p.proposer_dim == 64) {
    if (g.ndim != 2) return fail(CCWSIM_ERR_UNSUPPORTED, "the learned proposer runs on 2D training images");
    if (p.score_mode != 0) return fail(CCWSIM_ERR_UNSUPPORTED, "the learned proposer ranks squared-difference scores");
    if (p.shortlist != 0) return fail(CCWSIM_ERR_INVALID_ARG, "proposer_dim and shortlist exclude each other");
    if (!p.proposer) return fail(CCWSIM_ERR_INVALID_ARG, "proposer_dim 64 needs a proposer index");
    if (p.lp_probe < 1 || p.lp_probe > kLpProbeMax)
      return fail(CCWSIM_ERR_INVALID_ARG, "lp_probe must be in [1, %d]", kLpProbeMax);
    if (!(p.lp_gate == p.lp_gate)) return fail(CCWSIM_ERR_INVALID_ARG, "lp_gate is not a number");
  }
  g.wavelet = p.wavelet;
  if (p.wavelet == 1) g.shift = 1;
  if (p.max_hard_data < 0) return fail(CCWSIM_ERR_INVALID_ARG, "max_hard_data must be >= 0");
  if (p.proposer_dim != 0 && p.proposer_dim != 8 && p.proposer_dim != 16 && p.proposer_dim != 32 &&
      p.proposer_dim != 64)
    return fail(CCWSIM_ERR_INVALID_ARG, "proposer_dim must be 0, 8, 16, 32 or 64");
  if (p.proposer_dim && p.proposer_dim != 64) {
    if (p.score_mode != 0) return fail(CCWSIM_ERR_UNSUPPORTED, "the proposer bounds squared-difference scores only");
    if (p.shortlist != 0) return fail(CCWSIM_ERR_INVALID_ARG, "proposer_dim and shortlist exclude each other");
    if (g.tcells > kPcaMaxCells)
      return fail(CCWSIM_ERR_UNSUPPORTED, "the proposer supports templates of <= %d level-J blocks", kPcaMaxCells);
    if ((long long)g.cand[1] * g.cand[2] > 512)
      return fail(CCWSIM_ERR_UNSUPPORTED, "the proposer supports <= 512 candidate rows");
  }
  P.learn = p.proposer_dim == 64 ? 0 : p.proposer_dim;
  P.lp = p.proposer_dim == 64;
  const int nd = g.ndim;
  P.n_orient = 1 << nd;
  P.n_shapes = P.n_orient << nd;

  // overlap blocks per orientation: blocks touching any trailing band
  std::vector<std::vector<int>> klists(P.n_orient);
  int kmax_len = 0;
  long long ov_cells_max = 0;
  for (int o = 0; o < P.n_orient; ++o) {
    const int all = (1 << nd) - 1;
    long long cnt = 0;
    for (int bz = 0; bz < g.tc[2]; ++bz)
      for (int by = 0; by < g.tc[1]; ++by)
        for (int bx = 0; bx < g.tc[0]; ++bx) {
          bool hit = false;
          for (int uz = bz * g.b[2]; uz < std::min((bz + 1) * g.b[2], g.T[2]); ++uz)
            for (int uy = by * g.b[1]; uy < std::min((by + 1) * g.b[1], g.T[1]); ++uy)
              for (int ux = bx * g.b[0]; ux < std::min((bx + 1) * g.b[0], g.T[0]); ++ux) {
                const int u[3] = {ux, uy, uz};
                if (in_band(g, o, all, u)) {
                  hit = true;
                  ++cnt;
                }
              }
          if (hit) klists[o].push_back((bz * g.tc[1] + by) * g.tc[0] + bx);
        }
    kmax_len = std::max<int>(kmax_len, (int)klists[o].size());
    ov_cells_max = std::max(ov_cells_max, cnt);
  }
  P.kpad = std::max(16, (kmax_len + 15) / 16 * 16);
  if (P.kpad > kKMax) return fail(CCWSIM_ERR_UNSUPPORTED, "overlap spans %d blocks (> %d)", kmax_len, kKMax);
  if (p.wavelet == 1) {
    // 5/3 coefficients of codes in [0, max]: interval bound through the
    // J * ndim lifting passes (prediction, then update with rounding)
    long long lo = 0, hi = p.n_facies - 1 > 0 ? p.n_facies - 1 : 1;
    for (int k = 0; k < g.level * nd; ++k) {
      const long long dlo = lo - hi, dhi = hi - lo;
      const long long nlo = lo + floor_div(2 * dlo + 2, 4), nhi = hi + floor_div(2 * dhi + 2, 4);
      lo = nlo;
      hi = nhi;
    }
    const long long kb = std::max(-lo, hi);
    const long long lim = p.precision == 1 ? 256 : 2048;
    if (kb > lim)
      return fail(CCWSIM_ERR_UNSUPPORTED, "5/3 coefficients up to %lld are not exact in %s", kb,
                  p.precision == 1 ? "bf16" : "fp16");
    const long long cmax = (long long)kmax_len * kb * kb;
    if (cmax >= (1ll << 24)) return fail(CCWSIM_ERR_UNSUPPORTED, "cross sums up to %lld are not exact in fp32", cmax);
    if (3 * cmax >= (1ll << 31)) return fail(CCWSIM_ERR_UNSUPPORTED, "scores up to %lld overflow int32", 3 * cmax);
  } else {
    CCW_TRY(check_exact(g, p.n_facies - 1 > 0 ? p.n_facies - 1 : 1, ov_cells_max));
    if (p.precision == 1 && (long long)(p.n_facies > 1 ? p.n_facies - 1 : 1) * g.beta > 256)
      return fail(CCWSIM_ERR_UNSUPPORTED, "block sums up to %lld are not exact in bf16",
                  (long long)(p.n_facies - 1) * g.beta);
  }
  P.W = scan_strip_width(g);

  // schedule: anti-diagonal wavefronts when same-step windows are disjoint
  bool wave_ok = true;
  for (int a = 0; a < nd; ++a) wave_ok = wave_ok && g.T[a] >= 2 * g.OV[a];
  const long long nsteps = (long long)g.lat[0] * g.lat[1] * g.lat[2];
  if (nsteps > (1ll << 30)) return fail(CCWSIM_ERR_UNSUPPORTED, "lattice too large");
  P.nsteps_raster = (int)nsteps;
  std::vector<std::vector<FilterDev>> by_t;
  for (int r = 0; r < p.n_real; ++r) {
    int perm[3], flip[3];
    path_of(p, r, perm, flip);
    const int plen[3] = {g.lat[perm[0]], g.lat[perm[1]], g.lat[perm[2]]};
    int orient = 0;
    for (int a = 0; a < nd; ++a) orient |= flip[a] << a;
    for (long long s = 0; s < nsteps; ++s) {
      const int q[3] = {(int)(s % plen[0]), (int)((s / plen[0]) % plen[1]), (int)(s / ((long long)plen[0] * plen[1]))};
      FilterDev f = {};
      f.r = r;
      f.step = (int)s;
      int li[3];
      int bm = 0;
      for (int k = 0; k < 3; ++k) {
        const int a = perm[k];
        li[a] = flip[a] ? g.lat[a] - 1 - q[k] : q[k];
        if (a < nd && q[k] > 0) bm |= 1 << a;
      }
      for (int a = 0; a < 3; ++a) f.org[a] = li[a] * g.stride[a];
      f.orient = orient;
      f.bandmask = bm;
      f.shape = (orient << nd) | bm;
      const long long t = wave_ok ? (long long)q[0] + 2ll * q[1] + 4ll * q[2] : s;
      if ((long long)by_t.size() <= t) by_t.resize(t + 1);
      by_t[t].push_back(f);
    }
  }
  // Scan LDS for one tile per workgroup; up to 8 tiles of one orientation
  // may share a workgroup (and its A gather) when the LDS allows.
  {
    int kl = 0;
    for (int o = 0; o < P.n_orient; ++o) kl = std::max<int>(kl, (int)klists[o].size());
    P.kpad = std::max(16, (kl + 15) / 16 * 16);
    const int nrows = g.tc[1] * g.tc[2];
    P.scan_g_max = 1;
    for (int G : {2, 4, 8})
      if (!P.learn && P.kpad <= kScanGroupKMax && scan_group_lds(nrows, P.W, P.kpad, G) <= 64 * 1024)
        P.scan_g_max = G;
    P.scan_lds = scan_group_lds(nrows, P.W, P.kpad, 1);
    if (P.scan_lds > 64 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "scan strip needs %zu B of LDS", P.scan_lds);
  }

  // overlap blocks holding known cells, per shape (the method's K dimension)
  std::vector<int> shape_blocks(P.n_shapes, 0);
  for (int sh = 0; sh < P.n_shapes; ++sh) {
    const int o = sh >> nd, bm = sh & ((1 << nd) - 1);
    for (int bz = 0; bz < g.tc[2]; ++bz)
      for (int by = 0; by < g.tc[1]; ++by)
        for (int bx = 0; bx < g.tc[0]; ++bx) {
          bool hit = false;
          for (int uz = bz * g.b[2]; uz < std::min((bz + 1) * g.b[2], g.T[2]) && !hit; ++uz)
            for (int uy = by * g.b[1]; uy < std::min((by + 1) * g.b[1], g.T[1]) && !hit; ++uy)
              for (int ux = bx * g.b[0]; ux < std::min((bx + 1) * g.b[0], g.T[0]) && !hit; ++ux) {
                const int u[3] = {ux, uy, uz};
                hit = in_band(g, o, bm, u);
              }
          shape_blocks[sh] += hit;
        }
  }
  // overlap cells per shape
  std::vector<int> shape_cells(P.n_shapes, 0);
  for (int sh = 0; sh < P.n_shapes; ++sh) {
    const int o = sh >> nd, bm = sh & ((1 << nd) - 1);
    for (int uz = 0; uz < g.T[2]; ++uz)
      for (int uy = 0; uy < g.T[1]; ++uy)
        for (int ux = 0; ux < g.T[0]; ++ux) {
          const int u[3] = {ux, uy, uz};
          shape_cells[sh] += in_band(g, o, bm, u);
        }
  }
  std::vector<FilterDev> filters;
  std::vector<TileDev> tiles;
  std::vector<ScanRec> recs;
  std::vector<int2> groups;   // (first tile within the step, tiles)
  for (auto& lst : by_t) {
    for (const FilterDev& f : lst) {
      P.patches += 1;
      P.or_blocks += shape_blocks[f.shape];
      P.band_cells += shape_cells[f.shape];
    }
    if (lst.empty()) continue;   // e.g. odd t when the fast path axis has one patch
    std::stable_sort(lst.begin(), lst.end(), [](const FilterDev& x, const FilterDev& y) { return x.orient < y.orient; });
    StepRange sr;
    sr.fbegin = (int)filters.size();
    sr.fcount = (int)lst.size();
    sr.tbegin = (int)tiles.size();
    for (size_t i = 0; i < lst.size();) {
      size_t e = i;
      while (e < lst.size() && lst[e].orient == lst[i].orient && (int)(e - i) < kFiltersPerTile) ++e;
      uint32_t zm = 0;
      for (size_t q = i; q < e; ++q) zm |= (lst[q].bandmask == 0 ? 1u : 0u) << (q - i);
      TileDev t = {(int)i, (int)(e - i), lst[i].orient, zm};
      tiles.push_back(t);
      i = e;
    }
    sr.tcount = (int)tiles.size() - sr.tbegin;
    for (int gi = 0; gi < 4; ++gi) {
      const int G = 1 << gi;
      sr.gbegin[gi] = (int)groups.size();
      for (int k = sr.tbegin; k < sr.tbegin + sr.tcount;) {
        int e = k + 1;
        while (e < sr.tbegin + sr.tcount && e - k < G && tiles[e].orient == tiles[k].orient) ++e;
        groups.push_back({k - sr.tbegin, e - k});
        k = e;
      }
      sr.gcount[gi] = (int)groups.size() - sr.gbegin[gi];
    }
    for (int k = sr.tbegin; k < sr.tbegin + sr.tcount; ++k)
      for (int jj = 0; jj < kFiltersPerTile; ++jj) {
        ScanRec r = {-1, 0, 0, 0, 0};
        if (jj < tiles[k].count) {
          const FilterDev& f = lst[tiles[k].first + jj];
          r.gidx = sr.fbegin + tiles[k].first + jj;
          r.shape = f.shape;
          r.tkey = draw64(p.seed, kStreamTiebreak, (uint64_t)f.r, (uint64_t)f.step);
        }
        recs.push_back(r);
      }
    filters.insert(filters.end(), lst.begin(), lst.end());
    P.max_slots = std::max(P.max_slots, sr.fcount);
    P.steps.push_back(sr);
  }

  // Overlapping predecessors / successors of every patch.  A patch's overlap
  // cells are final once every earlier patch whose window overlaps it has
  // pasted; the last of them computes the patch's data event.
  P.nfilters = (int)filters.size();
  std::vector<int32_t> npred(filters.size(), 0), succ_off(filters.size() + 1, 0), succ;
  {
    const long long latc = (long long)g.lat[0] * g.lat[1] * g.lat[2];
    std::vector<int32_t> at((size_t)p.n_real * latc, -1);
    auto lat_of = [&](const FilterDev& f, int li[3]) {
      for (int a = 0; a < 3; ++a) li[a] = f.org[a] / g.stride[a];
    };
    for (size_t i = 0; i < filters.size(); ++i) {
      int li[3];
      lat_of(filters[i], li);
      at[(size_t)filters[i].r * latc + ((long long)li[2] * g.lat[1] + li[1]) * g.lat[0] + li[0]] = (int32_t)i;
    }
    int reach[3];
    for (int a = 0; a < 3; ++a) reach[a] = a < nd ? (g.T[a] - 1) / g.stride[a] : 0;  // |d| * s < T
    std::vector<std::vector<int32_t>> sl(filters.size());
    for (size_t i = 0; i < filters.size(); ++i) {
      int li[3];
      lat_of(filters[i], li);
      for (int dz = -reach[2]; dz <= reach[2]; ++dz)
        for (int dy = -reach[1]; dy <= reach[1]; ++dy)
          for (int dx = -reach[0]; dx <= reach[0]; ++dx) {
            if (!dx && !dy && !dz) continue;
            const int n[3] = {li[0] + dx, li[1] + dy, li[2] + dz};
            bool in = true;
            for (int a = 0; a < 3; ++a) in = in && n[a] >= 0 && n[a] < g.lat[a];
            if (!in) continue;
            const int32_t j = at[(size_t)filters[i].r * latc + ((long long)n[2] * g.lat[1] + n[1]) * g.lat[0] + n[0]];
            if (filters[j].step < filters[i].step) {
              npred[i] += 1;
              sl[j].push_back((int32_t)i);
            }
          }
    }
    for (size_t i = 0; i < filters.size(); ++i) {
      if (sl[i].size() > 64) return fail(CCWSIM_ERR_UNSUPPORTED, "a patch overlaps more than 64 later patches");
      succ_off[i + 1] = succ_off[i] + (int32_t)sl[i].size();
      filters[i].succ0 = succ_off[i];
      filters[i].nsucc = (int32_t)sl[i].size();
    }
    for (size_t i = 0; i < filters.size(); ++i)
      for (int32_t q : sl[i]) {
        succ.push_back(q);
        succ.push_back(npred[q]);
      }
    P.succ_links = (long long)succ.size() / 2;
    if (succ.empty()) {
      succ.push_back(-1);
      succ.push_back(0);
    }
  }

  // energy rows: known-cell count per block for each (orient, bandmask)
  std::vector<int32_t> nbt((size_t)P.n_shapes * g.tcells, 0);
  for (int sh = 0; sh < P.n_shapes; ++sh) {
    const int o = sh >> nd, bm = sh & ((1 << nd) - 1);
    for (int uz = 0; uz < g.T[2]; ++uz)
      for (int uy = 0; uy < g.T[1]; ++uy)
        for (int ux = 0; ux < g.T[0]; ++ux) {
          const int u[3] = {ux, uy, uz};
          if (!in_band(g, o, bm, u)) continue;
          const long long bi = ((long long)(uz / g.b[2]) * g.tc[1] + uy / g.b[1]) * g.tc[0] + ux / g.b[0];
          nbt[(size_t)sh * g.tcells + bi] += 1;
        }
    if (p.wavelet == 1)   // 5/3: every block with a known cell compares one coefficient
      for (long long i = 0; i < g.tcells; ++i) nbt[(size_t)sh * g.tcells + i] = nbt[(size_t)sh * g.tcells + i] > 0;
  }
  std::vector<int32_t> kbeta((size_t)P.n_orient * kKMax, -1);
  for (int o = 0; o < P.n_orient; ++o)
    for (size_t i = 0; i < klists[o].size(); ++i) kbeta[(size_t)o * kKMax + i] = klists[o][i];
  // fused scan: the overlap blocks of each orientation covered by segments
  // of 8 consecutive blocks of one block row (greedy from the row's first
  // uncovered block); each tap names its entry of the block list, or -1
  std::vector<int32_t> segoff((size_t)P.n_orient * kSegMax, 0), taps((size_t)P.n_orient * kSegMax * 8, -1);
  {
    const int cpad = ((g.cand[0] + 31) / 32) * 32;
    P.sel_W = scan_sel_width(cpad, g.tc[0]);
    int nseg_max = 0;
    bool fits = true;
    for (int o = 0; o < P.n_orient; ++o) {
      std::map<int, std::vector<std::pair<int, int>>> rows;   // block row -> (bx, list entry)
      for (size_t i = 0; i < klists[o].size(); ++i) {
        const int beta = klists[o][i];
        const int bx = beta % g.tc[0], rr = beta / g.tc[0];
        rows[rr].push_back({bx, (int)i});
      }
      int ns = 0;
      for (auto& kv : rows) {
        std::vector<std::pair<int, int>>& v = kv.second;
        std::sort(v.begin(), v.end());
        size_t i = 0;
        while (i < v.size()) {
          const int bx0 = v[i].first;
          if (ns < kSegMax) segoff[(size_t)o * kSegMax + ns] = kv.first * P.sel_W + bx0;
          for (; i < v.size() && v[i].first < bx0 + 8; ++i)
            if (ns < kSegMax) taps[((size_t)o * kSegMax + ns) * 8 + (v[i].first - bx0)] = v[i].second;
          ++ns;
        }
      }
      nseg_max = std::max(nseg_max, ns);
      fits = fits && ns <= kSegMax;
    }
    const int ks = std::max(4, ((nseg_max + 1) / 2 + 3) / 4 * 4);   // K-slices, a multiple of 4
    P.sel_kk = fits && ks <= kSegMax / 2 ? 16 * ks : 0;
  }

  // the coefficient tree layout serves J = 1 and 2, and J = 3 in 2D
  P.tree_level = p.wavelet == 0 && (g.level == 1 || g.level == 2 || (g.level == 3 && nd == 2)) ? g.level : 0;

  // finalize LDS: idwt buffers, pattern, keep mask, grid and hard-data
  // windows, keys of the best rows, cut scratch
  P.buf_cells = idwt_buf_cells(g);
  if (p.wavelet == 1) {
    // the successors' 5/3 windows (tc * b cells per axis) are lifted in
    // LDS: 7 rc / 4 int16 values (the window and two pass buffers) over
    // the idwt buffers and the four window-sized byte arrays behind them
    long long rc = 1;
    for (int a = 0; a < 3; ++a) rc *= (long long)g.tc[a] * g.b[a];
    const long long wpad5 = (g.wcells + 15) & ~15ll;
    const long long need = (7 * rc / 4 + 16) * 2;
    P.buf_cells = std::max(P.buf_cells, (need - 4 * wpad5 + 7) / 8);
  }
  const long long wpad = (g.wcells + 15) & ~15ll;
  int maxcols = 1;
  P.rows_max = 1;
  for (int a = 0; a < nd; ++a) {
    const int ra = a == 0 ? 1 : 0;
    P.rows_max = std::max(P.rows_max, g.T[ra]);
    maxcols = std::max(maxcols, g.OV[a]);
  }
  P.dp_wave = maxcols <= 16 && P.rows_max <= kSeamRowsMax;
  const int ksel = std::min(p.shortlist > 0 ? p.shortlist : p.top_k, g.ncand);
  const long long cand_bytes = (long long)ksel * g.cand[0] * 8;
  P.cand_cap = cand_bytes <= 24 * 1024 ? (long long)ksel * g.cand[0] : 0;
  if (ksel > kTopMax && (P.cand_cap == 0 || (long long)g.cand[1] * g.cand[2] > P.cand_cap))
    return fail(CCWSIM_ERR_UNSUPPORTED, "shortlist of %d needs %lld B of keys in LDS", ksel, cand_bytes);
  if (P.learn) P.cand_cap = 0;   // the proposer's selection has its own area
  const size_t fixed = (size_t)P.buf_cells * 8 + 4 * (size_t)wpad + (size_t)P.cand_cap * 8;
  const long long budget = 60 * 1024;
  if (P.dp_wave) {
    // squared differences of the seams, [wave][column][step] with a padded
    // step stride; the area begins at the key list, which is free by then
    P.dp_evs = (int)(((P.rows_max + 7) & ~7) + 4);
    const long long ev_bytes = 4ll * 16 * P.dp_evs * 4 + 16;
    P.dp_stride = (int)align256(std::max<long long>(256, ev_bytes - P.cand_cap * 8));
    P.dp_batch = 1;
  } else {
    P.dp_stride = (int)align256((long long)P.rows_max * maxcols + (long long)maxcols * 8 + 16);
    P.dp_batch = (int)std::min<long long>(kThreads, (budget - (long long)fixed) / P.dp_stride);
  }
  if (P.dp_batch < 1 || (long long)fixed + (long long)P.dp_stride * P.dp_batch > budget)
    return fail(CCWSIM_ERR_UNSUPPORTED, "pattern reconstruction needs more than %lld B of LDS", budget);
  P.fin_lds = fixed + (size_t)P.dp_batch * P.dp_stride + (size_t)((2 * g.tcells * 4 + 15) & ~15ll);
  const bool rows_try = !P.learn && p.score_mode == 0 && p.shortlist == 0 && p.wavelet == 0 &&
                        (long long)g.cand[1] * g.cand[2] <= 512 && P.kpad <= kKMax;
  if (P.learn || rows_try) {
    // rows by bound, the keys of a round of rows and their level-J rows (int16)
    const long long nrows = (long long)g.cand[1] * g.cand[2];
    P.learn_w = (int)((g.cand[0] + g.tc[0] - 1 + 1) & ~1);
    P.learn_off = (long long)((P.fin_lds + 15) & ~(size_t)15);
    // rows per round: with exact row minima the k best need at most k rows
    const int kbr_max = P.learn ? 4 : std::min(16, std::max(1, std::min(p.top_k, g.ncand)));
    for (P.learn_kbr = kbr_max; P.learn_kbr >= 1; --P.learn_kbr) {
      const long long bytes = nrows * 8 + ((nrows + 1) & ~1ll) * 4 + (long long)P.learn_kbr * g.cand[0] * 8 +
                              (long long)P.learn_kbr * g.tc[1] * g.tc[2] * P.learn_w * 2;
      if (P.learn_off + bytes <= 64 * 1024) {
        P.fin_lds = (size_t)(P.learn_off + bytes);
        break;
      }
    }
    if (P.learn && P.learn_kbr < 1) return fail(CCWSIM_ERR_UNSUPPORTED, "proposer row rescoring does not fit the LDS");
    P.rows_ok = rows_try && P.learn_kbr >= 1;
  }
  if (P.fin_lds > 64 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "finalize needs %zu B of LDS", P.fin_lds);
  // Selection fused into the scan (k_scan_sel): a lane's values fall into
  // 2^gbits groups; the fewest groups that still give every patch at least
  // ksel groups holding a candidate.
  {
    const int nchunks = (g.cand[0] + 31) / 32;
    P.sel_gbits = sel_group_bits(g.cand[0], nchunks, ksel);
    P.sel_n_bm = 1 << nd;
    const int nr = g.tc[1] * g.tc[2];
    P.sel_lds_nohd = scan_sel_lds(nr, P.sel_W, P.sel_kk, P.kpad, kEnStage, P.sel_n_bm, nchunks * 32, P.sel_gbits, false);
    P.sel_lds_hd = scan_sel_lds(nr, P.sel_W, P.sel_kk, P.kpad, kEnStage, P.sel_n_bm, nchunks * 32, P.sel_gbits, true);
    P.sel_fused_ok = !P.learn && g.cand[0] <= 4096 && P.cand_cap > 0 && P.sel_kk > 0 &&
                     std::max(P.sel_lds_nohd, P.sel_lds_hd) <= 64 * 1024 && !(p.max_hard_data > 0 && p.hd_direct);
  }
  // additive data events: the Haar block sums of a successor's overlap
  // change by what each predecessor's paste changes there; the sums of one
  // group of successors live in the inverse-DWT buffers, free by then
  P.ev_delta = p.wavelet == 0 && !P.learn && g.level > 0 && 2 * P.buf_cells >= g.tcells;
  // the coefficient staging area aliases the key list and the cut scratch
  const long long alias_bytes = P.cand_cap * 8 + (long long)P.dp_batch * P.dp_stride;
  P.coef_lds = p.wavelet == 0 && !P.tree_level && g.level > 0 && P.cand_cap > 0 &&
               idwt_coef_count(g) * 4 <= alias_bytes;

  // pinned table block
  P.off_kbeta = 0;
  P.off_segoff = align256(kbeta.size() * 4);
  P.off_taps = P.off_segoff + align256(segoff.size() * 4);
  P.off_nbt = P.off_taps + align256(taps.size() * 4);
  P.off_filters = P.off_nbt + align256(nbt.size() * 4);
  P.off_tiles = P.off_filters + align256(filters.size() * sizeof(FilterDev));
  P.off_recs = P.off_tiles + align256(tiles.size() * sizeof(TileDev));
  P.off_groups = P.off_recs + align256(recs.size() * sizeof(ScanRec));
  P.off_npred = P.off_groups + align256(groups.size() * sizeof(int2));
  P.nrecs = (long long)recs.size();
  P.off_succoff = P.off_npred + align256(npred.size() * 4);
  P.off_succ = P.off_succoff + align256(succ_off.size() * 4);
  P.tbl_bytes = P.off_succ + align256(succ.size() * 4);
  P.tbl_host.assign(P.tbl_bytes, 0);
  unsigned char* tb = P.tbl_host.data();
  memcpy(tb + P.off_kbeta, kbeta.data(), kbeta.size() * 4);
  memcpy(tb + P.off_segoff, segoff.data(), segoff.size() * 4);
  memcpy(tb + P.off_taps, taps.data(), taps.size() * 4);
  memcpy(tb + P.off_nbt, nbt.data(), nbt.size() * 4);
  memcpy(tb + P.off_filters, filters.data(), filters.size() * sizeof(FilterDev));
  memcpy(tb + P.off_tiles, tiles.data(), tiles.size() * sizeof(TileDev));
  memcpy(tb + P.off_recs, recs.data(), recs.size() * sizeof(ScanRec));
  memcpy(tb + P.off_groups, groups.data(), groups.size() * sizeof(int2));
  memcpy(tb + P.off_npred, npred.data(), npred.size() * 4);
  memcpy(tb + P.off_succoff, succ_off.data(), succ_off.size() * 4);
  memcpy(tb + P.off_succ, succ.data(), succ.size() * 4);

  // hard data: a grid cell lies in the virtual templates of at most
  // prod ceil((T + margin) / stride) patches of its realization
  long long per_cell = 1;
  for (int a = 0; a < nd; ++a) per_cell *= (g.T[a] + g.margin[a] + g.stride[a] - 1) / g.stride[a];
  P.hd_cap = (long long)p.max_hard_data * per_cell;

  // hard-data bit table: rows padded by the virtual-template margins, x
  // positions from floor(-margin / 2^J) to the last chunk's reach
  if (p.max_hard_data > 0 && !p.hd_direct) {
    HdmGeom& m = P.hm;
    const int bx = g.b[0];
    const int mx = g.margin[0], my = g.margin[1], mz = nd == 3 ? g.margin[2] : 0;
    const int nchunks = (g.cand[0] + 31) / 32;
    m.pb = (mx + bx - 1) / bx;
    const int avmax = (g.T[0] + mx - 1) / bx;
    m.nw = nchunks + ((avmax + m.pb) >> 5) + 2;
    m.py0 = my;
    m.ry = m.py0 + std::max(g.ti[1], (g.cand[1] - 1) * g.b[1] + g.T[1] + my);
    m.pz0 = mz;
    m.rz = m.pz0 + std::max(g.ti[2], (g.cand[2] - 1) * g.b[2] + g.T[2] + mz);
    m.nf = p.n_facies;
    m.ns = p.n_facies + 1;
    const long long rs = (long long)bx * m.ns * m.nw;
    const long long bytes = (long long)m.rz * m.ry * rs * 4;
    if (bytes <= (1ll << 30)) {
      m.rs = (int)rs;
      P.hdm = true;
    }
  }
  if (p.max_hard_data > 0 && !P.hdm) P.sel_fused_ok = false;   // its mismatches come from the bit table
  P.sel_fused = P.sel_fused_ok;   // before tuning
  if (P.lp) {
    // the patches the gate sends back go through the fused scan; the
    // proposal keeps the level-J grid in LDS as int8 or int16
    if (!P.sel_fused_ok)
      return fail(CCWSIM_ERR_UNSUPPORTED, "the learned proposer needs the selection fused into the scan");
    const long long kmax = (long long)(p.n_facies - 1) * g.beta;
    P.lp_kt = kmax <= 127 ? 1 : kmax <= 32767 ? 2 : 0;
    if (!P.lp_kt) return fail(CCWSIM_ERR_UNSUPPORTED, "block sums up to %lld exceed int16", kmax);
    P.lp_cap = kLpCandMax;
    P.lp_lds = (size_t)lp_prop_lds(g, P.lp_kt, P.lp_cap, P.kpad);
    if (P.lp_lds > 160 * 1024)
      return fail(CCWSIM_ERR_UNSUPPORTED, "the proposal needs %zu B of LDS (level-J grid too large)", P.lp_lds);
    for (const StepRange& sr : P.steps) P.lp_tmax = std::max(P.lp_tmax, sr.tcount);
    if (P.lp_tmax > 256) return fail(CCWSIM_ERR_UNSUPPORTED, "more than 256 scan tiles in one step");
    // the step's last proposal packs the gated patches in its LDS
    P.lp_cmp_lds = (size_t)P.max_slots * 16 + 1024;
    P.lp_lds = std::max(P.lp_lds, P.lp_cmp_lds);
    if (P.lp_lds > 160 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "too many patches in one step");
  }

  // workspace
  const long long gcells = (long long)g.G[0] * g.G[1] * g.G[2];
  const long long c1 = g.level >= 2 ? (long long)g.Gj[1][0] * g.Gj[1][1] * g.Gj[1][2] : 0;
  long long o = 0;
  P.ws_kh = o;        o += align256(gcells * 2);
  P.ws_ki = o;        o += align256(gcells * 4);
  P.ws_det = o;       o += align256(std::max(1ll, P.tree_level ? (long long)g.np[0] * g.np[1] * g.np[2] : g.det_total) * 4);
  P.ws_tmp = o;       o += align256(2 * c1 * 4);
  P.ws_energy = o;    o += align256((long long)P.n_shapes * g.ncand * 4);
  P.ws_tbl = o;       o += align256((long long)P.tbl_bytes);
  P.ws_sg = o;        o += align256((long long)p.n_real * g.pcells + 16);   // slack: window rows are read in 8-byte words
  P.ws_hdmap = o;     o += align256((long long)p.n_real * g.pcells + 16);
  P.ws_mbuf = o;      o += align256((long long)P.nfilters * kKMax * 4);
  P.ws_predcnt = o;   o += align256((long long)P.nfilters * 4);
  P.ws_report = o;    o += 256;
  P.ws_hdoff = o;     o += align256((long long)(P.nfilters + 1) * 4);
  P.ws_hdent = o;     o += align256(std::max(1ll, P.hd_cap) * (long long)sizeof(HdEnt));
  if (p.wavelet == 1) {   // two lifting buffers of half the padded TI each
    P.ws_lift = o;      o += 2 * align256(((long long)g.np[0] * g.np[1] * g.np[2] / 2 + 1) * 4);
  }
  if (P.hdm) {
    P.ws_hdmask = o;  o += align256((long long)P.hm.rz * P.hm.ry * P.hm.rs * 4);
    P.ws_hdbits = o;  o += align256(std::max(1ll, P.hd_cap) * (long long)sizeof(HdBits));
  }
  P.ws_keys = o;      o += align256((long long)P.max_slots * g.ncand * 8);
  P.ws_rowmin = o;    o += align256((long long)P.max_slots * g.cand[1] * g.cand[2] * 8);
  P.ws_rowcnt = o;    o += align256((long long)P.max_slots * g.cand[1] * g.cand[2] * 4);
  P.ws_err = o;       o += align256((long long)P.nfilters * 4);
  if (P.lp) {
    P.ws_lp_grid = o;   o += align256(lp_prop_grid_bytes(g, P.lp_kt));
    P.ws_lp_sel = o;    o += align256((long long)P.max_slots * p.top_k * 8);
    P.ws_lp_ok = o;     o += align256((long long)P.max_slots * 4);
    P.ws_lp_map = o;    o += align256((long long)P.max_slots * 4);
    P.ws_lp_dtiles = o; o += align256((long long)std::max(1, P.lp_tmax) * sizeof(TileDev));
    P.ws_lp_drecs = o;  o += align256((long long)std::max(1, P.lp_tmax) * kFiltersPerTile * sizeof(ScanRec));
    P.ws_lp_dcount = o; o += 256;
  }
  if (P.learn) {
    const long long n = g.tcells;
    P.ws_pca_part = o;  o += align256((long long)kPcaParts * (n * n + n) * 4);
    P.ws_pca_cov = o;   o += align256(n * n * 4);
    P.ws_pca_mu = o;    o += align256(n * 4);
    P.ws_pca_P = o;     o += align256((long long)P.learn * n * 4);
    P.ws_emb = o;       o += align256(g.ncand * P.learn * 4);
    P.ws_rn = o;        o += align256(g.ncand * 8);
    P.ws_qbuf = o;      o += align256((long long)P.nfilters * (P.learn + 4) * 8);
    P.proxy_lds = (size_t)g.cand[0] * P.learn * 4 + (size_t)g.cand[0] * 8;
    if (P.proxy_lds > 64 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "proposer scan needs %zu B of LDS", P.proxy_lds);
  }
  P.ws_total = o;

  return CCWSIM_OK;
}

int get_plan(const ccwsim_params& p, std::shared_ptr<Plan>* out) {
  std::string key((const char*)&p, sizeof p);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (size_t i = 0; i < g_plans.size(); ++i) {
    if (g_plans[i].key == key) {
      PlanEntry e = g_plans[i];
      g_plans.erase(g_plans.begin() + i);
      g_plans.push_back(e);
      *out = e.plan;
      return CCWSIM_OK;
    }
  }
  std::shared_ptr<Plan> P(new Plan);
  CCW_TRY(build_plan(p, *P));
  if (g_plans.size() >= kMaxPlans) {
    drop_graphs_of(g_plans.front().key);
    g_plans.erase(g_plans.begin());
  }
  g_plans.push_back({key, P});
  *out = P;
  return CCWSIM_OK;
}

// The pinned copy of a plan's tables (made once, on the first call that
// uploads them).
int plan_pin(Plan* P) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (P->tbl) return CCWSIM_OK;
  unsigned char* t = nullptr;
  if (hipHostMalloc((void**)&t, P->tbl_bytes, hipHostMallocDefault) != hipSuccess)
    return fail(CCWSIM_ERR_HIP, "hipHostMalloc of %zu bytes failed", P->tbl_bytes);
  memcpy(t, P->tbl_host.data(), P->tbl_bytes);
  P->tbl = t;
  return CCWSIM_OK;
}

// ---- simple per-call kernels ---------------------------------------------
__global__ void k_fill_i8(int8_t* __restrict__ p, long long n, int8_t v) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = v;
}

__global__ void k_scatter_hd(int8_t* __restrict__ sg, int8_t* __restrict__ hdmap, Geom g, int n_real,
                             long long n_hd, const int32_t* __restrict__ hr, const int32_t* __restrict__ hp,
                             const int8_t* __restrict__ hv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hd) return;
  const int r = hr[i];
  const int x = hp[3 * i], y = hp[3 * i + 1], z = hp[3 * i + 2];
  if (r < 0 || r >= n_real || x < 0 || y < 0 || z < 0 || x >= g.sg[0] || y >= g.sg[1] || z >= g.sg[2]) return;
  const long long at = (long long)r * g.pcells + idx3(x, y, z, g.pad);
  sg[at] = hv[i];
  hdmap[at] = hv[i];
}

__global__ void k_crop(const int8_t* __restrict__ sg, int8_t* __restrict__ out, Geom g, int n_real) {
  const long long cells = (long long)g.sg[0] * g.sg[1] * g.sg[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cells * n_real) return;
  const long long r = id / cells, c = id - r * cells;
  const int x = (int)(c % g.sg[0]), y = (int)((c / g.sg[0]) % g.sg[1]), z = (int)(c / ((long long)g.sg[0] * g.sg[1]));
  out[id] = sg[r * g.pcells + idx3(x, y, z, g.pad)];
}

// ---- data events (Algorithm 1: extract the overlap, its level-J DWT) ------
__device__ __forceinline__ bool dev_in_band(const Geom& g, int orient, int bandmask, int ux, int uy, int uz) {
  const int u[3] = {ux, uy, uz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= g.ndim || !((bandmask >> a) & 1)) continue;
    const int w = ((orient >> a) & 1) ? g.T[a] - 1 - u[a] : u[a];
    if (w < g.OV[a]) return true;
  }
  return false;
}

// Data events of every patch on the grid as it stands before the first
// step: per level-J block, the sum of the overlap cells (unknown cells hold
// -1, hard data their code).  The finalize step of each patch then adds,
// block by block, what its paste changes in its successors' overlaps.  Both
// are integer sums, so the order of the additions does not matter and a
// successor's scan reads the block sums of exactly the cells its
// predecessors left (Sec. 3.2: the data event is the level-J approximation
// of the overlap, a block sum for the Haar filters).  One workgroup per patch.
__global__ __launch_bounds__(kThreads) void k_event_init(Geom g, const FilterDev* __restrict__ filters,
                                                         const int32_t* __restrict__ kbeta,
                                                         const int8_t* __restrict__ sg, int32_t* __restrict__ mbuf,
                                                         int kpad) {
  extern __shared__ int s_bsum[];   // [window block]
  const FilterDev fq = filters[blockIdx.x];
  const int tid = threadIdx.x;
  for (int i = tid; i < (int)g.tcells; i += kThreads) s_bsum[i] = 0;
  __syncthreads();
  if (fq.bandmask) {
    const int8_t* sgq = sg + (long long)fq.r * g.pcells;
    const int lb = g.level, lbz = g.ndim == 3 ? g.level : 0;
    BoxWalk w(tid, kThreads, g.T[0], g.T[1]);
    for (int i = tid; i < (int)g.wcells; i += kThreads, w.next())
      if (dev_in_band(g, fq.orient, fq.bandmask, w.x, w.y, w.z))
        atomicAdd(&s_bsum[((w.z >> lbz) * g.tc[1] + (w.y >> lb)) * g.tc[0] + (w.x >> lb)],
                  (int)sgq[idx3(fq.org[0] + w.x, fq.org[1] + w.y, fq.org[2] + w.z, g.pad)]);
  }
  __syncthreads();
  for (int t = tid; t < kKMax; t += kThreads) {
    const int beta = t < kpad ? kbeta[fq.orient * kKMax + t] : -1;
    mbuf[(long long)blockIdx.x * kKMax + t] = beta >= 0 ? s_bsum[beta] : 0;
  }
}

// Copy the T-window of a padded grid at `org` into LDS (every load of a
// thread is issued before its stores).
__device__ __forceinline__ void load_window(int8_t* dst, const int8_t* __restrict__ grid, const int org[3],
                                            const Geom& g) {
  constexpr int U = 8;
  const int n = (int)g.wcells;
  BoxWalk w(threadIdx.x, kThreads, g.T[0], g.T[1]);
  for (int base = threadIdx.x; base < n; base += kThreads * U) {
    int8_t v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = base + q * kThreads;
      v[q] = 0;
      if (i < n) v[q] = grid[idx3(org[0] + w.x, org[1] + w.y, org[2] + w.z, g.pad)];
      w.next();
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = base + q * kThreads;
      if (i < n) dst[i] = v[q];
    }
  }
}

// Both windows (grid and hard-data map) in one pass; without hard data the
// second window is filled with -1.
__device__ __forceinline__ void load_windows(int8_t* d0, const int8_t* __restrict__ g0, int8_t* d1,
                                             const int8_t* __restrict__ g1, const int org[3], const Geom& g) {
  constexpr int U = 8;
  const int n = (int)g.wcells;
  BoxWalk w(threadIdx.x, kThreads, g.T[0], g.T[1]);
  for (int base = threadIdx.x; base < n; base += kThreads * U) {
    int8_t v0[U], v1[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = base + q * kThreads;
      v0[q] = 0;
      v1[q] = -1;
      if (i < n) {
        const long long at = idx3(org[0] + w.x, org[1] + w.y, org[2] + w.z, g.pad);
        v0[q] = g0[at];
        if (g1) v1[q] = g1[at];
      }
      w.next();
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = base + q * kThreads;
      if (i < n) {
        d0[i] = v0[q];
        d1[i] = v1[q];
      }
    }
  }
}

// Virtual template of patch f (template extended by the margin on the
// sides not yet simulated), clipped to the padded grid: origin lo, extent ext.
__device__ __forceinline__ int vbox(const Geom& g, const FilterDev& f, int lo[3], int ext[3]) {
  for (int d = 0; d < 3; ++d) {
    int l = 0, h = g.T[d];
    if (d < g.ndim) {
      if ((f.orient >> d) & 1) l = -g.margin[d];
      else h = g.T[d] + g.margin[d];
    }
    l = max(l, -f.org[d]);
    h = min(h, g.pad[d] - f.org[d]);
    lo[d] = l;
    ext[d] = max(0, h - l);
  }
  return ext[0] * ext[1] * ext[2];
}

// Hard data inside each patch's virtual template, binned once per call
// (they do not change during the simulation).  Pass 1 counts, an exclusive
// scan turns counts into offsets, pass 2 writes the entries.
template <bool FILL>
__global__ __launch_bounds__(kThreads) void k_hd_bin(Geom g, const FilterDev* __restrict__ filters,
                                                     const int8_t* __restrict__ hdmap, int32_t* __restrict__ hd_off,
                                                     HdEnt* __restrict__ hd_ent, long long cap,
                                                     HdBits* __restrict__ hd_bits, HdmGeom m) {
  __shared__ unsigned s_cnt;
  const int fg = blockIdx.x;
  const FilterDev f = filters[fg];
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  int lo[3], ext[3];
  const int vc = vbox(g, f, lo, ext);
  const int8_t* hm = hdmap + (long long)f.r * g.pcells;
  const long long base_off = FILL ? hd_off[fg] : 0;
  for (int i = threadIdx.x; i < vc; i += kThreads) {
    int ux, uy, uz;
    split3(i, ext[0], ext[1], ux, uy, uz);
    ux += lo[0];
    uy += lo[1];
    uz += lo[2];
    const int8_t v = hm[idx3(f.org[0] + ux, f.org[1] + uy, f.org[2] + uz, g.pad)];
    if (v >= 0) {
      const unsigned p = atomicAdd(&s_cnt, 1u);
      if (FILL && base_off + p < cap) {
        HdEnt e;
        e.u[0] = (int16_t)ux;
        e.u[1] = (int16_t)uy;
        e.u[2] = (int16_t)uz;
        e.v = v;
        hd_ent[base_off + p] = e;
        if (hd_bits) {   // where the datum's vector starts in the bit table
          const int bx = g.b[0];
          const int r = ((ux % bx) + bx) % bx;
          const int av = (ux - r) / bx;
          const int slot = v < m.nf ? v : m.nf;
          HdBits hb;
          hb.woff = ((((uz + m.pz0) * m.ry + (uy + m.py0)) * bx + r) * m.ns + slot) * m.nw + ((av + m.pb) >> 5);
          hb.sh = (av + m.pb) & 31;
          hd_bits[base_off + p] = hb;
        }
      }
    }
  }
  __syncthreads();
  if (!FILL && threadIdx.x == 0) hd_off[fg] = (int32_t)s_cnt;
}

// The hard-data bit table (layout with HdmGeom): one thread per word.
__global__ __launch_bounds__(kThreads) void k_hd_mask(Geom g, HdmGeom m, const int8_t* __restrict__ ti,
                                                      uint32_t* __restrict__ out, long long nwords) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nwords) return;
  const int bx = g.b[0];
  long long t = id;
  const int w = (int)(t % m.nw);
  t /= m.nw;
  const int slot = (int)(t % m.ns);
  t /= m.ns;
  const int r = (int)(t % bx);
  t /= bx;
  const int y = (int)(t % m.ry) - m.py0, z = (int)(t / m.ry) - m.pz0;
  uint32_t bits = 0;
  if (y >= 0 && y < g.ti[1] && z >= 0 && z < g.ti[2]) {
    const int8_t* trow = ti + ((long long)z * g.ti[1] + y) * g.ti[0];
    for (int b = 0; b < 32; ++b) {
      const int x = (w * 32 + b - m.pb) * bx + r;
      if (x >= 0 && x < g.ti[0] && (slot == m.nf || trow[x] != slot)) bits |= 1u << b;
    }
  }
  out[id] = bits;
}

// One LeGall 5/3 integer lifting level along `axis` of an image of extent
// e (even along that axis), keeping the low-pass half: dst has e[axis] / 2
// samples along it.  Samples outside [0, n) mirror about the end samples.
// Prediction d[k] = x[2k+1] - floor((x[2k] + x[2k+2]) / 2), update
// s[k] = x[2k] + floor((d[k-1] + d[k] + 2) / 4).  FROM_TI: the source is the
// int8 TI, edge-replicated beyond its extent (the padded TI); dst_h, if
// given, receives the operand-type copy.  One thread per output sample.
__device__ __forceinline__ int mirror53(int i, int n) {
  if (i < 0) i = -i;
  if (i >= n) i = 2 * (n - 1) - i;
  if (i < 0) i = -i;   // only for n = 2
  return i;
}

template <bool FROM_TI>
__global__ __launch_bounds__(kThreads) void k_lift53(const void* __restrict__ src, int32_t* __restrict__ dst,
                                                     _Float16* __restrict__ dst_h, int e0, int e1, int e2, int axis,
                                                     Geom g) {
  int o[3] = {e0, e1, e2};
  const int e[3] = {e0, e1, e2};
  o[axis] >>= 1;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)o[0] * o[1] * o[2]) return;
  int c[3];
  split3((int)id, o[0], o[1], c[0], c[1], c[2]);
  const int n = e[axis], k = c[axis];
  auto at = [&](int i) -> int {
    int u[3] = {c[0], c[1], c[2]};
    u[axis] = mirror53(i, n);
    if (FROM_TI) {
      const int x = min(u[0], g.ti[0] - 1), y = min(u[1], g.ti[1] - 1), z = min(u[2], g.ti[2] - 1);
      return ((const int8_t*)src)[((long long)z * g.ti[1] + y) * g.ti[0] + x];
    }
    return ((const int32_t*)src)[idx3i(u[0], u[1], u[2], e)];
  };
  const int x0 = at(2 * k - 2), x1 = at(2 * k - 1), x2 = at(2 * k), x3 = at(2 * k + 1), x4 = at(2 * k + 2);
  const int dl = x1 - ((x0 + x2) >> 1), dr = x3 - ((x2 + x4) >> 1);
  const int s = x2 + ((dl + dr + 2) >> 2);
  dst[id] = s;
  if (dst_h) dst_h[id] = (_Float16)(float)s;
}

// Hard-data ranges of the scan records, from the binned offsets.
__global__ void k_recs_hd(ScanRec* __restrict__ recs, long long n, const int32_t* __restrict__ hd_off) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int gi = recs[i].gidx;
  if (gi < 0) return;
  recs[i].hd0 = hd_off[gi];
  recs[i].nhd = hd_off[gi + 1] - hd_off[gi];
}

// In-place exclusive scan of n counts (one workgroup); x[n] receives the total.
__global__ __launch_bounds__(kThreads) void k_exclusive_scan(int32_t* __restrict__ x, int n) {
  __shared__ int s_part[kThreads];
  const int tid = threadIdx.x;
  const int per = (n + kThreads - 1) / kThreads;
  const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
  int sum = 0;
  for (int i = b0; i < b1; ++i) sum += x[i];
  s_part[tid] = sum;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const int v = tid >= off ? s_part[tid - off] : 0;
    __syncthreads();
    s_part[tid] += v;
    __syncthreads();
  }
  int run = s_part[tid] - sum;
  for (int i = b0; i < b1; ++i) {
    const int c = x[i];
    x[i] = run;
    run += c;
  }
  if (tid == kThreads - 1) x[n] = s_part[tid];
}

__global__ void k_fill_i32(int32_t* __restrict__ p, long long n, int32_t v) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = v;
}

// ---- choose, rebuild, cut, paste (Algorithm 1 lines K best .. paste) ----
struct FinArgs {
  Geom g;
  const FilterDev* filters;       // of this step
  const FilterDev* filters_all;   // every patch of the call
  int fbegin;                     // global index of this step's first patch
  const int32_t* npred;
  const int32_t* succ_off;
  const int32_t* succ;
  int32_t* predcnt;
  const int32_t* kbeta;
  const int32_t* nbt;             // [shape][window block] known-cell counts
  int32_t* mbuf;                  // [patch][kKMax] data events
  int ev_delta;                   // 1: add the paste's changes to the successors' events
  unsigned long long* report;     // shortlist report: max |bulk - exact|, rescored, changed, patches
  int kpad;
  int shortlist;
  int score_mode;
  const uint64_t* keys;
  const uint64_t* rowmin;
  const int32_t* rowcnt;          // fused selection: keys at the start of each row's segment, else null
  const int32_t* lp_map;          // learned proposer: [slot] packed scan slot, or -1 (proposal stands)
  const uint64_t* lp_sel;         // learned proposer: [slot][top_k] the proposal's K best keys
  int32_t* drawn;                 // [patch] the drawn candidate
  const int32_t* Ki;
  const int32_t* det;
  const int32_t* tree;  // block-subtree coefficients (tree path)
  int8_t* sg;
  const int8_t* hdmap;
  int32_t* chosen_log;
  uint64_t seed;
  long long buf_cells;
  long long cand_cap;   // keys of the best rows staged in LDS (0: read all keys from memory)
  long long coef_lds;   // 1: stage the window's coefficients in LDS (aliases the key/cut area)
  int top_k;
  int cut;
  int nsteps;
  int rows_max;         // longest seam (cells)
  int has_hd;
  int dp_wave;          // 1: every overlap <= 16 cells, one 16-lane group per seam
  int dp_evs;           // step stride of the seam error buffer (wavefront DP)
  int dp_stride, dp_batch;
  // learned proposer (learn = D > 0), or the row-minima selection
  int learn;
  int rescore_rows;               // select by exact rescoring of rows in order of their minima / bounds
  int rows_exact;                 // the row keys are exact keys (row-minima selection)
  const uint32_t* hdm;            // hard-data bit table, or null
  const HdBits* hd_bits;
  HdmGeom hm;
  double* qbuf;                   // [patch][D + 4] queries of the data events (fp64)
  const float* pca_P;             // [D][template blocks]
  const float* pca_mu;            // [template blocks]
  const int32_t* energy;          // [shape][ncand]
  const int32_t* hd_off;          // [patch + 1]
  const HdEnt* hd_ent;
  const int8_t* ti;
  long long learn_off;            // LDS offset of the row-rescoring area
  int learn_kbr;                  // candidate rows rescored per round
  int learn_w;                    // staged K-row length (int16)
  // the step's patch records by value when they fit, so that reading a
  // workgroup's record overlaps the argument load instead of following it
  int n_inline;
  FilterDev recs_inline[kFinInline];
};

// Window cell of a seam: w along the band axis ax (counted from the side
// that faces the already simulated neighbour), y along the seam axis ra, sl
// on the slice axis sa (or none).  Built with selects, not array indexing,
// so everything stays in registers.
__device__ __forceinline__ int seam_cell(const Geom& g, int orient, int ax, int ra, int sa, int sl, int y, int w) {
  const int wc = ((orient >> ax) & 1) ? (ax == 0 ? g.T[0] : ax == 1 ? g.T[1] : g.T[2]) - 1 - w : w;
  const int ux = ax == 0 ? wc : ra == 0 ? y : sa == 0 ? sl : 0;
  const int uy = ax == 1 ? wc : ra == 1 ? y : sa == 1 ? sl : 0;
  const int uz = ax == 2 ? wc : ra == 2 ? y : sa == 2 ? sl : 0;
  return ux + g.T[0] * (uy + g.T[1] * uz);
}

// Squared code difference between the grid and the new pattern at that cell.
__device__ __forceinline__ int seam_err(const Geom& g, const int8_t* s_sg, const int8_t* P, int orient, int ax,
                                        int ra, int sa, int sl, int y, int w) {
  const int c = seam_cell(g, orient, ax, ra, sa, sl, y, w);
  const int d = (int)s_sg[c] - (int)P[c];
  return d * d;
}


// Minimal-error boundary cut of every seam of one patch, one wavefront per
// seam (overlap <= 16 cells, seam <= 64 cells).  Lane w holds column w
// (w = 0 faces the already simulated neighbour).  Row by row the cumulative
// error is E'[w] = e[w] + min(E[w], E[w-1], E[w+1]); the wavefront keeps its
// complement F = ~E instead, for which the recurrence reads
// F'[w] = max(F[w], F[w-1], F[w+1]) - e[w] (saturating at 0), and a column
// outside the overlap, or outside the 16-lane row of a row shift, reads as
// F = 0, i.e. E = infinity.  The seam is padded at the top to a multiple of
// 8 rows with rows of zero error, which leave F unchanged, so the row loop
// needs no per-row bound checks.  The errors e of the whole seam are first
// written to LDS by all 64 lanes (lane = step), so the row loop reads four
// rows per load.  Each row also records, per column, the step to the row
// above (0, -1 or +1; ties prefer the same column, then w - 1, then w + 1),
// off the dependency chain of F.  The trace back starts at the smallest end
// value (smallest column on ties) and costs one register read per row; the
// seam column of step s is kept in lane s, and the cells before the seam are
// marked in parallel afterwards.  Lanes 16..63 run the row loop on copies
// that never reach lanes 0..15.
template <int ND>
__device__ void seam_dp_wave(const Geom& g, const FilterDev& f, const int8_t* s_sg, const int8_t* P,
                             uint8_t* keep, int n0, int n1, int n2, uint32_t* s_ev, int evs) {
  constexpr int NS = kSeamRowsMax;
  constexpr uint32_t kBig = 0xFFFFFFFFu;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ndp = __builtin_amdgcn_readfirstlane(n0 + n1 + n2);
  uint32_t* my_ev = s_ev + wave * 16 * evs;   // [column][step]
  for (int dd = wave; dd < ndp; dd += kThreads / 64) {
    // seam parameters are the same for the whole wavefront: keep them scalar
    const int ax = __builtin_amdgcn_readfirstlane(dd < n0 ? 0 : dd < n0 + n1 ? 1 : 2);
    const int sl = __builtin_amdgcn_readfirstlane(dd - (ax == 0 ? 0 : ax == 1 ? n0 : n0 + n1));
    const int ra = ax == 0 ? 1 : 0;
    const int sa = ND == 3 ? 3 - ax - ra : -1;
    const int rows = __builtin_amdgcn_readfirstlane(ra == 0 ? g.T[0] : g.T[1]);
    const int cols = __builtin_amdgcn_readfirstlane(ax == 0 ? g.OV[0] : ax == 1 ? g.OV[1] : g.OV[2]);
    const int flip = (f.orient >> ax) & 1;
    // window strides: cell(y, w) = y * rs + wc(w) * as + sl * ss
    const int st[3] = {1, g.T[0], g.T[0] * g.T[1]};
    const int rs = ra == 0 ? st[0] : st[1];
    const int as = ax == 0 ? st[0] : ax == 1 ? st[1] : st[2];
    const int ss = sa < 0 ? 0 : sa == 0 ? st[0] : sa == 1 ? st[1] : st[2];
    const int tax = ax == 0 ? g.T[0] : ax == 1 ? g.T[1] : g.T[2];
    const int steps = (rows + 7) & ~7;   // rows padded at the top
    const int pad = steps - rows;        // step s holds row s - pad
    // errors of the seam: lane s fills step s of every column
    {
      const bool real = lane >= pad && lane < steps;
      const int rowc = min(max(lane - pad, 0), rows - 1) * rs + sl * ss;
      int d[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) {
        const int c = rowc + (flip ? tax - 1 - min(w, tax - 1) : min(w, tax - 1)) * as;
        d[w] = (int)s_sg[c] - (int)P[c];
      }
      asm volatile("" : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]), "+v"(d[3]), "+v"(d[4]), "+v"(d[5]), "+v"(d[6]),
                   "+v"(d[7]), "+v"(d[8]), "+v"(d[9]), "+v"(d[10]), "+v"(d[11]), "+v"(d[12]), "+v"(d[13]),
                   "+v"(d[14]), "+v"(d[15]));
      if (lane < steps) {
#pragma unroll
        for (int w = 0; w < 16; ++w)
          my_ev[w * evs + lane] = w >= cols ? kBig : real ? (uint32_t)__mul24(d[w], d[w]) : 0u;
      }
    }
    const uint32_t* ev_row = my_ev + (lane & 15) * evs;
    int D[NS];   // step to the row above, per step and column
    uint32_t Fc = lane < cols ? kBig : 0u;
#pragma unroll
    for (int s0 = 0; s0 < NS; s0 += 8) {
      if (s0 < steps) {   // one scalar branch per 8 rows
        const uint4 e0 = *(const uint4*)(ev_row + s0);
        const uint4 e1 = *(const uint4*)(ev_row + s0 + 4);
        const uint32_t ev[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t l = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)Fc, 0x111, 0xF, 0xF, true);
          const uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)Fc, 0x101, 0xF, 0xF, true);
          const uint32_t lr = max(l, r);
          D[s0 + e] = Fc >= lr ? 0 : (l >= r ? -1 : 1);
          const uint32_t m = max(Fc, lr);
          Fc = m > ev[e] ? m - ev[e] : 0u;
        }
      }
    }
    // end of the seam: largest F (smallest error), smallest column on ties;
    // lane 15 ends with the largest F of lanes 0..15
    uint32_t mx = Fc;
    mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x111, 0xF, 0xF, true));
    mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x112, 0xF, 0xF, true));
    mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x114, 0xF, 0xF, true));
    mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x118, 0xF, 0xF, true));
    const uint32_t fmax = (uint32_t)__builtin_amdgcn_readlane((int)mx, 15);
    const unsigned long long hit = __ballot(Fc == fmax) & 0xFFFFull;
    int sc = __builtin_amdgcn_readfirstlane(__builtin_ctzll(hit | (1ull << 15)));
    int seam_of_step = 0;   // lane s: seam column at step s
#pragma unroll
    for (int s0 = NS - 8; s0 >= 0; s0 -= 8) {
      if (s0 < steps) {
#pragma unroll
        for (int e = 7; e >= 0; --e) {
          seam_of_step = lane == s0 + e ? sc : seam_of_step;
          sc += __builtin_amdgcn_readlane(D[s0 + e], sc);
        }
      }
    }
    const int y = lane - pad;
    if (y >= 0 && lane < steps) {
      const int rb = y * rs + sl * ss;
      const int sc_y = min(seam_of_step, cols);
      for (int ww = 0; ww < sc_y; ++ww) keep[rb + (flip ? tax - 1 - ww : ww) * as] = 1;
    }
  }
}

template <int ND, int TJ>
__global__ __launch_bounds__(kThreads) void k_finalize(FinArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ TopkShared sh;
  __shared__ int s_rows[kShortMax];
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const int slot = blockIdx.x;
  // scalar loads from the arguments, issued together with the count that
  // decides whether they are used (the empty asm takes both before the branch)
  const int n_inline = a.n_inline;
  const FilterDev f_arg = a.recs_inline[min(slot, kFinInline - 1)];
  __asm__ volatile("" ::"s"(n_inline), "s"(f_arg.r));
  FilterDev f;
  if (slot < n_inline) {
    f = f_arg;
    __asm__ volatile("" ::: "memory");  // keeps the two loads apart (no generic pointer)
  } else {
    f = a.filters[slot];
  }
  // learned proposer: the patch's slot in the scan's packed output, or -1
  // where the proposal stands
  const int kslot = a.lp_map ? a.lp_map[slot] : slot;
  const bool from_lp = kslot < 0;
  // the row minima depend on the slot only: fetch them with the record
  const int nrows_c = g.cand[1] * g.cand[2];
  uint64_t rm_pre = ~0ull;
  int rc_pre = 0;
  if (!from_lp && (a.cand_cap > 0 || a.rescore_rows) && tid < nrows_c) {
    rm_pre = a.rowmin[(long long)kslot * nrows_c + tid];
    if (a.rowcnt) rc_pre = a.rowcnt[(long long)kslot * nrows_c + tid];
  }
  // keys per candidate row (fused selection: the row's survivors)
  constexpr int kRcLds = 512;
  __shared__ int s_rc[kRcLds];
  if (a.rowcnt && tid < nrows_c && tid < kRcLds) s_rc[tid] = rc_pre;
  const long long wpad = (g.wcells + 15) & ~15ll;
  int32_t* bufA = (int32_t*)smem;
  int32_t* bufB = bufA + a.buf_cells;
  int8_t* P = (int8_t*)(bufB + a.buf_cells);
  uint8_t* keep = (uint8_t*)(P + wpad);
  int8_t* s_sg = (int8_t*)(keep + wpad);
  int8_t* s_hd = s_sg + wpad;
  uint64_t* s_cand = (uint64_t*)(s_hd + wpad);
  unsigned char* dps = (unsigned char*)(s_cand + a.cand_cap);

  // successor list of this patch (used at the very end), fetched early
  __shared__ int s_mine[kMaxSucc];
  __shared__ FilterDev s_fq[kMaxSucc];
  __shared__ int s_nmine;
  const int my_nsucc = min(f.nsucc, kMaxSucc);
  static_assert(sizeof(FilterDev) == 40, "successor record is moved as five int2");
  int2 my_fq[5] = {};   // the successor's record (fetched after the selection), kept in registers
  // (successor, its predecessor count), meaningful for tid < my_nsucc; read
  // unconditionally (entry 0 always exists) so that nothing waits for it here
  const int2 succ_e = ((const int2*)a.succ)[tid < my_nsucc ? f.succ0 + tid : 0];
  // the block list of this realization's orientation (shared by successors)
  const int my_beta = tid < a.kpad ? a.kbeta[f.orient * kKMax + tid] : -1;

  // windows of the grid and of the hard-data map.  They are first read by
  // the cut.  When they fit one batch, each thread loads up to kWinWords
  // aligned 8-byte words of the window rows (a row of T0 cells starts at
  // any byte, so it spans at most (T0 + 14) / 8 words), keeps them in
  // registers through the selection and unpacks their bytes into LDS after
  // it, so the loads' latency overlaps the selection.  The grids carry 16
  // bytes of slack for the words that reach past a row's end.
  constexpr int kWinWords = 4;
  const int win_wpr = (g.T[0] + 14) >> 3;
  const int win_nw = g.T[1] * g.T[2] * win_wpr;
  const bool win_defer = win_wpr <= 64 && win_nw <= kWinWords * kThreads;
  const int8_t* win_sg = a.sg + (long long)f.r * g.pcells;
  const int8_t* win_hd = a.has_hd ? a.hdmap + (long long)f.r * g.pcells : nullptr;
  uint64_t wv0[kWinWords], wv1[kWinWords];
  int wrow[kWinWords], wx0[kWinWords];   // window row of each word, window x of its first byte
  auto issue_windows = [&]() {
    const unsigned mdiv = (65536u + win_wpr - 1) / win_wpr;   // j / wpr exactly for j < 2^16 / wpr
#pragma unroll
    for (int q = 0; q < kWinWords; ++q) {
      const int j = tid + q * kThreads;
      wv0[q] = 0;
      wv1[q] = ~0ull;   // no hard data: every byte -1
      wrow[q] = -1;
      wx0[q] = 0;
      if (j < win_nw) {
        const int row = (int)(((unsigned)j * mdiv) >> 16), w = j - row * win_wpr;
        const int z = g.T[2] > 1 ? row / g.T[1] : 0, y = row - z * g.T[1];
        const long long c0 = idx3(f.org[0], f.org[1] + y, f.org[2] + z, g.pad);
        const int lead = (int)((uintptr_t)(win_sg + c0) & 7);   // the same for both maps (256-aligned bases)
        const long long wo = c0 - lead + 8ll * w;
        wv0[q] = *(const uint64_t*)(win_sg + wo);
        if (win_hd) wv1[q] = *(const uint64_t*)(win_hd + wo);
        wrow[q] = row;
        wx0[q] = 8 * w - lead;
      }
    }
  };
  // With stored keys the windows' loads go out after the row minima are
  // ranked, beside the loads of the best rows' keys: the staging of the row
  // minima would otherwise wait for them too.
  const bool win_late = win_defer && !from_lp && !a.rescore_rows && a.cand_cap > 0;
  if (!win_defer) load_windows(s_sg, win_sg, s_hd, win_hd, f.org, g);
  else if (!win_late) issue_windows();
  for (int i = tid; i < (int)g.wcells; i += kThreads) keep[i] = 0;

  // K best keys.  The smallest key of every candidate row is known from the
  // scan; the K best keys lie in the K rows with the smallest minima, so only
  // those rows are read.
  const uint64_t tkey = draw64(a.seed, kStreamTiebreak, (uint64_t)f.r, (uint64_t)f.step);
  const int k = min(a.top_k, g.ncand);
  const uint64_t* kf = a.keys + (long long)max(kslot, 0) * g.ncand;
  // ksel best bulk keys: k, or the shortlist that is rescored exactly below
  __shared__ uint64_t s_rowtop[kShortMax];
  __shared__ uint64_t s_sel[kShortMax];
  __shared__ uint64_t s_fin[kShortMax];
  __shared__ unsigned s_cnt;
  const int ksel = a.shortlist > 0 ? min(a.shortlist, g.ncand) : k;
  bool done = false;
  if (from_lp) {
    if (tid < k) s_sel[tid] = a.lp_sel[(long long)slot * a.top_k + tid];
    __syncthreads();
    done = true;
  } else if (a.rescore_rows) {
    // The scan wrote, per candidate row, the smallest key of the row (the
    // row-minima selection) or the smallest lower bound of its keys (the
    // learned proposer).  Rows are rescored exactly in order of their
    // minimum or bound, a few at a time, until the k best exact keys lie
    // below the minimum or bound of every row left (certified), so the k
    // best equal the full scan's.  With exact minima that takes at most k
    // rows: a row holding one of the k best keys has its minimum among them.
    const int nrows = g.cand[1] * g.cand[2];
    const int C0 = g.cand[0];
    const uint64_t* rm = a.rowmin + (long long)kslot * nrows;
    const bool exact_rows = a.rows_exact || f.bandmask == 0;   // no overlap: the row keys are exact keys
    unsigned char* lb = smem + a.learn_off;
    uint64_t* s_rk = (uint64_t*)lb;                                  // [nrows] sort keys
    int* s_order = (int*)(s_rk + nrows);                             // [nrows] rows by bound
    uint64_t* s_bkey = (uint64_t*)(s_order + ((nrows + 1) & ~1));    // [kbr * C0] batch keys
    int16_t* s_stage = (int16_t*)(s_bkey + a.learn_kbr * C0);        // [kbr][K rows][W] int16
    __shared__ int s_koff[kKMax], s_km[kKMax];
    __shared__ int s_row_of[16];
    const int nkr = g.tc[1] * g.tc[2];
    const int W = a.learn_w;
    // block list of this orientation with the exact data event
    if (tid < a.kpad) {
      int off = -1, m = 0;
      if (my_beta >= 0) {
        int bx, by, bz;
        split3(my_beta, g.tc[0], g.tc[1], bx, by, bz);
        off = (bz * g.tc[1] + by) * W + bx;
        m = f.bandmask ? (int)a.mbuf[(long long)(a.fbegin + slot) * kKMax + tid] : 0;
      }
      s_koff[tid] = off;
      s_km[tid] = m;
    }
    // the orientation's block list ends at its first -1
    const int nk = __syncthreads_count(tid < a.kpad && my_beta >= 0);
    // sort keys: a bound's tie field carries the row index (distinct keys)
    for (int i = tid; i < nrows; i += kThreads) {
      const uint64_t v = i < kThreads ? rm_pre : rm[i];
      s_rk[i] = exact_rows ? v : ((v & ~(uint64_t)kMask20) | (uint64_t)i);
      s_order[i] = i;
    }
    __syncthreads();
    for (int i = tid; i < nrows; i += kThreads) {
      const uint64_t x = s_rk[i];
      int rank = 0;
      for (int jj = 0; jj < nrows; ++jj) rank += s_rk[jj] < x ? 1 : 0;
      s_order[rank] = i;
    }
    const int hd0 = a.has_hd ? a.hd_off[a.fbegin + slot] : 0;
    const int nhd = a.has_hd ? a.hd_off[a.fbegin + slot + 1] - hd0 : 0;
    const int32_t* erow = a.energy + (long long)f.shape * g.ncand;
    const int shift = g.shift;
    int nsel = 0, pos = 0;
    while (pos < nrows) {
      __syncthreads();
      if (nsel == k) {
        const uint64_t nb = s_rk[min(max(s_order[pos], 0), nrows - 1)];
        const uint64_t bound = exact_rows ? nb : (nb & ~(uint64_t)kMask20);
        if (s_sel[k - 1] < bound) break;   // certified: no row left can hold a better key
      }
      const int nb_rows = min(a.learn_kbr, nrows - pos);
      if (tid < nb_rows) s_row_of[tid] = min(max(s_order[pos + tid], 0), nrows - 1);
      __syncthreads();
      // stage the level-J rows these candidate rows read, as int16; every
      // load of a thread's share is issued before any of them is stored
      {
        constexpr int U = 16;
        const int total = nb_rows * nkr * W;
        for (int base = tid; base < total; base += kThreads * U) {
          int16_t v[U];
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int i = base + q * kThreads;
            v[q] = 0;
            if (i < total) {
              const int b = i / (nkr * W), rest = i - b * (nkr * W);
              const int kr = rest / W, x = rest - kr * W;
              const int row = s_row_of[b];
              const int cy = row % g.cand[1], cz = row / g.cand[1];
              const int by = kr % g.tc[1], bz = kr / g.tc[1];
              if (x < g.G[0]) v[q] = (int16_t)a.Ki[idx3i(x, cy + by, cz + bz, g.G)];
            }
          }
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int i = base + q * kThreads;
            if (i < total) s_stage[i] = v[q];
          }
        }
      }
      __syncthreads();
      // exact keys of every candidate of the batch
      const int J = g.level, Jz = g.ndim == 3 ? J : 0;
      for (int i = tid; i < nb_rows * C0; i += kThreads) {
        const int b = i / C0, cx = i - b * C0;
        const int row = s_row_of[b];
        const int cy = row % g.cand[1], cz = row / g.cand[1];
        const int16_t* st = s_stage + b * nkr * W + cx;
        int C = 0;
#pragma unroll 8
        for (int kk = 0; kk < nk; ++kk) C += s_km[kk] * (int)st[s_koff[kk]];
        const long long idx = (long long)row * C0 + cx;
        const int S = erow[idx] - (C << shift);
        unsigned mis = 0;
        if (a.hdm) {   // bit cx + sh of the datum's vector for this row
          const uint32_t* mb = a.hdm + ((cz << Jz) * a.hm.ry + (cy << J)) * a.hm.rs;
          for (int h = 0; h < nhd; ++h) {
            const HdBits hb = a.hd_bits[hd0 + h];
            mis += (mb[hb.woff + ((cx + hb.sh) >> 5)] >> ((cx + hb.sh) & 31)) & 1u;
          }
        } else {
          for (int h = 0; h < nhd; ++h) {
            const HdEnt e = a.hd_ent[hd0 + h];
            const int fx = (cx << J) + e.u[0], fy = (cy << J) + e.u[1], fz = (cz << Jz) + e.u[2];
            if (fx >= 0 && fy >= 0 && fz >= 0 && fx < g.ti[0] && fy < g.ti[1] && fz < g.ti[2])
              mis += a.ti[(fz * g.ti[1] + fy) * g.ti[0] + fx] != e.v ? 1u : 0u;
          }
        }
        s_bkey[i] = make_key(mis, f.bandmask ? S : 0, tie_perm((uint32_t)idx, tkey));
      }
      __syncthreads();
      // the k best of the kept keys and the batch
      const int nkeep = nsel, nbk = nb_rows * C0;
      block_topk(nkeep + nbk, min(k, nkeep + nbk),
                 [&](long long q) { return q < nkeep ? s_sel[q] : s_bkey[q - nkeep]; }, sh);
      nsel = min(k, nkeep + nbk);
      if (tid < nsel) s_sel[tid] = sh.top[tid];
      pos += nb_rows;
    }
    __syncthreads();
    if (tid == 0 && a.learn) {
      atomicAdd(&a.report[4], 1ull);                       // patches selected through the proposer
      atomicAdd(&a.report[5], (unsigned long long)pos);    // candidate rows rescored exactly
    }
    done = true;
  } else if (a.cand_cap > 0) {
    // 1. the kr smallest row minima, by rank (rows are few)
    const int nrows = g.cand[1] * g.cand[2];
    const uint64_t* rm = a.rowmin + (long long)kslot * nrows;
    const int kr = min(ksel, nrows);
    uint64_t* s_rm = s_cand;   // staging; the candidate list reuses it afterwards
    if (nrows <= a.cand_cap) {
      if (tid < nrows) s_rm[tid] = rm_pre;
      for (int i = tid + kThreads; i < nrows; i += kThreads) s_rm[i] = rm[i];
      if (tid == 0) s_cnt = 0;
      __syncthreads();
      block_rank_select(s_rm, nrows, kr, s_rowtop);
    } else {   // only reached with kr <= 16 (checked when the plan is built)
      block_topk(nrows, kr, [&](long long i) { return rm[i]; }, sh);
      if (tid < kr) s_rowtop[tid] = sh.top[tid];
      if (tid == 0) s_cnt = 0;
      __syncthreads();
    }
    if (tid < kr) {
      const int id = (int)tie_perm_inv((uint32_t)(s_rowtop[tid] & kMask20), tkey);
      s_rows[tid] = min(max(id / g.cand[0], 0), nrows - 1);
    }
    if (win_late) issue_windows();
    __syncthreads();
    // 2. every key of those rows at or below the kr-th row minimum (when
    //    there are fewer rows than ksel, every key of every row); the list
    //    holds at most kr * C_x <= cand_cap keys
    const uint64_t thr = kr == ksel ? s_rowtop[kr - 1] : ~0ull;
    const int cx = g.cand[0];
    const int nc = kr * cx;
    constexpr int U = 8;
    BoxWalk w(tid, kThreads, cx, 1 << 30);   // (x, y) = (column, list row)
    for (int base = tid; base < nc; base += kThreads * U) {
      uint64_t v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        v[q] = ~0ull;
        if (i < nc) {
          const int rr = s_rows[w.y];
          const int n_in_row =
              !a.rowcnt ? cx : rr < kRcLds ? s_rc[rr] : a.rowcnt[(long long)kslot * nrows + rr];
          if (w.x < n_in_row) v[q] = kf[(long long)rr * cx + w.x];
        }
        w.next();
      }
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (v[q] <= thr && v[q] != ~0ull) s_cand[atomicAdd(&s_cnt, 1u)] = v[q];
    }
    __syncthreads();
    const int n = (int)s_cnt;
    if (n <= 512) {
      // 3. the ksel smallest of the short list, by rank
      block_rank_select(s_cand, n, ksel, s_sel);
    } else {
      // long list: ksel rounds of "smallest key above the previous one"
      uint64_t prev = 0;
      for (int r = 0; r < ksel; ++r) {
        uint64_t mm = ~0ull;
        for (int i = tid; i < n; i += kThreads) {
          const uint64_t key = s_cand[i];
          if ((r == 0 || key > prev) && key < mm) mm = key;
        }
        mm = wave_min64(mm);
        __syncthreads();
        if ((tid & 63) == 0) sh.small[tid >> 6] = mm;
        __syncthreads();
        uint64_t best = sh.small[0];
        for (int w = 1; w < kThreads / 64; ++w) best = sh.small[w] < best ? sh.small[w] : best;
        prev = best;
        if (tid == 0) s_sel[r] = best;
      }
      __syncthreads();
    }
    done = true;
  }
  if (!done) {   // only reached with ksel <= 16 (checked when the plan is built)
    block_topk(g.ncand, ksel, [&](long long i) { return kf[i]; }, sh);
    if (tid < ksel) s_sel[tid] = sh.top[tid];
    __syncthreads();
  }

  if (a.shortlist > 0) {
    // Exact rescoring of the shortlist in integers from the int32 grid and
    // the exact data event; the K best of the rescored keys are drawn from.
    __shared__ int s_bk[kKMax], s_mk[kKMax], s_nk[kKMax];
    __shared__ uint64_t s_resc[kShortMax];
    const int fgi = a.fbegin + slot;
    if (tid < a.kpad) {
      s_bk[tid] = my_beta;
      s_mk[tid] = (my_beta >= 0 && f.bandmask) ? (int)a.mbuf[(long long)fgi * kKMax + tid] : 0;
      s_nk[tid] = my_beta >= 0 ? a.nbt[(long long)f.shape * g.tcells + my_beta] : 0;
    }
    __syncthreads();
    const int ci = tid >> 3, sub = tid & 7;   // 8 lanes per shortlisted candidate
    long long C = 0, E = 0;
    uint64_t key = 0;
    int c0[3] = {0, 0, 0};
    if (ci < ksel) {
      key = s_sel[ci];
      const int id = min(max((int)tie_perm_inv((uint32_t)(key & kMask20), tkey), 0), g.ncand - 1);
      split3(id, g.cand[0], g.cand[1], c0[0], c0[1], c0[2]);
      for (int kk = sub; kk < a.kpad; kk += 8) {
        const int beta = s_bk[kk];
        if (beta < 0) continue;
        int bx, by, bz;
        split3(beta, g.tc[0], g.tc[1], bx, by, bz);
        const long long kv = a.Ki[idx3(c0[0] + bx, c0[1] + by, c0[2] + bz, g.G)];
        C += (long long)s_mk[kk] * kv;
        E += (long long)s_nk[kk] * kv * kv;
      }
    }
#pragma unroll
    for (int m = 4; m >= 1; m >>= 1) {
      C += __shfl_xor(C, m, 8);
      E += __shfl_xor(E, m, 8);
    }
    if (ci < ksel && sub == 0) {
      const long long sx = a.score_mode == 0 ? E - 2ll * g.beta * C : -C;
      const long long sb = (long long)((key >> 20) & 0xFFFFFFFFull) - 2147483648ll;
      const unsigned long long err = (unsigned long long)(sx > sb ? sx - sb : sb - sx);
      s_resc[ci] = make_key((uint32_t)(key >> 52), (int32_t)sx, (uint32_t)(key & kMask20));
      if (err) atomicMax(&a.report[0], err);
    }
    __syncthreads();
    block_rank_select(s_resc, ksel, k, s_fin);
    if (tid == 0) {
      atomicAdd(&a.report[1], (unsigned long long)ksel);
      atomicAdd(&a.report[3], 1ull);
      bool changed = false;
      for (int i = 0; i < k; ++i) changed = changed || ((s_fin[i] ^ s_sel[i]) & kMask20) != 0;
      if (changed) atomicAdd(&a.report[2], 1ull);
    }
  } else if (tid < k) {
    s_fin[tid] = s_sel[tid];
  }
  __syncthreads();
  // the successors' records: their loads go out now, after the selection's
  // waits, and arrive while the pattern is rebuilt
  const int my_succ = succ_e.x, my_npred = succ_e.y;
  if (tid < my_nsucc) {
    const int2* src = (const int2*)(a.filters_all + my_succ);
#pragma unroll
    for (int q = 0; q < 5; ++q) my_fq[q] = src[q];
  }
  const uint64_t u = draw64(a.seed, kStreamDraw, (uint64_t)f.r, (uint64_t)f.step) >> 32;
  const int jpick = (int)((u * (uint64_t)k) >> 32);
  int idx = (int)tie_perm_inv((uint32_t)(s_fin[jpick] & kMask20), tkey);
  idx = min(max(idx, 0), g.ncand - 1);  // always in range for keys written by the scan
  if (tid == 0 && a.chosen_log) a.chosen_log[(long long)f.r * a.nsteps + f.step] = idx;
  if (tid == 0) a.drawn[a.fbegin + slot] = idx;
  const int cx = idx % g.cand[0], cy = (idx / g.cand[0]) % g.cand[1], cz = idx / (g.cand[0] * g.cand[1]);

  if (win_defer) {
#pragma unroll
    for (int q = 0; q < kWinWords; ++q) {
      if (wrow[q] < 0) continue;
      int8_t* ds = s_sg + wrow[q] * g.T[0];
      int8_t* dh = s_hd + wrow[q] * g.T[0];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int x = wx0[q] + b;
        if (x >= 0 && x < g.T[0]) {
          ds[x] = (int8_t)(wv0[q] >> (8 * b));
          dh[x] = (int8_t)(wv1[q] >> (8 * b));
        }
      }
    }
  }
  // rebuild the pattern from the coefficient pyramid (5/3: by perfect
  // reconstruction the TI's own window)
  if constexpr (TJ > 0) {
    idwt_window_tree<ND, TJ>(a.tree, g, cx, cy, cz, P);
  } else if (g.wavelet == 1) {
    for (int i = tid; i < (int)g.wcells; i += kThreads) {
      int x, y, z;
      split3(i, g.T[0], g.T[1], x, y, z);
      P[i] = a.ti[((long long)(g.b[2] * cz + z) * g.ti[1] + g.b[1] * cy + y) * g.ti[0] + g.b[0] * cx + x];
    }
    __syncthreads();
  } else if (a.coef_lds) idwt_window_lds<ND>(a.Ki, a.det, g, cx, cy, cz, (int32_t*)s_cand, bufA, bufB, P);
  else idwt_window<ND>(a.Ki, a.det, g, cx, cy, cz, bufA, bufB, P);
  // additive data events: the successors' records, the block list and the
  // zeroed sums of the first group of successors go to LDS now (the inverse
  // DWT is done with its buffers), so the barriers of the cut cover them
  // additive data events: the successors' records, the block list and the
  // zeroed sums of the first group of successors go to LDS now (the inverse
  // DWT is done with its buffers), under the barrier the cut needs anyway
  __shared__ int s_betas[kKMax];
  const int ev_tcl = (int)g.tcells;
  const int ev_ng = a.ev_delta ? max(1, min(my_nsucc, (int)(2 * a.buf_cells / ev_tcl))) : 0;
  int* s_dsum = bufA;
  if (a.ev_delta) {
    for (int i = tid; i < ev_ng * ev_tcl; i += kThreads) s_dsum[i] = 0;
    if (tid < a.kpad) s_betas[tid] = my_beta;
    if (tid < my_nsucc) {
      s_mine[tid] = my_succ;
#pragma unroll
      for (int q = 0; q < 5; ++q) ((int2*)&s_fq[tid])[q] = my_fq[q];
    }
  }
  if (win_defer || a.ev_delta) __syncthreads();   // the windows' LDS stores, for the cut

  int8_t* sgw = a.sg + (long long)f.r * g.pcells;
  bool interior_done = false;   // cells outside every band already pasted
  if (a.cut && f.bandmask) {
    // seams: one per present band, per slice in 3D
    // seams of band 0 first, then band 1, then band 2; n_a seams per band
    const int n0 = (f.bandmask & 1) ? (ND == 3 ? g.T[2] : 1) : 0;
    const int n1 = (f.bandmask & 2) ? (ND == 3 ? g.T[2] : 1) : 0;
    const int n2 = (ND == 3 && (f.bandmask & 4)) ? g.T[1] : 0;
    const int ndp = n0 + n1 + n2;
    auto dp_of = [&](int dd, int& ax, int& ra, int& sa, int& sl) {
      ax = dd < n0 ? 0 : dd < n0 + n1 ? 1 : 2;
      sl = dd - (ax == 0 ? 0 : ax == 1 ? n0 : n0 + n1);
      ra = ax == 0 ? 1 : 0;
      sa = ND == 3 ? 3 - ax - ra : -1;
    };
    if (a.dp_wave) {
      // 16-byte aligned, as an offset from the LDS base: an integer round
      // trip of the pointer would lose its address space (FLAT accesses)
      uint32_t* s_ev = (uint32_t*)(smem + ((((unsigned char*)s_cand - smem) + 15) & ~15ll));
      seam_dp_wave<ND>(g, f, s_sg, P, keep, n0, n1, n2, s_ev, a.dp_evs);
      // wavefronts without a seam paste the cells outside every band meanwhile
      const int busy = min(ndp, kThreads / 64);
      if (busy < kThreads / 64) {
        interior_done = true;
        const int t0 = tid - busy * 64, nt = kThreads - busy * 64;
        if (t0 >= 0) {
          BoxWalk w(t0, nt, g.T[0], g.T[1]);
          for (int i = t0; i < (int)g.wcells; i += nt, w.next())
            if (s_hd[i] < 0 && !dev_in_band(g, f.orient, f.bandmask, w.x, w.y, w.z))
              sgw[idx3(f.org[0] + w.x, f.org[1] + w.y, f.org[2] + w.z, g.pad)] = P[i];
        }
      }
      __syncthreads();
    } else {
      // wide overlaps: one thread per seam
      for (int base = 0; base < ndp; base += a.dp_batch) {
        const int nb = min(a.dp_batch, ndp - base);
        if (tid < nb) {
          int ax, ra, sa, sl;
          dp_of(base + tid, ax, ra, sa, sl);
          const int rows = g.T[ra], cols = g.OV[ax];
          unsigned char* scr = dps + (long long)tid * a.dp_stride;
          int32_t* Ep = (int32_t*)scr;
          int32_t* Ec = Ep + cols;
          uint8_t* from = (uint8_t*)(Ec + cols);
          for (int w = 0; w < cols; ++w) Ep[w] = seam_err(g, s_sg, P, f.orient, ax, ra, sa, sl, 0, w);
          for (int y = 1; y < rows; ++y) {
            for (int w = 0; w < cols; ++w) {
              int best = w, bv = Ep[w];
              if (w > 0 && Ep[w - 1] < bv) { best = w - 1; bv = Ep[w - 1]; }
              if (w + 1 < cols && Ep[w + 1] < bv) { best = w + 1; bv = Ep[w + 1]; }
              Ec[w] = seam_err(g, s_sg, P, f.orient, ax, ra, sa, sl, y, w) + bv;
              from[y * cols + w] = (uint8_t)best;
            }
            int32_t* t = Ep; Ep = Ec; Ec = t;
          }
          int sc = 0;
          for (int w = 1; w < cols; ++w)
            if (Ep[w] < Ep[sc]) sc = w;
          for (int y = rows - 1; y >= 0; --y) {
            for (int w = 0; w < sc; ++w) keep[seam_cell(g, f.orient, ax, ra, sa, sl, y, w)] = 1;
            if (y > 0) sc = from[y * cols + sc];
          }
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // paste the new side of every seam, keep hard data
  if (interior_done) {
    // only the band is left: its cells as up to three disjoint boxes, the
    // slab of each band axis minus the slabs of the axes before it
#pragma unroll 1
    for (int ax = 0; ax < ND; ++ax) {
      if (!((f.bandmask >> ax) & 1)) continue;
      int lo[3] = {0, 0, 0}, ex[3] = {g.T[0], g.T[1], g.T[2]};
      lo[ax] = ((f.orient >> ax) & 1) ? g.T[ax] - g.OV[ax] : 0;
      ex[ax] = g.OV[ax];
      for (int b = 0; b < ax; ++b)
        if ((f.bandmask >> b) & 1) {
          lo[b] = ((f.orient >> b) & 1) ? 0 : g.OV[b];
          ex[b] = g.T[b] - g.OV[b];
        }
      auto put = [&](int x, int y, int z) {
        const int c = idx3i(x, y, z, g.T);
        const int8_t pv = P[c], hv = s_hd[c];
        const uint8_t kv = keep[c];
        if (hv < 0 && !kv) sgw[idx3(f.org[0] + x, f.org[1] + y, f.org[2] + z, g.pad)] = pv;
      };
      if (ND == 2) {   // a 16 x 16 thread tile over the box: no divisions
        const int tx = tid & 15, ty = tid >> 4;
#pragma unroll 1
        for (int y = ty; y < ex[1]; y += 16)
#pragma unroll 1
          for (int x = tx; x < ex[0]; x += 16) put(lo[0] + x, lo[1] + y, 0);
      } else {
        const int nbox = ex[0] * ex[1] * ex[2];
        BoxWalk w(tid, kThreads, max(ex[0], 1), max(ex[1], 1));
#pragma unroll 1
        for (int i = tid; i < nbox; i += kThreads, w.next()) put(lo[0] + w.x, lo[1] + w.y, lo[2] + w.z);
      }
    }
  } else {
    // every cell (the LDS reads of eight cells are issued before the first test)
    constexpr int U = 8;
    const int n = (int)g.wcells;
    BoxWalk w(tid, kThreads, g.T[0], g.T[1]);
    for (int base = tid; base < n; base += kThreads * U) {
      int8_t pv[U], hv[U];
      uint8_t kv[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = min(base + q * kThreads, n - 1);
        pv[q] = P[i];
        hv[q] = s_hd[i];
        kv[q] = keep[i];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (base + q * kThreads < n && hv[q] < 0 && !kv[q])
          sgw[((f.org[2] + w.z) * g.pad[1] + f.org[1] + w.y) * g.pad[0] + f.org[0] + w.x] = pv[q];
        w.next();
      }
    }
  }
  if (a.ev_delta) {
    // Additive data events: what this paste changed in each successor's
    // overlap is added to that successor's block sums.  A cell changes where
    // the paste wrote it (no hard datum, new side of every seam); the old
    // value is the window read before the cut.  The sums of a group of
    // successors are gathered in the inverse-DWT buffers, then each listed
    // block goes out as one device-scope atomic add (fire and forget).  This
    // runs once per launch on each CU, so the loops are kept compact: their
    // code is fetched cold.
    const int lb = g.level, lbz = g.ndim == 3 ? g.level : 0;
#pragma unroll 1
    for (int m0 = 0; m0 < my_nsucc; m0 += ev_ng) {
      const int gm = min(ev_ng, my_nsucc - m0);
      if (m0 > 0) {
        for (int i = tid; i < gm * ev_tcl; i += kThreads) s_dsum[i] = 0;
        __syncthreads();
      }
#pragma unroll 1
      for (int mm = 0; mm < gm; ++mm) {
        const FilterDev q = s_fq[m0 + mm];   // in registers: the atomics below alias LDS
        int d[3], lo[3], ex[3];   // the box both windows cover, in this window's coordinates
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          d[ax] = f.org[ax] - q.org[ax];
          lo[ax] = max(0, -d[ax]);
          ex[ax] = max(0, min(g.T[ax], g.T[ax] - d[ax]) - lo[ax]);
        }
        int* dsum = s_dsum + mm * ev_tcl;
        auto cell = [&](int x, int y, int z) {
          const int c = idx3i(x, y, z, g.T);
          const int o = s_sg[c], h = s_hd[c], k = keep[c], p = P[c];   // one wait for all four
          const int nv = (h < 0 && !k) ? p : o;
          const int sx = x + d[0], sy = y + d[1], sz = z + d[2];
          if (nv != o && dev_in_band(g, q.orient, q.bandmask, sx, sy, sz))
            atomicAdd(&dsum[((sz >> lbz) * g.tc[1] + (sy >> lb)) * g.tc[0] + (sx >> lb)], nv - o);
        };
        if (ND == 2) {   // a 16 x 16 thread tile over the box: no divisions
          const int tx = tid & 15, ty = tid >> 4;
#pragma unroll 1
          for (int y = ty; y < ex[1]; y += 16)
#pragma unroll 1
            for (int x = tx; x < ex[0]; x += 16) cell(lo[0] + x, lo[1] + y, 0);
        } else {
          const int nbox = ex[0] * ex[1] * ex[2];
          BoxWalk w(tid, kThreads, max(ex[0], 1), max(ex[1], 1));
#pragma unroll 1
          for (int i = tid; i < nbox; i += kThreads, w.next()) cell(lo[0] + w.x, lo[1] + w.y, lo[2] + w.z);
        }
      }
      __syncthreads();
      // one thread per (successor, listed block)
#pragma unroll 1
      for (int i = tid; i < gm * a.kpad; i += kThreads) {
        const int mm = i / a.kpad, t = i - mm * a.kpad;
        const int beta = s_betas[t];
        const int v = beta >= 0 ? s_dsum[mm * ev_tcl + beta] : 0;
        if (v != 0)
          __hip_atomic_fetch_add(&a.mbuf[(long long)s_mine[m0 + mm] * kKMax + t], v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
      if (m0 + gm < my_nsucc) __syncthreads();
    }
    return;
  }
  // Successors whose last overlapping predecessor is this patch get their
  // data event here.  Every wavefront first waits for its own stores of the
  // paste; then one lane per successor counts this patch in with an
  // acquire-release atomic at device scope (its release publishes the paste,
  // its acquire makes the other predecessors' cells visible), and the patch
  // that completes a successor's count computes that successor's block sums.
  __builtin_amdgcn_s_waitcnt(0);
  if (tid == 0) s_nmine = 0;
  __syncthreads();
  if (tid < my_nsucc) {
    if (__hip_atomic_fetch_add(&a.predcnt[my_succ], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1 ==
        my_npred) {
      const int m = atomicAdd(&s_nmine, 1);
      s_mine[m] = my_succ;
#pragma unroll
      for (int q = 0; q < 5; ++q) ((int2*)&s_fq[m])[q] = my_fq[q];
    }
  }
  __syncthreads();
  const int nmine = min(s_nmine, kMaxSucc);
  int* s_msum = (int*)(dps + (long long)a.dp_batch * a.dp_stride);   // [2][tcells]
  // overlap cells of the successors, summed per level-J block; with two or
  // more left, each half of the block takes one, so both sets of reads are
  // in flight together
  constexpr int U = 16;
  const int n = (int)g.wcells;
  const int lb = g.level;   // block of a cell: coordinates shifted by J on the used axes
  const int lbz = g.ndim == 3 ? lb : 0;
  if (g.wavelet == 1) {
    // 5/3: each successor's data event is the level-J approximation of its
    // zero-filled overlap window (tc * b cells per axis), lifted in LDS;
    // blocks without a known cell of the successor compare nothing
    const int r0 = g.tc[0] * g.b[0], r1 = g.tc[1] * g.b[1], r2 = g.tc[2] * g.b[2];
    const int rc = r0 * r1 * r2;
    // int16 buffers (every lifted value is bounded by the plan's check,
    // <= 2048) over the idwt buffers and the pattern / mask / window area,
    // all free once the paste is done: the window (rc values), then the
    // passes' outputs (rc / 2, rc / 4, ...) alternating behind it
    int16_t* const lW = (int16_t*)bufA;
    int16_t* const lA = lW + rc;
    int16_t* const lB = lA + rc / 2;
    for (int mm = 0; mm < nmine; ++mm) {
      const FilterDev& fq = s_fq[mm];
      const int8_t* sgq = a.sg + (long long)fq.r * g.pcells;
      // the zero-filled window: every load of a thread's share in flight at once
      {
        constexpr int U = 8;
        BoxWalk w(tid, kThreads, r0, r1);
        for (int base = tid; base < rc; base += kThreads * U) {
          int16_t v[U];
#pragma unroll
          for (int q = 0; q < U; ++q) {
            v[q] = 0;
            if (base + q * kThreads < rc && w.x < g.T[0] && w.y < g.T[1] && w.z < g.T[2] &&
                dev_in_band(g, fq.orient, fq.bandmask, w.x, w.y, w.z))
              v[q] = sgq[((fq.org[2] + w.z) * g.pad[1] + fq.org[1] + w.y) * g.pad[0] + fq.org[0] + w.x];
            w.next();
          }
#pragma unroll
          for (int q = 0; q < U; ++q)
            if (base + q * kThreads < rc) lW[base + q * kThreads] = v[q];
        }
      }
      __syncthreads();
      int e[3] = {r0, r1, r2};
      int16_t* src = lW;
      int16_t* dst = lA;
      for (int j = 0; j < g.level; ++j)
        for (int axis = 0; axis < g.ndim; ++axis) {
          int o[3] = {e[0], e[1], e[2]};
          o[axis] >>= 1;
          const int n = e[axis];
          const int oc = o[0] * o[1] * o[2];
          const int sa = axis == 0 ? 1 : axis == 1 ? e[0] : e[0] * e[1];   // input stride along the axis
          BoxWalk w(tid, kThreads, o[0], o[1]);
          for (int i = tid; i < oc; i += kThreads, w.next()) {
            const int k2 = 2 * (axis == 0 ? w.x : axis == 1 ? w.y : w.z);
            // the line through this output: input index of position 0
            const int line = idx3i(axis == 0 ? 0 : w.x, axis == 1 ? 0 : w.y, axis == 2 ? 0 : w.z, e);
            const int x0 = src[line + mirror53(k2 - 2, n) * sa], x1 = src[line + mirror53(k2 - 1, n) * sa];
            const int x2 = src[line + k2 * sa], x3 = src[line + mirror53(k2 + 1, n) * sa];
            const int x4 = src[line + mirror53(k2 + 2, n) * sa];
            const int dl = x1 - ((x0 + x2) >> 1), dr = x3 - ((x2 + x4) >> 1);
            dst[i] = (int16_t)(x2 + ((dl + dr + 2) >> 2));
          }
          __syncthreads();
          e[axis] = o[axis];
          src = dst;
          dst = dst == lA ? lB : lA;
        }
      if (tid < a.kpad) {
        int v = 0;
        if (my_beta >= 0 && a.nbt[(long long)fq.shape * g.tcells + my_beta]) v = src[my_beta];
        a.mbuf[(long long)s_mine[mm] * kKMax + tid] = v;
      }
      __syncthreads();
    }
  }
  for (int m0 = 0; m0 < (g.wavelet == 1 ? 0 : nmine);) {
    const int gm = nmine - m0 >= 2 ? 2 : 1;
    for (int i = tid; i < gm * (int)g.tcells; i += kThreads) s_msum[i] = 0;
    __syncthreads();
    const int half = gm == 2 ? tid / (kThreads / 2) : 0;
    const int t0 = gm == 2 ? tid - half * (kThreads / 2) : tid, nt = kThreads / gm;
    const FilterDev& fq = s_fq[m0 + half];
    int* msum = s_msum + half * (int)g.tcells;
    const int8_t* sgq = a.sg + (long long)fq.r * g.pcells;
    BoxWalk w(t0, nt, g.T[0], g.T[1]);
    for (int base = t0; base < n; base += nt * U) {
      int v[U], bi[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        v[q] = 0;
        bi[q] = -1;
        if (base + q * nt < n && dev_in_band(g, fq.orient, fq.bandmask, w.x, w.y, w.z)) {
          v[q] = sgq[((fq.org[2] + w.z) * g.pad[1] + fq.org[1] + w.y) * g.pad[0] + fq.org[0] + w.x];
          bi[q] = ((w.z >> lbz) * g.tc[1] + (w.y >> lb)) * g.tc[0] + (w.x >> lb);
        }
        w.next();
      }
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (bi[q] >= 0) atomicAdd(&msum[bi[q]], v[q]);
    }
    __syncthreads();
    if (a.learn)   // the successors' queries for the proposer
      for (int mm = 0; mm < gm; ++mm)
        pca_query(s_msum + mm * (int)g.tcells, (int)g.tcells, a.learn, a.pca_P, a.pca_mu,
                  a.qbuf + (long long)s_mine[m0 + mm] * (a.learn + 4));
    if (tid < a.kpad)
      for (int mm = 0; mm < gm; ++mm)
        a.mbuf[(long long)s_mine[m0 + mm] * kKMax + tid] =
            my_beta >= 0 ? s_msum[mm * (int)g.tcells + my_beta] : 0;
    __syncthreads();
    m0 += gm;
  }
}

}  // namespace

namespace {
// One kernel per (dimension, depth of the coefficient tree).
void launch_finalize(int ndim, int tree_level, unsigned blocks, size_t lds, hipStream_t st, const FinArgs& fa,
                     hipEvent_t e0, hipEvent_t e1) {
#define CCW_FIN(ND, TJ) \
  hipExtLaunchKernelGGL((k_finalize<ND, TJ>), dim3(blocks), dim3(kThreads), (uint32_t)lds, st, e0, e1, 0, fa)
  if (ndim == 2) {
    if (tree_level == 1) CCW_FIN(2, 1);
    else if (tree_level == 2) CCW_FIN(2, 2);
    else if (tree_level == 3) CCW_FIN(2, 3);
    else CCW_FIN(2, 0);
  } else {
    if (tree_level == 1) CCW_FIN(3, 1);
    else if (tree_level == 2) CCW_FIN(3, 2);
    else CCW_FIN(3, 0);
  }
#undef CCW_FIN
}
}  // namespace

extern "C" int64_t ccwsim_simulate_workspace_size(const ccwsim_params* p) {
  if (!p) {
    fail(CCWSIM_ERR_INVALID_ARG, "null params");
    return -1;
  }
  std::shared_ptr<Plan> Ph;
  if (get_plan(*p, &Ph)) return -1;
  Plan* P = Ph.get();
  return P->ws_total;
}

namespace {
// Scan variant for this plan: the forced value (tests), else the tuned
// one, within what the LDS allows.
int scan_group_of(const Plan* P) {
  const int V = g_scan_g_force != 0 ? g_scan_g_force : P->scan_g;
  if (V == kScanFilterMajor) return V;
  const int G = V > P->scan_g_max ? P->scan_g_max : V;
  return G >= 8 ? 8 : G >= 4 ? 4 : G >= 2 ? 2 : 1;
}
int group_index(int V) { return V == 8 ? 3 : V == 4 ? 2 : V == 2 ? 1 : 0; }   // filter-major: single tiles
bool sel_fused_of(const Plan* P) {
  if (!P->sel_fused_ok) return false;
  if (g_sel_force != 0) return g_sel_force == 3;
  if (g_scan_g_force != 0) return false;   // a forced scan layout runs with stored keys
  return P->sel_fused;
}
bool sel_rows_of(const Plan* P) {
  if (!P->rows_ok || sel_fused_of(P)) return false;
  return g_sel_force != 0 ? g_sel_force == 2 : P->sel_rows;
}

int enqueue_simulate(const Plan* P, const ccwsim_params* p, const int8_t* ti, int64_t n_hd, const int32_t* hd_real,
                     const int32_t* hd_pos, const int8_t* hd_val, int8_t* out, int32_t* chosen, void* workspace,
                     hipStream_t st) {
  const Geom& g = P->g;
  unsigned char* ws = (unsigned char*)workspace;
  _Float16* Kh = (_Float16*)(ws + P->ws_kh);
  int32_t* Ki = (int32_t*)(ws + P->ws_ki);
  int32_t* det = (int32_t*)(ws + P->ws_det);
  int32_t* tmp = (int32_t*)(ws + P->ws_tmp);
  int32_t* energy = (int32_t*)(ws + P->ws_energy);
  unsigned char* tbl = ws + P->ws_tbl;
  int8_t* sg = (int8_t*)(ws + P->ws_sg);
  int8_t* hdmap = (int8_t*)(ws + P->ws_hdmap);
  int32_t* mbuf = (int32_t*)(ws + P->ws_mbuf);
  unsigned long long* report = (unsigned long long*)(ws + P->ws_report);
  int32_t* predcnt = (int32_t*)(ws + P->ws_predcnt);
  int32_t* hd_off = (int32_t*)(ws + P->ws_hdoff);
  HdEnt* hd_ent = (HdEnt*)(ws + P->ws_hdent);
  uint32_t* hdmask = P->hdm ? (uint32_t*)(ws + P->ws_hdmask) : nullptr;
  HdBits* hd_bits = P->hdm ? (HdBits*)(ws + P->ws_hdbits) : nullptr;
  uint64_t* keys = (uint64_t*)(ws + P->ws_keys);
  uint64_t* rowmin = (uint64_t*)(ws + P->ws_rowmin);
  int32_t* rowcnt = (int32_t*)(ws + P->ws_rowcnt);
  int32_t* drawn = (int32_t*)(ws + P->ws_err);
  // the learned proposer's patches that fall back are scanned with the fused selection
  const bool fused = P->lp || sel_fused_of(P);
  const bool sel_rows = !fused && sel_rows_of(P);
  const int32_t* kbeta = (const int32_t*)(tbl + P->off_kbeta);
  const int32_t* nbt = (const int32_t*)(tbl + P->off_nbt);
  const FilterDev* filters = (const FilterDev*)(tbl + P->off_filters);
  const TileDev* tiles = (const TileDev*)(tbl + P->off_tiles);
  ScanRec* recs = (ScanRec*)(tbl + P->off_recs);
  const int2* groups = (const int2*)(tbl + P->off_groups);
  const int32_t* npred = (const int32_t*)(tbl + P->off_npred);
  const int32_t* succ_off = (const int32_t*)(tbl + P->off_succoff);
  const int32_t* succ = (const int32_t*)(tbl + P->off_succ);

  HIP_TRY(hipMemcpyAsync(tbl, P->tbl, P->tbl_bytes, hipMemcpyHostToDevice, st));
  // TI transform and energy rows (depend on the TI only)
  {
    ProfScope ps(CCWSIM_KIND_DWT, st);
    if (g.wavelet == 1) {
      // J levels of x, y (, z) lifting passes, ping-pong through two
      // buffers; the last pass writes the approximation grid
      int32_t* lb[2] = {(int32_t*)(ws + P->ws_lift),
                        (int32_t*)(ws + P->ws_lift + align256(((long long)g.np[0] * g.np[1] * g.np[2] / 2 + 1) * 4))};
      int e[3] = {g.np[0], g.np[1], g.np[2]};
      const void* srcp = ti;
      const int npass = g.level * g.ndim;
      for (int q = 0; q < npass; ++q) {
        const int axis = q % g.ndim;
        const bool last = q == npass - 1;
        int32_t* dstp = last ? Ki : lb[q & 1];
        const long long outc = (long long)e[0] * e[1] * e[2] / 2;
        if (q == 0)
          k_lift53<true><<<nblocks(outc), kThreads, 0, st>>>(srcp, dstp, last ? Kh : nullptr, e[0], e[1], e[2],
                                                             axis, g);
        else
          k_lift53<false><<<nblocks(outc), kThreads, 0, st>>>(srcp, dstp, last ? Kh : nullptr, e[0], e[1], e[2],
                                                              axis, g);
        e[axis] >>= 1;
        srcp = dstp;
      }
      if (npass == 0) CCW_TRY(launch_dwt(g, ti, Ki, Kh, det, tmp, st));   // J = 0: the TI itself
      HIP_TRY(hipGetLastError());
    } else if (P->tree_level) {
      const long long gc = (long long)g.G[0] * g.G[1] * g.G[2];
      if (g.ndim == 2 && g.level == 1) k_dwt_tree<2, 1><<<nblocks(gc), kThreads, 0, st>>>(ti, det, Ki, Kh, g);
      else if (g.ndim == 2 && g.level == 3) k_dwt_tree<2, 3><<<nblocks(gc), kThreads, 0, st>>>(ti, det, Ki, Kh, g);
      else if (g.ndim == 2) k_dwt_tree<2, 2><<<nblocks(gc), kThreads, 0, st>>>(ti, det, Ki, Kh, g);
      else if (g.level == 1) k_dwt_tree<3, 1><<<nblocks(gc), kThreads, 0, st>>>(ti, det, Ki, Kh, g);
      else k_dwt_tree<3, 2><<<nblocks(gc), kThreads, 0, st>>>(ti, det, Ki, Kh, g);
      HIP_TRY(hipGetLastError());
    } else {
      CCW_TRY(launch_dwt(g, ti, Ki, Kh, det, tmp, st));
    }
    if (p->precision == 1) {
      const long long gc = (long long)g.G[0] * g.G[1] * g.G[2];
      k_to_bf16<<<nblocks(gc), kThreads, 0, st>>>(Ki, (__bf16*)Kh, gc);
      HIP_TRY(hipGetLastError());
    }
  }
  if (p->score_mode == 0) {
    ProfScope ps(CCWSIM_KIND_ENERGY, st);
    k_energy<<<nblocks((long long)P->n_shapes * g.ncand), kThreads, 0, st>>>(Ki, nbt, P->n_shapes, energy, g);
    HIP_TRY(hipGetLastError());
  }
  // learned proposer: principal components of the candidates' windows
  double* qbuf = P->learn ? (double*)(ws + P->ws_qbuf) : nullptr;
  float* pca_mu = P->learn ? (float*)(ws + P->ws_pca_mu) : nullptr;
  float* pca_P = P->learn ? (float*)(ws + P->ws_pca_P) : nullptr;
  float* emb = P->learn ? (float*)(ws + P->ws_emb) : nullptr;
  float2* rn = P->learn ? (float2*)(ws + P->ws_rn) : nullptr;
  if (P->learn) {
    ProfScope ps(CCWSIM_KIND_LEARN, st);
    float* part = (float*)(ws + P->ws_pca_part);
    float* cov = (float*)(ws + P->ws_pca_cov);
    const int n = (int)g.tcells;
    const int R = (n * n + kThreads - 1) / kThreads;
    if (R <= 9) k_pca_moments<9><<<kPcaParts, kThreads, 0, st>>>(Ki, g, part);
    else if (R <= 36) k_pca_moments<36><<<kPcaParts, kThreads, 0, st>>>(Ki, g, part);
    else if (R <= 81) k_pca_moments<81><<<kPcaParts, kThreads, 0, st>>>(Ki, g, part);
    else k_pca_moments<144><<<kPcaParts, kThreads, 0, st>>>(Ki, g, part);
    k_pca_reduce<<<nblocks((long long)n * n + n), kThreads, 0, st>>>(part, kPcaParts, g, cov, pca_mu);
    k_pca_fit<<<1, kThreads, 0, st>>>(cov, pca_mu, g, P->learn, pca_P);
    if (g_pca_skew != 0.f)
      k_pca_skew<<<nblocks((long long)g.tcells), kThreads, 0, st>>>(pca_P, P->learn, (int)g.tcells, g_pca_skew);
    k_pca_embed<<<nblocks(g.ncand), kThreads, 0, st>>>(Ki, g, P->learn, pca_mu, pca_P, emb, rn);
    HIP_TRY(hipGetLastError());
  }
  // learned proposer: the level-J grid narrowed for the proposal's LDS
  void* lp_grid = P->lp ? (void*)(ws + P->ws_lp_grid) : nullptr;
  if (P->lp) {
    ProfScope ps(CCWSIM_KIND_LEARN, st);
    k_fill_i32<<<1, kThreads, 0, st>>>((int32_t*)(ws + P->ws_lp_dcount), 64, 0);   // count and ticket
    const long long gc = (long long)g.G[0] * g.G[1] * g.G[2];
    const long long npad = lp_prop_grid_bytes(g, P->lp_kt) / P->lp_kt;
    if (P->lp_kt == 1) k_lp_narrow<int8_t><<<nblocks(npad), kThreads, 0, st>>>(Ki, gc, npad, (int8_t*)lp_grid);
    else k_lp_narrow<int16_t><<<nblocks(npad), kThreads, 0, st>>>(Ki, gc, npad, (int16_t*)lp_grid);
    HIP_TRY(hipGetLastError());
  }
  // grids start unknown (-1) except for hard data
  const long long allp = (long long)p->n_real * g.pcells;
  {
    ProfScope ps(CCWSIM_KIND_INIT, st);
    k_fill_i8<<<nblocks(allp), kThreads, 0, st>>>(sg, allp, (int8_t)-1);
    k_fill_i8<<<nblocks(allp), kThreads, 0, st>>>(hdmap, allp, (int8_t)-1);
    if (n_hd > 0)
      k_scatter_hd<<<nblocks(n_hd), kThreads, 0, st>>>(sg, hdmap, g, p->n_real, n_hd, hd_real, hd_pos, hd_val);
    k_fill_i32<<<nblocks(P->nfilters), kThreads, 0, st>>>(predcnt, P->nfilters, 0);
    k_fill_i32<<<1, kThreads, 0, st>>>((int32_t*)report, 32, 0);
    if (P->ev_delta)
      k_event_init<<<(unsigned)P->nfilters, kThreads, (size_t)g.tcells * 4, st>>>(g, filters, kbeta, sg, mbuf,
                                                                                   P->kpad);
    if (n_hd > 0) {
      k_hd_bin<false><<<(unsigned)P->nfilters, kThreads, 0, st>>>(g, filters, hdmap, hd_off, hd_ent, P->hd_cap,
                                                                   nullptr, P->hm);
      k_exclusive_scan<<<1, kThreads, 0, st>>>(hd_off, P->nfilters);
      k_hd_bin<true><<<(unsigned)P->nfilters, kThreads, 0, st>>>(g, filters, hdmap, hd_off, hd_ent, P->hd_cap,
                                                                  hd_bits, P->hm);
      if (hdmask) {
        const long long nw = (long long)P->hm.rz * P->hm.ry * P->hm.rs;
        k_hd_mask<<<nblocks(nw), kThreads, 0, st>>>(g, P->hm, ti, hdmask, nw);
      }
      k_recs_hd<<<nblocks(P->nrecs), kThreads, 0, st>>>(recs, P->nrecs, hd_off);
    }
    HIP_TRY(hipGetLastError());
  }

  ScanArgs sa = {};
  sa.g = g;
  sa.Kop = Kh;
  sa.kbeta = kbeta;
  sa.mbuf = mbuf;
  sa.hd_ent = hd_ent;
  sa.hm = P->hm;
  sa.hdm = n_hd > 0 ? hdmask : nullptr;
  sa.hd_bits = hd_bits;
  sa.energy = energy;
  sa.ti = ti;
  sa.keys = keys;
  sa.rowmin = rowmin;
  sa.seed = p->seed;
  sa.kpad = P->kpad;
  sa.W = P->W;
  sa.score_mode = p->score_mode;
  sa.rowmin_only = !P->learn && sel_rows;
  sa.standalone = 0;
  sa.has_hd = n_hd > 0;
  sa.rowcnt = rowcnt;
  sa.ksel = std::min(p->shortlist > 0 ? p->shortlist : p->top_k, g.ncand);
  sa.gbits = P->sel_gbits;
  sa.n_bm = P->sel_n_bm;

  FinArgs fa = {};
  fa.g = g;
  fa.keys = keys;
  fa.rowmin = rowmin;
  fa.rowcnt = fused ? rowcnt : nullptr;
  fa.filters_all = filters;
  fa.npred = npred;
  fa.succ_off = succ_off;
  fa.succ = succ;
  fa.predcnt = predcnt;
  fa.kbeta = kbeta;
  fa.nbt = nbt;
  fa.mbuf = mbuf;
  fa.ev_delta = P->ev_delta ? 1 : 0;
  fa.report = report;
  fa.kpad = P->kpad;
  fa.shortlist = p->shortlist;
  fa.score_mode = p->score_mode;
  fa.cand_cap = P->cand_cap;
  fa.coef_lds = P->coef_lds;
  fa.rows_max = P->rows_max;
  fa.has_hd = n_hd > 0;
  fa.dp_wave = P->dp_wave;
  fa.dp_evs = P->dp_evs;
  fa.Ki = Ki;
  fa.det = det;
  fa.tree = det;
  fa.sg = sg;
  fa.hdmap = hdmap;
  fa.chosen_log = chosen;
  fa.seed = p->seed;
  fa.buf_cells = P->buf_cells;
  fa.top_k = p->top_k;
  fa.cut = p->cut;
  fa.nsteps = P->nsteps_raster;
  fa.dp_stride = P->dp_stride;
  fa.dp_batch = P->dp_batch;
  fa.learn = P->learn;
  fa.rescore_rows = P->learn || sel_rows;
  fa.drawn = drawn;
  fa.rows_exact = !P->learn;
  fa.hdm = n_hd > 0 ? hdmask : nullptr;
  fa.hd_bits = hd_bits;
  fa.hm = P->hm;
  fa.qbuf = qbuf;
  fa.pca_P = pca_P;
  fa.pca_mu = pca_mu;
  fa.energy = energy;
  fa.hd_off = hd_off;
  fa.hd_ent = hd_ent;
  fa.ti = ti;
  fa.learn_off = P->learn_off;
  fa.learn_kbr = P->learn_kbr;
  fa.learn_w = P->learn_w;

  ProxyArgs xa = {};
  xa.g = g;
  xa.qbuf = qbuf;
  xa.emb = emb;
  xa.rn = rn;
  xa.energy = energy;
  xa.hd_ent = hd_ent;
  xa.ti = ti;
  xa.rowmin = rowmin;
  xa.D = P->learn;
  xa.has_hd = n_hd > 0;

  const unsigned rows = (unsigned)(g.cand[1] * g.cand[2]);
  const int G = scan_group_of(P);
  const int gix = group_index(G);
  const size_t scan_lds = scan_group_lds(g.tc[1] * g.tc[2], P->W, P->kpad, G == kScanFilterMajor ? 1 : G);
  for (const StepRange& s : P->steps) {
    sa.fbegin = s.fbegin;
    sa.tiles = tiles + s.tbegin;
    sa.recs = recs + (long long)s.tbegin * kFiltersPerTile;
    sa.ntiles = s.tcount;
    sa.groups = groups + s.gbegin[gix];
    sa.n_ginline = s.gcount[gix] <= kScanGroupsInline ? s.gcount[gix] : 0;
    if (sa.n_ginline)
      memcpy(sa.groups_inline, P->tbl_host.data() + P->off_groups + (size_t)s.gbegin[gix] * sizeof(int2),
             (size_t)s.gcount[gix] * sizeof(int2));
    if (P->lp) {
      // proposals, then the patches the gate sends back packed into scan
      // tiles, then the scan over those
      LpPropArgs la = {};
      la.g = g;
      la.index = (const unsigned char*)p->proposer;
      la.grid = lp_grid;
      la.probe = p->lp_probe;
      la.cap = P->lp_cap;
      la.top_k = p->top_k;
      la.kpad = P->kpad;
      la.gate = p->lp_gate;
      la.seed = p->seed;
      la.filters = filters + s.fbegin;
      la.fbegin = s.fbegin;
      la.kbeta = kbeta;
      la.nbt = nbt;
      la.mbuf = mbuf;
      la.hd_off = n_hd > 0 ? hd_off : nullptr;
      la.sel = (uint64_t*)(ws + P->ws_lp_sel);
      la.ok = (int32_t*)(ws + P->ws_lp_ok);
      la.report = report;
      la.ticket = (int32_t*)(ws + P->ws_lp_dcount) + 16;
      LpCompactArgs& ca = la.cmp;
      ca.tiles = tiles + s.tbegin;
      ca.recs = recs + (long long)s.tbegin * kFiltersPerTile;
      ca.ntiles = s.tcount;
      ca.nf = s.fcount;
      ca.n_orient = P->n_orient;
      ca.fbegin = s.fbegin;
      ca.ok = la.ok;
      ca.dtiles = (TileDev*)(ws + P->ws_lp_dtiles);
      ca.drecs = (ScanRec*)(ws + P->ws_lp_drecs);
      ca.map = (int32_t*)(ws + P->ws_lp_map);
      ca.dcount = (int32_t*)(ws + P->ws_lp_dcount);
      {
        ProfKernel pk(CCWSIM_KIND_LEARN);
        if (P->lp_kt == 1)
          hipExtLaunchKernelGGL(k_lp_propose<int8_t>, dim3((unsigned)s.fcount), dim3(kThreads), P->lp_lds, st, pk.a,
                                pk.b, 0, la);
        else
          hipExtLaunchKernelGGL(k_lp_propose<int16_t>, dim3((unsigned)s.fcount), dim3(kThreads), P->lp_lds, st, pk.a,
                                pk.b, 0, la);
      }
      ScanArgs sf = sa;
      sf.kpad = P->sel_kk;
      sf.klist = P->kpad;
      sf.W = P->sel_W;
      sf.segoff = (const int32_t*)(tbl + P->off_segoff);
      sf.taps = (const int32_t*)(tbl + P->off_taps);
      sf.n_tinline = 0;
      sf.tiles = ca.dtiles;
      sf.recs = ca.drecs;
      sf.fbegin = 0;
      sf.ntiles_dyn = ca.dcount;
      ProfKernel pk(CCWSIM_KIND_SCAN);
      launch_scan_sel(p->precision, n_hd > 0, kEnStage, rows, s.tcount, n_hd > 0 ? P->sel_lds_hd : P->sel_lds_nohd,
                      st, sf, pk.a, pk.b);
    } else if (P->learn) {
      xa.tiles = tiles + s.tbegin;
      xa.recs = recs + (long long)s.tbegin * kFiltersPerTile;
      xa.fbegin = s.fbegin;
      ProfScope ps(CCWSIM_KIND_SCAN, st);
      k_proxy<<<dim3(rows, (unsigned)s.tcount), kThreads, P->proxy_lds, st>>>(xa);
    } else if (fused) {
      ScanArgs sf = sa;
      sf.kpad = P->sel_kk;
      sf.klist = P->kpad;
      sf.W = P->sel_W;
      sf.segoff = (const int32_t*)(tbl + P->off_segoff);
      sf.taps = (const int32_t*)(tbl + P->off_taps);
      sf.n_tinline = s.tcount <= 32 ? s.tcount : 0;
      if (sf.n_tinline)
        memcpy(sf.tiles_inline, P->tbl_host.data() + P->off_tiles + (size_t)s.tbegin * sizeof(TileDev),
               (size_t)s.tcount * sizeof(TileDev));
      ProfKernel pk(CCWSIM_KIND_SCAN);
      launch_scan_sel(p->precision, n_hd > 0, kEnStage, rows, s.tcount, n_hd > 0 ? P->sel_lds_hd : P->sel_lds_nohd,
                      st, sf, pk.a, pk.b);
    } else {
      ProfKernel pk(CCWSIM_KIND_SCAN);
      launch_scan(p->precision, G, rows, s.gcount[gix], scan_lds, st, sa, pk.a, pk.b);
    }
    fa.filters = filters + s.fbegin;
    fa.fbegin = s.fbegin;
    if (P->lp) {
      fa.lp_map = (const int32_t*)(ws + P->ws_lp_map);
      fa.lp_sel = (const uint64_t*)(ws + P->ws_lp_sel);
    }
    fa.n_inline = s.fcount <= kFinInline ? s.fcount : 0;
    if (fa.n_inline)
      memcpy(fa.recs_inline, P->tbl_host.data() + P->off_filters + (size_t)s.fbegin * sizeof(FilterDev),
             (size_t)s.fcount * sizeof(FilterDev));
    {
      ProfKernel pk(CCWSIM_KIND_FINALIZE);
      launch_finalize(g.ndim, P->tree_level, (unsigned)s.fcount, P->fin_lds, st, fa, pk.a, pk.b);
    }
  }
  HIP_TRY(hipGetLastError());
  {
    ProfScope ps(CCWSIM_KIND_CROP, st);
    k_crop<<<nblocks((long long)p->n_real * g.sg[0] * g.sg[1] * g.sg[2]), kThreads, 0, st>>>(sg, out, g, p->n_real);
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}
}  // namespace

namespace {
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;   // most recent last
bool g_graphs_on = true;
constexpr size_t kMaxGraphs = 64;

void drop_graphs() {
  for (GraphEntry& e : g_graphs) (void)hipGraphExecDestroy(e.exec);
  g_graphs.clear();
}
}  // namespace

namespace {
// Graph keys begin with the bytes of the parameters, i.e. the plan key.
void drop_graphs_of(const std::string& plan_key) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    if (g_graphs[i].key.compare(0, plan_key.size(), plan_key) == 0) {
      (void)hipGraphExecDestroy(g_graphs[i].exec);
      g_graphs.erase(g_graphs.begin() + i);
    } else {
      ++i;
    }
  }
}
}  // namespace

namespace {
// Tuned tile counts per scan workgroup, keyed by the scan's shape; kept in
// memory and, when CCWSIM_TUNE_FILE names a file, in that JSON object.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const Plan* P, const ccwsim_params* p) {
  const Geom& g = P->g;
  int maxt = 0;
  for (const StepRange& s : P->steps) maxt = std::max(maxt, s.tcount);
  char buf[256];
  snprintf(buf, sizeof buf, "d%d_cand%dx%dx%d_tc%dx%dx%d_k%d_tiles%d_prec%d_hd%d", g.ndim, g.cand[0], g.cand[1],
           g.cand[2], g.tc[0], g.tc[1], g.tc[2], P->kpad, maxt, p->precision, p->max_hard_data > 0 ? 1 : 0);
  return buf;
}

void tune_load_once() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* f = getenv("CCWSIM_TUNE_FILE");
  if (!f) return;
  FILE* fp = fopen(f, "r");
  if (!fp) return;
  char line[512], key[400];
  int v = 0;
  while (fgets(line, sizeof line, fp))
    if (sscanf(line, " \"%399[^\"]\" : %d", key, &v) == 2) {
      const int b = v > 150 ? v - 200 : v > 50 ? v - 100 : v;
      if (b == -1 || b == 1 || b == 2 || b == 4 || b == 8) g_tune[key] = v;
    }
  fclose(fp);
}

void tune_save() {
  const char* f = getenv("CCWSIM_TUNE_FILE");
  if (!f) return;
  FILE* fp = fopen(f, "w");
  if (!fp) return;
  fprintf(fp, "{\n");
  size_t i = 0;
  for (const auto& kv : g_tune) fprintf(fp, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < g_tune.size() ? "," : "");
  fprintf(fp, "}\n");
  fclose(fp);
}

// Before tuning: the largest tile count that still gives two workgroups per
// CU on the widest step.
int scan_group_guess(const Plan* P) {
  int maxt = 0;
  for (const StepRange& s : P->steps) maxt = std::max(maxt, s.tcount);
  const long long rows = (long long)P->g.cand[1] * P->g.cand[2];
  int G = 1;
  for (int c : {2, 4, 8})
    if (c <= P->scan_g_max && c <= maxt && rows * ((maxt + c - 1) / c) >= 512) G = c;
  return G;
}
}  // namespace

extern "C" int ccwsim_set_scan_group(int g) {
  if (g != 0 && g != -1 && g != 1 && g != 2 && g != 4 && g != 8)
    return fail(CCWSIM_ERR_INVALID_ARG, "tiles per scan workgroup must be 0 (tuned), -1 (filter-major), 1, 2, 4 or 8");
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    drop_graphs();   // captured graphs hold the previous choice
  }
  g_scan_g_force = g;
  return CCWSIM_OK;
}

extern "C" int ccwsim_set_selection(int mode) {
  if (mode < 0 || mode > 3)
    return fail(CCWSIM_ERR_INVALID_ARG,
                "selection must be 0 (tuned), 1 (stored keys), 2 (row minima) or 3 (fused into the scan)");
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    drop_graphs();   // captured graphs hold the previous choice
  }
  g_sel_force = mode;
  return CCWSIM_OK;
}

extern "C" int ccwsim_set_proposer_skew(float s) {
  if (!(s == s) || s < 0.f || s > 4.f) return fail(CCWSIM_ERR_INVALID_ARG, "skew must be in [0, 4]");
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    drop_graphs();
  }
  g_pca_skew = s;
  return CCWSIM_OK;
}

extern "C" int ccwsim_simulate(const ccwsim_params* p, const int8_t* ti, int64_t n_hd, const int32_t* hd_real,
                               const int32_t* hd_pos, const int8_t* hd_val, int8_t* out, int32_t* chosen,
                               void* workspace, int64_t workspace_bytes, void* stream) {
  if (!p || !ti || !out) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (n_hd < 0 || (n_hd > 0 && (!hd_real || !hd_pos || !hd_val)))
    return fail(CCWSIM_ERR_INVALID_ARG, "hard data pointers");
  std::shared_ptr<Plan> Ph;
  CCW_TRY(get_plan(*p, &Ph));
  Plan* P = Ph.get();
  if (!workspace || workspace_bytes < P->ws_total)
    return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", (long long)P->ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (n_hd > p->max_hard_data)
    return fail(CCWSIM_ERR_INVALID_ARG, "%lld hard data exceed max_hard_data = %d", (long long)n_hd, p->max_hard_data);
  CCW_TRY(plan_pin(P));
  hipStream_t st = as_stream(stream);
  if (P->lp) {
    // the index header, read back unless the stream is being captured (the
    // proposal kernel checks it again and sends every patch to the scan
    // when it does not match)
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cst));
    if (cst == hipStreamCaptureStatusNone && P->lp_checked != p->proposer) {
      CCW_TRY(lp_index_check(p->proposer, P->g, st, nullptr));
      P->lp_checked = p->proposer;
    }
    CCW_TRY(lp_lds_allow(P->lp_kt, P->lp_lds));
  }
  bool prof;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof = g_prof_on;
  }
  // First call of a plan: look the scan shape up in the tuning table, else
  // run eagerly once (a full, valid call) and time the widest step's scan
  // for each variant (output layout, tiles per workgroup).
  if (!P->tuned && g_scan_g_force == 0 && g_sel_force == 0 && !P->learn && !P->lp) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_once();
    const std::string tk = tune_key(P, p);
    const auto it = g_tune.find(tk);
    if (it != g_tune.end()) {
      // stored as the tiles per workgroup, plus 100 for the row-minima
      // selection, plus 200 for the selection fused into the scan
      const int v = it->second;
      P->sel_fused = v > 150 && P->sel_fused_ok;
      P->sel_rows = v > 50 && v < 150 && P->rows_ok;
      P->scan_g = v > 150 ? v - 200 : v > 50 ? v - 100 : v;
      P->tuned = true;
    } else {
      hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
      HIP_TRY(hipStreamIsCapturing(st, &cst));
      P->scan_g = scan_group_guess(P);
      if (cst == hipStreamCaptureStatusNone) {
        // every variant gives the same realizations, so each timed run is a
        // valid call; the last one's output is returned
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        float best_ms = 3.4e38f;
        int best = 1, rc = CCWSIM_OK;
        bool best_rows = false, best_fused = false;
        auto try_variant = [&](int c, bool rows, bool fusedv = false) {
          P->scan_g = c;
          P->sel_rows = rows;
          P->sel_fused = fusedv;
          HIP_TRY(hipEventRecord(e0, st));
          rc = enqueue_simulate(P, p, ti, n_hd, hd_real, hd_pos, hd_val, out, chosen, workspace, st);
          if (rc != CCWSIM_OK) return rc;
          HIP_TRY(hipEventRecord(e1, st));
          HIP_TRY(hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best_ms * 0.95f) {   // another variant must beat the first by 5 %
            best_ms = ms;
            best = c;
            best_rows = rows;
            best_fused = fusedv;
          }
          return CCWSIM_OK;
        };
        // one untimed call first: the first call of a process pays one-time
        // costs (kernel loading, cold caches) that would bias the first variant
        P->scan_g = 1;
        P->sel_rows = false;
        P->sel_fused = P->sel_fused_ok;
        rc = enqueue_simulate(P, p, ti, n_hd, hd_real, hd_pos, hd_val, out, chosen, workspace, st);
        if (rc != CCWSIM_OK) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return rc;
        }
        // the selection fused into the scan first (it writes the fewest keys)
        if (P->sel_fused_ok) try_variant(1, false, true);
        // the scan's layout and tiles with stored keys, then the row-minima
        // selection (no stored keys, exact rescoring of the best rows) with
        // the best layout and with single tiles
        for (int c : {1, kScanFilterMajor, 2, 4, 8}) {
          if (rc != CCWSIM_OK || c > P->scan_g_max) break;
          if (try_variant(c, false) != CCWSIM_OK) break;
        }
        if (rc == CCWSIM_OK && P->rows_ok) {
          const int kb = best_fused ? 1 : best;
          if (try_variant(kb, true) == CCWSIM_OK && kb != 1) try_variant(1, true);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        P->scan_g = best;
        P->sel_rows = best_rows;
        P->sel_fused = best_fused;
        if (rc == CCWSIM_OK) {
          P->tuned = true;
          g_tune[tk] = best + (best_fused ? 200 : best_rows ? 100 : 0);
          tune_save();
        }
        return rc;
      }
    }
  }
  if (prof || !g_graphs_on)
    return enqueue_simulate(P, p, ti, n_hd, hd_real, hd_pos, hd_val, out, chosen, workspace, st);

  // The launch sequence depends only on the parameters and the buffers, so it
  // is captured once into a HIP graph and replayed on the caller's stream.
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::string key((const char*)p, sizeof *p);
  const void* ptrs[8] = {ti, hd_real, hd_pos, hd_val, out, chosen, workspace, (const void*)(intptr_t)n_hd};
  key.append((const char*)ptrs, sizeof ptrs);
  key.append((const char*)&dev, sizeof dev);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size(); ++i) {
    if (g_graphs[i].key == key) {
      GraphEntry e = g_graphs[i];
      g_graphs.erase(g_graphs.begin() + i);
      g_graphs.push_back(e);
      HIP_TRY(hipGraphLaunch(e.exec, st));
      return CCWSIM_OK;
    }
  }
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(CCWSIM_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  const int rc = enqueue_simulate(P, p, ti, n_hd, hd_real, hd_pos, hd_val, out, chosen, workspace, cs);
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc != CCWSIM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(CCWSIM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(CCWSIM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  if (g_graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(g_graphs.front().exec);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back({key, exec});
  HIP_TRY(hipGraphLaunch(exec, st));
  return CCWSIM_OK;
}

extern "C" int ccwsim_set_graphs(int on) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  g_graphs_on = on != 0;
  if (!g_graphs_on) drop_graphs();
  return CCWSIM_OK;
}

extern "C" void ccwsim_release_caches(void) {
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    drop_graphs();
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = false;
  }
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.clear();
}

extern "C" int ccwsim_cache_counts(int64_t* plans, int64_t* graphs) {
  if (!plans || !graphs) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    *plans = (int64_t)g_plans.size();
  }
  std::lock_guard<std::mutex> lk(g_graph_mu);
  *graphs = (int64_t)g_graphs.size();
  return CCWSIM_OK;
}

extern "C" int ccwsim_simulate_stats(const ccwsim_params* p, ccwsim_plan_stats* out) {
  if (!p || !out) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  std::shared_ptr<Plan> Ph;
  CCW_TRY(get_plan(*p, &Ph));
  Plan* P = Ph.get();
  const Geom& g = P->g;
  out->patches = P->patches;
  out->wavefront_steps = (int64_t)P->steps.size();
  out->candidates = g.ncand;
  out->or_blocks = P->or_blocks;
  out->scan_flops = 2.0 * (double)P->or_blocks * (double)g.ncand;
  out->key_bytes = 2.0 * 8.0 * (double)P->patches * (double)g.ncand;
  out->cells = (double)p->n_real * g.sg[0] * g.sg[1] * g.sg[2];
  const double rows = (double)g.cand[1] * g.cand[2];
  const double krows = std::min<double>(std::min(p->shortlist > 0 ? p->shortlist : p->top_k, g.ncand), rows);
  // windows, row minima, the best rows' keys, coefficients, paste; then the
  // successors' events: read back from the grid and written once (4 B per
  // listed block), or added to by every predecessor (4 B per listed block
  // and successor link)
  const double per_patch = 2.0 * g.wcells + 8.0 * rows + 8.0 * krows * g.cand[0] + 4.0 * g.wcells + g.wcells;
  out->fin_bytes = per_patch * (double)P->patches +
                   (P->ev_delta ? 4.0 * P->kpad * (double)P->succ_links
                                : (double)P->band_cells + 4.0 * P->kpad * (double)P->patches);
  return CCWSIM_OK;
}

extern "C" int ccwsim_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return CCWSIM_OK;
}

extern "C" int ccwsim_profile_read(double* ms, int64_t* launches) {
  if (!ms || !launches) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int k = 0; k < CCWSIM_NUM_KINDS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  int rc = CCWSIM_OK;
  for (const ProfRec& r : g_prof_recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      rc = fail(CCWSIM_ERR_HIP, "profiling events could not be read");
    ms[r.kind] += t;
    launches[r.kind] += 1;
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  return rc;
}

extern "C" int ccwsim_simulate_report(const ccwsim_params* p, const void* workspace, int64_t workspace_bytes,
                                      int64_t* out, void* stream) {
  if (!p || !workspace || !out) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  std::shared_ptr<Plan> Ph;
  CCW_TRY(get_plan(*p, &Ph));
  Plan* P = Ph.get();
  if (workspace_bytes < P->ws_total) return fail(CCWSIM_ERR_WORKSPACE, "workspace too small");
  unsigned long long v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipStream_t st = as_stream(stream);
  HIP_TRY(hipMemcpyAsync(v, (const unsigned char*)workspace + P->ws_report, sizeof v, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < 8; ++i) out[i] = (int64_t)v[i];
  return CCWSIM_OK;
}

namespace {
// Every patch's data event as the scan takes it (known cells and code sums
// per template block), with its realization and raster step.
__global__ __launch_bounds__(kThreads) void k_export_events(Geom g, const FilterDev* __restrict__ filters,
                                                            const int32_t* __restrict__ kbeta,
                                                            const int32_t* __restrict__ nbt,
                                                            const int32_t* __restrict__ mbuf, int kpad,
                                                            int32_t* __restrict__ or_n, int32_t* __restrict__ or_m,
                                                            int32_t* __restrict__ real, int32_t* __restrict__ step) {
  const int pi = blockIdx.x, tid = threadIdx.x;
  const FilterDev f = filters[pi];
  const long long tcl = g.tcells;
  for (int i = tid; i < (int)tcl; i += kThreads) {
    or_n[pi * tcl + i] = 0;
    or_m[pi * tcl + i] = 0;
  }
  __syncthreads();
  if (tid < kpad && f.bandmask) {
    const int beta = kbeta[f.orient * kKMax + tid];
    if (beta >= 0) {
      or_n[pi * tcl + beta] = nbt[(long long)f.shape * tcl + beta];
      or_m[pi * tcl + beta] = mbuf[(long long)pi * kKMax + tid];
    }
  }
  if (tid == 0) {
    if (real) real[pi] = f.r;
    if (step) step[pi] = f.step;
  }
}
}  // namespace

extern "C" int ccwsim_simulate_events(const ccwsim_params* p, const void* workspace, int64_t workspace_bytes,
                                      int32_t* or_n, int32_t* or_m, int32_t* realization, int32_t* step,
                                      void* stream) {
  if (!p || !workspace || !or_n || !or_m) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  std::shared_ptr<Plan> Ph;
  CCW_TRY(get_plan(*p, &Ph));
  Plan* P = Ph.get();
  if (workspace_bytes < P->ws_total) return fail(CCWSIM_ERR_WORKSPACE, "workspace too small");
  const unsigned char* ws = (const unsigned char*)workspace;
  const unsigned char* tbl = ws + P->ws_tbl;
  k_export_events<<<(unsigned)P->nfilters, kThreads, 0, as_stream(stream)>>>(
      P->g, (const FilterDev*)(tbl + P->off_filters), (const int32_t*)(tbl + P->off_kbeta),
      (const int32_t*)(tbl + P->off_nbt), (const int32_t*)(ws + P->ws_mbuf), P->kpad, or_n, or_m, realization, step);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

namespace {
// Match error of each patch's drawn candidate c, from the data event the
// call left in the workspace and the level-J grid:
// (S + sum |beta|^2 m^2 / n) / (|beta|^2 sum n) with S = sum n K^2 - 2^s sum m K.
__global__ __launch_bounds__(kThreads) void k_match_errors(Geom g, const FilterDev* __restrict__ filters,
                                                           const int32_t* __restrict__ kbeta,
                                                           const int32_t* __restrict__ nbt,
                                                           const int32_t* __restrict__ mbuf,
                                                           const int32_t* __restrict__ drawn,
                                                           const int32_t* __restrict__ Ki, int kpad, float* __restrict__ out) {
  __shared__ double s_r[4][kThreads / 64];
  const int pi = blockIdx.x, tid = threadIdx.x;
  const FilterDev f = filters[pi];
  const int c = min(max(drawn[pi], 0), (int)g.ncand - 1);
  int cx, cy, cz;
  split3(c, g.cand[0], g.cand[1], cx, cy, cz);
  double t = 0.0, nn = 0.0, E = 0.0, C = 0.0;
  if (tid < kpad && f.bandmask) {
    const int beta = kbeta[f.orient * kKMax + tid];
    if (beta >= 0) {
      const int n = nbt[(long long)f.shape * g.tcells + beta];
      if (n > 0) {
        const double B = (double)(1 << (g.shift - 1));
        const double m = (double)mbuf[(long long)pi * kKMax + tid];
        int bx, by, bz;
        split3(beta, g.tc[0], g.tc[1], bx, by, bz);
        const double k = (double)Ki[idx3i(cx + bx, cy + by, cz + bz, g.G)];
        t = B * B * m * m / (double)n;
        nn = (double)n;
        E = (double)n * k * k;
        C = m * k;
      }
    }
  }
  double v[4] = {t, nn, E, C};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if ((tid & 63) == 0) s_r[q][tid >> 6] = v[q];
  }
  __syncthreads();
  if (tid == 0) {
    double r[4];
    for (int q = 0; q < 4; ++q) r[q] = s_r[q][0] + s_r[q][1] + s_r[q][2] + s_r[q][3];
    const double B = (double)(1 << (g.shift - 1));
    const double S = r[2] - (double)(1 << g.shift) * r[3];
    out[pi] = r[1] > 0.0 ? (float)((S + r[0]) / (B * B * r[1])) : -1.f;
  }
}
}  // namespace

extern "C" int ccwsim_simulate_match_errors(const ccwsim_params* p, const void* workspace, int64_t workspace_bytes,
                                            float* out, void* stream) {
  if (!p || !workspace || !out) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  std::shared_ptr<Plan> Ph;
  CCW_TRY(get_plan(*p, &Ph));
  Plan* P = Ph.get();
  if (workspace_bytes < P->ws_total) return fail(CCWSIM_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = as_stream(stream);
  if (p->score_mode != 0) {
    k_fill_i32<<<nblocks(P->nfilters), kThreads, 0, st>>>((int32_t*)out, P->nfilters, (int32_t)0xBF800000u);
  } else {
    const unsigned char* ws = (const unsigned char*)workspace;
    const unsigned char* tbl = ws + P->ws_tbl;
    k_match_errors<<<(unsigned)P->nfilters, kThreads, 0, st>>>(
        P->g, (const FilterDev*)(tbl + P->off_filters), (const int32_t*)(tbl + P->off_kbeta),
        (const int32_t*)(tbl + P->off_nbt), (const int32_t*)(ws + P->ws_mbuf), (const int32_t*)(ws + P->ws_err),
        (const int32_t*)(ws + P->ws_ki), P->kpad, out);
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// ---- realization statistics (Sec. 5.2, 5.3, 5.8) ----
namespace {
constexpr int kStatMaxLag = 4096;
constexpr int kStatRowLds = 16000;   // widest row k_st_conn_x stages in LDS

int stat_shape(const ccwsim_shape& sh, StatShape& s) {
  if (sh.ndim != 2 && sh.ndim != 3) return fail(CCWSIM_ERR_SHAPE, "ndim must be 2 or 3");
  long long cells = 1;
  for (int a = 0; a < 3; ++a) {
    const int n = sh.n[a];
    if (n < 1) return fail(CCWSIM_ERR_SHAPE, "extent %d on axis %d", n, a);
    if (a >= sh.ndim && n != 1) return fail(CCWSIM_ERR_SHAPE, "extent of unused axis %d must be 1", a);
    s.n[a] = n;
    cells *= n;
  }
  if (cells > 0x7fffffffll) return fail(CCWSIM_ERR_UNSUPPORTED, "images of more than 2^31 - 1 cells");
  s.cells = cells;
  s.rows = s.n[1] * s.n[2];
  s.nwx = (s.n[0] + 31) / 32;
  s.nwp = s.nwx + 1;
  return CCWSIM_OK;
}

long long stat_bits_bytes(const StatShape& s, int n_img) { return align256((long long)n_img * s.rows * s.nwp * 4); }

int stat_common(const int8_t* codes, const ccwsim_shape& shape, int n_img, int n_facies, StatShape& s) {
  CCW_TRY(stat_shape(shape, s));
  if (n_img < 0 || n_img > 65535) return fail(CCWSIM_ERR_INVALID_ARG, "n_img must be in [0, 65535]");
  if (n_facies < 1 || n_facies > 127) return fail(CCWSIM_ERR_INVALID_ARG, "n_facies must be in [1, 127]");
  if (n_img > 0 && !codes) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  return CCWSIM_OK;
}

int stat_lags(const ccwsim_shape& shape, int axis, int max_lag) {
  if (axis < 0 || axis >= shape.ndim) return fail(CCWSIM_ERR_INVALID_ARG, "axis must be in [0, ndim)");
  if (max_lag < 1 || max_lag > shape.n[axis] - 1 || max_lag > kStatMaxLag)
    return fail(CCWSIM_ERR_INVALID_ARG, "max_lag must be in [1, min(n[axis] - 1, %d)]", kStatMaxLag);
  return CCWSIM_OK;
}

unsigned stat_blocks(long long work, int n_img) {
  const long long per = std::max(1ll, 2048ll / std::max(1, n_img));
  return (unsigned)std::max(1ll, std::min(per, (work + kThreads - 1) / kThreads));
}
}  // namespace

extern "C" int64_t ccwsim_stats_workspace_size(ccwsim_shape shape, int32_t n_img) {
  StatShape s;
  if (stat_shape(shape, s)) return -1;
  if (n_img < 0) {
    fail(CCWSIM_ERR_INVALID_ARG, "n_img must be >= 0");
    return -1;
  }
  return stat_bits_bytes(s, n_img) + align256((long long)n_img * s.cells * 4);
}

extern "C" int ccwsim_stats_histogram(const int8_t* codes, ccwsim_shape shape, int32_t n_img, int32_t n_facies,
                                      int64_t* per_image, int32_t* per_cell, void* stream) {
  StatShape s;
  CCW_TRY(stat_common(codes, shape, n_img, n_facies, s));
  if (!per_image) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (n_img == 0) return CCWSIM_OK;
  hipStream_t st = as_stream(stream);
  unsigned long long* pi = (unsigned long long*)per_image;
  k_st_fill_u64<<<nblocks((long long)n_img * n_facies), kThreads, 0, st>>>(pi, (long long)n_img * n_facies);
  k_st_hist_images<<<dim3(stat_blocks(s.cells, n_img), (unsigned)n_img), kThreads, 0, st>>>(codes, s.cells,
                                                                                             n_facies, pi);
  if (per_cell) k_st_hist_cells<<<nblocks(s.cells), kThreads, 0, st>>>(codes, s.cells, n_img, n_facies, per_cell);
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int ccwsim_stats_variogram(const int8_t* codes, ccwsim_shape shape, int32_t n_img, int32_t n_facies,
                                      int32_t axis, int32_t max_lag, int64_t* diff, void* workspace,
                                      int64_t workspace_bytes, void* stream) {
  StatShape s;
  CCW_TRY(stat_common(codes, shape, n_img, n_facies, s));
  CCW_TRY(stat_lags(shape, axis, max_lag));
  if (!diff) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (n_img == 0) return CCWSIM_OK;
  if (!workspace || workspace_bytes < stat_bits_bytes(s, n_img))
    return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", (long long)stat_bits_bytes(s, n_img));
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  uint32_t* bits = (uint32_t*)workspace;
  unsigned long long* out = (unsigned long long*)diff;
  const long long nout = (long long)n_img * n_facies * max_lag;
  k_st_fill_u64<<<nblocks(nout), kThreads, 0, st>>>(out, nout);
  const long long words = (long long)n_img * s.rows * s.nwp;
  // rows per block: a block's count for one lag (at most rb * nx pairs) stays
  // within its 32-bit counter
  const int rb = (int)std::max(1ll, std::min(32ll, 0x7fffffffll / s.n[0]));
  for (int f = 0; f < n_facies; ++f) {
    k_st_pack<<<nblocks(words), kThreads, 0, st>>>(codes, s, n_img, f, bits);
    k_st_pairs<<<dim3((unsigned)((s.rows + rb - 1) / rb), (unsigned)n_img), kThreads, (size_t)max_lag * 4, st>>>(
        bits, s, axis, max_lag, rb, out + (long long)f * max_lag, (long long)n_facies * max_lag);
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

extern "C" int ccwsim_stats_connectivity(const int8_t* codes, ccwsim_shape shape, int32_t n_img, int32_t n_facies,
                                         int32_t axis, int32_t max_lag, int64_t* both, int64_t* connected,
                                         void* workspace, int64_t workspace_bytes, void* stream) {
  StatShape s;
  CCW_TRY(stat_common(codes, shape, n_img, n_facies, s));
  CCW_TRY(stat_lags(shape, axis, max_lag));
  if (!both || !connected) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (n_img == 0) return CCWSIM_OK;
  const long long need = ccwsim_stats_workspace_size(shape, n_img);
  if (!workspace || workspace_bytes < need) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", need);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  uint32_t* bits = (uint32_t*)workspace;
  int32_t* L = (int32_t*)((unsigned char*)workspace + stat_bits_bytes(s, n_img));
  unsigned long long* ob = (unsigned long long*)both;
  unsigned long long* oc = (unsigned long long*)connected;
  const long long nout = (long long)n_img * n_facies * max_lag;
  k_st_fill_u64<<<nblocks(nout), kThreads, 0, st>>>(ob, nout);
  k_st_fill_u64<<<nblocks(nout), kThreads, 0, st>>>(oc, nout);
  const long long words = (long long)n_img * s.rows * s.nwp;
  const long long cells = (long long)n_img * s.cells;
  // x-axis counting: rows per block for about 2048 blocks, and a block's
  // count for one lag (at most rbx * nx pairs) within 32 bits
  const int rbx = (int)std::max(1ll, std::min({(long long)s.rows * n_img / 2048 + 1, 0x7fffffffll / s.n[0],
                                               (long long)s.rows}));
  for (int f = 0; f < n_facies; ++f) {
    k_st_pack<<<nblocks(words), kThreads, 0, st>>>(codes, s, n_img, f, bits);
    k_st_ccl_init<<<nblocks(cells), kThreads, 0, st>>>(bits, s, n_img, L);
    k_st_ccl_merge<<<nblocks((long long)n_img * s.rows * s.nwx), kThreads, 0, st>>>(bits, s, n_img, L);
    k_st_ccl_flatten<true><<<nblocks(cells), kThreads, 0, st>>>(s, n_img, L);
    k_st_ccl_flatten<false><<<nblocks(cells), kThreads, 0, st>>>(s, n_img, L);
    if (axis == 0 && s.n[0] <= kStatRowLds) {
      k_st_conn_x<<<dim3((unsigned)((s.rows + rbx - 1) / rbx), (unsigned)n_img), kThreads,
                    (size_t)(s.n[0] + 4) * 4, st>>>(L, s, max_lag, rbx, ob + (long long)f * max_lag,
                                                    oc + (long long)f * max_lag, (long long)n_facies * max_lag);
    } else if (axis > 0) {
      const int nxb = (s.n[0] + kThreads - 1) / kThreads;
      const int lines = axis == 1 ? s.n[2] : s.n[1];
      k_st_conn_col<<<dim3((unsigned)(nxb * lines), (unsigned)((max_lag + 7) / 8), (unsigned)n_img), kThreads, 0,
                      st>>>(L, s, axis, max_lag, ob + (long long)f * max_lag, oc + (long long)f * max_lag,
                            (long long)n_facies * max_lag);
    } else {
      k_st_conn<<<dim3(stat_blocks(s.cells, n_img), (unsigned)n_img), kThreads, (size_t)max_lag * 8, st>>>(
          L, s, axis, max_lag, ob + (long long)f * max_lag, oc + (long long)f * max_lag,
          (long long)n_facies * max_lag);
    }
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// ===========================================================================
// CDF 9/7 in floating point (Sec. 4.2: the mother wavelet is a choice)
// ===========================================================================
namespace {

// Workspace of the 9/7 transforms: three float buffers of the padded TI.
long long c97_ws_bytes(const Geom& g) { return 3 * align256((long long)g.np[0] * g.np[1] * g.np[2] * 4); }

// Level-J 9/7 DWT of the TI into approx and the detail layout of the other
// wavelets (band-stacked passes, as for 5/3).
int launch_dwt97(const Geom& g, const int8_t* x, float* approx, float* details, unsigned char* ws, hipStream_t st) {
  const long long npc = (long long)g.np[0] * g.np[1] * g.np[2];
  float* C = (float*)ws;
  float* A = (float*)(ws + align256(npc * 4));
  float* B = (float*)(ws + 2 * align256(npc * 4));
  k_c97_pad<<<nblocks(npc), kThreads, 0, st>>>(x, g.level == 0 ? approx : C, g);
  int e[3] = {g.np[0], g.np[1], g.np[2]};
  for (int j = 1; j <= g.level; ++j) {
    const float* src = C;
    float* bufs[2] = {A, B};
    float* dst = nullptr;
    for (int a = 0; a < g.ndim; ++a) {
      dst = bufs[a & 1];
      const long long outc = (long long)e[0] * e[1] * e[2] / 2 * (1 << a);
      k_c97_fwd<<<nblocks(outc), kThreads, 0, st>>>(src, dst, e[0], e[1], e[2], a, 1 << a);
      e[a] >>= 1;
      src = dst;
    }
    const long long band = (long long)e[0] * e[1] * e[2];
    HIP_TRY(hipMemcpyAsync(details + g.det_off[j], dst + band, band * ((1 << g.ndim) - 1) * 4,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(j == g.level ? approx : C, dst, band * 4, hipMemcpyDeviceToDevice, st));
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

// Inverse from approx and details into `image` (the padded extent).
int launch_idwt97(const Geom& g, const float* approx, const float* details, float* image, unsigned char* ws,
                  hipStream_t st) {
  const long long npc = (long long)g.np[0] * g.np[1] * g.np[2];
  float* C = (float*)ws;
  float* A = (float*)(ws + align256(npc * 4));
  float* B = (float*)(ws + 2 * align256(npc * 4));
  const int nd = g.ndim;
  int e[3] = {g.G[0], g.G[1], g.G[2]};
  if (g.level == 0) {
    HIP_TRY(hipMemcpyAsync(image, approx, npc * 4, hipMemcpyDeviceToDevice, st));
    return CCWSIM_OK;
  }
  const float* cur = approx;
  for (int j = g.level; j >= 1; --j) {
    const long long band = (long long)e[0] * e[1] * e[2];
    float* bufs[2] = {A, B};
    HIP_TRY(hipMemcpyAsync(A, cur, band * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(A + band, details + g.det_off[j], band * ((1 << nd) - 1) * 4, hipMemcpyDeviceToDevice, st));
    const float* src = A;
    float* dst = nullptr;
    for (int a = nd - 1, i = 1; a >= 0; --a, ++i) {
      dst = a > 0 ? bufs[i & 1] : (j == 1 ? image : C);
      e[a] <<= 1;
      const long long pairs = (long long)e[0] * e[1] * e[2] / 2 * (1 << a);
      k_c97_inv<<<nblocks(pairs), kThreads, 0, st>>>(src, dst, e[0], e[1], e[2], a, 1 << a);
      src = dst;
    }
    cur = C;
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}

struct C97Plan {
  Geom g;
  int kpad = 0, W = 0, R = 0, seg = kC97Seg;
  bool exact = true, want_scores = false, want_keys = false;
  size_t lds = 0;
  long long ws_cnt = 0, ws_off = 0, ws_soff = 0, ws_val = 0, ws_kmax = 0, ws_map = -1, ws_bulk = -1, ws_short = -1, ws_cext = -1,
            ws_total = 0;
};

int c97_plan(ccwsim_shape ti, int32_t level, int32_t precision, const int32_t tmpl[3], int32_t n_filters,
             int32_t top_k, int32_t shortlist, bool want_scores, bool want_keys, bool scores_given, C97Plan& p) {
  Geom& g = p.g;
  CCW_TRY(geom_ti(g, ti, level));
  if (!tmpl) return fail(CCWSIM_ERR_INVALID_ARG, "null template");
  CCW_TRY(geom_tmpl(g, tmpl));
  if (n_filters < 1 || n_filters > (1 << 19)) return fail(CCWSIM_ERR_INVALID_ARG, "n_filters must be in [1, 2^19]");
  if (precision != 0 && precision != 1) return fail(CCWSIM_ERR_INVALID_ARG, "precision must be 0 (fp16) or 1 (bf16)");
  if (!want_scores && !want_keys) return fail(CCWSIM_ERR_INVALID_ARG, "neither scores nor top-K keys requested");
  if (g.tcells > kC97BlocksMax) return fail(CCWSIM_ERR_UNSUPPORTED, "template has %lld blocks (> %d)", g.tcells, kC97BlocksMax);
  if (c97_map_width(g) == 0)
    return fail(CCWSIM_ERR_UNSUPPORTED, "template of %d block rows of %d blocks is too tall for the score map's strip",
                g.tc[1] * g.tc[2], g.tc[0]);
  p.want_scores = want_scores;
  p.want_keys = want_keys;
  if (want_keys) {
    if (top_k < 1 || top_k > kTopMax) return fail(CCWSIM_ERR_UNSUPPORTED, "top_k must be in [1, %d]", kTopMax);
    if (top_k > g.ncand) return fail(CCWSIM_ERR_INVALID_ARG, "top_k exceeds the %d candidates", g.ncand);
    if (shortlist != 0 && (shortlist < top_k || shortlist > kC97ShortMax))
      return fail(CCWSIM_ERR_INVALID_ARG, "shortlist must be 0 (every candidate rescored) or in [top_k, %d]",
                  kC97ShortMax);
    p.R = shortlist == 0 ? g.ncand : std::min(shortlist, g.ncand);
    p.exact = p.R == g.ncand;
  }
  const long long nf = n_filters;
  long long o = 0;
  p.ws_cnt = o;   o += align256(nf * 4);
  p.ws_off = o;   o += align256(nf * kC97BlocksMax * 4);
  p.ws_soff = o;  o += align256(nf * kC97BlocksMax * 4);
  p.ws_val = o;   o += align256(nf * kC97BlocksMax * 4);
  const long long nchk = (long long)g.cand[1] * g.cand[2] * ((g.cand[0] + 31) / 32);
  if (want_keys && p.exact && !scores_given) {
    p.ws_map = o; o += align256(nf * g.ncand * 4);
  }
  if (want_keys) {
    p.ws_cext = o; o += align256(nf * nchk * 4);
  }
  if (want_keys && !p.exact) {
    const int nrows = g.tc[1] * g.tc[2];
    p.kpad = (int)((2 * g.tcells + 15) / 16 * 16);
    // the widest row segment whose strips fit the LDS
    for (p.seg = kC97Seg; p.seg > 32 && c97_bulk_lds(nrows, p.seg + g.tc[0] - 1, p.kpad) > 64 * 1024; p.seg -= 32) {}
    p.W = p.seg + g.tc[0] - 1;
    p.lds = c97_bulk_lds(nrows, p.W, p.kpad);
    if (p.lds > 64 * 1024) return fail(CCWSIM_ERR_UNSUPPORTED, "bulk scan needs %zu bytes of LDS", p.lds);
    p.ws_kmax = o;  o += align256(kC97MaxParts * 4);
    p.ws_bulk = o;  o += align256(nf * g.ncand * 4);
    p.ws_short = o; o += align256(nf * p.R * 4);
  }
  p.ws_total = o;
  return CCWSIM_OK;
}

}  // namespace

extern "C" int64_t ccwsim_dwt97_workspace_size(ccwsim_shape s, int32_t level) {
  Geom g;
  if (geom_ti(g, s, level)) return -1;
  return c97_ws_bytes(g);
}

extern "C" int ccwsim_dwt97(const int8_t* x, ccwsim_shape s, int32_t level, float* approx, float* details,
                            void* workspace, int64_t workspace_bytes, void* stream) {
  Geom g;
  CCW_TRY(geom_ti(g, s, level));
  if (!x || !approx || (level > 0 && !details)) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  const long long need = c97_ws_bytes(g);
  if (!workspace || workspace_bytes < need) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", need);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return launch_dwt97(g, x, approx, details, (unsigned char*)workspace, as_stream(stream));
}

extern "C" int ccwsim_idwt97(const float* approx, const float* details, ccwsim_shape ti, int32_t level, float* image,
                             void* workspace, int64_t workspace_bytes, void* stream) {
  Geom g;
  CCW_TRY(geom_ti(g, ti, level));
  if (!approx || !image || (level > 0 && !details)) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  const long long need = c97_ws_bytes(g);
  if (!workspace || workspace_bytes < need) return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", need);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return launch_idwt97(g, approx, details, image, (unsigned char*)workspace, as_stream(stream));
}

extern "C" int64_t ccwsim_ccf_scan97_workspace_size(ccwsim_shape ti, int32_t level, int32_t precision,
                                                    const int32_t tmpl[3], int32_t n_filters, int32_t top_k,
                                                    int32_t shortlist, int32_t want_scores, int32_t want_keys) {
  C97Plan p;
  if (c97_plan(ti, level, precision, tmpl, n_filters, top_k, shortlist, want_scores != 0, want_keys != 0,
               want_scores != 0, p))
    return -1;
  return p.ws_total;
}

extern "C" int ccwsim_ccf_scan97(ccwsim_shape ti, int32_t level, int32_t precision, const float* approx,
                                 const int32_t tmpl[3], const int32_t* or_n, const float* or_m, int32_t n_filters,
                                 float* scores, int32_t top_k, int32_t shortlist, uint64_t seed,
                                 const int32_t* realization, const int64_t* step, uint64_t* topk_keys,
                                 int32_t* shortlist_out, void* workspace, int64_t workspace_bytes, void* stream) {
  C97Plan p;
  CCW_TRY(c97_plan(ti, level, precision, tmpl, n_filters, top_k, shortlist, scores != nullptr, topk_keys != nullptr,
                   scores != nullptr, p));
  if (!approx || !or_n || !or_m) return fail(CCWSIM_ERR_INVALID_ARG, "null pointer");
  if (topk_keys && (!realization || !step)) return fail(CCWSIM_ERR_INVALID_ARG, "top-K keys need realization and step");
  if (shortlist_out && (!topk_keys || p.exact))
    return fail(CCWSIM_ERR_INVALID_ARG, "shortlist_out needs top-K keys and a shortlist smaller than the candidates");
  if (!workspace || workspace_bytes < p.ws_total)
    return fail(CCWSIM_ERR_WORKSPACE, "workspace of %lld bytes needed", p.ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(CCWSIM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const Geom& g = p.g;
  hipStream_t st = as_stream(stream);
  unsigned char* ws = (unsigned char*)workspace;
  int32_t* cnt = (int32_t*)(ws + p.ws_cnt);
  int32_t* off = (int32_t*)(ws + p.ws_off);
  float* val = (float*)(ws + p.ws_val);
  const int sw = c97_map_width(g);
  const size_t mlds = c97_map_lds(sw, g);
  int32_t* soff = (int32_t*)(ws + p.ws_soff);
  k_c97_pack<<<(unsigned)((n_filters + kThreads / 64 - 1) / (kThreads / 64)), kThreads, 0, st>>>(
      or_n, or_m, n_filters, g, c97_map_wc(sw, g), cnt, off, soff, val);
  const unsigned nseg = (unsigned)((g.cand[0] + sw - 1) / sw);
  const dim3 mgrid(nseg * (unsigned)(g.cand[1] * g.cand[2]), (unsigned)((n_filters + kC97MapEvents - 1) / kC97MapEvents));
  float* cext = topk_keys ? (float*)(ws + p.ws_cext) : nullptr;
  if (scores) k_c97_map<<<mgrid, kThreads, mlds, st>>>(approx, g, sw, cnt, soff, val, n_filters, scores, p.exact ? cext : nullptr);
  if (topk_keys) {
    if (p.exact) {
      float* map = scores ? scores : (float*)(ws + p.ws_map);
      if (!scores) k_c97_map<<<mgrid, kThreads, mlds, st>>>(approx, g, sw, cnt, soff, val, n_filters, map, cext);
      k_c97_best<<<(unsigned)n_filters, kThreads, 0, st>>>(map, cext, g, top_k, seed, realization, step, topk_keys);
    } else {
      float* kmax = (float*)(ws + p.ws_kmax);
      float* bulk = (float*)(ws + p.ws_bulk);
      int32_t* sl = shortlist_out ? shortlist_out : (int32_t*)(ws + p.ws_short);
      const long long gcells = (long long)g.G[0] * g.G[1] * g.G[2];
      k_c97_absmax<<<kC97MaxParts, kThreads, 0, st>>>(approx, gcells, kmax);
      C97BulkArgs a = {};
      a.g = g;
      a.K = approx;
      a.cnt = cnt;
      a.blk = off;
      a.val = val;
      a.kmax = kmax;
      a.n_filters = n_filters;
      a.kpad = p.kpad;
      a.seg = p.seg;
      a.W = p.W;
      a.bulk = bulk;
      a.cmax = cext;
      const dim3 bgrid((unsigned)(g.cand[1] * g.cand[2]), (unsigned)((n_filters + 31) / 32),
                       (unsigned)((g.cand[0] + p.seg - 1) / p.seg));
      if (precision == 1) k_c97_bulk<__bf16><<<bgrid, kThreads, p.lds, st>>>(a);
      else k_c97_bulk<_Float16><<<bgrid, kThreads, p.lds, st>>>(a);
      k_c97_short<<<(unsigned)n_filters, kThreads, 0, st>>>(bulk, cext, g, p.R, sl);
      k_c97_rescore<<<(unsigned)n_filters, kThreads, 0, st>>>(approx, g, cnt, off, val, sl, p.R, top_k, seed,
                                                             realization, step, topk_keys);
    }
  }
  HIP_TRY(hipGetLastError());
  return CCWSIM_OK;
}
