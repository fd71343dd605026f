// dev_scan.h -- the CCW scan on MFMA (Sec. 4.3): every candidate of the TI
// approximation grid against a tile of up to 32 data events ("filters").
//
// The contraction C[c][f] = sum_k K[c + beta_k] * m[f][k] is a GEMM with
// M = candidates, N = filters, K = the level-J blocks of the overlap.  One
// workgroup owns one row of candidates (fixed cy, cz) and one filter tile.
// It stages the K-grid rows the row touches (T_c,y * T_c,z rows of the fp16
// grid) in LDS, so the A operand is gathered from LDS without forming the
// im2col matrix: A[i][k] = strip[off(beta_k) + cx_i].  Each wavefront takes
// 32-candidate chunks and runs v_mfma_f32_32x32x16_f16 over the K dimension.
// Inputs are integers <= 2048 and every partial sum stays below 2^24, so the
// fp16-in / fp32-accumulate contraction is exact; the score is then formed
// in int32: S = E - 2 |beta| C (squared-difference mode) or S = -C.
#pragma once

#include "dev_kernels.h"

namespace ccw {

constexpr int kKMax = 256;   // longest padded list of overlap blocks
constexpr int kScanGroupKMax = 128;   // longest list for workgroups of several tiles
constexpr int kFiltersPerTile = 32;

struct FilterDev {     // one (realization, patch) pair active in a step
  int32_t r;           // realization
  int32_t step;        // raster step of the patch
  int32_t org[3];      // patch origin in the padded grid
  int32_t shape;       // energy row: orient * 2^ndim + bandmask
  int32_t orient;      // bit a: axis a walked from its high end
  int32_t bandmask;    // bit a: overlap band present on axis a
  int32_t succ0;       // first entry of this patch's successor list
  int32_t nsucc;       // later patches whose windows overlap this one
};

struct TileDev {
  int32_t first;       // first filter (index within the step)
  int32_t count;       // filters in this tile (<= 32)
  int32_t orient;      // shared orientation of the tile
  uint32_t zmask;      // bit j: filter j has no overlap yet (first patch)
};

struct ScanRec {       // one filter lane of one scan tile (simulate)
  int32_t gidx;        // patch index over the whole plan, -1 for an empty lane
  int32_t shape;       // energy row
  uint64_t tkey;       // tie-break key of the patch
  int32_t hd0, nhd;    // hard data of the patch's virtual template (set per call)
};

struct HdEnt {         // one hard datum inside a virtual template
  int16_t u[3];        // offset from the patch origin
  int16_t v;           // code
};

// Hard-data bit table (built once per call from the TI).  Rows are the TI's
// (y, z) rows padded by py0 / pz0 rows before the TI (and enough after it)
// so that every row a virtual template reaches exists; a padded row holds
// zeros.  Row (ry, rz) holds, for each x phase r < 2^J and code slot c
// (0 .. nf-1, and nf for a code that no TI cell holds), a bit vector of nw
// words over the level-J x positions bx, bit bx + pb set where the cell
// (2^J bx + r, y, z) lies in the TI and its code differs from c.  A
// candidate's mismatch with datum (u, v) is then bit cx + floor(u_x / 2^J)
// + pb of the vector (row of y, z; phase u_x mod 2^J; slot of v), so the
// 32 candidates of a chunk read two adjacent words per datum.
struct HdmGeom {
  int pb;          // bit of bx = 0
  int py0, pz0;    // padding rows before y = 0 and z = 0
  int ry, rz;      // padded rows per axis
  int nw;          // words per (row, phase, slot)
  int ns, nf;      // slots (n_facies + 1) and n_facies
  int rs;          // words per padded row: 2^J * ns * nw
};

struct HdBits {        // one hard datum: where its bit vector starts
  int32_t woff;        // word of the vector for candidates 0..31 of row (cy, cz) = (0, 0)
  int32_t sh;          // bit of candidate 0 within that word pair
};

constexpr int kScanGroupsInline = 64;   // group-table entries passed by value to a scan launch

struct ScanArgs {
  Geom g;
  HdmGeom hm;
  const uint32_t* hdm;         // simulate: hard-data bit table, or null (read TI codes)
  const HdBits* hd_bits;       // simulate: entries parallel to hd_ent (with hdm)
  const void* Kop;             // level-J grid in the operand type (fp16 or bf16)
  const int32_t* kbeta;        // [orient][kKMax] block index or -1 (simulate)
  const TileDev* tiles;        // simulate: tiles of this step
  const ScanRec* recs;         // simulate: [tile][kFiltersPerTile] records of this step
  const int32_t* mbuf;         // [patch][kKMax] data-event block sums (standalone: [filter])
  const int32_t* energy;       // simulate: [shape][ncand]
  const HdEnt* hd_ent;
  const int8_t* ti;
  uint64_t* keys;              // simulate: [slot][ncand]
  uint64_t* rowmin;            // simulate: [slot][candidate rows] smallest key of each row
  int32_t* scores;             // standalone: [filter][ncand], holds E on entry
  uint64_t seed;
  int fbegin;                  // simulate: global index of this step's first patch
  int kpad;                    // padded K dimension (multiple of 16)
  int W;                       // LDS strip row length (halves)
  int score_mode;
  int rowmin_only;             // simulate: write the row minima only (no per-candidate keys)              // 0 squared difference, 1 raw
  int standalone;              // 1: filters/tiles/kbeta are implicit
  int n_filters;               // standalone: number of filters
  int has_hd;
  int ntiles;                  // tiles of this launch
  const int2* groups;          // simulate: per workgroup column (first tile, tiles), one orientation
  // the step's group table by value when it fits, so that a workgroup's
  // entry arrives with the arguments instead of after them
  int n_ginline;
  int2 groups_inline[kScanGroupsInline];
  // fused selection (k_scan_sel): per (patch, candidate row) only the
  // candidates that can be among the row's ksel best keys are written
  int32_t* rowcnt;             // [slot][candidate rows] keys written at the start of the row's segment
  const int32_t* nbuf;         // standalone with the energy in the contraction: [filter][kKMax] known cells
  const int32_t* fil_real;     // standalone: realization of each filter (tie-break key), or null
  const int64_t* fil_step;     // standalone: raster step of each filter (tie-break key), or null
  int ksel;                    // keys the selection keeps per row (K, or the shortlist)
  int ng_shift;                // value v of a lane joins group v >> ng_shift of its lane
  int n_bm;                    // band masks per orientation (energy rows per tile)
};

template <typename OT>
struct MfmaOp;
template <>
struct MfmaOp<_Float16> {
  typedef _Float16 vec8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ float16_t mma(vec8 a, vec8 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaOp<__bf16> {
  typedef __bf16 vec8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ float16_t mma(vec8 a, vec8 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// LDS bytes of a scan workgroup taking G tiles.
inline size_t scan_group_lds(int nrows, int W, int kpad, int G) {
  const size_t strip = ((size_t)nrows * W * 2 + 15) & ~(size_t)15;
  return strip + (size_t)kpad * 4 + (size_t)G * kFiltersPerTile * (kpad + 8) * 2 +
         (size_t)G * kFiltersPerTile * (sizeof(ScanRec) + 8);
}

// Operand type OT: _Float16 (exact for integers <= 2048) or __bf16 (exact for
// integers <= 256); accumulation is fp32 either way.  Up to G tiles of one
// orientation per workgroup: the candidate row's A fragments are gathered
// once per 32-candidate chunk and serve all of them (they share one block
// list), so the strip staging, the gather and the prologue's memory round
// trips are paid once per group.
template <typename OT, int G>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(G == 1 ? 4 : 2)))
void k_scan(ScanArgs a) {
  typedef typename MfmaOp<OT>::vec8 vec8;
  constexpr int KS = kScanGroupKMax / 16;   // K slices kept for a group (G > 1)
  const OT* Kop = (const OT*)a.Kop;
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = blockIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int W = a.W, kpad = a.kpad;
  const int nrows = g.tc[1] * g.tc[2];
  const int j = lane & 31;          // A row (candidate in chunk) and B/D column (filter)
  const int g8 = (lane >> 5) * 8;   // this lane's 8 entries of each 16-wide K slice
  int tile0, nt;
  if (a.standalone) {
    tile0 = blockIdx.y * G;
    nt = min(G, a.ntiles - tile0);
  } else if (G == 1) {   // one tile per workgroup: the group table is the identity
    tile0 = blockIdx.y;
    nt = 1;
  } else {
    // scalar loads of the arguments, issued with the count that decides
    // whether they are used (the empty asm takes both before the branch)
    const int n_gi = a.n_ginline;
    const int2 g_arg = a.groups_inline[min((int)blockIdx.y, kScanGroupsInline - 1)];
    __asm__ volatile("" ::"s"(n_gi), "s"(g_arg.x));
    int2 grp;
    if ((int)blockIdx.y < n_gi) {
      grp = g_arg;
      __asm__ volatile("" ::: "memory");   // keeps the two loads apart (no generic pointer)
    } else {
      grp = a.groups[blockIdx.y];
    }
    tile0 = grp.x;
    nt = grp.y;
  }

  OT* s_strip = (OT*)smem;
  const int strip_bytes = ((nrows * W * 2) + 15) & ~15;
  int* s_off = (int*)(smem + strip_bytes);
  OT* s_B = (OT*)(smem + strip_bytes + kpad * 4);
  const int bstride = kpad + 8;   // halves per filter row (keeps 16 B alignment)
  ScanRec* s_rec = (ScanRec*)(smem + strip_bytes + kpad * 4 + G * kFiltersPerTile * bstride * 2);
  unsigned long long* s_rowmin = (unsigned long long*)(s_rec + G * kFiltersPerTile);
  __shared__ TileDev s_tile[G];

  // tiles and per-lane filter records first (one round trip reaches every
  // epilogue input); the first tile's record also goes to registers
  auto tile_of = [&](int gi) {
    TileDev t;
    if (a.standalone) {
      t.first = (tile0 + gi) * kFiltersPerTile;
      t.count = min(kFiltersPerTile, a.n_filters - t.first);
      t.orient = 0;
      t.zmask = 0;
    } else {
      t = a.tiles[tile0 + gi];
    }
    return t;
  };
  auto rec_of = [&](int gi, int jj, const TileDev& t) {
    ScanRec r = {};
    if (a.standalone) r.gidx = jj < t.count ? 0 : -1;
    else r = a.recs[(tile0 + gi) * kFiltersPerTile + jj];
    return r;
  };
  const TileDev t0 = tile_of(0);
  const ScanRec rec0 = rec_of(0, j, t0);
  if (tid < nt) s_tile[tid] = tile_of(tid);
  if (tid < nt * kFiltersPerTile) {
    const int gi = tid / kFiltersPerTile;
    s_rec[tid] = rec_of(gi, tid - gi * kFiltersPerTile, tile_of(gi));
    s_rowmin[tid] = ~0ull;
  }

  const int shift = g.shift;
  const int nchunks = (g.cand[0] + 31) / 32;
  const long long rowbase = (long long)g.cand[0] * row;
  // epilogue inputs of a 32-candidate chunk that do not depend on the
  // contraction: energy and hard-data mismatch counts
  auto epilogue_inputs = [&](int ch, const ScanRec& rec, int slot, int (&ev)[16], unsigned (&mis)[16]) {
    const bool fvalid = rec.gidx >= 0;
    const int32_t* erow = a.standalone ? a.scores + (long long)slot * g.ncand
                                       : a.energy + (long long)rec.shape * g.ncand;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int cx = ch * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      ev[v] = (fvalid && a.score_mode == 0 && cx < g.cand[0]) ? erow[rowbase + cx] : 0;
      mis[v] = 0;
    }
    // hard data: the next entry is read while the current one's 16 TI
    // reads (at clamped, always valid cells) are in flight; a datum counts
    // where it lies inside the TI and the TI differs
    const int nhd = fvalid ? rec.nhd : 0;
    const int J = g.level;   // block factor 2^J on every used axis
    const int Jz = g.ndim == 3 ? J : 0;
    if (a.hdm) {
      // bit table: per datum two words cover the chunk; byte counters
      // (4 candidates per register) take up to 255 data between flushes
      const uint32_t* mb = a.hdm + ((cz << Jz) * a.hm.ry + (cy << J)) * a.hm.rs + ch;
      const HdBits* hb = a.hd_bits + rec.hd0;
      const int hs = 4 * (lane >> 5);
      for (int h0 = 0; h0 < nhd; h0 += 255) {
        const int hn = min(nhd, h0 + 255);
        uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        for (int h = h0; h < hn; h += 4) {
          HdBits b[4];
          uint32_t lo[4], hi[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) b[q] = hb[min(h + q, hn - 1)];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            lo[q] = mb[b[q].woff];
            hi[q] = mb[b[q].woff + 1];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t w = h + q < hn ? __builtin_amdgcn_alignbit(hi[q], lo[q], (uint32_t)b[q].sh) >> hs : 0u;
            c0 += w & 0x01010101u;
            c1 += (w >> 1) & 0x01010101u;
            c2 += (w >> 2) & 0x01010101u;
            c3 += (w >> 3) & 0x01010101u;
          }
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const uint32_t c = (v & 3) == 0 ? c0 : (v & 3) == 1 ? c1 : (v & 3) == 2 ? c2 : c3;
          mis[v] += (c >> (8 * (v >> 2))) & 0xFFu;
        }
      }
      return;
    }
    HdEnt e = {};
    if (nhd > 0) e = a.hd_ent[rec.hd0];
    for (int h = 0; h < nhd; ++h) {
      const HdEnt en = a.hd_ent[rec.hd0 + min(h + 1, nhd - 1)];
      const int fy = (cy << J) + e.u[1], fz = (cz << Jz) + e.u[2];
      const unsigned ok = (fy >= 0 && fz >= 0 && fy < g.ti[1] && fz < g.ti[2]) ? 1u : 0u;
      const int8_t* trow =
          a.ti + (min(max(fz, 0), g.ti[2] - 1) * g.ti[1] + min(max(fy, 0), g.ti[1] - 1)) * g.ti[0];
      int8_t tv[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int cx = ch * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        tv[v] = trow[min(max((cx << J) + e.u[0], 0), g.ti[0] - 1)];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int cx = ch * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int fx = (cx << J) + e.u[0];
        const unsigned inb = (fx >= 0 && fx < g.ti[0] && cx < g.cand[0]) ? ok : 0u;
        mis[v] += inb & (tv[v] != e.v ? 1u : 0u);
      }
      e = en;
    }
  };

  // K-grid strip: issue every load of a thread before storing any of them
  {
    constexpr int U = 8;
    const int n = nrows * W;
    BoxWalk w(tid, kThreads, W, g.tc[1]);   // (x, by, bz) of strip entry i
    for (int base = tid; base < n; base += kThreads * U) {
      OT v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        v[q] = (OT)0.0f;
        if (i < n && w.x < g.G[0]) v[q] = Kop[idx3i(w.x, cy + w.y, cz + w.z, g.G)];
        w.next();
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        if (i < n) s_strip[i] = v[q];
      }
    }
  }
  for (int k = tid; k < kpad; k += kThreads) {
    int beta;
    if (a.standalone) beta = k < (int)g.tcells ? k : -1;
    else beta = a.kbeta[t0.orient * kKMax + k];
    int off = 0;
    if (beta >= 0) {
      const int bx = beta % g.tc[0], by = (beta / g.tc[0]) % g.tc[1], bz = beta / (g.tc[0] * g.tc[1]);
      off = (bz * g.tc[1] + by) * W + bx;
    }
    s_off[k] = off;
  }
  // data events of every tile: 8 int32 (32 B) per load, converted to the
  // operand type
  typedef int32_t int8v_t __attribute__((ext_vector_type(8)));
  const int k8n = kpad / 8;
  for (int i = tid; i < nt * kFiltersPerTile * k8n; i += kThreads) {
    const int row_f = i / k8n, k8 = (i - row_f * k8n) * 8;
    const int gi = row_f / kFiltersPerTile, jj = row_f - gi * kFiltersPerTile;
    const TileDev t = tile_of(gi);
    int8v_t m = {};
    if (jj < t.count && !((t.zmask >> jj) & 1u))
      m = *(const int8v_t*)(a.mbuf + (long long)(a.fbegin + t.first + jj) * kKMax + k8);
    vec8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (OT)(float)m[e];
    *(vec8*)(s_B + row_f * bstride + k8) = v;
  }
  // the first chunk's epilogue reads go out before the barrier
  int ev[16];
  unsigned mis[16];
  if (wave < nchunks) epilogue_inputs(wave, rec0, t0.first + j, ev, mis);
  __syncthreads();

  // (chunk, tile) pairs of this wavefront; a pair's epilogue reads go out
  // before its contraction
  const int my_chunks = wave < nchunks ? (nchunks - 1 - wave) / (kThreads / 64) + 1 : 0;
  const int npairs = my_chunks * nt;
  vec8 afr[KS];
  for (int p = 0; p < npairs; ++p) {
    const int ch = wave + (kThreads / 64) * (p / nt), gi = p - (p / nt) * nt;
    const TileDev t = s_tile[gi];
    const ScanRec rec = s_rec[gi * kFiltersPerTile + j];
    if (p > 0) epilogue_inputs(ch, rec, t.first + j, ev, mis);
    const int cbase = ch * 32 + j;
    float16_t acc = {};
    const OT* brow = s_B + (gi * kFiltersPerTile + j) * bstride + g8;
    if constexpr (G == 1) {
      for (int kc = 0; kc < kpad; kc += 16) {
        vec8 av;
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = s_strip[s_off[kc + g8 + e] + cbase];
        acc = MfmaOp<OT>::mma(av, *(const vec8*)(brow + kc), acc);
      }
    } else {
      if (gi == 0) {   // gather this chunk's A fragments once for the group
#pragma unroll
        for (int q = 0; q < KS; ++q) {
          if (q * 16 < kpad) {
#pragma unroll
            for (int e = 0; e < 8; ++e) afr[q][e] = s_strip[s_off[q * 16 + g8 + e] + cbase];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < KS; ++q)
        if (q * 16 < kpad) acc = MfmaOp<OT>::mma(afr[q], *(const vec8*)(brow + q * 16), acc);
    }
    const bool fvalid = rec.gidx >= 0;
    const int slot = t.first + j;
    uint64_t lane_min = ~0ull;
    if (fvalid) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int cx = ch * 32 + i;
        if (cx >= g.cand[0]) continue;
        const long long idx = rowbase + cx;
        const int C = (int)acc[v];
        const int S = (a.score_mode == 0) ? ev[v] - (C << shift) : -C;
        if (a.standalone) {
          a.scores[(long long)slot * g.ncand + idx] = S;
          continue;
        }
        const uint64_t key = make_key(mis[v], S, tie_perm((uint32_t)idx, rec.tkey));
        if (!a.rowmin_only) a.keys[(long long)slot * g.ncand + idx] = key;
        lane_min = key < lane_min ? key : lane_min;
      }
    }
    if (!a.standalone) {
      // lanes j and j + 32 hold the same filter; the wavefronts meet in LDS
      const uint64_t other = shfl_xor64(lane_min, 32);
      lane_min = other < lane_min ? other : lane_min;
      if (lane < 32 && fvalid) atomicMin(&s_rowmin[gi * kFiltersPerTile + j], (unsigned long long)lane_min);
    }
  }
  if (a.standalone) return;
  __syncthreads();
  if (tid < nt * kFiltersPerTile) {
    const int gi = tid / kFiltersPerTile, jj = tid - gi * kFiltersPerTile;
    const TileDev t = s_tile[gi];
    if (jj < t.count) a.rowmin[(long long)(t.first + jj) * (g.cand[1] * g.cand[2]) + row] = s_rowmin[tid];
  }
}

// Filter-major variant (one tile per workgroup).  The MFMA takes the data
// events as its A operand and the gathered K values as its B operand, so
// lane l ends with one candidate (column l % 32) against 16 patches
// (rows 8(v/4) + 4(l/32) + v%4).  For a fixed v the 32 lanes of a half
// wavefront then hold 32 consecutive candidates of one patch: the energy
// reads and the key stores are contiguous runs instead of 32 scattered
// lines.  Each lane keeps its 16 row minima across its chunks; they are
// reduced over the half wavefront once at the end.
template <typename OT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_scan_fm(ScanArgs a) {
  typedef typename MfmaOp<OT>::vec8 vec8;
  const OT* Kop = (const OT*)a.Kop;
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = blockIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int W = a.W, kpad = a.kpad;
  const int nrows = g.tc[1] * g.tc[2];
  const int j = lane & 31, half = lane >> 5;
  const int g8 = half * 8;
  const int tile = (int)blockIdx.y;   // one tile per workgroup: the group table is the identity

  OT* s_strip = (OT*)smem;
  const int strip_bytes = ((nrows * W * 2) + 15) & ~15;
  int* s_off = (int*)(smem + strip_bytes);
  OT* s_B = (OT*)(smem + strip_bytes + kpad * 4);
  const int bstride = kpad + 8;
  ScanRec* s_rec = (ScanRec*)(smem + strip_bytes + kpad * 4 + kFiltersPerTile * bstride * 2);
  unsigned long long* s_rowmin = (unsigned long long*)(s_rec + kFiltersPerTile);

  TileDev t;
  if (a.standalone) {
    t.first = tile * kFiltersPerTile;
    t.count = min(kFiltersPerTile, a.n_filters - t.first);
    t.orient = 0;
    t.zmask = 0;
  } else {
    t = a.tiles[tile];
  }
  if (tid < kFiltersPerTile) {
    ScanRec r = {};
    if (a.standalone) r.gidx = tid < t.count ? 0 : -1;
    else r = a.recs[tile * kFiltersPerTile + tid];
    s_rec[tid] = r;
    s_rowmin[tid] = ~0ull;
  }
  {
    constexpr int U = 8;
    const int n = nrows * W;
    BoxWalk w(tid, kThreads, W, g.tc[1]);
    for (int base = tid; base < n; base += kThreads * U) {
      OT v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        v[q] = (OT)0.0f;
        if (i < n && w.x < g.G[0]) v[q] = Kop[idx3i(w.x, cy + w.y, cz + w.z, g.G)];
        w.next();
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        if (i < n) s_strip[i] = v[q];
      }
    }
  }
  for (int k = tid; k < kpad; k += kThreads) {
    int beta;
    if (a.standalone) beta = k < (int)g.tcells ? k : -1;
    else beta = a.kbeta[t.orient * kKMax + k];
    int off = 0;
    if (beta >= 0) {
      const int bx = beta % g.tc[0], by = (beta / g.tc[0]) % g.tc[1], bz = beta / (g.tc[0] * g.tc[1]);
      off = (bz * g.tc[1] + by) * W + bx;
    }
    s_off[k] = off;
  }
  typedef int32_t int8v_t __attribute__((ext_vector_type(8)));
  const int k8n = kpad / 8;
  for (int i = tid; i < kFiltersPerTile * k8n; i += kThreads) {
    const int jj = i / k8n, k8 = (i - jj * k8n) * 8;
    int8v_t m = {};
    if (jj < t.count && !((t.zmask >> jj) & 1u))
      m = *(const int8v_t*)(a.mbuf + (long long)(a.fbegin + t.first + jj) * kKMax + k8);
    vec8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (OT)(float)m[e];
    *(vec8*)(s_B + jj * bstride + k8) = v;
  }
  __syncthreads();

  const int shift = g.shift;
  const int nchunks = (g.cand[0] + 31) / 32;
  const long long rowbase = (long long)g.cand[0] * row;
  const int J = g.level, Jz = g.ndim == 3 ? J : 0;
  const int fy0 = cy << J, fz0 = cz << Jz;
  uint64_t lmin[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) lmin[v] = ~0ull;
  const OT* brow = s_B + j * bstride + g8;
  for (int ch = wave; ch < nchunks; ch += kThreads / 64) {
    const int cx = ch * 32 + j;
    const bool cval = cx < g.cand[0];
    const long long idx = rowbase + min(cx, g.cand[0] - 1);
    // energy of this candidate for each of the lane's 16 patches (contiguous
    // over the half wavefront), read before the contraction
    int ev[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * half + (v & 3);
      const ScanRec& r = s_rec[i];
      ev[v] = 0;
      if (r.gidx >= 0 && a.score_mode == 0)
        ev[v] = a.standalone ? a.scores[(long long)(t.first + i) * g.ncand + idx] : a.energy[(long long)r.shape * g.ncand + idx];
    }
    float16_t acc = {};
    for (int kc = 0; kc < kpad; kc += 16) {
      vec8 av;
#pragma unroll
      for (int e = 0; e < 8; ++e) av[e] = s_strip[s_off[kc + g8 + e] + ch * 32 + j];
      acc = MfmaOp<OT>::mma(*(const vec8*)(brow + kc), av, acc);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * half + (v & 3);
      const ScanRec r = s_rec[i];
      if (r.gidx < 0 || !cval) continue;
      const int C = (int)acc[v];
      const int S = (a.score_mode == 0) ? ev[v] - (C << shift) : -C;
      const long long o = (long long)(t.first + i) * g.ncand + idx;
      if (a.standalone) {
        a.scores[o] = S;
        continue;
      }
      // hard-data mismatch of this candidate for patch i (the next entry is
      // read while the current one's TI read is in flight)
      unsigned mis = 0;
      if (r.nhd > 0 && a.hdm) {
        // bit table: candidate cx of patch i is bit j + sh of the datum's
        // words from chunk ch on
        const uint32_t* mb = a.hdm + (fz0 * a.hm.ry + fy0) * a.hm.rs + ch;
        const HdBits* hb = a.hd_bits + r.hd0;
        for (int h = 0; h < r.nhd; ++h) {
          const HdBits b = hb[h];
          mis += (mb[b.woff + ((j + b.sh) >> 5)] >> ((j + b.sh) & 31)) & 1u;
        }
      } else if (r.nhd > 0) {
        HdEnt e = a.hd_ent[r.hd0];
        for (int h = 0; h < r.nhd; ++h) {
          const HdEnt en = a.hd_ent[r.hd0 + min(h + 1, r.nhd - 1)];
          const int fx = (cx << J) + e.u[0], fy = fy0 + e.u[1], fz = fz0 + e.u[2];
          const bool in = fx >= 0 && fy >= 0 && fz >= 0 && fx < g.ti[0] && fy < g.ti[1] && fz < g.ti[2];
          const int8_t tv = a.ti[(min(max(fz, 0), g.ti[2] - 1) * g.ti[1] + min(max(fy, 0), g.ti[1] - 1)) * g.ti[0] +
                                 min(max(fx, 0), g.ti[0] - 1)];
          mis += (in && tv != e.v) ? 1u : 0u;
          e = en;
        }
      }
      const uint64_t key = make_key(mis, S, tie_perm((uint32_t)idx, r.tkey));
      if (!a.rowmin_only) a.keys[o] = key;
      lmin[v] = key < lmin[v] ? key : lmin[v];
    }
  }
  if (a.standalone) return;
  // row minima: reduce each of the 16 patches over the 32 candidates of the
  // half wavefront, then across wavefronts in LDS
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    uint64_t m = lmin[v];
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) {
      const uint64_t o = shfl_xor64(m, off);
      m = o < m ? o : m;
    }
    lmin[v] = m;
  }
  if (j == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * half + (v & 3);
      if (i < t.count) atomicMin(&s_rowmin[i], (unsigned long long)lmin[v]);
    }
  }
  __syncthreads();
  if (tid < t.count) a.rowmin[(long long)(t.first + tid) * (g.cand[1] * g.cand[2]) + row] = s_rowmin[tid];
}

// ---------------------------------------------------------------------------
// Scan with the selection of the K best fused into it (Sec. 4.4: the K best
// candidates of the score map; the map itself is never written).
//
// One workgroup takes one candidate row and one tile of 32 patches
// (candidate-major MFMA layout: lane l holds patch l % 32 against 16
// candidates of a 32-candidate chunk).  For every patch it writes only the
// candidates that can be among the row's ksel best keys, at the start of the
// row's key segment, with their count and the row's smallest key:
//   1. Every score is formed and reduced to a selection value q, a
//      non-decreasing function of the key without its tie-break field
//      (q = S, or (mismatch, S) with hard data).  Each lane keeps the
//      minima of q over groups of its values (disjoint sets of candidates);
//      the ksel-th smallest of a patch's group minima, tau, bounds the q of
//      its ksel-th best candidate from above: ksel candidates have q <= tau,
//      and a candidate with q > tau has ksel keys below its own.
//   2. Candidates with q <= tau (the survivors) get their full key (with the
//      keyed tie-break) and are written out.  Survivors are collected per
//      wavefront into an LDS queue with ballots, so the keys of a sparse
//      set of survivors are built densely, 64 at a time.
// A row's best keys are therefore among its survivors, and the K best keys
// of a patch are among the survivors of the K rows with the smallest minima.
//
// Energy source EN: kEnStage -- the energy rows of the tile's orientation
// (one per band mask) are staged in LDS; kEnFold -- the MFMA also contracts
// K^2 against the known-cell counts n (a second accumulator, exact when
// K^2 <= 2048 and sum n K^2 < 2^24); kEnMem -- per filter energy rows read
// from memory (standalone).  HD: hard-data mismatch counts from the bit
// table enter the key.
// ---------------------------------------------------------------------------
constexpr int kSelQueue = 512;   // survivor queue entries per wavefront
enum { kEnStage = 0, kEnFold = 1, kEnMem = 2 };

// LDS bytes of k_scan_sel.
inline size_t scan_sel_lds(int nrows, int W, int kpad, int en, int n_bm, int cpad, int ng_shift, bool hd) {
  size_t o = ((size_t)nrows * W * 2 * (en == kEnFold ? 2 : 1) + 15) & ~(size_t)15;
  const int kk = en == kEnFold ? 2 * kpad : kpad;
  o += (size_t)kpad * 4;
  o += (size_t)kFiltersPerTile * (kk + 8) * 2;
  o += (size_t)kFiltersPerTile * sizeof(ScanRec);
  if (en == kEnStage) o += (size_t)n_bm * cpad * 4;
  const int nwv = std::min(kThreads / 64, cpad / 32);
  o += (size_t)kFiltersPerTile * (nwv * 2 * (16 >> ng_shift)) * (hd ? 8 : 4);
  o += (size_t)(kThreads / 64) * kSelQueue * 8;
  return o;
}

template <bool HD> struct SelVal;
template <> struct SelVal<false> {
  typedef int32_t T;
  static __device__ __forceinline__ T inf() { return 0x7FFFFFFF; }
  static __device__ __forceinline__ T make(uint32_t, int32_t S) { return S; }
  static __device__ __forceinline__ int32_t score(T q) { return q; }
  static __device__ __forceinline__ uint32_t mis(T) { return 0u; }
};
template <> struct SelVal<true> {
  typedef uint64_t T;
  static __device__ __forceinline__ T inf() { return ~0ull; }
  static __device__ __forceinline__ T make(uint32_t m, int32_t S) {
    return ((uint64_t)(m > 4095u ? 4095u : m) << 32) | (uint64_t)((uint32_t)S ^ 0x80000000u);
  }
  static __device__ __forceinline__ int32_t score(T q) { return (int32_t)((uint32_t)q ^ 0x80000000u); }
  static __device__ __forceinline__ uint32_t mis(T q) { return (uint32_t)(q >> 32); }
};

template <typename OT, bool HD, int EN>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HD ? 2 : 4)))
void k_scan_sel(ScanArgs a) {
  typedef typename MfmaOp<OT>::vec8 vec8;
  typedef SelVal<HD> SV;
  typedef typename SV::T qt;
  const OT* Kop = (const OT*)a.Kop;
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = blockIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int W = a.W, kpad = a.kpad;
  const int nrows = g.tc[1] * g.tc[2];
  const int j = lane & 31, h = lane >> 5;
  const int g8 = h * 8;
  const int C0 = g.cand[0];
  const int nchunks = (C0 + 31) / 32;
  const int cpad = nchunks * 32;
  const int kk = EN == kEnFold ? 2 * kpad : kpad;
  const int bstride = kk + 8;
  const int ng_shift = a.ng_shift;
  const int NG = 16 >> ng_shift;
  const int nwv = min(kThreads / 64, nchunks);   // wavefronts holding chunks
  const int G8 = nwv * 2 * NG;                   // groups per patch

  const int strip_n = nrows * W;
  OT* s_strip = (OT*)smem;
  size_t o = ((size_t)strip_n * 2 * (EN == kEnFold ? 2 : 1) + 15) & ~(size_t)15;
  int* s_off = (int*)(smem + o);
  o += (size_t)kpad * 4;
  OT* s_B = (OT*)(smem + o);
  o += (size_t)kFiltersPerTile * bstride * 2;
  ScanRec* s_rec = (ScanRec*)(smem + o);
  o += (size_t)kFiltersPerTile * sizeof(ScanRec);
  int32_t* s_E = (int32_t*)(smem + o);
  if (EN == kEnStage) o += (size_t)a.n_bm * cpad * 4;
  qt* s_gm = (qt*)(smem + o);
  o += (size_t)kFiltersPerTile * G8 * sizeof(qt);
  uint2* s_q = (uint2*)(smem + o) + wave * kSelQueue;
  __shared__ unsigned s_cnt[kFiltersPerTile];
  __shared__ unsigned long long s_rmin[kFiltersPerTile];
  __shared__ qt s_tau[kFiltersPerTile];

  TileDev t;
  if (a.standalone) {
    t.first = blockIdx.y * kFiltersPerTile;
    t.count = min(kFiltersPerTile, a.n_filters - t.first);
    t.orient = 0;
    t.zmask = 0;
  } else {
    t = a.tiles[blockIdx.y];
  }
  ScanRec rec = {};
  if (a.standalone) {
    rec.gidx = j < t.count ? 0 : -1;
    if (j < t.count && a.fil_real)
      rec.tkey = draw64(a.seed, kStreamTiebreak, (uint64_t)a.fil_real[t.first + j], (uint64_t)a.fil_step[t.first + j]);
  } else {
    rec = a.recs[blockIdx.y * kFiltersPerTile + j];
  }
  if (tid < kFiltersPerTile) {
    s_rec[tid] = rec;
    s_cnt[tid] = 0;
    s_rmin[tid] = ~0ull;
  }
  const long long rowbase = (long long)C0 * row;
  // K-grid strip (and its squares): every load of a thread before any store
  {
    constexpr int U = 8;
    BoxWalk w(tid, kThreads, W, g.tc[1]);
    for (int base = tid; base < strip_n; base += kThreads * U) {
      OT v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        v[q] = (OT)0.0f;
        if (i < strip_n && w.x < g.G[0]) v[q] = Kop[idx3i(w.x, cy + w.y, cz + w.z, g.G)];
        w.next();
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = base + q * kThreads;
        if (i < strip_n) {
          s_strip[i] = v[q];
          if (EN == kEnFold) {
            const float f = (float)v[q];
            s_strip[strip_n + i] = (OT)(f * f);
          }
        }
      }
    }
  }
  for (int k = tid; k < kpad; k += kThreads) {
    int beta;
    if (a.standalone) beta = k < (int)g.tcells ? k : -1;
    else beta = a.kbeta[t.orient * kKMax + k];
    int off = 0;
    if (beta >= 0) {
      const int bx = beta % g.tc[0], by = (beta / g.tc[0]) % g.tc[1], bz = beta / (g.tc[0] * g.tc[1]);
      off = (bz * g.tc[1] + by) * W + bx;
    }
    s_off[k] = off;
  }
  // data events (and, folded, the known-cell counts) as the B operand
  typedef int32_t int8v_t __attribute__((ext_vector_type(8)));
  const int k8n = kk / 8, k8m = kpad / 8;
  for (int i = tid; i < kFiltersPerTile * k8n; i += kThreads) {
    const int jj = i / k8n, k8i = i - jj * k8n;
    const bool second = k8i >= k8m;
    const int k8 = (second ? k8i - k8m : k8i) * 8;
    int8v_t m = {};
    if (jj < t.count && !((t.zmask >> jj) & 1u)) {
      const int32_t* src = second ? a.nbuf : a.mbuf;
      m = *(const int8v_t*)(src + (long long)(a.fbegin + t.first + jj) * kKMax + k8);
    }
    vec8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (OT)(float)m[e];
    *(vec8*)(s_B + jj * bstride + k8i * 8) = v;
  }
  // energy rows of the tile's orientation, one per band mask
  if (EN == kEnStage && a.score_mode == 0) {
    const int nb = a.n_bm;
    for (int i = tid; i < nb * cpad; i += kThreads) {
      const int bm = i / cpad, cx = i - bm * cpad;
      s_E[i] = cx < C0 ? a.energy[(long long)((t.orient * nb) | bm) * g.ncand + rowbase + cx] : 0;
    }
  }
  __syncthreads();

  const bool fvalid = rec.gidx >= 0;
  const int shift = g.shift;
  const int J = g.level, Jz = g.ndim == 3 ? J : 0;
  const int bm_j = EN == kEnStage ? (rec.shape & (a.n_bm - 1)) : 0;
  const int32_t* erow = EN == kEnMem ? a.energy + (long long)(t.first + j) * g.ncand + rowbase : nullptr;
  const OT* brow = s_B + j * bstride + g8;

  // selection values of one 32-candidate chunk (invalid entries: infinity)
  auto chunk_values = [&](int ch, qt (&q)[16]) {
    int ev[16];
    unsigned mis[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      ev[v] = 0;
      mis[v] = 0;
    }
    if (a.score_mode == 0 && EN != kEnFold) {
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        const int cx0 = ch * 32 + 8 * qd + 4 * h;
        int4 e4;
        if (EN == kEnStage) {
          e4 = *(const int4*)(s_E + bm_j * cpad + cx0);
        } else {
          e4.x = cx0 < C0 ? erow[cx0] : 0;
          e4.y = cx0 + 1 < C0 ? erow[cx0 + 1] : 0;
          e4.z = cx0 + 2 < C0 ? erow[cx0 + 2] : 0;
          e4.w = cx0 + 3 < C0 ? erow[cx0 + 3] : 0;
        }
        ev[4 * qd] = e4.x;
        ev[4 * qd + 1] = e4.y;
        ev[4 * qd + 2] = e4.z;
        ev[4 * qd + 3] = e4.w;
      }
    }
    if (HD && fvalid && rec.nhd > 0) {
      // bit table: per datum two words cover the chunk; byte counters (four
      // candidates per register) take up to 255 data between flushes
      const uint32_t* mb = a.hdm + ((cz << Jz) * a.hm.ry + (cy << J)) * a.hm.rs + ch;
      const HdBits* hb = a.hd_bits + rec.hd0;
      const int hs = 4 * h;
      const int nhd = rec.nhd;
      for (int h0 = 0; h0 < nhd; h0 += 255) {
        const int hn = min(nhd, h0 + 255);
        uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        for (int hh = h0; hh < hn; hh += 4) {
          HdBits b[4];
          uint32_t lo[4], hi[4];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) b[qq] = hb[min(hh + qq, hn - 1)];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            lo[qq] = mb[b[qq].woff];
            hi[qq] = mb[b[qq].woff + 1];
          }
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const uint32_t w = hh + qq < hn ? __builtin_amdgcn_alignbit(hi[qq], lo[qq], (uint32_t)b[qq].sh) >> hs : 0u;
            c0 += w & 0x01010101u;
            c1 += (w >> 1) & 0x01010101u;
            c2 += (w >> 2) & 0x01010101u;
            c3 += (w >> 3) & 0x01010101u;
          }
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const uint32_t c = (v & 3) == 0 ? c0 : (v & 3) == 1 ? c1 : (v & 3) == 2 ? c2 : c3;
          mis[v] += (c >> (8 * (v >> 2))) & 0xFFu;
        }
      }
    }
    const int cbase = ch * 32 + j;
    float16_t acc = {}, acc2 = {};
    for (int kc = 0; kc < kpad; kc += 16) {
      vec8 av;
#pragma unroll
      for (int e = 0; e < 8; ++e) av[e] = s_strip[s_off[kc + g8 + e] + cbase];
      acc = MfmaOp<OT>::mma(av, *(const vec8*)(brow + kc), acc);
      if (EN == kEnFold) {
        vec8 a2;
#pragma unroll
        for (int e = 0; e < 8; ++e) a2[e] = s_strip[strip_n + s_off[kc + g8 + e] + cbase];
        acc2 = MfmaOp<OT>::mma(a2, *(const vec8*)(brow + kpad + kc), acc2);
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int cx = ch * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
      const int C = (int)acc[v];
      const int E = EN == kEnFold ? (int)acc2[v] : ev[v];
      const int S = a.score_mode == 0 ? E - (C << shift) : -C;
      q[v] = (fvalid && cx < C0) ? SV::make(mis[v], S) : SV::inf();
    }
  };

  // pass 1: selection values, their group minima; the first two chunks of
  // a wavefront stay in registers for pass 2
  const int my_chunks = wave < nchunks ? (nchunks - 1 - wave) / (kThreads / 64) + 1 : 0;
  qt qv0[16], qv1[16], vmin[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    vmin[v] = SV::inf();
    qv0[v] = SV::inf();
    qv1[v] = SV::inf();
  }
  for (int p = 0; p < my_chunks; ++p) {
    qt q[16];
    chunk_values(wave + (kThreads / 64) * p, q);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      vmin[v] = q[v] < vmin[v] ? q[v] : vmin[v];
      if (p == 0) qv0[v] = q[v];
      if (p == 1) qv1[v] = q[v];
    }
  }
  // minima of groups of 2^ng_shift adjacent values
  if (ng_shift >= 1) {
#pragma unroll
    for (int v = 0; v < 16; v += 2) vmin[v] = vmin[v + 1] < vmin[v] ? vmin[v + 1] : vmin[v];
  }
  if (ng_shift >= 2) {
#pragma unroll
    for (int v = 0; v < 16; v += 4) vmin[v] = vmin[v + 2] < vmin[v] ? vmin[v + 2] : vmin[v];
  }
  if (ng_shift >= 3) {
#pragma unroll
    for (int v = 0; v < 16; v += 8) vmin[v] = vmin[v + 4] < vmin[v] ? vmin[v + 4] : vmin[v];
  }
  if (ng_shift >= 4) vmin[0] = vmin[8] < vmin[0] ? vmin[8] : vmin[0];
  if (wave < nwv) {
    qt* gm = s_gm + j * G8 + (wave * 2 + h) * NG;
    const int gmask = (1 << ng_shift) - 1;
#pragma unroll
    for (int v = 0; v < 16; ++v)
      if ((v & gmask) == 0) gm[v >> ng_shift] = vmin[v];
  }
  __syncthreads();
  // tau of each patch: the ksel-th smallest of its group minima (ties by
  // position)
  for (int pi = tid; pi < kFiltersPerTile * G8; pi += kThreads) {
    const int jj = pi / G8, i = pi - jj * G8;
    const qt* gm = s_gm + jj * G8;
    const qt x = gm[i];
    int rank = 0;
    for (int i2 = 0; i2 < G8; ++i2) {
      const qt y = gm[i2];
      rank += (y < x || (y == x && i2 < i)) ? 1 : 0;
    }
    if (rank == a.ksel - 1) s_tau[jj] = x;
  }
  __syncthreads();

  // pass 2: survivors, their keys
  const qt tau = s_tau[j];
  int qn = 0;   // entries in this wavefront's queue (uniform)
  auto flush = [&]() {
    __builtin_amdgcn_wave_barrier();   // the queue entries other lanes wrote come first
    for (int i = lane; i < qn; i += 64) {
      const uint2 e = s_q[i];
      const int jj = (int)((e.y >> 12) & 31u), cx = (int)(e.y & 4095u);
      const uint32_t mm = e.y >> 20;
      const long long idx = rowbase + cx;
      const uint64_t key = make_key(mm, (int32_t)e.x, tie_perm((uint32_t)idx, s_rec[jj].tkey));
      const unsigned pos = atomicAdd(&s_cnt[jj], 1u);
      a.keys[(long long)(t.first + jj) * g.ncand + rowbase + pos] = key;
      atomicMin(&s_rmin[jj], (unsigned long long)key);
    }
    __builtin_amdgcn_wave_barrier();
    qn = 0;
  };
  const unsigned jbits = (unsigned)j << 12;
  for (int p = 0; p < my_chunks; ++p) {
    const int ch = wave + (kThreads / 64) * p;
    qt q[16];
    if (p == 0) {
#pragma unroll
      for (int v = 0; v < 16; ++v) q[v] = qv0[v];
    } else if (p == 1) {
#pragma unroll
      for (int v = 0; v < 16; ++v) q[v] = qv1[v];
    } else {
      chunk_values(ch, q);
    }
#pragma unroll
    for (int v4 = 0; v4 < 16; v4 += 4) {
      if (qn > kSelQueue - 256) flush();
#pragma unroll
      for (int v = v4; v < v4 + 4; ++v) {
        const bool sv = q[v] != SV::inf() && q[v] <= tau;
        const uint64_t m = __ballot(sv);
        if (m) {
          if (sv) {
            const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const int cx = ch * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            s_q[pos] = make_uint2((uint32_t)SV::score(q[v]), (uint32_t)cx | jbits | (SV::mis(q[v]) << 20));
          }
          qn += __builtin_popcountll(m);
        }
      }
    }
  }
  flush();
  __syncthreads();
  if (tid < t.count && s_rec[tid].gidx >= 0) {
    const long long o2 = (long long)(t.first + tid) * (g.cand[1] * g.cand[2]) + row;
    a.rowcnt[o2] = (int32_t)s_cnt[tid];
    a.rowmin[o2] = s_rmin[tid];
  }
}

// Energy term E(c) = sum_beta n_beta K[c + beta]^2 for each shape (rows of
// nbt), int32.  One thread per (shape, candidate).
__global__ __launch_bounds__(kThreads) void k_energy(const int32_t* __restrict__ K,
                                                     const int32_t* __restrict__ nbt, int n_shapes,
                                                     int32_t* __restrict__ out, Geom g) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)n_shapes * g.ncand) return;
  const int shape = (int)(id / g.ncand);
  const long long c = id - (long long)shape * g.ncand;
  const int cx = (int)(c % g.cand[0]), cy = (int)((c / g.cand[0]) % g.cand[1]);
  const int cz = (int)(c / ((long long)g.cand[0] * g.cand[1]));
  const int32_t* nb = nbt + (long long)shape * g.tcells;
  int e = 0;
  for (int bz = 0; bz < g.tc[2]; ++bz)
    for (int by = 0; by < g.tc[1]; ++by)
      for (int bx = 0; bx < g.tc[0]; ++bx) {
        const int n = nb[(bz * g.tc[1] + by) * g.tc[0] + bx];
        if (n) {
          const int kv = K[idx3(cx + bx, cy + by, cz + bz, g.G)];
          e += n * kv * kv;
        }
      }
  out[id] = e;
}

}  // namespace ccw
