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
  const int32_t* segoff;       // fused: [orient][kSegMax] strip offset of each 8-tap segment's first block
  const int32_t* taps;         // fused: [orient][kSegMax * 8] data-event entry of each tap, or -1
  int klist;                   // fused, simulation: entries of the orientation block lists (a multiple of 16)
  int n_tinline;               // fused, simulation: tiles passed by value (the step's first ones)
  TileDev tiles_inline[32];
  int ksel;                    // keys the selection keeps per row (K, or the shortlist)
  int gbits;                   // value v of a lane joins group v & (2^gbits - 1) of its lane
  int n_bm;                    // band masks per orientation (energy rows per tile)
  const int32_t* ntiles_dyn;   // fused, simulation: tiles of this launch counted on the device, or null
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
//      minima of q over groups of its values (disjoint sets of candidates,
//      spread along the row); the ksel-th smallest of a patch's group
//      minima, tau, bounds the q of its ksel-th best candidate from above:
//      ksel candidates have q <= tau, and a candidate with q > tau has ksel
//      keys below its own.
//   2. Candidates with q <= tau (the survivors) get their full key (with the
//      keyed tie-break) and are written out.  Survivors are collected per
//      wavefront into an LDS queue with ballots, so the keys of a sparse
//      set of survivors are built densely, 64 at a time.
// A row's best keys are therefore among its survivors, and the K best keys
// of a patch are among the survivors of the K rows with the smallest minima.
//
// The contraction uses the Toeplitz structure of the correlation: along a
// row of template blocks, block bx of candidate cx reads K[cx + bx].  The
// overlap's blocks are covered by segments of 8 consecutive blocks of one
// block row (a block outside the overlap inside a segment gets weight 0),
// and one MFMA K-slice of 16 taps is two segments.  Lane (candidate c,
// half h) then needs the 8 consecutive values K[c + bx0 .. c + bx0 + 7] of
// its segment: four aligned 32-bit LDS reads from one of two copies of the
// strip, the second shifted by one value, picked by the parity of c + bx0.
//
// Energy source EN: kEnStage -- the energy rows of the tile's orientation
// (one per band mask) are staged in LDS; kEnFold -- the MFMA also contracts
// K^2 against the known-cell counts n (a second accumulator, exact when
// K^2 <= 2048 and sum n K^2 < 2^24); kEnMem -- per filter energy rows read
// from memory (standalone).  HD: hard-data mismatch counts from the bit
// table enter the key.
// ---------------------------------------------------------------------------
constexpr int kSelQueue = 256;   // survivor queue entries per wavefront
constexpr int kSegMax = 32;      // segments of 8 taps (16 MFMA K-slices)
enum { kEnStage = 0, kEnFold = 1, kEnMem = 2 };

// Strip row length (values) of the fused scan: the candidate chunks, the
// template row and one segment of slack.
inline int scan_sel_width(int cpad, int tc0) { return (cpad + ((tc0 + 7) / 8) * 8 + 8 + 3) & ~3; }

// LDS bytes of k_scan_sel.
inline size_t scan_sel_lds(int nrows, int W, int kk, int klist, int en, int n_bm, int cpad, int gbits, bool hd) {
  const size_t cs = ((size_t)nrows * W * 2 + 15) & ~(size_t)15;
  size_t o = cs * 2;
  o += 4 * kSegMax / 2 * 4;                                   // segment addresses
  o += (size_t)kFiltersPerTile * (kk * (en == kEnFold ? 2 : 1) + 8) * 2;   // B operand
  o += (size_t)kFiltersPerTile * sizeof(ScanRec);
  if (en == kEnStage) o += (size_t)(n_bm + 2) * cpad * 4;
  const int nwv = std::min(kThreads / 64, cpad / 32);
  o += (size_t)kFiltersPerTile * (nwv * 2 * (1 << gbits)) * (hd ? 8 : 4);
  o += std::max((size_t)(kThreads / 64) * kSelQueue * 8, (size_t)kFiltersPerTile * klist * 2);
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
  constexpr bool FOLD = EN == kEnFold;
  const OT* Kop = (const OT*)a.Kop;
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = blockIdx.x;
  const int cy = row % g.cand[1], cz = row / g.cand[1];
  const int W = a.W, kk = a.kpad;          // kk: taps (16 per K-slice, a multiple of 64)
  const int KS = kk / 16;
  const int nrows = g.tc[1] * g.tc[2];
  const int j = lane & 31, h = lane >> 5;
  const int C0 = g.cand[0];
  const int nchunks = (C0 + 31) / 32;
  const int cpad = nchunks * 32;
  const int kb = FOLD ? 2 * kk : kk;       // B operand length (taps, then known-cell counts)
  const int bstride = kb + 8;
  const int gbits = a.gbits;
  const int NG = 1 << gbits;
  const int nwv = min(kThreads / 64, nchunks);   // wavefronts holding chunks
  const int G8 = nwv * 2 * NG;                   // groups per patch

  const int strip_n = nrows * W;
  const int cs = (strip_n * 2 + 15) & ~15;       // bytes per strip copy
  unsigned char* s_strip = smem;                 // copies: K, K shifted by one
  size_t o = (size_t)cs * 2;
  int* s_seg = (int*)(smem + o);                 // [h][parity of c][slice] byte address of the segment
  o += 4 * kSegMax / 2 * 4;
  OT* s_B = (OT*)(smem + o);
  o += (size_t)kFiltersPerTile * bstride * 2;
  ScanRec* s_rec = (ScanRec*)(smem + o);
  o += (size_t)kFiltersPerTile * sizeof(ScanRec);
  int32_t* s_E = (int32_t*)(smem + o);           // [band mask][cpad], then a zero row and an infinite row
  if (EN == kEnStage) o += (size_t)(a.n_bm + 2) * cpad * 4;
  qt* s_gm = (qt*)(smem + o);
  o += (size_t)kFiltersPerTile * G8 * sizeof(qt);
  unsigned char* s_qbase = smem + o;   // survivor queues; before pass 1 the event staging
  uint2* s_q = (uint2*)s_qbase + wave * kSelQueue;
  __shared__ unsigned s_cnt[kFiltersPerTile];
  __shared__ unsigned long long s_rmin[kFiltersPerTile];
  __shared__ qt s_tau[kFiltersPerTile];

  // tiles packed on the device: the grid covers the most there can be
  if (a.ntiles_dyn && (int)blockIdx.y >= *a.ntiles_dyn) return;
  TileDev t;
  if (a.standalone) {
    t.first = blockIdx.y * kFiltersPerTile;
    t.count = min(kFiltersPerTile, a.n_filters - t.first);
    t.orient = 0;
    t.zmask = 0;
  } else {
    // the tile record by value when the step's tiles fit the arguments, so
    // it arrives with them (the empty asm takes both loads before the branch)
    const int n_ti = a.n_tinline;
    const TileDev t_arg = a.tiles_inline[min((int)blockIdx.y, 31)];
    __asm__ volatile("" ::"s"(n_ti), "s"(t_arg.first));
    if ((int)blockIdx.y < n_ti) {
      t = t_arg;
      __asm__ volatile("" ::: "memory");
    } else {
      t = a.tiles[blockIdx.y];
    }
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
  // strip copies: copy 0 holds K[x], copy 1 K[x + 1].  Lane l of a
  // wavefront loads 4 values of a block row with one 8-byte load and
  // stores them to copy 0; copy 1 takes values 1..3 of the lane and value 0
  // of the next lane (a lane shuffle), so each value is loaded once.  The
  // wavefronts take the rows in turn; near the grid's edge a lane loads
  // value by value.
  {
    const int nq = W / 4;   // 4-value groups per row (W is a multiple of 4)
    for (int rr = wave; rr < nrows; rr += kThreads / 64) {
      const int by = rr % g.tc[1], bz = rr / g.tc[1];
      const OT* krow = Kop + (long long)g.G[0] * ((cy + by) + (long long)g.G[1] * (cz + bz));
      for (int xq0 = 0; xq0 < nq + 1; xq0 += 64) {
        const int xq = xq0 + lane;
        const int x = 4 * xq;
        uint64_t w0 = 0;
        if (x + 4 <= g.G[0]) {
          __builtin_memcpy(&w0, krow + x, 8);
        } else if (x < g.G[0]) {
          OT v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = x + e < g.G[0] ? krow[x + e] : (OT)0.0f;
          __builtin_memcpy(&w0, v, 8);
        }
        // value 0 of the next lane; the last lane of a pass loads its own
        uint32_t nxt = (uint32_t)__shfl_down((int)(uint32_t)w0, 1, 64);
        if (lane == 63) {
          OT v0 = (OT)0.0f;
          if (x + 4 < g.G[0]) v0 = krow[x + 4];
          uint16_t b16;
          __builtin_memcpy(&b16, &v0, 2);
          nxt = b16;
        }
        const uint64_t w1 = (w0 >> 16) | ((uint64_t)(nxt & 0xFFFFu) << 48);
        if (xq < nq) {
          *(uint64_t*)(s_strip + 2 * (rr * W + x)) = w0;
          *(uint64_t*)(s_strip + cs + 2 * (rr * W + x)) = w1;
        }
      }
    }
  }
  // data events (and, folded, the known-cell counts) as the B operand:
  // standalone events arrive in tap order and are copied with 32-byte
  // loads; a simulation's arrive in the order of the orientation's block
  // list and are staged in LDS with 32-byte loads, then moved to their taps
  // after the barrier.  Thread tid takes filter tid % 32 and every eighth
  // group of 8 entries from tid / 32 on.
  typedef int32_t int8v_t __attribute__((ext_vector_type(8)));
  const int kl = a.standalone ? kk : a.klist;   // entries per event row
  OT* s_mst = (OT*)s_qbase;                     // staging (simulation), aliases the survivor queues
  {
    const int jj = tid & (kFiltersPerTile - 1);
    const bool on = jj < t.count && !((t.zmask >> jj) & 1u);
    // packed tiles name their patches in the records (rec is lane jj's)
    const long long fo = (long long)(a.ntiles_dyn ? rec.gidx : a.fbegin + t.first + jj) * kKMax;
    for (int k8 = (tid >> 5) * 8; k8 < kl; k8 += 64) {
      int8v_t m = {}, n = {};
      if (on) {
        m = *(const int8v_t*)(a.mbuf + fo + k8);
        if (FOLD) n = *(const int8v_t*)(a.nbuf + fo + k8);
      }
      vec8 v, w;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        v[e] = (OT)(float)m[e];
        if (FOLD) w[e] = (OT)(float)n[e];
      }
      if (a.standalone) {
        *(vec8*)(s_B + jj * bstride + k8) = v;
        if (FOLD) *(vec8*)(s_B + jj * bstride + kk + k8) = w;
      } else {
        *(vec8*)(s_mst + jj * kl + k8) = v;
      }
    }
  }
  // energy rows of the tile's orientation (one per band mask), a zero row
  // and an infinite row; 4 candidates per thread and load
  if (EN == kEnStage) {
    const int nb = a.n_bm;
    const int c4 = cpad / 4;
    for (int i = tid; i < (nb + 2) * c4; i += kThreads) {
      const int bm = i / c4, cx = (i - bm * c4) * 4;
      int4 e4 = make_int4(0, 0, 0, 0);
      if (bm == nb + 1) {
        e4 = make_int4(0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF);
      } else if (bm < nb && a.score_mode == 0) {
        const int32_t* er = a.energy + (long long)((t.orient * nb) | bm) * g.ncand + rowbase + cx;
        if (cx + 4 <= C0 && ((uintptr_t)er & 15) == 0) {
          e4 = *(const int4*)er;
        } else {
          e4.x = cx < C0 ? er[0] : 0;
          e4.y = cx + 1 < C0 ? er[1] : 0;
          e4.z = cx + 2 < C0 ? er[2] : 0;
          e4.w = cx + 3 < C0 ? er[3] : 0;
        }
      }
      *(int4*)(s_E + bm * cpad + cx) = e4;
    }
  }
  // the first tap entries of this thread's scatter (after the barrier)
  int4 tq0[2] = {make_int4(-1, -1, -1, -1), make_int4(-1, -1, -1, -1)};
  if (!a.standalone && tid < kFiltersPerTile * (kk / 8)) {
    const int tp = (tid >> 5) * 8;
    tq0[0] = *(const int4*)(a.taps + t.orient * (kSegMax * 8) + tp);
    tq0[1] = *(const int4*)(a.taps + t.orient * (kSegMax * 8) + tp + 4);
  }
  // segments of this orientation: byte address, per lane parity, of the
  // four aligned words holding taps bx0 .. bx0 + 7 for candidate c = parity
  if (tid < kSegMax) {
    const int sg = tid;
    int so = 0;
    if (sg < 2 * KS) {
      if (a.standalone) {
        const int spr = (g.tc[0] + 7) / 8;   // segments per block row
        const int r = sg / spr, bx0 = (sg - r * spr) * 8;
        so = r < nrows ? r * W + bx0 : 0;
      } else {
        so = a.segoff[t.orient * kSegMax + sg];
      }
    }
#pragma unroll
    for (int jp = 0; jp < 2; ++jp) {
      const int p = (so + jp) & 1;
      s_seg[((sg & 1) * 2 + jp) * (kSegMax / 2) + (sg >> 1)] = p * cs + 2 * (so + jp - p);
    }
  }
  lds_barrier();
  if (!a.standalone) {
    // events to their taps, 8 taps of one filter per thread and step (the
    // tap entries were loaded before the barrier)
    const int tg = kk / 8;
    for (int i = tid, it = 0; i < kFiltersPerTile * tg; i += kThreads, ++it) {
      const int jj = i & (kFiltersPerTile - 1), tp = (i >> 5) * 8;
      const int4 k0 = it == 0 ? tq0[0] : *(const int4*)(a.taps + t.orient * (kSegMax * 8) + tp);
      const int4 k1 = it == 0 ? tq0[1] : *(const int4*)(a.taps + t.orient * (kSegMax * 8) + tp + 4);
      const int kq[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
      vec8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = kq[e] >= 0 ? s_mst[jj * kl + kq[e]] : (OT)0.0f;
      *(vec8*)(s_B + jj * bstride + tp) = v;
    }
    lds_barrier();
  }

  const bool fvalid = rec.gidx >= 0;
  const int shift = g.shift;
  const int J = g.level, Jz = g.ndim == 3 ? J : 0;
  // S = E - mul * C: mul = 2^shift (squared difference) or 1 (raw, E = 0);
  // an invalid lane reads the infinite row with mul = 0
  const int mul = !fvalid ? 0 : a.score_mode == 0 ? (1 << shift) : 1;
  const int32_t* erow_s = EN == kEnStage
                              ? s_E + (!fvalid ? a.n_bm + 1 : a.score_mode == 0 ? (rec.shape & (a.n_bm - 1)) : a.n_bm) * cpad
                              : nullptr;
  const int32_t* erow_m = EN == kEnMem ? a.energy + (long long)(fvalid ? t.first + j : t.first) * g.ncand + rowbase : nullptr;
  const int einf = fvalid ? 0 : 0x7FFFFFFF;   // fold / memory energy of an invalid lane
  const int lane_b = 2 * (j & ~1);            // bytes of the even part of c within a chunk
  const int jp = j & 1;
  const int* segp = s_seg + (h * 2 + jp) * (kSegMax / 2);
  const OT* brow = s_B + j * bstride + 8 * h;

  // selection values of one 32-candidate chunk (invalid entries: infinity)
  auto chunk_values = [&](int ch, qt (&q)[16]) {
    int ev[16];
    unsigned mis[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) mis[v] = 0;
    if (EN == kEnStage) {
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        const int4 e4 = *(const int4*)(erow_s + ch * 32 + 8 * qd + 4 * h);
        ev[4 * qd] = e4.x;
        ev[4 * qd + 1] = e4.y;
        ev[4 * qd + 2] = e4.z;
        ev[4 * qd + 3] = e4.w;
      }
    } else if (EN == kEnMem) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int cx = ch * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        ev[v] = (a.score_mode == 0 && cx < C0) ? erow_m[cx] : 0;
        if (!fvalid) ev[v] = 0x7FFFFFFF;
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
    // contraction: four K-slices at a time, every read of a group issued
    // before its MFMAs
    float16_t acc = {}, acc2 = {};
    const int cb = lane_b + ch * 64;
    for (int q0 = 0; q0 < KS; q0 += 4) {
      const int4 sa4 = *(const int4*)(segp + q0);
      const int sa[4] = {sa4.x, sa4.y, sa4.z, sa4.w};
      vec8 av[4], bv[4], a2[4], b2[4];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const unsigned char* p = s_strip + sa[qq] + cb;
        uint32_t w4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) w4[e] = *(const uint32_t*)(p + 4 * e);
        av[qq] = __builtin_bit_cast(vec8, w4);
        bv[qq] = *(const vec8*)(brow + (q0 + qq) * 16);
        if (FOLD) {   // K^2 from the same values: exact, K^2 stays below the operand's integer range
          a2[qq] = av[qq] * av[qq];
          b2[qq] = *(const vec8*)(brow + kk + (q0 + qq) * 16);
        }
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        acc = MfmaOp<OT>::mma(av[qq], bv[qq], acc);
        if (FOLD) acc2 = MfmaOp<OT>::mma(a2[qq], b2[qq], acc2);
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int C = (int)acc[v];
      const int E = FOLD ? (int)acc2[v] + einf : ev[v];
      q[v] = SV::make(mis[v], E - __mul24(mul, C));
    }
    if (ch * 32 + 32 > C0) {   // the row's last chunk: candidates past the row
#pragma unroll
      for (int v = 0; v < 16; ++v)
        if (ch * 32 + 8 * (v >> 2) + 4 * h + (v & 3) >= C0) q[v] = SV::inf();
    }
    if (HD && !fvalid) {
#pragma unroll
      for (int v = 0; v < 16; ++v) q[v] = SV::inf();
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
  // group g of a lane: its values v with v mod NG = g.  Value v holds
  // candidate 8 (v / 4) + 4 h + v % 4 of a chunk, so the candidates of one
  // group are spread along the row and a run of good neighbouring
  // candidates lands in different groups (a tighter tau).
  if (gbits <= 3) {
#pragma unroll
    for (int v = 0; v < 8; ++v) vmin[v] = vmin[v + 8] < vmin[v] ? vmin[v + 8] : vmin[v];
  }
  if (gbits <= 2) {
#pragma unroll
    for (int v = 0; v < 4; ++v) vmin[v] = vmin[v + 4] < vmin[v] ? vmin[v + 4] : vmin[v];
  }
  if (gbits <= 1) {
#pragma unroll
    for (int v = 0; v < 2; ++v) vmin[v] = vmin[v + 2] < vmin[v] ? vmin[v + 2] : vmin[v];
  }
  if (gbits <= 0) vmin[0] = vmin[1] < vmin[0] ? vmin[1] : vmin[0];
  if (wave < nwv) {
    qt* gm = s_gm + j * G8 + (wave * 2 + h) * NG;
#pragma unroll
    for (int v = 0; v < 16; ++v)
      if (v < NG) gm[v] = vmin[v];
  }
  lds_barrier();
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
  lds_barrier();

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
    const unsigned cxb = (unsigned)(ch * 32 + 4 * h) | jbits;
#pragma unroll
    for (int v2 = 0; v2 < 16; v2 += 2) {
      if (qn > kSelQueue - 128) flush();
#pragma unroll
      for (int v = v2; v < v2 + 2; ++v) {
        const bool sv = q[v] <= tau && q[v] != SV::inf();
        const uint64_t m = __ballot(sv);
        if (m) {
          if (sv) {
            const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            s_q[pos] = make_uint2((uint32_t)SV::score(q[v]),
                                  (cxb + (unsigned)(8 * (v >> 2) + (v & 3))) | (SV::mis(q[v]) << 20));
          }
          qn += __builtin_popcountll(m);
        }
      }
    }
  }
  flush();
  lds_barrier();
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
