/*
 * ccwsim_oracle.c -- plain, slow CPU oracle of the CCWSIM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: every step below is written out again from
 * the paper (Bavandsavadkoohi et al., "CCWSIM", arXiv 2404.00441) with plain
 * loops and 64-bit integer arithmetic.
 *
 * Method steps and where they come from (paper sections / equations):
 *   - Haar DWT of the training image, level J: Sec. 3.1 (filter-and-downsample
 *     steps, the 2D expansion and its basis), Haar scaling/wavelet functions in
 *     Sec. 4.2.  Algorithm 1, step "compute DWT of TI".
 *   - Inverse DWT of the chosen pattern: Sec. 3.1 (bijective filters),
 *     Sec. 3.2 (details keep what the approximation drops), Algorithm 1
 *     step "Inv-DWT".
 *   - Raster-path lattice and overlapping region (L-shaped / vertical /
 *     horizontal): Sec. 4.1 and Fig. 3a-c.  Randomised origin and direction:
 *     Algorithm 1, step "Randomize(origin, direction)".
 *   - CCW similarity of approximation coefficients: Sec. 4.3, CCW equation.
 *   - Top-K candidates and uniform random draw: Sec. 4.4, Algorithm 1.
 *   - Conditioning by a virtual template and sequential search over the
 *     sorted scores: end of Sec. 4.4 (defers to MS-CCSIM).
 *   - Minimal-error boundary cut between patches: Sec. 2 (image quilting) and
 *     Sec. 4.1 (the OR resembles image quilting).
 *   - Another mother wavelet (Sec. 4.2 calls Haar particularly suitable, so a
 *     choice exists): the LeGall 5/3 biorthogonal wavelet in the integer
 *     lifting form of Calderbank, Daubechies, Sweldens and Yeo ("Wavelet
 *     transforms that map integers to integers", 1998), the reversible filter
 *     of JPEG 2000, with whole-sample symmetric extension.
 *
 * Integer conventions (the paper's normalisation is orthonormal; every
 * ranking below is scale-invariant, so the oracle works on the unnormalised
 * integer Haar transform: low = e + o, high = e - o per axis and level; the
 * orthonormal coefficient is the integer times 2^(-p/2) after p passes).
 *
 * Readings of the paper taken where it is silent or garbled are listed in the
 * repository's design notes; each function below names the reading it uses.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_SHAPE 2
#define ORC_ERR_RANGE 3
#define ORC_ERR_NOMEM 4

/* RNG stream identifiers (counter-based generator, see orc_rng). */
#define ORC_STREAM_PATH 1u
#define ORC_STREAM_TIEBREAK 2u
#define ORC_STREAM_DRAW 3u

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t ti_n[3];       /* TI extent, [0] = x (fastest) */
    int32_t sg_n[3];       /* simulation grid extent */
    int32_t tmpl[3];       /* template T per axis */
    int32_t overlap[3];    /* overlap OV per axis */
    int32_t level;         /* J */
    int32_t top_k;         /* K */
    int32_t n_real;        /* realizations */
    int32_t n_facies;      /* facies codes are 0 .. n_facies-1 */
    uint64_t seed;
    int32_t path_mode;     /* 0 fixed raster, 1 seeded corner (+ major axis in 2D) */
    int32_t score_mode;    /* 0 SSD, 1 raw CCW */
    int32_t nc_margin[3];  /* virtual-template margin; negative -> overlap */
    int32_t cut;           /* 1 min-error boundary cut, 0 plain paste */
    int32_t wavelet;       /* 0 Haar, 1 LeGall 5/3 integer lifting */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers.                                             */
/* The paper draws "randomly" (Algorithm 1) without naming a generator.      */
/* Reading: every draw is a pure function of (seed, stream, a, b) so that a  */
/* result does not depend on the order in which patches are processed.       */
/* The mixer is SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state advance  */
/* by the golden-ratio increment, then the variant-13 finaliser.             */
/* ------------------------------------------------------------------------ */
static uint64_t orc_splitmix_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static const uint64_t ORC_GOLDEN = 0x9e3779b97f4a7c15ULL;

/* First SplitMix64 output from state x (so orc_splitmix_first(0) is the
 * published first output of a generator seeded with 0). */
uint64_t orc_splitmix_first(uint64_t x)
{
    return orc_splitmix_finalise(x + ORC_GOLDEN);
}

/* Absorb one 64-bit word into a running hash: xor it in, then one SplitMix64
 * step. */
static uint64_t orc_absorb(uint64_t h, uint64_t w)
{
    return orc_splitmix_finalise((h ^ w) + ORC_GOLDEN);
}

uint64_t orc_rng(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b)
{
    uint64_t h = orc_splitmix_first(seed);
    h = orc_absorb(h, stream);
    h = orc_absorb(h, a);
    h = orc_absorb(h, b);
    return h;
}

/* Keyed bijection on 20-bit integers used to break score ties (reading: the
 * paper is silent on ties; a lowest-index rule would bias every draw towards
 * the TI origin on binary images, where ties are huge).  Each step is
 * invertible on [0, 2^20): xor with a key, multiply by an odd constant,
 * xor with a right shift of itself. */
uint32_t orc_perm20(uint32_t x, uint64_t key)
{
    const uint32_t M = 0xFFFFFu;
    uint32_t k1 = (uint32_t)(key & M);
    uint32_t k2 = (uint32_t)((key >> 20) & M);
    uint32_t k3 = (uint32_t)((key >> 40) & M);
    x &= M;
    x ^= k1;
    x = (x * 0x6B5A5u) & M;
    x ^= x >> 10;
    x ^= k2;
    x = (x * 0x3A8F3u) & M;
    x ^= x >> 9;
    x ^= k3;
    return x & M;
}

/* ------------------------------------------------------------------------ */
/* Small geometry helpers.                                                   */
/* ------------------------------------------------------------------------ */
static int64_t orc_idx3(int64_t x, int64_t y, int64_t z, const int64_t d[3])
{
    return x + d[0] * (y + d[1] * z);
}

/* Per-axis block factor: 2^J on the active axes, 1 on an unused third axis. */
static void orc_block_factor(int ndim, int J, int64_t b[3])
{
    for (int a = 0; a < 3; a++) b[a] = (a < ndim) ? ((int64_t)1 << J) : 1;
}

/* ------------------------------------------------------------------------ */
/* Haar DWT, integer form (Sec. 3.1 steps: filter rows with the low- and     */
/* high-pass filters and keep every second column, then do the same on the   */
/* columns; Sec. 4.2 Haar functions: scaling function = box, wavelet = +1 on */
/* the first half and -1 on the second).  Low-pass (e, o) -> e + o,          */
/* high-pass (e, o) -> e - o.  Reading on boundaries: the image is first     */
/* extended by edge replication to a multiple of 2^J on every axis.          */
/*                                                                          */
/* Output layout:                                                           */
/*   approx:  level-J approximation (= integer block sums), size G = Np/2^J. */
/*   details: for j = 1..J, for sub-band s = 1 .. 2^ndim-1 (bit a of s set   */
/*            when axis a took the high-pass), an array of Np/2^j cells,     */
/*            x fastest.  Levels are concatenated in increasing j.          */
/* ------------------------------------------------------------------------ */

/* One analysis pass along axis `a`: src has extent d, the two outputs have
 * extent d with d[a] halved. */
static void orc_analysis_pass(const int64_t *src, const int64_t d[3], int a,
                              int64_t *lo, int64_t *hi)
{
    int64_t h[3] = {d[0], d[1], d[2]};
    h[a] /= 2;
    for (int64_t z = 0; z < h[2]; z++)
        for (int64_t y = 0; y < h[1]; y++)
            for (int64_t x = 0; x < h[0]; x++) {
                int64_t pe[3] = {x, y, z}, po[3] = {x, y, z};
                pe[a] = 2 * pe[a];
                po[a] = 2 * po[a] + 1;
                int64_t e = src[orc_idx3(pe[0], pe[1], pe[2], d)];
                int64_t o = src[orc_idx3(po[0], po[1], po[2], d)];
                lo[orc_idx3(x, y, z, h)] = e + o;
                hi[orc_idx3(x, y, z, h)] = e - o;
            }
}

/* Padded extent of the image and number of detail values. */
static void orc_padded(const int32_t n[3], int ndim, int J, int64_t np[3])
{
    int64_t b[3];
    orc_block_factor(ndim, J, b);
    for (int a = 0; a < 3; a++) np[a] = ((n[a] + b[a] - 1) / b[a]) * b[a];
}

int64_t orc_details_count(const int32_t n[3], int32_t ndim, int32_t J)
{
    int64_t np[3];
    orc_padded(n, ndim, J, np);
    int64_t total = 0;
    int nsub = (1 << ndim) - 1;
    for (int j = 1; j <= J; j++) {
        int64_t cells = 1;
        for (int a = 0; a < 3; a++) cells *= (a < ndim) ? (np[a] >> j) : np[a];
        total += nsub * cells;
    }
    return total;
}

int orc_dwt(const int8_t *ti, const int32_t n[3], int32_t ndim, int32_t J,
            int64_t *approx, int64_t *details)
{
    if (ndim < 2 || ndim > 3 || J < 0) return ORC_ERR_ARG;
    if (ndim == 2 && n[2] != 1) return ORC_ERR_SHAPE;
    int64_t np[3];
    orc_padded(n, ndim, J, np);
    int64_t ncell = np[0] * np[1] * np[2];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * ncell);
    if (!cur) return ORC_ERR_NOMEM;
    int64_t d[3] = {n[0], n[1], n[2]};
    /* edge-replicating extension */
    for (int64_t z = 0; z < np[2]; z++)
        for (int64_t y = 0; y < np[1]; y++)
            for (int64_t x = 0; x < np[0]; x++) {
                int64_t sx = x < n[0] ? x : n[0] - 1;
                int64_t sy = y < n[1] ? y : n[1] - 1;
                int64_t sz = z < n[2] ? z : n[2] - 1;
                cur[orc_idx3(x, y, z, np)] = ti[orc_idx3(sx, sy, sz, d)];
            }
    int64_t cd[3] = {np[0], np[1], np[2]};
    int nsub = 1 << ndim;
    int64_t det_off = 0;
    for (int j = 1; j <= J; j++) {
        /* subs[s] holds the sub-band whose high-pass axes are the bits of s */
        int64_t *subs[8] = {0};
        int64_t sd[3] = {cd[0], cd[1], cd[2]};
        subs[0] = cur;
        int have = 1;
        for (int a = 0; a < ndim; a++) {
            int64_t hd[3] = {sd[0], sd[1], sd[2]};
            hd[a] /= 2;
            int64_t hcells = hd[0] * hd[1] * hd[2];
            for (int s = 0; s < have; s++) {
                int64_t *lo = (int64_t *)malloc(sizeof(int64_t) * hcells);
                int64_t *hi = (int64_t *)malloc(sizeof(int64_t) * hcells);
                if (!lo || !hi) return ORC_ERR_NOMEM;
                orc_analysis_pass(subs[s], sd, a, lo, hi);
                free(subs[s]);
                subs[s] = lo;
                subs[s | (1 << a)] = hi;
            }
            have *= 2;
            sd[a] = hd[a];
        }
        int64_t scells = sd[0] * sd[1] * sd[2];
        for (int s = 1; s < nsub; s++) {
            memcpy(details + det_off, subs[s], sizeof(int64_t) * scells);
            det_off += scells;
            free(subs[s]);
        }
        cur = subs[0];
        cd[0] = sd[0];
        cd[1] = sd[1];
        cd[2] = sd[2];
    }
    memcpy(approx, cur, sizeof(int64_t) * cd[0] * cd[1] * cd[2]);
    free(cur);
    return ORC_OK;
}

/* One synthesis pass along axis `a` (inverse of orc_analysis_pass):
 * e = (lo + hi) / 2, o = (lo - hi) / 2; the divisions are exact because
 * lo and hi always have the same parity. */
static void orc_synthesis_pass(const int64_t *lo, const int64_t *hi,
                               const int64_t h[3], int a, int64_t *dst)
{
    int64_t d[3] = {h[0], h[1], h[2]};
    d[a] *= 2;
    for (int64_t z = 0; z < h[2]; z++)
        for (int64_t y = 0; y < h[1]; y++)
            for (int64_t x = 0; x < h[0]; x++) {
                int64_t l = lo[orc_idx3(x, y, z, h)];
                int64_t g = hi[orc_idx3(x, y, z, h)];
                int64_t pe[3] = {x, y, z}, po[3] = {x, y, z};
                pe[a] = 2 * pe[a];
                po[a] = 2 * po[a] + 1;
                dst[orc_idx3(pe[0], pe[1], pe[2], d)] = (l + g) / 2;
                dst[orc_idx3(po[0], po[1], po[2], d)] = (l - g) / 2;
            }
}

/* Inverse DWT of a region of the pyramid.  The region starts at level-J
 * block `c0` and spans `nc` level-J blocks per axis; it is rebuilt level by
 * level from the level-J approximation and the detail sub-bands that cover
 * it (Haar atoms never straddle a dyadic block, so the region needs nothing
 * outside it).  `out` receives (nc * 2^J) cells per active axis, x fastest.
 * With c0 = 0 and nc = G this is the full inverse transform. */
int orc_idwt_region(const int64_t *approx, const int64_t *details,
                    const int32_t n[3], int32_t ndim, int32_t J,
                    const int32_t c0[3], const int32_t nc[3], int64_t *out)
{
    if (ndim < 2 || ndim > 3 || J < 0) return ORC_ERR_ARG;
    int64_t np[3];
    orc_padded(n, ndim, J, np);
    int64_t G[3];
    for (int a = 0; a < 3; a++) G[a] = (a < ndim) ? (np[a] >> J) : np[a];
    for (int a = 0; a < 3; a++)
        if (c0[a] < 0 || nc[a] < 1 || c0[a] + nc[a] > G[a]) return ORC_ERR_RANGE;
    /* current approximation region at level j, start cs, extent ce */
    int64_t ce[3] = {nc[0], nc[1], nc[2]};
    int64_t cs[3] = {c0[0], c0[1], c0[2]};
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * ce[0] * ce[1] * ce[2]);
    if (!cur) return ORC_ERR_NOMEM;
    for (int64_t z = 0; z < ce[2]; z++)
        for (int64_t y = 0; y < ce[1]; y++)
            for (int64_t x = 0; x < ce[0]; x++)
                cur[orc_idx3(x, y, z, ce)] =
                    approx[orc_idx3(cs[0] + x, cs[1] + y, cs[2] + z, G)];
    int nsub = 1 << ndim;
    for (int j = J; j >= 1; j--) {
        /* locate level-j details: skip levels 1..j-1 */
        int64_t off = 0;
        for (int jj = 1; jj < j; jj++) {
            int64_t cells = 1;
            for (int a = 0; a < 3; a++) cells *= (a < ndim) ? (np[a] >> jj) : np[a];
            off += (int64_t)(nsub - 1) * cells;
        }
        int64_t Gj[3];
        for (int a = 0; a < 3; a++) Gj[a] = (a < ndim) ? (np[a] >> j) : np[a];
        int64_t gcells = Gj[0] * Gj[1] * Gj[2];
        int64_t rcells = ce[0] * ce[1] * ce[2];
        int64_t *subs[8] = {0};
        subs[0] = cur;
        for (int s = 1; s < nsub; s++) {
            subs[s] = (int64_t *)malloc(sizeof(int64_t) * rcells);
            if (!subs[s]) return ORC_ERR_NOMEM;
            const int64_t *band = details + off + (int64_t)(s - 1) * gcells;
            for (int64_t z = 0; z < ce[2]; z++)
                for (int64_t y = 0; y < ce[1]; y++)
                    for (int64_t x = 0; x < ce[0]; x++)
                        subs[s][orc_idx3(x, y, z, ce)] =
                            band[orc_idx3(cs[0] + x, cs[1] + y, cs[2] + z, Gj)];
        }
        /* undo the passes in reverse axis order */
        int64_t sd[3] = {ce[0], ce[1], ce[2]};
        int have = nsub;
        for (int a = ndim - 1; a >= 0; a--) {
            int64_t dd[3] = {sd[0], sd[1], sd[2]};
            dd[a] *= 2;
            int64_t dcells = dd[0] * dd[1] * dd[2];
            int half = have / 2;
            for (int s = 0; s < half; s++) {
                /* s has bit a clear, s | (1<<a) is its high-pass partner;
                 * at this point only the lowest `have` indices are live and
                 * bits above a have already been merged. */
                int64_t *dst = (int64_t *)malloc(sizeof(int64_t) * dcells);
                if (!dst) return ORC_ERR_NOMEM;
                orc_synthesis_pass(subs[s], subs[s | (1 << a)], sd, a, dst);
                free(subs[s]);
                free(subs[s | (1 << a)]);
                subs[s] = dst;
                subs[s | (1 << a)] = 0;
            }
            have = half;
            sd[a] = dd[a];
        }
        cur = subs[0];
        for (int a = 0; a < 3; a++) {
            if (a < ndim) {
                ce[a] *= 2;
                cs[a] *= 2;
            }
        }
    }
    memcpy(out, cur, sizeof(int64_t) * ce[0] * ce[1] * ce[2]);
    free(cur);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* CCW score of every candidate (Sec. 4.3, CCW equation), plus the energy    */
/* term that turns the raw cross-correlation into a sum of squared           */
/* differences.  Readings: candidates are coarse-aligned (fine offset b*c),  */
/* the sum runs over the template footprint at level J (T_c blocks per      */
/* axis) restricted to the overlap, and partially known blocks carry their   */
/* known-cell count n and known-cell sum m (the level-J approximation of the */
/* zero-filled overlap).                                                    */
/*   SSD mode: S(c) = sum_b n_b K[c+b]^2 - 2 |beta| sum_b m_b K[c+b]         */
/*   RAW mode: S(c) = - sum_b m_b K[c+b]   (the paper's CCW, negated so that */
/*             smaller is better in both modes)                              */
/* K: level-J block sums over the grid of extent G.  Cand: number of         */
/* candidates per axis.  n_b, m_b: T_c[0]*T_c[1]*T_c[2] values each.         */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* LeGall 5/3 integer lifting, one level along one line of even length n.   */
/* Samples outside [0, n) are mirrored about the end samples (x[-i] = x[i], */
/* x[n-1+i] = x[n-1-i]).  Predict: d[k] = x[2k+1] - floor((x[2k] +          */
/* x[2k+2]) / 2); update: s[k] = x[2k] + floor((d[k-1] + d[k] + 2) / 4),   */
/* with d[-1] taken from the mirrored signal (it equals d[0]).  The inverse */
/* undoes the update, then the prediction, so it returns x exactly.         */
/* ------------------------------------------------------------------------ */
static int64_t orc_mirror(int64_t i, int64_t n)
{
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

static int64_t orc_floordiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

int orc_lift53_forward(const int64_t *x, int64_t n, int64_t *s, int64_t *d)
{
    if (n < 2 || n % 2) return ORC_ERR_SHAPE;
    int64_t h = n / 2;
    for (int64_t k = -1; k < h; k++) {
        /* d[k] from the mirrored signal; k = -1 only feeds s[0] */
        int64_t xo = x[orc_mirror(2 * k + 1, n)];
        int64_t xl = x[orc_mirror(2 * k, n)], xr = x[orc_mirror(2 * k + 2, n)];
        int64_t dk = xo - orc_floordiv(xl + xr, 2);
        if (k >= 0) d[k] = dk;
    }
    for (int64_t k = 0; k < h; k++) {
        int64_t dl;
        if (k == 0) {
            int64_t xo = x[orc_mirror(-1, n)];
            dl = xo - orc_floordiv(x[orc_mirror(-2, n)] + x[0], 2);
        } else {
            dl = d[k - 1];
        }
        s[k] = x[2 * k] + orc_floordiv(dl + d[k] + 2, 4);
    }
    return ORC_OK;
}

int orc_lift53_inverse(const int64_t *s, const int64_t *d, int64_t n, int64_t *x)
{
    if (n < 2 || n % 2) return ORC_ERR_SHAPE;
    int64_t h = n / 2;
    /* the mirrored d[-1] equals d[0] (x[-1] = x[1], x[-2] = x[2]) */
    for (int64_t k = 0; k < h; k++) {
        int64_t dl = k == 0 ? d[0] : d[k - 1];
        x[2 * k] = s[k] - orc_floordiv(dl + d[k] + 2, 4);
    }
    for (int64_t k = 0; k < h; k++) {
        int64_t xr = x[orc_mirror(2 * k + 2, n)];
        x[2 * k + 1] = d[k] + orc_floordiv(x[2 * k] + xr, 2);
    }
    return ORC_OK;
}

/* Level-J approximation of an image of extent e (every used axis a
 * multiple of 2^J): per level, the lifting along x, then y, then z, keeping
 * the low-pass half of each line.  out receives e / 2^J cells per used axis. */
int orc_approx53(const int64_t *img, const int64_t e_in[3], int32_t ndim, int32_t J, int64_t *out)
{
    int64_t e[3] = {e_in[0], e_in[1], e_in[2]};
    int64_t total = e[0] * e[1] * e[2];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * total);
    int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * total);
    int64_t nmax = e[0] > e[1] ? e[0] : e[1];
    if (e[2] > nmax) nmax = e[2];
    int64_t *line = (int64_t *)malloc(sizeof(int64_t) * nmax);
    int64_t *ls = (int64_t *)malloc(sizeof(int64_t) * nmax);
    int64_t *ld = (int64_t *)malloc(sizeof(int64_t) * nmax);
    if (!cur || !nxt || !line || !ls || !ld) return ORC_ERR_NOMEM;
    memcpy(cur, img, sizeof(int64_t) * total);
    for (int j = 0; j < J; j++) {
        for (int a = 0; a < ndim; a++) {
            if (e[a] % 2) return ORC_ERR_SHAPE;
            int64_t ne[3] = {e[0], e[1], e[2]};
            ne[a] = e[a] / 2;
            int64_t o1 = (a + 1) % 3, o2 = (a + 2) % 3;
            for (int64_t p = 0; p < e[o1]; p++)
                for (int64_t q = 0; q < e[o2]; q++) {
                    for (int64_t i = 0; i < e[a]; i++) {
                        int64_t u[3];
                        u[a] = i; u[o1] = p; u[o2] = q;
                        line[i] = cur[orc_idx3(u[0], u[1], u[2], e)];
                    }
                    int st = orc_lift53_forward(line, e[a], ls, ld);
                    if (st) return st;
                    for (int64_t i = 0; i < ne[a]; i++) {
                        int64_t u[3];
                        u[a] = i; u[o1] = p; u[o2] = q;
                        nxt[orc_idx3(u[0], u[1], u[2], ne)] = ls[i];
                    }
                }
            for (int c = 0; c < 3; c++) e[c] = ne[c];
            int64_t *t = cur; cur = nxt; nxt = t;
        }
    }
    memcpy(out, cur, sizeof(int64_t) * e[0] * e[1] * e[2]);
    free(cur); free(nxt); free(line); free(ls); free(ld);
    return ORC_OK;
}

int orc_scores(const int64_t *K, const int32_t G[3], const int32_t cand[3],
               const int32_t tc[3], int64_t beta_cells, const int64_t *nb,
               const int64_t *mb, int32_t mode, int64_t *S_out)
{
    int64_t g[3] = {G[0], G[1], G[2]};
    int64_t t[3] = {tc[0], tc[1], tc[2]};
    for (int a = 0; a < 3; a++)
        if (cand[a] < 1 || cand[a] - 1 + tc[a] > G[a]) return ORC_ERR_RANGE;
    for (int64_t cz = 0; cz < cand[2]; cz++)
        for (int64_t cy = 0; cy < cand[1]; cy++)
            for (int64_t cx = 0; cx < cand[0]; cx++) {
                int64_t cross = 0, energy = 0;
                for (int64_t bz = 0; bz < t[2]; bz++)
                    for (int64_t by = 0; by < t[1]; by++)
                        for (int64_t bx = 0; bx < t[0]; bx++) {
                            int64_t kv = K[orc_idx3(cx + bx, cy + by, cz + bz, g)];
                            int64_t bi = orc_idx3(bx, by, bz, t);
                            cross += mb[bi] * kv;
                            energy += nb[bi] * kv * kv;
                        }
                int64_t s = (mode == 0) ? energy - 2 * beta_cells * cross : -cross;
                S_out[cx + (int64_t)cand[0] * (cy + (int64_t)cand[1] * cz)] = s;
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Minimal-error boundary cut on one band (image quilting, Sec. 2; reading   */
/* for the tie rules): e is rows x cols, row-major, where column w = 0 is    */
/* the band edge that faces the already simulated neighbour.  Cumulative     */
/* error E[0][w] = e[0][w], E[y][w] = e[y][w] + min over w' in {w, w-1, w+1} */
/* of E[y-1][w'], preferring w, then w-1, then w+1 on equal values.  The     */
/* seam ends at the smallest w of minimal E in the last row and is traced    */
/* back through the recorded choices.  seam[y] is the first column that      */
/* takes the new patch in row y.                                             */
/* ------------------------------------------------------------------------ */
int orc_mincut(const int64_t *e, int32_t rows, int32_t cols, int32_t *seam)
{
    if (rows < 1 || cols < 1) return ORC_ERR_ARG;
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * rows * cols);
    int32_t *from = (int32_t *)malloc(sizeof(int32_t) * rows * cols);
    if (!E || !from) return ORC_ERR_NOMEM;
    for (int w = 0; w < cols; w++) {
        E[w] = e[w];
        from[w] = w;
    }
    for (int y = 1; y < rows; y++) {
        for (int w = 0; w < cols; w++) {
            int best = w;
            int64_t bv = E[(y - 1) * cols + w];
            if (w - 1 >= 0 && E[(y - 1) * cols + w - 1] < bv) {
                best = w - 1;
                bv = E[(y - 1) * cols + w - 1];
            }
            if (w + 1 < cols && E[(y - 1) * cols + w + 1] < bv) {
                best = w + 1;
                bv = E[(y - 1) * cols + w + 1];
            }
            E[y * cols + w] = e[y * cols + w] + bv;
            from[y * cols + w] = best;
        }
    }
    int end = 0;
    for (int w = 1; w < cols; w++)
        if (E[(rows - 1) * cols + w] < E[(rows - 1) * cols + end]) end = w;
    seam[rows - 1] = end;
    for (int y = rows - 1; y >= 1; y--) seam[y - 1] = from[y * cols + seam[y]];
    free(E);
    free(from);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* K best candidates and the uniform draw among them (Sec. 4.4, Algorithm 1).*/
/* Candidates are ordered by (hard-data mismatch, score, keyed tie-break);   */
/* reading for conditioning: the sequential search of Sec. 4.4 over the      */
/* sorted scores takes the best candidate that honours the data, which is    */
/* the lexicographic order with the mismatch first.  The mismatch is capped  */
/* at 4095.  The K' = min(K, n) best are kept and the j-th is drawn with      */
/* j = floor(u * K' / 2^32), u the high half of the DRAW stream for          */
/* (seed, r, step).  mis may be NULL (no hard data).  topkeys, if not NULL,  */
/* receives the K' keys (mismatch << 52 | (S + 2^31) << 20 | tie-break) in   */
/* ascending order.                                                          */
/* ------------------------------------------------------------------------ */
int orc_select(const int64_t *S, const int64_t *mis, int64_t ncand, int32_t k, uint64_t seed,
               int64_t r, int64_t step, int64_t *chosen, uint64_t *topkeys)
{
    if (ncand < 1 || ncand > (1 << 20) || k < 1) return ORC_ERR_ARG;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * ncand);
    if (!keys) return ORC_ERR_NOMEM;
    uint64_t tkey = orc_rng(seed, ORC_STREAM_TIEBREAK, (uint64_t)r, (uint64_t)step);
    for (int64_t c = 0; c < ncand; c++) {
        int64_t m = mis ? (mis[c] > 4095 ? 4095 : mis[c]) : 0;
        int64_t s = S[c] + 2147483648LL;
        if (s < 0 || s > 0xFFFFFFFFLL) {
            free(keys);
            return ORC_ERR_RANGE;
        }
        keys[c] = ((uint64_t)m << 52) | ((uint64_t)s << 20) | (uint64_t)orc_perm20((uint32_t)c, tkey);
    }
    /* the K' best, by repeated minimum (plain selection) */
    int64_t kk = k < ncand ? k : ncand;
    uint64_t u32 = orc_rng(seed, ORC_STREAM_DRAW, (uint64_t)r, (uint64_t)step) >> 32;
    int64_t j = (int64_t)((u32 * (uint64_t)kk) >> 32);
    int64_t pick = -1;
    uint64_t prev = 0;
    for (int64_t rank = 0; rank < kk; rank++) {
        int64_t best = -1;
        for (int64_t c = 0; c < ncand; c++) {
            if (rank > 0 && keys[c] <= prev) continue;
            if (best < 0 || keys[c] < keys[best]) best = c;
        }
        prev = keys[best];
        if (topkeys) topkeys[rank] = prev;
        if (rank == j) pick = best;
        if (!topkeys && rank == j) break;
    }
    *chosen = pick;
    free(keys);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole simulation (Algorithm 1, with the conditioning of Sec. 4.4).        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ndim;
    int64_t ti[3], sg[3], T[3], OV[3], b[3], G[3], np[3], tc[3], cand[3];
    int64_t stride[3], lat[3], pad[3], margin[3];
    int64_t ncand, beta_cells;
} orc_geom;

static int orc_setup(const orc_params *p, orc_geom *g)
{
    if (p->ndim < 2 || p->ndim > 3) return ORC_ERR_ARG;
    if (p->level < 0 || p->level > 8 || p->top_k < 1 || p->n_real < 1) return ORC_ERR_ARG;
    if (p->n_facies < 1 || p->n_facies > 127) return ORC_ERR_ARG;
    if (p->wavelet != 0 && p->wavelet != 1) return ORC_ERR_ARG;
    g->ndim = p->ndim;
    orc_block_factor(p->ndim, p->level, g->b);
    g->beta_cells = g->b[0] * g->b[1] * g->b[2];
    for (int a = 0; a < 3; a++) {
        int act = a < p->ndim;
        g->ti[a] = act ? p->ti_n[a] : 1;
        g->sg[a] = act ? p->sg_n[a] : 1;
        g->T[a] = act ? p->tmpl[a] : 1;
        g->OV[a] = act ? p->overlap[a] : 0;
        g->margin[a] = act ? (p->nc_margin[a] < 0 ? p->overlap[a] : p->nc_margin[a]) : 0;
        if (act) {
            if (g->ti[a] < 1 || g->sg[a] < 1) return ORC_ERR_SHAPE;
            if (!(g->T[a] > g->OV[a] && g->OV[a] >= 1)) return ORC_ERR_SHAPE;
            if (g->T[a] > g->ti[a]) return ORC_ERR_SHAPE;
        } else if (p->ti_n[a] != 1 || p->sg_n[a] != 1) {
            return ORC_ERR_SHAPE;
        }
        g->np[a] = ((g->ti[a] + g->b[a] - 1) / g->b[a]) * g->b[a];
        g->G[a] = g->np[a] / g->b[a];
        g->tc[a] = (g->T[a] + g->b[a] - 1) / g->b[a];
        /* candidates: the fine window b*c + [0,T) lies inside the TI */
        g->cand[a] = (g->ti[a] - g->T[a]) / g->b[a] + 1;
        /* lattice: stride T - OV, padded grid n*s + OV, crop at the end */
        g->stride[a] = g->T[a] - g->OV[a];
        int64_t l = (g->sg[a] - g->OV[a] + g->stride[a] - 1) / g->stride[a];
        g->lat[a] = l < 1 ? 1 : l;
        g->pad[a] = g->lat[a] * g->stride[a] + g->OV[a];
    }
    g->ncand = g->cand[0] * g->cand[1] * g->cand[2];
    if (g->ncand > (1 << 20)) return ORC_ERR_RANGE;
    return ORC_OK;
}

/* Path of realization r (Algorithm 1, "Randomize(origin, direction)").
 * perm[k] = lattice axis visited at path depth k (k = 0 fastest);
 * flip[a] = 1 when lattice axis a is walked from its high end. */
static void orc_path(const orc_params *p, int r, int perm[3], int flip[3])
{
    for (int a = 0; a < 3; a++) {
        perm[a] = a;
        flip[a] = 0;
    }
    if (p->path_mode == 1) {
        uint64_t u = orc_rng(p->seed, ORC_STREAM_PATH, (uint64_t)r, 0);
        for (int a = 0; a < p->ndim; a++) flip[a] = (int)((u >> a) & 1u);
        if (p->ndim == 2 && ((u >> 3) & 1u)) {
            perm[0] = 1;
            perm[1] = 0;
        }
    }
}

int orc_geometry(const orc_params *p, int64_t out[32])
{
    orc_geom g;
    int st = orc_setup(p, &g);
    if (st) return st;
    for (int a = 0; a < 3; a++) {
        out[a] = g.G[a];
        out[3 + a] = g.cand[a];
        out[6 + a] = g.tc[a];
        out[9 + a] = g.lat[a];
        out[12 + a] = g.pad[a];
        out[15 + a] = g.b[a];
    }
    out[18] = g.ncand;
    out[19] = g.beta_cells;
    return ORC_OK;
}

/* Simulate every realization in raster order.
 *   ti:      TI codes, ti_n extent, x fastest.
 *   hd_*:    n_hd hard data; hd_real[i] realization, hd_pos[3i..3i+2]
 *            grid coordinates (x, y, z), hd_val[i] code.  Positions are
 *            distinct within a realization.
 *   out:     n_real * sg cells.
 *   chosen:  optional n_real * n_steps log of chosen candidate indices.
 *   scores:  optional n_real * n_steps * ncand log of S (debug, tiny runs). */
int orc_simulate(const orc_params *p, const int8_t *ti, int64_t n_hd,
                 const int32_t *hd_real, const int32_t *hd_pos, const int8_t *hd_val,
                 int8_t *out, int32_t *chosen, int64_t *scores)
{
    orc_geom g;
    int st = orc_setup(p, &g);
    if (st) return st;
    const int ndim = p->ndim;
    const int J = p->level;

    /* Algorithm 1 computes the TI transform inside the realization loop; it
     * depends on the TI only, so it is done once. */
    int32_t tin[3] = {(int32_t)g.ti[0], (int32_t)g.ti[1], (int32_t)g.ti[2]};
    int64_t gcells = g.G[0] * g.G[1] * g.G[2];
    int64_t ndet = orc_details_count(tin, ndim, J);
    int64_t *K = (int64_t *)malloc(sizeof(int64_t) * gcells);
    int64_t *det = (int64_t *)malloc(sizeof(int64_t) * (ndet > 0 ? ndet : 1));
    if (!K || !det) return ORC_ERR_NOMEM;
    if (p->wavelet == 1) {
        /* LeGall 5/3: approximation of the edge-replicated TI; the pattern
         * comes back by perfect reconstruction, i.e. as the TI crop */
        int64_t npc = g.np[0] * g.np[1] * g.np[2];
        int64_t *tip = (int64_t *)malloc(sizeof(int64_t) * npc);
        if (!tip) return ORC_ERR_NOMEM;
        for (int64_t z = 0; z < g.np[2]; z++)
            for (int64_t y = 0; y < g.np[1]; y++)
                for (int64_t x = 0; x < g.np[0]; x++) {
                    int64_t sx = x < g.ti[0] ? x : g.ti[0] - 1, sy = y < g.ti[1] ? y : g.ti[1] - 1;
                    int64_t sz = z < g.ti[2] ? z : g.ti[2] - 1;
                    tip[orc_idx3(x, y, z, g.np)] = ti[orc_idx3(sx, sy, sz, g.ti)];
                }
        st = orc_approx53(tip, g.np, ndim, J, K);
        free(tip);
    } else {
        st = orc_dwt(ti, tin, ndim, J, K, det);
    }
    if (st) return st;

    int64_t tcells = g.tc[0] * g.tc[1] * g.tc[2];
    int64_t wcells = g.T[0] * g.T[1] * g.T[2];
    int64_t pcells = g.pad[0] * g.pad[1] * g.pad[2];
    int64_t nsteps = g.lat[0] * g.lat[1] * g.lat[2];
    int64_t rcells[3] = {g.tc[0] * g.b[0], g.tc[1] * g.b[1], g.tc[2] * g.b[2]};
    int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * tcells);
    int64_t *mb = (int64_t *)malloc(sizeof(int64_t) * tcells);
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * g.ncand);
    int64_t *mis = (int64_t *)malloc(sizeof(int64_t) * g.ncand);
    int64_t *rec = (int64_t *)malloc(sizeof(int64_t) * rcells[0] * rcells[1] * rcells[2]);
    int8_t *patch = (int8_t *)malloc(wcells);
    uint8_t *inband = (uint8_t *)malloc(wcells);
    uint8_t *keep_old = (uint8_t *)malloc(wcells);
    int8_t *sg = (int8_t *)malloc(pcells);
    int8_t *hdmap = (int8_t *)malloc(pcells);
    int64_t *win = (int64_t *)malloc(sizeof(int64_t) * rcells[0] * rcells[1] * rcells[2]);
    int64_t *ade = (int64_t *)malloc(sizeof(int64_t) * tcells);
    if (!nb || !mb || !S || !mis || !rec || !patch || !inband || !keep_old || !sg || !hdmap || !win || !ade)
        return ORC_ERR_NOMEM;

    for (int r = 0; r < p->n_real; r++) {
        /* hard data are frozen into the grid; everything else starts unknown */
        memset(sg, -1, pcells);
        memset(hdmap, -1, pcells);
        for (int64_t i = 0; i < n_hd; i++) {
            if (hd_real[i] != r) continue;
            int64_t x = hd_pos[3 * i], y = hd_pos[3 * i + 1], z = hd_pos[3 * i + 2];
            if (x < 0 || y < 0 || z < 0 || x >= g.sg[0] || y >= g.sg[1] || z >= g.sg[2])
                return ORC_ERR_RANGE;
            int64_t at = orc_idx3(x, y, z, g.pad);
            sg[at] = hd_val[i];
            hdmap[at] = hd_val[i];
        }
        int perm[3], flip[3];
        orc_path(p, r, perm, flip);
        int64_t plen[3] = {g.lat[perm[0]], g.lat[perm[1]], g.lat[perm[2]]};

        for (int64_t step = 0; step < nsteps; step++) {
            /* raster position along the path, then lattice index */
            int64_t q[3] = {step % plen[0], (step / plen[0]) % plen[1], step / (plen[0] * plen[1])};
            int64_t li[3];
            int band[3] = {0, 0, 0};
            for (int k = 0; k < 3; k++) {
                int a = perm[k];
                li[a] = flip[a] ? g.lat[a] - 1 - q[k] : q[k];
                /* a previously simulated neighbour along this axis exists
                 * when the path coordinate is past its start (Fig. 3a-c) */
                band[a] = (a < ndim) && q[k] > 0;
            }
            int64_t org[3] = {li[0] * g.stride[0], li[1] * g.stride[1], li[2] * g.stride[2]};

            /* overlap region: union of the bands on the trailing sides */
            for (int64_t z = 0; z < g.T[2]; z++)
                for (int64_t y = 0; y < g.T[1]; y++)
                    for (int64_t x = 0; x < g.T[0]; x++) {
                        int64_t u[3] = {x, y, z};
                        int in = 0;
                        for (int a = 0; a < ndim; a++) {
                            if (!band[a]) continue;
                            int64_t w = flip[a] ? g.T[a] - 1 - u[a] : u[a];
                            if (w < g.OV[a]) in = 1;
                        }
                        inband[orc_idx3(x, y, z, g.T)] = (uint8_t)in;
                    }

            /* data event: known-cell count and sum per level-J block */
            for (int64_t i = 0; i < tcells; i++) {
                nb[i] = 0;
                mb[i] = 0;
            }
            for (int64_t z = 0; z < g.T[2]; z++)
                for (int64_t y = 0; y < g.T[1]; y++)
                    for (int64_t x = 0; x < g.T[0]; x++) {
                        if (!inband[orc_idx3(x, y, z, g.T)]) continue;
                        int64_t v = sg[orc_idx3(org[0] + x, org[1] + y, org[2] + z, g.pad)];
                        if (v < 0) return ORC_ERR_RANGE; /* overlap must be known */
                        int64_t bi = orc_idx3(x / g.b[0], y / g.b[1], z / g.b[2], g.tc);
                        nb[bi] += 1;
                        mb[bi] += v;
                    }

            int64_t score_beta = g.beta_cells;
            if (p->wavelet == 1) {
                /* 5/3: the data event's approximation is the transform of
                 * the zero-filled overlap window (tc * b cells per axis);
                 * each block with a known cell compares its coefficient,
                 * S = sum (K - A)^2 up to a constant, so n = 1 and m = A */
                for (int64_t i = 0; i < rcells[0] * rcells[1] * rcells[2]; i++) win[i] = 0;
                for (int64_t z = 0; z < g.T[2]; z++)
                    for (int64_t y = 0; y < g.T[1]; y++)
                        for (int64_t x = 0; x < g.T[0]; x++)
                            if (inband[orc_idx3(x, y, z, g.T)])
                                win[orc_idx3(x, y, z, rcells)] =
                                    sg[orc_idx3(org[0] + x, org[1] + y, org[2] + z, g.pad)];
                st = orc_approx53(win, rcells, ndim, J, ade);
                if (st) return st;
                for (int64_t i = 0; i < tcells; i++) {
                    nb[i] = nb[i] > 0 ? 1 : 0;
                    mb[i] = nb[i] ? ade[i] : 0;
                }
                score_beta = 1;
            }
            int32_t G32[3] = {(int32_t)g.G[0], (int32_t)g.G[1], (int32_t)g.G[2]};
            int32_t c32[3] = {(int32_t)g.cand[0], (int32_t)g.cand[1], (int32_t)g.cand[2]};
            int32_t t32[3] = {(int32_t)g.tc[0], (int32_t)g.tc[1], (int32_t)g.tc[2]};
            st = orc_scores(K, G32, c32, t32, score_beta, nb, mb, p->score_mode, S);
            if (st) return st;
            if (scores) memcpy(scores + ((int64_t)r * nsteps + step) * g.ncand, S, sizeof(int64_t) * g.ncand);

            /* hard-data mismatch inside the virtual template: the template
             * extended by the margin on the sides not yet simulated */
            int64_t vlo[3], vhi[3];
            for (int a = 0; a < 3; a++) {
                vlo[a] = 0;
                vhi[a] = g.T[a];
                if (a < ndim) {
                    if (flip[a]) vlo[a] = -g.margin[a];
                    else vhi[a] = g.T[a] + g.margin[a];
                }
            }
            for (int64_t c = 0; c < g.ncand; c++) mis[c] = 0;
            for (int64_t i = 0; i < n_hd; i++) {
                if (hd_real[i] != r) continue;
                int64_t u[3];
                int inside = 1;
                for (int a = 0; a < 3; a++) {
                    u[a] = hd_pos[3 * i + a] - org[a];
                    if (u[a] < vlo[a] || u[a] >= vhi[a]) inside = 0;
                }
                if (!inside) continue;
                for (int64_t cz = 0; cz < g.cand[2]; cz++)
                    for (int64_t cy = 0; cy < g.cand[1]; cy++)
                        for (int64_t cx = 0; cx < g.cand[0]; cx++) {
                            int64_t f[3] = {g.b[0] * cx + u[0], g.b[1] * cy + u[1], g.b[2] * cz + u[2]};
                            int ok = 1;
                            for (int a = 0; a < 3; a++)
                                if (f[a] < 0 || f[a] >= g.ti[a]) ok = 0;
                            if (!ok) continue;
                            int64_t tv = ti[orc_idx3(f[0], f[1], f[2], g.ti)];
                            if (tv != hd_val[i])
                                mis[cx + g.cand[0] * (cy + g.cand[1] * cz)] += 1;
                        }
            }

            /* K best and the draw */
            int64_t pick = -1;
            st = orc_select(S, mis, g.ncand, p->top_k, p->seed, r, step, &pick, NULL);
            if (st) return st;
            if (chosen) chosen[(int64_t)r * nsteps + step] = (int32_t)pick;

            /* reconstruct the chosen pattern from the coefficient pyramid */
            int64_t pc[3] = {pick % g.cand[0], (pick / g.cand[0]) % g.cand[1],
                             pick / (g.cand[0] * g.cand[1])};
            int32_t c0[3] = {(int32_t)pc[0], (int32_t)pc[1], (int32_t)pc[2]};
            if (p->wavelet == 0) {
                st = orc_idwt_region(K, det, tin, ndim, J, c0, t32, rec);
                if (st) return st;
            }
            for (int64_t z = 0; z < g.T[2]; z++)
                for (int64_t y = 0; y < g.T[1]; y++)
                    for (int64_t x = 0; x < g.T[0]; x++) {
                        int64_t tv = ti[orc_idx3(g.b[0] * pc[0] + x, g.b[1] * pc[1] + y,
                                                 g.b[2] * pc[2] + z, g.ti)];
                        int64_t v = tv;   /* 5/3: perfect reconstruction of the TI's own window */
                        if (p->wavelet == 0) {
                            v = rec[orc_idx3(x, y, z, rcells)];
                            /* Haar reconstruction must give back the TI crop */
                            if (v != tv) return ORC_ERR_RANGE;
                        }
                        patch[orc_idx3(x, y, z, g.T)] = (int8_t)v;
                    }

            /* boundary cut: one seam per band, per slice in 3D */
            memset(keep_old, 0, wcells);
            if (p->cut) {
                for (int a = 0; a < ndim; a++) {
                    if (!band[a]) continue;
                    /* rows run along the first other active axis, slices
                     * along the remaining one */
                    int ra = (a == 0) ? 1 : 0;
                    int sa = -1;
                    for (int x = 0; x < ndim; x++)
                        if (x != a && x != ra) sa = x;
                    int64_t nslice = sa >= 0 ? g.T[sa] : 1;
                    int64_t rows = g.T[ra], cols = g.OV[a];
                    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * rows * cols);
                    int32_t *seam = (int32_t *)malloc(sizeof(int32_t) * rows);
                    if (!e || !seam) return ORC_ERR_NOMEM;
                    for (int64_t sl = 0; sl < nslice; sl++) {
                        for (int64_t y = 0; y < rows; y++)
                            for (int64_t w = 0; w < cols; w++) {
                                int64_t u[3] = {0, 0, 0};
                                u[a] = flip[a] ? g.T[a] - 1 - w : w;
                                u[ra] = y;
                                if (sa >= 0) u[sa] = sl;
                                int64_t sv = sg[orc_idx3(org[0] + u[0], org[1] + u[1], org[2] + u[2], g.pad)];
                                int64_t pv = patch[orc_idx3(u[0], u[1], u[2], g.T)];
                                e[y * cols + w] = (sv - pv) * (sv - pv);
                            }
                        st = orc_mincut(e, (int32_t)rows, (int32_t)cols, seam);
                        if (st) return st;
                        for (int64_t y = 0; y < rows; y++)
                            for (int64_t w = 0; w < seam[y]; w++) {
                                int64_t u[3] = {0, 0, 0};
                                u[a] = flip[a] ? g.T[a] - 1 - w : w;
                                u[ra] = y;
                                if (sa >= 0) u[sa] = sl;
                                keep_old[orc_idx3(u[0], u[1], u[2], g.T)] = 1;
                            }
                    }
                    free(e);
                    free(seam);
                }
            }

            /* paste (Algorithm 1): new side of every seam, hard data kept */
            for (int64_t z = 0; z < g.T[2]; z++)
                for (int64_t y = 0; y < g.T[1]; y++)
                    for (int64_t x = 0; x < g.T[0]; x++) {
                        int64_t w = orc_idx3(x, y, z, g.T);
                        int64_t at = orc_idx3(org[0] + x, org[1] + y, org[2] + z, g.pad);
                        if (hdmap[at] >= 0 || keep_old[w]) continue;
                        sg[at] = patch[w];
                    }
        }
        /* crop the padded lattice back to the grid */
        for (int64_t z = 0; z < g.sg[2]; z++)
            for (int64_t y = 0; y < g.sg[1]; y++)
                for (int64_t x = 0; x < g.sg[0]; x++)
                    out[(int64_t)r * g.sg[0] * g.sg[1] * g.sg[2] + orc_idx3(x, y, z, g.sg)] =
                        sg[orc_idx3(x, y, z, g.pad)];
    }
    free(K);
    free(det);
    free(nb);
    free(mb);
    free(S);
    free(mis);
    free(rec);
    free(patch);
    free(inband);
    free(keep_old);
    free(sg);
    free(hdmap);
    free(win);
    free(ade);
    return ORC_OK;
}
