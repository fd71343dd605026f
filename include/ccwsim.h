/*
 * ccwsim.h -- C ABI of the CCWSIM hot path on AMD Instinct MI355X (gfx950).
 *
 * CCWSIM (Bavandsavadkoohi et al., arXiv 2404.00441) simulates a categorical
 * grid patch by patch along a raster path.  For every patch it
 *   1. takes the overlap with already simulated patches as a data event
 *      (Sec. 4.1, Fig. 3a-c),
 *   2. compares the data event's Haar approximation with every candidate
 *      position of the training image's approximation grid through the CCW
 *      cross-correlation (Sec. 4.3),
 *   3. keeps the K best candidates and draws one uniformly (Sec. 4.4,
 *      Algorithm 1),
 *   4. rebuilds the chosen pattern by inverse DWT from the stored detail
 *      coefficients (Sec. 3.1, Algorithm 1) and pastes it behind a
 *      minimal-error boundary cut (image quilting, Sec. 2 and Sec. 4.1).
 *
 * Conventions shared by every entry point
 *   - Extents and coordinates are (x, y, z) with x fastest in memory; a 2D
 *     problem has ndim = 2 and extent 1 (template 1, overlap 0) on z.
 *   - Codes are int8 facies indices 0 .. n_facies-1 (n_facies <= 127).
 *   - The Haar transform is kept in exact integer form: per axis and level
 *     the low-pass is e + o and the high-pass e - o (e, o = even and odd
 *     sample; the wavelet is +1 on its first half, Sec. 4.2).  The level-J
 *     approximation is therefore the integer block sum over 2^J cells per
 *     axis; orthonormal coefficients are these integers times 2^(-p/2) after
 *     p filter passes.  Images whose extent is not a multiple of 2^J are
 *     extended by edge replication first.
 *   - Unless stated otherwise every pointer is a DEVICE pointer owned by the
 *     caller; `stream` is a hipStream_t passed as void* (NULL = default
 *     stream).  Calls are asynchronous on `stream` and return a status; a
 *     fault inside a kernel shows up at the caller's next synchronisation.
 *   - Argument errors are reported before anything is launched.  The text of
 *     the last error on the calling thread is ccwsim_last_error().
 *   - Calls never abort or throw.  Calls on different streams must not share
 *     output buffers or workspaces.
 */
#ifndef CCWSIM_H
#define CCWSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CCWSIM_OK 0
#define CCWSIM_ERR_INVALID_ARG 1 /* null pointer, bad enum, bad count      */
#define CCWSIM_ERR_SHAPE 2       /* extents / template / overlap invalid   */
#define CCWSIM_ERR_WORKSPACE 3   /* workspace missing or too small         */
#define CCWSIM_ERR_HIP 4         /* a HIP runtime call failed              */
#define CCWSIM_ERR_UNSUPPORTED 5 /* valid input outside what is built      */

const char* ccwsim_status_string(int status);
/* Text of the last failure on the calling thread ("" if none). */
const char* ccwsim_last_error(void);

/* ---- shapes and parameters --------------------------------------------- */
typedef struct {
  int32_t ndim; /* 2 or 3                                            */
  int32_t n[3]; /* extent per axis, n[0] = x; n[2] = 1 when ndim = 2  */
} ccwsim_shape;

/* Problem statement of Algorithm 1 (TI, template size, overlap size, level
 * J, K, number of realizations) plus the choices the paper leaves open. */
typedef struct {
  ccwsim_shape ti;      /* training image extent                          */
  ccwsim_shape grid;    /* simulation grid extent (per realization)       */
  int32_t tmpl[3];      /* template T per axis (T > OV >= 1 on used axes) */
  int32_t overlap[3];   /* overlap OV per axis                            */
  int32_t level;        /* wavelet decomposition level J, 0 <= J <= 6     */
  int32_t top_k;        /* K best candidates kept for the draw, >= 1      */
  int32_t n_real;       /* realizations simulated together, >= 1          */
  int32_t n_facies;     /* codes are 0 .. n_facies-1, 1 <= n_facies <= 127*/
  uint64_t seed;        /* every random draw is a function of
                           (seed, realization, raster step)              */
  int32_t path_mode;    /* 0: raster from the low corner, x fastest;
                           1: per realization a seeded start corner (and,
                           in 2D, which axis is walked fastest)          */
  int32_t score_mode;   /* 0: squared difference of approximations
                           (CCW cross term + energy term, smaller = better);
                           1: negated raw CCW                             */
  int32_t nc_margin[3]; /* non-causal margin of the virtual template used
                           for hard data; < 0 means "= overlap"          */
  int32_t cut;          /* 1: minimal-error boundary cut; 0: plain paste  */
  int32_t precision;    /* bulk scan operands, fp32 accumulation:
                           0 fp16 (exact for block sums <= 2048),
                           1 bf16 (exact for block sums <= 256);
                           ccwsim_simulate refuses inexact combinations  */
  int32_t shortlist;    /* 0, or S in [top_k, 32]: the S best candidates by
                           the bulk score are rescored exactly in integers
                           and the K best of those are drawn from        */
  int32_t max_hard_data;/* most hard data a call passes (sizes the
                           workspace); 0 = unconditional only            */
  int32_t proposer_dim; /* 64: the learned convolutional proposer (see
                           ccwsim_lp_*): each patch's data event is encoded
                           (query encoder), the lp_probe inverted lists of
                           `proposer` whose centroids score best are
                           scored exactly (Sec. 4.3, in integers) and the
                           K best of those are drawn from, unless the gate
                           sends the patch to the full scan (empty overlap,
                           hard data in the virtual template, fewer than K
                           members, or a best match error above lp_gate).
                           Not identical to proposer_dim = 0 by design;
                           2D, score_mode 0, Haar, shortlist 0.
                           D in {8, 16, 32}: a certified proposer.  A
                           D-dimensional principal-component basis of the
                           candidates' level-J windows is fitted on the
                           device from the TI (every call); each patch's
                           data event is encoded against it, the scan then
                           bounds every candidate's score from below, and
                           the exact scores of whole candidate rows are
                           computed in order of their bound until the K
                           best are certified.  Results are identical to
                           proposer_dim = 0.  Needs score_mode 0 and
                           shortlist 0.                                   */
  int32_t hd_direct;    /* 0: the scan counts hard-data mismatches from a
                           bit table built once per call (for every TI
                           row, x phase below 2^J and code: one bit per
                           level-J x position, set where the TI cell
                           lies inside the TI and holds another code),
                           when that table takes at most 1 GiB, else as
                           1; 1: it reads the TI codes directly.  Both
                           give the same results.                         */
  int32_t wavelet;      /* mother wavelet of the search (Sec. 4.2 calls Haar
                           particularly suitable): 0 Haar (the default);
                           1 LeGall 5/3 in the integer lifting form of
                           Calderbank, Daubechies, Sweldens and Yeo (the
                           reversible filter of JPEG 2000), whole-sample
                           symmetric extension, x then y then z per level.
                           With 5/3 a candidate's score is the squared
                           difference between the TI's level-J
                           approximation at its blocks and that of the
                           zero-filled overlap window, over the blocks
                           holding a known cell (n = 1, m = the window's
                           coefficient), and the pattern is rebuilt by
                           perfect reconstruction, i.e. as the TI window.
                           Needs shortlist 0 and proposer_dim 0.          */
  int32_t lp_probe;     /* proposer_dim = 64: inverted lists probed per
                           data event, 1 .. 64                            */
  float lp_gate;        /* proposer_dim = 64: largest best match error a
                           proposal may have (below: the full scan
                           decides); < 0 sends every patch to the scan   */
  const void* proposer; /* proposer_dim = 64: device index from
                           ccwsim_lp_build_index for this TI, level and
                           template (NULL otherwise)                      */
} ccwsim_params;

/* ---- A1: training-image transform (Sec. 3.1 DWT; Sec. 4.2 the mother
 * wavelet; Algorithm 1, DWT of TI) ---
 * Level-J DWT of x (int8, extent s) with wavelet 0 (Haar, in the integer
 * form above) or 1 (LeGall 5/3 integer lifting: per line d[k] = x[2k+1] -
 * floor((x[2k] + x[2k+2]) / 2), s[k] = x[2k] + floor((d[k-1] + d[k] + 2) / 4),
 * whole-sample symmetric extension, x then y then z per level).  The image
 * is extended by edge replication to Np = ceil(n / 2^J) * 2^J per used axis.
 *   approx:  level-J approximation, G = Np / 2^J cells per used axis, int32
 *            (for Haar the integer block sums).
 *   details: for j = 1..J, for sub-band q = 1 .. 2^ndim - 1 (bit a of q set
 *            when axis a took the high-pass), Np / 2^j cells per used axis,
 *            int32; levels concatenated in increasing j.
 *   workspace: device memory of workspace_bytes (ccwsim_dwt_sizes), 256-byte
 *            aligned, owned by the caller (may be NULL when 0 bytes).
 * ccwsim_dwt_sizes returns the element counts of both outputs and the
 * workspace bytes (host call, no device work).  Returns CCWSIM_ERR_SHAPE for
 * bad extents or J > 6, CCWSIM_ERR_INVALID_ARG for another wavelet. */
int ccwsim_dwt_sizes(ccwsim_shape s, int32_t level, int32_t wavelet, int64_t* n_approx, int64_t* n_details,
                     int64_t* workspace_bytes);
int ccwsim_dwt(const int8_t* x, ccwsim_shape s, int32_t level, int32_t wavelet, int32_t* approx, int32_t* details,
               void* workspace, int64_t workspace_bytes, void* stream);

/* ---- A3/A4 (+A6): CCW scan (Sec. 4.3, CCW equation; Sec. 4.4 K best) ----
 * Scores every candidate of the TI approximation grid against n_filters
 * data events.  Candidates are coarse-aligned: candidate c = (cx, cy, cz)
 * has its fine window at 2^J * c, fully inside the TI, so there are
 * C_a = (n_a - T_a) / 2^J + 1 candidates per axis, index cx + C_x*(cy + C_y*cz).
 * A data event is given per level-J block of the template footprint
 * (T_c = ceil(T / 2^J) blocks per axis, x fastest): or_n = number of known
 * overlap cells in the block, or_m = sum of their codes (the level-J
 * approximation of the zero-filled overlap), int32 [n_filters][T_c cells].
 *   score_mode 0: S = sum n K^2 - 2^s sum m K   (s = 1 + J * ndim for Haar,
 *                 s = 1 for LeGall 5/3, whose n is 0 or 1)
 *   score_mode 1: S = - sum m K
 * with K = approx[c + beta], the level-J approximation from ccwsim_dwt with
 * the same wavelet (0 Haar, 1 LeGall 5/3).  Two outputs, either or both:
 *   scores:    int32 [n_filters][C cells], the whole score map, or NULL;
 *   topk_keys: uint64 [n_filters][K'] ascending, K' = min(top_k, C cells),
 *              or NULL: the K best candidates of each filter under the key
 *              (S + 2^31, pi(index)) of ccwsim_select (pi keyed by seed,
 *              realization[f], step[f]; int32 / int64 [n_filters] device
 *              arrays).  The selection is fused into the scan: per candidate
 *              row only the candidates that can be among the row's K best
 *              keys are kept, and the score map is never written.
 *              1 <= top_k <= 16.
 * precision: 0 fp16, 1 bf16 MFMA operands (fp32 accumulation).  The call
 * returns CCWSIM_ERR_UNSUPPORTED if the values could leave the range in
 * which that arithmetic is exact (the bound uses max_code, the largest code
 * in the TI; 0 < max_code <= 126).
 * workspace: device memory of at least ccwsim_ccf_scan_workspace_size(...)
 * bytes (the same arguments; want_scores / want_keys say which outputs will
 * be non-NULL), 256-byte aligned, owned by the caller; nothing is allocated.
 * ccwsim_ccf_scan_workspace_size is a host call and returns -1 on invalid
 * arguments (text in ccwsim_last_error). */
int64_t ccwsim_ccf_scan_workspace_size(ccwsim_shape ti, int32_t level, int32_t wavelet, int32_t max_code,
                                       int32_t precision, const int32_t tmpl[3], int32_t n_filters,
                                       int32_t score_mode, int32_t top_k, int32_t want_scores, int32_t want_keys);
int ccwsim_ccf_scan(ccwsim_shape ti, int32_t level, int32_t wavelet, int32_t max_code, int32_t precision,
                    const int32_t* approx, const int32_t tmpl[3], const int32_t* or_n, const int32_t* or_m,
                    int32_t n_filters, int32_t score_mode, int32_t* scores, int32_t top_k, uint64_t seed,
                    const int32_t* realization, const int64_t* step, uint64_t* topk_keys, void* workspace,
                    int64_t workspace_bytes, void* stream);

/* ---- CDF 9/7 wavelet in floating point (Sec. 4.2: the mother wavelet is a
 * choice; Sec. 4.3 scores over the approximation) ----
 * The Cohen-Daubechies-Feauveau 9/7 biorthogonal wavelet in the lifting
 * factorisation of Daubechies and Sweldens: per line of even length,
 * d += alpha (s + s'), s += beta (d' + d), d += gamma (s + s'),
 * s += delta (d' + d) on the even (s) and odd (d) samples (primes are the
 * right / left neighbours), then s *= zeta, d /= zeta, with alpha =
 * -1.586134342059924, beta = -0.052980118572961, gamma = 0.882911075530934,
 * delta = 0.443506852043971, zeta = 1.149604398860241 (low-pass gain sqrt 2
 * at DC); whole-sample symmetric extension; x then y then z per level; the
 * TI edge-replicated to Np = ceil(n / 2^J) * 2^J per used axis.  fp32
 * arithmetic throughout.
 *   ccwsim_dwt97: approx float32 [G cells] and details float32 in the layout
 *     of ccwsim_dwt (counts from ccwsim_dwt_sizes with any wavelet).
 *   ccwsim_idwt97: the inverse, image float32 [Np cells] (the edge-replicated
 *     TI, up to rounding).
 *   workspace: ccwsim_dwt97_workspace_size bytes (-1 on a bad shape),
 *     256-byte aligned, caller-owned.
 * ccwsim_ccf_scan97 scores every candidate (coarse-aligned as for
 * ccwsim_ccf_scan) against n_filters data events, each a known-block mask
 * or_n (int32 0/1 [n_filters][T_c cells]: the blocks holding a known cell)
 * and the event's own level-J approximation or_m (float32, same shape; read
 * where or_n is 1):  S(c) = sum over blocks b with or_n = 1 of
 * (approx[c + b] - or_m[b])^2, evaluated in fp32 in block order (x fastest).
 *   scores:    float32 [n_filters][C cells], the whole map, or NULL.
 *   topk_keys: uint64 [n_filters][top_k] ascending, or NULL: key =
 *              (bits of the fp32 S) << 20 | pi(index), pi keyed by seed,
 *              realization[f], step[f] as in ccwsim_select; 1 <= top_k <= 16,
 *              top_k <= C cells.
 *   shortlist: 0 or R >= C cells: every candidate's fp32 S decides the keys.
 *              top_k <= R < C cells (R <= 128): precision split.  A bulk pass
 *              ranks every candidate by sum n (A K - K^2 / 2) with MFMA
 *              operands in fp16 (precision 0; K^2 scaled by a power of two
 *              fitting the largest |approx|, values clamped to the fp16
 *              range) or bf16 (precision 1), fp32 accumulation; the R
 *              candidates with the largest bulk value (ties to the smaller
 *              index) are rescored in fp32 and the keys come from them.
 *   shortlist_out: int32 [n_filters][R] ascending candidate indices of the
 *              shortlist, or NULL (only with a shortlist smaller than C).
 * The fp32 S of a candidate is the same value in the map and in its key.
 * workspace: ccwsim_ccf_scan97_workspace_size(...) bytes (want_scores /
 * want_keys say which outputs will be non-NULL), 256-byte aligned,
 * caller-owned; -1 on invalid arguments.  T_c cells <= 256; a template of
 * more than about 240 block rows of one block (too tall for the map's LDS
 * strip) is refused with CCWSIM_ERR_UNSUPPORTED. */
int64_t ccwsim_dwt97_workspace_size(ccwsim_shape s, int32_t level);
int ccwsim_dwt97(const int8_t* x, ccwsim_shape s, int32_t level, float* approx, float* details, void* workspace,
                 int64_t workspace_bytes, void* stream);
int ccwsim_idwt97(const float* approx, const float* details, ccwsim_shape ti, int32_t level, float* image,
                  void* workspace, int64_t workspace_bytes, void* stream);
int64_t ccwsim_ccf_scan97_workspace_size(ccwsim_shape ti, int32_t level, int32_t precision, const int32_t tmpl[3],
                                         int32_t n_filters, int32_t top_k, int32_t shortlist, int32_t want_scores,
                                         int32_t want_keys);
int ccwsim_ccf_scan97(ccwsim_shape ti, int32_t level, int32_t precision, const float* approx, const int32_t tmpl[3],
                      const int32_t* or_n, const float* or_m, int32_t n_filters, float* scores, int32_t top_k,
                      int32_t shortlist, uint64_t seed, const int32_t* realization, const int64_t* step,
                      uint64_t* topk_keys, int32_t* shortlist_out, void* workspace, int64_t workspace_bytes,
                      void* stream);

/* ---- the scan without a workspace -----------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).
 * ccwsim_ccf_scan_noalloc computes exactly what ccwsim_ccf_scan computes
 * (same arguments, same outputs, which the caller still owns) but keeps its
 * temporaries in a static device array of ccwsim_ccf_scan_noalloc_capacity()
 * bytes (64 MiB) that every device the library runs on holds from module
 * load until the process ends; it calls no allocator and records no
 * profiler events.  A call whose temporaries (the value
 * ccwsim_ccf_scan_workspace_size returns for the same arguments) exceed the
 * array returns CCWSIM_ERR_UNSUPPORTED before launching anything.  All calls
 * on one device share that device's array: calls that overlap in time on
 * one device (different streams or host threads) race and must not be
 * issued; nothing in the array needs clearing between calls. */
int64_t ccwsim_ccf_scan_noalloc_capacity(void);
int ccwsim_ccf_scan_noalloc(ccwsim_shape ti, int32_t level, int32_t wavelet, int32_t max_code, int32_t precision,
                            const int32_t* approx, const int32_t tmpl[3], const int32_t* or_n, const int32_t* or_m,
                            int32_t n_filters, int32_t score_mode, int32_t* scores, int32_t top_k, uint64_t seed,
                            const int32_t* realization, const int64_t* step, uint64_t* topk_keys, void* stream);

/* ---- A9 learned proposer: encoders and training (Sec. 4.3: the search
 * runs on the approximation coefficients; Sec. 4.4: the K best are drawn
 * from) ----
 * Two convolutional encoders over level-J approximation coefficients rank
 * candidate positions for a data event; the exact CCW score of a shortlist
 * then decides.  Key encoder: input K / |beta| (one channel, the TI's
 * approximation grid); query encoder: input m / |beta| and n / |beta| over
 * the event's T_c blocks (two channels, zero off the overlap).  Events
 * come as for ccwsim_ccf_scan: or_n / or_m int32 [batch][T_c cells].  Each: 3x3 convolutions with dilations 1, 2, 4
 * and 32 channels (ReLU), then a 1x1 convolution to 64 channels.  The key
 * of candidate c is the key map at c + T_c / 2; the query is the query map
 * at T_c / 2; the proposer's score is their dot product.  2D TIs only.
 * Weights: one float32 buffer of n_weights values (key encoder layers 0..3,
 * then the query encoder's; per layer weights [cout][cin][taps] then
 * biases).
 *   ccwsim_lp_sizes:  weights count, workspace bytes for `batch` events and
 *                     the candidate count (host call, no device work);
 *   ccwsim_lp_init:   He-uniform weights from the seed (biases zero);
 *   ccwsim_lp_encode: keys float32 [n_cand][64], queries [batch][64] and
 *                     scores [batch][n_cand] (each may be NULL);
 *   ccwsim_lp_train_step: one Adam step (lr, beta 0.9 / 0.999, eps 1e-8,
 *                     step >= 1 counts the updates) on the mean over the
 *                     batch of the cross-entropy between the softmax of the
 *                     scores over every candidate and the labels, int32
 *                     [batch][n_pos] distinct candidate indices (1 <= n_pos
 *                     <= 32; the best exact scores), loss = -log of the
 *                     softmax mass on them; writes the per-example loss
 *                     (float32 [batch]) and, when grad_out is not NULL, the
 *                     gradient before the update;
 *   ccwsim_lp_shortlist: the k (<= 256) highest scores' candidate indices
 *                     per row of scores (ties to the smaller index), in
 *                     ascending index order;
 *   ccwsim_lp_labels: the same for exact int32 scores (Sec. 4.3 S), the k
 *                     smallest: the training labels.
 * Every pointer is a device pointer owned by the caller; workspaces are
 * 256-byte aligned. */
int ccwsim_lp_sizes(ccwsim_shape ti, int32_t level, const int32_t tmpl[3], int32_t batch, int64_t* n_weights,
                    int64_t* workspace_bytes, int64_t* n_cand);
int ccwsim_lp_init(float* weights, uint64_t seed, void* stream);
int ccwsim_lp_encode(const float* weights, const int32_t* approx, ccwsim_shape ti, int32_t level, const int32_t tmpl[3],
                     const int32_t* or_n, const int32_t* or_m, int32_t batch, float* keys_out, float* queries_out,
                     float* scores_out, void* workspace, int64_t workspace_bytes, void* stream);
int ccwsim_lp_train_step(float* weights, float* adam_m, float* adam_v, int32_t step, float lr, const int32_t* approx,
                         ccwsim_shape ti, int32_t level, const int32_t tmpl[3], const int32_t* or_n,
                         const int32_t* or_m, const int32_t* labels, int32_t n_pos, int32_t batch, float* loss,
                         float* grad_out, void* workspace, int64_t workspace_bytes, void* stream);
int ccwsim_lp_shortlist(const float* scores, int32_t batch, int64_t n_cand, int32_t k, int32_t* idx_out, void* stream);
int ccwsim_lp_labels(const int32_t* scores, int32_t batch, int64_t n_cand, int32_t k, int32_t* idx_out, void* stream);

/* Inverted lists of the keys and the proposal (Sec. 4.3 exact score of a
 * shortlist, Sec. 4.4 K best of it).
 *   ccwsim_lp_index_size: bytes of an index with n_lists lists (1 .. 1024)
 *     and of the workspace that builds it (host call);
 *   ccwsim_lp_build_index: keys of every candidate from the key encoder,
 *     then `iters` rounds of Lloyd's k-means (squared distance; starting
 *     centroids at evenly spaced candidates; a list's centroid is the mean
 *     of its members, an empty list keeps its centroid), each candidate in
 *     the list of its nearest centroid.  The index (device memory of
 *     index_bytes, 256-byte aligned, owned by the caller) holds a header
 *     with the geometry, the query encoder's weights, the centroids and the
 *     lists; ccwsim_simulate takes it as `proposer`;
 *   ccwsim_lp_propose: for each data event (or_n / or_m as for
 *     ccwsim_ccf_scan), the query (the query encoder's output at the
 *     window's centre block), the `probe` lists whose centroids have the
 *     largest inner product with it (ties to the smaller list), and their
 *     members in that order, up to 1792 (the first list alone may be cut),
 *     each scored exactly in integers, S = sum n K^2 - 2 |beta| sum m K.
 *     Outputs: topk_keys uint64 [n_filters][top_k] the min(top_k, n_cand)
 *     best keys (S + 2^31, pi(index)) of ccwsim_select (all ones when fewer
 *     members were scored); members int32 [n_filters][1792] and n_members
 *     int32 [n_filters], queries float32 [n_filters][64] and best_error
 *     float32 [n_filters] (the best key's match error, see
 *     ccwsim_simulate_match_errors; -1 when fewer than top_k members),
 *     each may be NULL.  The index must match ti, level and tmpl
 *     (CCWSIM_ERR_INVALID_ARG otherwise; the header is read back, which
 *     synchronises `stream`).  workspace: ccwsim_lp_propose_workspace_size
 *     bytes, 256-byte aligned. */
int ccwsim_lp_index_size(ccwsim_shape ti, int32_t level, const int32_t tmpl[3], int32_t n_lists, int64_t* index_bytes,
                         int64_t* workspace_bytes);
int ccwsim_lp_build_index(const float* weights, const int32_t* approx, ccwsim_shape ti, int32_t level,
                          const int32_t tmpl[3], int32_t n_lists, int32_t iters, void* index, int64_t index_bytes,
                          void* workspace, int64_t workspace_bytes, void* stream);
int64_t ccwsim_lp_propose_workspace_size(ccwsim_shape ti, int32_t level, int32_t max_code, const int32_t tmpl[3]);
int ccwsim_lp_propose(const void* index, const int32_t* approx, ccwsim_shape ti, int32_t level, int32_t max_code,
                      const int32_t tmpl[3], const int32_t* or_n, const int32_t* or_m, int32_t n_filters,
                      int32_t probe, int32_t top_k, uint64_t seed, const int32_t* realization, const int64_t* step,
                      uint64_t* topk_keys, int32_t* members, int32_t* n_members, float* queries, float* best_error,
                      void* workspace, int64_t workspace_bytes, void* stream);

/* ---- A6: top-K and draw (Sec. 4.4; Algorithm 1, K best and random draw) ---
 * For each filter f, candidates are ordered by the key
 *   (min(mismatch, 4095), S + 2^31, pi(index))
 * where pi is a keyed bijection of the 20-bit index (ties between equal
 * scores are broken by a seeded order, not by position).  The K' = min(K,
 * n_cand) smallest are kept and the j-th is chosen with
 * j = floor(u * K' / 2^32), u the high 32 bits of the draw for (seed,
 * realization[f], step[f]).
 *   scores:   int32 [n_filters][n_cand]
 *   mismatch: uint16 [n_filters][n_cand] hard-data mismatch counts, or NULL
 *   realization, step: int32 / int64 [n_filters] (device)
 *   chosen:   int32 [n_filters] chosen candidate index
 *   topk_keys: uint64 [n_filters][K'] ascending keys, or NULL
 * 1 <= top_k <= 16, 1 <= n_cand <= 2^20. */
int ccwsim_select(const int32_t* scores, const uint16_t* mismatch, int64_t n_cand,
                  int32_t n_filters, int32_t top_k, uint64_t seed, const int32_t* realization,
                  const int64_t* step, int32_t* chosen, uint64_t* topk_keys, void* stream);

/* ---- A7: inverse DWT of chosen patterns (Sec. 3.1; Algorithm 1 Inv-DWT) ---
 * Rebuilds n patterns of extent `patch` (fine cells, <= 64 x 64 x 64 and
 * <= 16384 cells) whose level-J block origins are block_origins (int32
 * [n][3], x y z) from the approx/details layout of ccwsim_dwt (same
 * wavelet) of a TI of extent ti.  patches: int8 [n][patch cells].  The block
 * range [origin, origin + ceil(patch / 2^J)) must lie inside the
 * approximation grid; a pattern whose origin does not is filled with -1.
 * Haar rebuilds each pattern from its own blocks' coefficients and needs no
 * workspace; LeGall 5/3 (whose synthesis filters reach across blocks)
 * inverts the whole image into the workspace (ccwsim_idwt_workspace_size
 * bytes, 256-byte aligned, caller-owned) and crops the patterns from it. */
int64_t ccwsim_idwt_workspace_size(ccwsim_shape ti, int32_t level, int32_t wavelet);
int ccwsim_idwt(const int32_t* approx, const int32_t* details, ccwsim_shape ti, int32_t level, int32_t wavelet,
                const int32_t* block_origins, int32_t n, const int32_t patch[3], int8_t* patches, void* workspace,
                int64_t workspace_bytes, void* stream);

/* ---- whole hot path (Algorithm 1 and the conditioning of Sec. 4.4) --------
 * Simulates p->n_real realizations of p->grid from the TI (device int8).
 * Hard data (may be n_hd = 0 and NULL pointers): hd_real int32 [n_hd]
 * realization index, hd_pos int32 [n_hd][3] grid coordinates (x, y, z),
 * hd_val int8 [n_hd] code.  Hard-data cells are never overwritten; entries
 * outside the grid or with a realization outside [0, n_real) are ignored;
 * positions must be distinct within a realization.
 *   out:    int8 [n_real][grid cells]
 *   chosen: int32 [n_real][lattice patches] chosen candidate per raster
 *           step, or NULL
 *   workspace: device memory of at least ccwsim_simulate_workspace_size(p)
 *           bytes, 256-byte aligned, owned by the caller; its contents on
 *           entry do not matter.
 * The result does not depend on how patches are scheduled: patches whose
 * windows do not overlap run concurrently (anti-diagonal wavefronts when
 * T >= 2 OV on every axis), and every draw is keyed by the raster step. */
int64_t ccwsim_simulate_workspace_size(const ccwsim_params* p);
int ccwsim_simulate(const ccwsim_params* p, const int8_t* ti, int64_t n_hd, const int32_t* hd_real,
                    const int32_t* hd_pos, const int8_t* hd_val, int8_t* out, int32_t* chosen,
                    void* workspace, int64_t workspace_bytes, void* stream);

/* Host-side caches.  A plan (the schedule and the tables of one parameter
 * set, the seed included) is built on the first call that names its
 * parameters; at most 16 plans are kept, the least recently used dropped
 * first together with the graphs captured on it.  ccwsim_release_caches
 * frees every plan, graph and the in-memory tuning table (not thread-safe
 * with concurrent ccwsim_simulate calls); ccwsim_cache_counts reports how
 * many plans and graphs are held (host call, no device work). */
void ccwsim_release_caches(void);
int ccwsim_cache_counts(int64_t* plans, int64_t* graphs);

/* ---- measurement --------------------------------------------------------
 * Work of one ccwsim_simulate call as the method defines it (not counting
 * padding the kernels add): patches = (realization, patch) pairs, or_blocks =
 * sum over patches of the level-J blocks holding known overlap cells,
 * scan_flops = 2 * or_blocks * candidates (one multiply-add per block and
 * candidate, Sec. 4.3).  Host call, no device work (it builds or reuses the
 * plan, which needs no device either; so does
 * ccwsim_simulate_workspace_size). */
typedef struct {
  int64_t patches;
  int64_t wavefront_steps;
  int64_t candidates;      /* per patch */
  int64_t or_blocks;
  double scan_flops;
  double key_bytes;        /* candidate keys written by the scan and read by the selection */
  double cells;            /* simulated grid cells, all realizations */
  double fin_bytes;        /* bytes the per-patch finalize step must move, summed over patches:
                              grid and hard-data windows (2 T^d), the row minima (8 per candidate
                              row), the keys of the k best rows, the pattern's coefficients
                              (4 T^d), the pasted window (T^d) and the successor data event it
                              completes (its overlap cells plus 2 bytes per block) */
} ccwsim_plan_stats;
int ccwsim_simulate_stats(const ccwsim_params* p, ccwsim_plan_stats* out);

/* Report of the last ccwsim_simulate call on this workspace (synchronises
 * `stream`), int64 out[8].  Shortlist rescoring: out[0] largest |bulk score -
 * exact score|, out[1] candidates rescored, out[2] patches whose K best
 * changed after rescoring, out[3] patches rescored (all zero without a
 * shortlist).  Proposer: out[4] patches selected through it; out[5]
 * candidate rows (dimensions 8 to 32) or candidates (64) whose exact keys
 * were computed for them; out[6] patches the learned proposer's gate sent
 * to the full scan; out[7] 0 (zero without a proposer). */
int ccwsim_simulate_report(const ccwsim_params* p, const void* workspace, int64_t workspace_bytes,
                           int64_t* out, void* stream);

/* After a ccwsim_simulate call on this workspace, stream-ordered (Sec. 4.3:
 * the data event of each patch; Sec. 4.4: the choice among the K best):
 *   ccwsim_simulate_events: every patch's data event in the scan's input
 *     form, or_n / or_m int32 [patches][T_c cells] (zero on blocks outside
 *     the overlap; all zero for a first patch), and, where not NULL, its
 *     realization int32 [patches] and raster step int32 [patches];
 *   ccwsim_simulate_match_errors: float32 [patches], the match error of the
 *     drawn candidate, (S + sum |beta|^2 m^2 / n) / (|beta|^2 sum n) for
 *     score_mode 0: the squared difference between the level-J
 *     approximations of the TI window and of the overlap, in orthonormal
 *     coefficients, per known cell (|beta| = 1 for LeGall 5/3); -1 where the
 *     overlap is empty or score_mode is 1.
 * Patches are in the order of the plan (ccwsim_simulate_stats counts
 * them); the buffers are device memory owned by the caller. */
int ccwsim_simulate_events(const ccwsim_params* p, const void* workspace, int64_t workspace_bytes, int32_t* or_n,
                           int32_t* or_m, int32_t* realization, int32_t* step, void* stream);
int ccwsim_simulate_match_errors(const ccwsim_params* p, const void* workspace, int64_t workspace_bytes, float* out,
                                 void* stream);

/* Kernel kinds timed by the profiler. */
#define CCWSIM_KIND_DWT 0
#define CCWSIM_KIND_ENERGY 1
#define CCWSIM_KIND_INIT 2
#define CCWSIM_KIND_PREPARE 3
#define CCWSIM_KIND_SCAN 4
#define CCWSIM_KIND_FINALIZE 5
#define CCWSIM_KIND_CROP 6
#define CCWSIM_KIND_LEARN 7   /* the proposer's fit (principal components, embeddings) */
#define CCWSIM_NUM_KINDS 8
/* When enabled, ccwsim_simulate times its kernels with pairs of hipEvents on
 * the caller's stream: the per-step scan and finalize launches carry start
 * and stop events recorded by their own dispatch (the kernel's run time);
 * the other launches are bracketed by event records.  ccwsim_profile_read
 * synchronises those
 * events, writes per-kind total milliseconds and launch counts (arrays of
 * CCWSIM_NUM_KINDS) and clears the record.  Host calls; the events add a
 * little launch overhead, so time throughput with profiling disabled. */
int ccwsim_profile_enable(int on);
int ccwsim_profile_read(double* ms, int64_t* launches);

/* ccwsim_simulate captures its launch sequence into a HIP graph the first
 * time it sees a (parameters, buffers) combination and replays the graph on
 * later calls (up to 64 graphs are kept, least recently used dropped first; the profiler
 * bypasses them).
 * ccwsim_set_graphs(0) switches to plain launches and drops the graphs. */
int ccwsim_set_graphs(int on);

/* Scan variant.  The scan has two output layouts: candidate-major (each
 * lane holds one patch against 16 candidates; up to 1, 2, 4 or 8 tiles of
 * 32 patches of one orientation share a workgroup and its gather of the
 * TI approximation) and filter-major (each lane holds one candidate
 * against 16 patches, so energy reads and key stores are contiguous; one
 * tile per workgroup).  0 (the default) lets the library choose: on the
 * first call of a parameter set it runs the call eagerly, times the widest
 * step's scan for every variant and keeps the fastest for that scan shape
 * (in memory, and in the JSON object of the file named by the environment
 * variable CCWSIM_TUNE_FILE if set; ccwsim_release_caches forgets the
 * in-memory table).  1, 2, 4 or 8 force the candidate-major layout with
 * that many tiles (within what the LDS allows), -1 the filter-major one
 * (for tests; results do not depend on the variant).  Drops captured
 * graphs.  Returns CCWSIM_ERR_INVALID_ARG for other values. */
int ccwsim_set_scan_group(int g);

/* Selection of the K best candidates (Sec. 4.4).  Stored keys: the scan
 * writes every candidate's key and the row minimum of every candidate row;
 * the finalize step reads the keys of the K rows with the smallest minima.
 * Row minima: the scan writes only the row minima and the finalize step
 * recomputes the exact keys of rows in order of their minima until the K
 * best are certified (at most K rows); the scan then stores 8 bytes per
 * candidate row instead of per candidate.  Both give the same results.  The
 * row minima need score_mode 0, no shortlist and at most 512 candidate rows
 * (else the stored keys are used).  Fused (3): the scan keeps, per
 * candidate row, only the candidates that can be among the row's K best
 * keys (a threshold from minima over disjoint groups of the row's
 * candidates bounds the K-th best from above) and writes their keys, their
 * count and the row minimum; the finalize step reads the survivors of the K
 * rows with the smallest minima.  It needs at most 4096 candidates per row,
 * the hard-data bit table when there are hard data, and no proposer.
 * 0 (the default) lets the tuner of ccwsim_set_scan_group choose on the
 * first call of a parameter set (the fused selection is tried first and is
 * used before tuning); 1, 2 and 3 force stored keys, row minima or the fused
 * selection (for tests).  Drops captured graphs.
 * Returns CCWSIM_ERR_INVALID_ARG for other values. */
int ccwsim_set_selection(int mode);

/* Test hook of the certified proposer (proposer_dim 8 to 32): s > 0 skews
 * the fitted basis (row 0 scaled by 1 + s and added s times to every other
 * row), so that it is neither orthogonal nor normalised; its bounds, and so
 * the results, must not change.  0 (the default) turns it off; s in [0, 4].
 * Drops captured graphs. */
int ccwsim_set_proposer_skew(float s);

/* ---- A17/A18: realization statistics (Sec. 5.2 Fig. 7b ensemble map;
 * Sec. 5.3 Fig. 9 variograms and probability of connection; Sec. 5.8
 * Fig. 16b facies proportions) ----
 * The paper compares realizations with the TI through these statistics
 * without writing them out; the entry points return the integer counts of
 * their textbook forms, from which the ratios follow on the host:
 *   proportion of f in image i   = per_image[i][f] / cells
 *   ensemble map of f            = per_cell[f][c] / n_img
 *   indicator variogram          = diff[i][f][h-1] / (2 N(h)),
 *       N(h) = cells whose neighbour h cells further along `axis` exists
 *   probability of connection    = connected[i][f][h-1] / both[i][f][h-1]
 * codes: int8 DEVICE stack of n_img (<= 65535) images, [image][z][y][x] with x
 * fastest, extent `shape` (ndim 2 or 3, at most 2^31 - 1 cells per image);
 * codes outside 0 .. n_facies-1 belong to no facies.  axis: 0 = x (the
 * paper's east-west), 1 = y (north-south), 2 = z.  Lags h = 1 .. max_lag
 * cells, 1 <= max_lag <= min(n[axis] - 1, 4096).  Outputs are DEVICE
 * arrays owned by the caller and fully overwritten.  n_img = 0 returns
 * CCWSIM_OK without touching anything.  Errors: CCWSIM_ERR_SHAPE,
 * CCWSIM_ERR_INVALID_ARG (counts, axis, lags, null pointers),
 * CCWSIM_ERR_WORKSPACE (missing, too small or not 256-byte aligned),
 * CCWSIM_ERR_UNSUPPORTED (images above 2^31 - 1 cells). */

/* Workspace bytes of ccwsim_stats_variogram / _connectivity for n_img
 * images of this extent (-1 on a bad shape). */
int64_t ccwsim_stats_workspace_size(ccwsim_shape shape, int32_t n_img);

/* per_image int64 [n_img][n_facies]: cells of image i holding f.
 * per_cell int32 [n_facies][cells] (may be NULL): images holding f at each
 * cell.  No workspace. */
int ccwsim_stats_histogram(const int8_t* codes, ccwsim_shape shape, int32_t n_img, int32_t n_facies,
                           int64_t* per_image, int32_t* per_cell, void* stream);

/* diff int64 [n_img][n_facies][max_lag]: pairs of cells (x, x + h e_axis)
 * inside the image whose indicators [code == f] differ. */
int ccwsim_stats_variogram(const int8_t* codes, ccwsim_shape shape, int32_t n_img, int32_t n_facies,
                           int32_t axis, int32_t max_lag, int64_t* diff, void* workspace,
                           int64_t workspace_bytes, void* stream);

/* both, connected int64 [n_img][n_facies][max_lag]: pairs at lag h along
 * `axis` whose two cells hold f, and those of them whose cells lie in one
 * connected component of f, cells being connected through shared faces (4
 * neighbours in 2D, 6 in 3D). */
int ccwsim_stats_connectivity(const int8_t* codes, ccwsim_shape shape, int32_t n_img, int32_t n_facies,
                              int32_t axis, int32_t max_lag, int64_t* both, int64_t* connected,
                              void* workspace, int64_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CCWSIM_H */
