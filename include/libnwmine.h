/*
 * libnwmine -- comparable-corpus mining hot path on one AMD Instinct MI355X
 * (gfx950): score every source x target sentence pair of a batch of document
 * pairs, align each pair's two sentence sequences with Needleman-Wunsch, keep
 * the aligned pairs whose similarity reaches the threshold, and differentiate
 * the alignment score for tuning.
 *
 * Method: Wolk & Marasek, "Unsupervised comparable corpora preparation and
 * exploration for bi-lingual translation equivalents", arXiv 1512.01641.
 *   Sec. 4    similarity = a classifier's likelihood in [0,1] (SVM distance
 *             through a sigmoid) over a dictionary with translation
 *             probabilities; sequence aligner maximising the summed pair
 *             similarity; pairs below the threshold are excluded.
 *   Sec. 5    one session over many document pairs, multi-threaded.
 *   Sec. 5.1  Needleman-Wunsch: similarity matrix, gap penalty, DP matrix
 *             with (0,0) = 0, first row/column initialised, every cell from
 *             its top, left and top-left neighbours (Figs. 1-2, eq. (1)); the
 *             GPU computes each anti-diagonal in parallel.
 *   Sec. 5.2  threshold and penalty are tuned against reference alignments.
 *
 * Conventions for every entry point
 *   - Pointers marked "device" are HIP device (or managed) memory on the
 *     context's device; "host" pointers are read before the call returns.
 *     The caller owns every buffer; the library keeps no pointer to caller
 *     memory after a call returns.
 *   - Host-visible arguments are validated synchronously.  On success the
 *     work is enqueued on `stream` (a hipStream_t, NULL = the null stream)
 *     and the call returns NWM_OK; outputs are valid once the stream has
 *     reached that point.  Kernel launch failures return NWM_EDEVICE.
 *   - No entry point allocates device memory except nwm_plan_create.
 *   - A context (and the plans made from it) must be used by one host thread
 *     at a time.  Calls that overlap on one stream are ordered by it.
 *   - Token ids outside [0, V) and non-finite similarities are not checked
 *     (undefined results).
 */
#ifndef LIBNWMINE_H
#define LIBNWMINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NWM_OK = 0,
  NWM_EINVAL = 1,       /* NULL required pointer, negative size, non-finite gap/threshold */
  NWM_ESHAPE = 2,       /* arguments disagree with each other or with the plan */
  NWM_ENOMEM = 3,       /* allocation failed (plan creation only) */
  NWM_EDEVICE = 4,      /* a HIP call or kernel launch failed */
  NWM_EUNSUPPORTED = 5  /* a documented size limit is exceeded */
} nwm_status;

/* Operand type of the similarity contraction.  The DP always runs in FP32. */
typedef enum { NWM_FP32 = 0, NWM_BF16 = 1 } nwm_prec;

typedef struct nwm_ctx nwm_ctx;
typedef struct nwm_plan nwm_plan;

/* Bilingual dictionary D (Sec. 4: a dictionary with translation
 * probabilities): V x V sparse, CSR.  Row t lists target words u with
 * probability d = D[t][u].  Device arrays; max_deg is a host-known upper bound
 * on the entries of any row. */
typedef struct {
  int32_t V;
  int32_t max_deg;
  const int32_t *row_off;  /* device [V+1] */
  const int32_t *col;      /* device [row_off[V]], values in [0, V) */
  const float *val;        /* device [row_off[V]] */
} nwm_dict;

/* Logistic scorer over the features (S_raw, rho):
 *   z = w0 * S_raw + w1 * rho + b,   S = 1 / (1 + exp(-z))
 * (Sec. 4: a classifier distance mapped into [0,1] by a sigmoid). */
typedef struct {
  float w0, w1, b;
} nwm_scorer;

/* A batch of B document pairs.  Pair b has n_b source and m_b target
 * sentences.  Sentences of all pairs are concatenated in pair order (pair b
 * owns source sentences [sum_{c<b} n_c, sum_{c<=b} n_c), likewise targets);
 * each sentence is a bag of token ids given as a CSR over tokens. */
typedef struct {
  int32_t B;                 /* number of document pairs, >= 0 */
  int32_t V;                 /* hashed vocabulary size of both languages */
  const int32_t *n_host;     /* host [B] source sentence counts, >= 0 */
  const int32_t *m_host;     /* host [B] target sentence counts, >= 0 */
  int64_t src_tokens;        /* host: src_off[sum n], total source tokens */
  int64_t tgt_tokens;        /* host: tgt_off[sum m], total target tokens */
  int32_t max_sent_tokens;   /* host: upper bound on the tokens of any source sentence */
  const int64_t *src_off;    /* device [sum n + 1] token offsets, src_off[0] = 0 */
  const int32_t *src_tok;    /* device [src_tokens] token ids in [0, V) */
  const int64_t *tgt_off;    /* device [sum m + 1] */
  const int32_t *tgt_tok;    /* device [tgt_tokens] */
} nwm_batch;

/* Buffer sizes a plan needs (all chosen by nwm_plan_create). */
typedef struct {
  size_t S_elems;    /* floats in S, S_raw and grad_S: sum_b n_b * m_b */
  size_t kept_cap;   /* (i, j) pair capacity of `kept`: sum_b min(n_b, m_b) */
  size_t tb_bytes;   /* bytes of the opaque traceback buffer */
  size_t ws_bytes;   /* bytes of the workspace */
} nwm_sizes;

/* --- context -------------------------------------------------------------- */

/* Create a context bound to HIP device `hip_device`.  Fails with NWM_EDEVICE
 * if the device is absent or not gfx950. */
nwm_status nwm_create(nwm_ctx **ctx, int hip_device);
/* Destroy a context.  Plans made from it may be destroyed before or after. */
void nwm_destroy(nwm_ctx *ctx);
const char *nwm_strerror(nwm_status s);
/* Name of the HIP error behind the last NWM_EDEVICE an entry point returned
 * on the calling thread ("none" if there was none).  Entry points clear an
 * error left by an earlier, unrelated HIP call before they launch, so the
 * error named here is the library's own.  The string is static. */
const char *nwm_last_device_error(void);

/* --- plan ----------------------------------------------------------------- */

/* Plan a batch (host-only work plus one small upload): per-pair offsets of S,
 * kept pairs and traceback, the tile lists of the contraction and the
 * longest-first order of the DP, and the workspace layout.  Uses only the
 * batch's host fields and `max_deg`; the device pointers of `batch` may be
 * NULL here.  Limits (NWM_EUNSUPPORTED): V <= 32768, max_deg <= 64,
 * m_b <= 2^22, max_sent_tokens * max_deg <= 1024.
 * Allocates one small device buffer of per-pair metadata owned by the plan. */
nwm_status nwm_plan_create(nwm_ctx *ctx, const nwm_batch *batch, int32_t max_deg,
                           nwm_prec prec, nwm_plan **plan);
nwm_status nwm_plan_sizes(const nwm_plan *plan, nwm_sizes *sizes);
void nwm_plan_destroy(nwm_plan *plan);

/* --- hot path --------------------------------------------------------------- */

/* Similarity of every sentence pair of every document pair (Sec. 4).
 *   S_raw[i][j] = (1/l_i) * sum_u T[i][u] * Y[j][u],  T = (count of each token
 *     of source sentence i) . D,  Y[j][u] = [u occurs in target sentence j]
 *     (l_i = tokens of source sentence i; S_raw = 0 when l_i = 0);
 *   rho[i][j]   = min(l_i, l'_j) / max(l_i, l'_j)  (1 when both are 0);
 *   S = sigmoid(w0 * S_raw + w1 * rho + b).
 * The contraction runs on MFMA with `prec` operands and FP32 accumulation.
 * Outputs (device, FP32, row-major n_b x m_b blocks, pair b at element
 * offset sum_{c<b} n_c m_c): S [S_elems]; S_raw [S_elems] or NULL.
 * ws: device workspace of ws_bytes, contents need not persist. */
nwm_status nwm_score_pairs(nwm_plan *plan, const nwm_batch *batch, const nwm_dict *dict,
                           nwm_scorer scorer, float *S, float *S_raw, void *ws, void *stream);

/* Needleman-Wunsch global alignment of every pair (Sec. 5.1) and the
 * threshold filter (Sec. 4).  For pair b, with H[0][0] = 0,
 * H[i][0] = fl32(i*gap), H[0][j] = fl32(j*gap) and for i, j >= 1
 *   up = H[i-1][j] + gap, left = H[i][j-1] + gap, diag = H[i-1][j-1] + S[i-1][j-1]
 *   H[i][j] = first maximum of (up, left, diag) in that order (FP32, compare
 *   with '>', so exact ties resolve UP > LEFT > DIAG).
 * The traceback from (n, m) yields the aligned (DIAG) pairs.
 *   S       device [S_elems] similarity, layout as nwm_score_pairs;
 *   gap     signed additive gap score (e.g. -0.2), finite;
 *   threshold  pairs with S >= threshold are kept, finite;
 *   score   device [B] H[n_b][m_b];
 *   n_diag  device [B] number of aligned pairs k_b (the gap count is n+m-2k);
 *   kept    device int32 [2 * kept_cap]: pair b's kept (i, j) pairs, 0-based,
 *           ascending, start at pair index sum_{c<b} min(n_c, m_c);
 *   n_kept  device [B];
 *   tb      device [tb_bytes] opaque traceback (direction bits + path), read
 *           by nwm_align_backward;
 *   ws      device [ws_bytes].
 * The strips of a tall pair run on different waves that hand rows to each
 * other; a wave that waits longer than its poll limit (NWM_PARAM_DP_SPIN_LIMIT)
 * gives up.  The call still returns NWM_OK (it does not wait for the
 * kernels); the failed pairs get score NaN, n_diag 0 and n_kept 0, and
 * nwm_align_check reports the failure. */
nwm_status nwm_align_batch(nwm_plan *plan, const float *S, float gap, float threshold,
                           float *score, int32_t *n_diag, int32_t *kept, int32_t *n_kept,
                           void *tb, void *ws, void *stream);

/* Status of the last nwm_align_batch or nwm_mine that ran on workspace `ws`
 * with this plan: waits for `stream` (synchronous), then returns NWM_EDEVICE
 * if a DP wave gave up waiting for the strip above it (the pairs concerned
 * have a NaN score and no aligned or kept pairs), else NWM_OK.  `failed`
 * (host, nullable) receives 1 or 0 likewise.  NWM_EINVAL for a NULL plan or
 * (B > 0) a NULL ws. */
nwm_status nwm_align_check(const nwm_plan *plan, const void *ws, int32_t *failed, void *stream);

/* nwm_align_batch for callers that cannot allocate device memory or pass a
 * workspace: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, outputs and layouts as
 * nwm_align_batch, without `ws`; it calls no allocating routine.  Its
 * scratch (the DP's queue heads and error flag, the boundary rows handed
 * between the strips of a pair) is a fixed
 * device array of the library, 32 MiB on every GPU the library runs on, held
 * until the process ends and reached through its device address, taken once
 * per device by nwm_create.  A plan needs 256 + 8 * (published-row slots +
 * 2) bytes of it, where a pair of n_b x m_b sentences publishes
 * (ceil(n_b / 64) - 1) rows of about m_b + 194 slots; larger plans return
 * NWM_EUNSUPPORTED (a batch of 4096 pairs of median 60 sentences needs about
 * 17 MiB).  Every call on a GPU shares that GPU's array and leaves its
 * contents behind; the call clears what must start at zero itself, by a
 * kernel.  Calls that overlap on one GPU (two streams, two threads, two
 * plans) race on the array and must be ordered by the caller.  A DP wave that
 * gives up waiting shows only as a NaN score of its pair (nwm_align_check
 * reads a workspace and does not apply). */
nwm_status nwm_align_batch_noalloc(nwm_plan *plan, const float *S, float gap, float threshold,
                                   float *score, int32_t *n_diag, int32_t *kept, int32_t *n_kept,
                                   void *tb, void *stream);

/* Backward of L = sum_b grad_score[b] * Score_b + sum_ij grad_S_extra[ij] * S[ij]
 * through the alignment and the logistic scorer, for gradient tuning of the
 * scorer and the gap penalty (Sec. 5.2 tunes threshold and penalty against
 * reference alignments).  The NW score (Sec. 5.1) is a maximum of affine path
 * sums, so dScore_b/dS = P_b (indicator of the aligned cells of the traced
 * path) and dScore_b/dgap = n_b + m_b - 2 k_b, exact where the optimal path is
 * unique; the chain through the sigmoid (Sec. 4) uses dS/dz = S (1 - S).
 *   tb, n_diag   from nwm_align_batch on the same plan (read only when
 *                grad_score is given; path cells outside a pair are skipped);
 *   grad_score   device [B] dL/dScore_b (FP32), or NULL: no score term (the
 *                path is not read, grad_gap is 0);
 *   grad_S_extra device [S_elems] or NULL: extra dense dL/dS;
 *   grad_S       device [S_elems] or NULL: receives dL/dS (FP32);
 *   grad_gap     device double [1] or NULL: dL/dgap;
 *   S, S_raw     device [S_elems] from nwm_score_pairs (needed if grad_wb);
 *   grad_wb      device double [3] or NULL: dL/d(w0, w1, b).
 * Per-pair partial sums are FP32; the batch reduction is FP64 in a fixed
 * order, so results are run-to-run deterministic. */
nwm_status nwm_align_backward(nwm_plan *plan, const nwm_batch *batch, const void *tb,
                              const int32_t *n_diag, const float *grad_score,
                              const float *grad_S_extra, float *grad_S, double *grad_gap,
                              const float *S, const float *S_raw, nwm_scorer scorer,
                              double *grad_wb, void *ws, void *stream);

/* Score then align (nwm_score_pairs followed by nwm_align_batch, same
 * arguments and layouts) in one call.  With graphs enabled on the plan
 * (nwm_plan_set_graph), the first call for a given set of arguments captures
 * the plan's kernels into a HIP graph on a stream of the library's own and
 * every later call with the same arguments replays the whole path with one
 * graph launch on `stream` (Sec. 5: one session over many document pairs).
 * Changing any argument recaptures.  Per-kernel timing is not recorded for
 * graph replays. */
nwm_status nwm_mine(nwm_plan *plan, const nwm_batch *batch, const nwm_dict *dict, nwm_scorer scorer, float gap,
                    float threshold, float *S, float *S_raw, float *score, int32_t *n_diag, int32_t *kept,
                    int32_t *n_kept, void *tb, void *ws, void *stream);
nwm_status nwm_plan_set_graph(nwm_plan *plan, int on);

/* --- bi-directional mining ----------------------------------------------------- */

/* Union of the aligned pairs two mining directions keep (Sec. 5.4, Table 3
 * "BI": a second classifier trained in the reverse direction adds pairs the
 * first misses).  `plan` is the forward plan.  The reverse direction is a
 * plan of the same document pairs with the roles swapped (target sentences
 * as the source side, a target-to-source dictionary); both have the same
 * kept-pair offsets, p_off[b] = sum over c < b of min(n_c, m_c).
 *   kept_fwd    [kept_cap][2] int32, device: (i, j) of the forward plan's
 *               nwm_align_batch; n_kept_fwd [B] its counts.
 *   kept_rev    [kept_cap][2] int32, device: the reverse plan's kept pairs,
 *               as that plan reports them: (target index, source index);
 *               n_kept_rev [B].
 *   kept_out    [2 kept_cap][2] int32, device, caller-owned: pair b's union
 *               at 2 p_off[b], as (i, j) = (source, target) in ascending
 *               order, each sentence pair once; n_out [B] its size
 *               (<= 2 min(n_b, m_b)).
 * Both inputs must be strictly increasing in i and in j per pair, as
 * nwm_align_batch writes them (other inputs give an unspecified but
 * in-bounds result).  Asynchronous on `stream`.  NWM_EINVAL for null
 * pointers the sizes need. */
nwm_status nwm_union_kept(const nwm_plan *plan, const int32_t *kept_fwd, const int32_t *n_kept_fwd,
                          const int32_t *kept_rev, const int32_t *n_kept_rev, int32_t *kept_out, int32_t *n_out,
                          void *stream);

/* --- launch parameters (for the autotuner) ------------------------------------ */

/* Launch shapes that do not change any result, only the time (all but
 * SCORE_COMPACT):
 *   NWM_PARAM_FILL_WAVES_PER_CU   persistent DP waves per compute unit
 *                                 (0 = as many as fit; default 0; the LDS-ring
 *                                 fill runs whole workgroups of four waves)
 *   NWM_PARAM_MERGE_WAVES_PER_CU  dictionary-merge waves per compute unit
 *                                 (0 = as many as the LDS allows; default 0)
 *   NWM_PARAM_SCORE_XCD_MAP       1 = contraction tiles of one pair on one XCD
 *                                 (shared L2), 0 = dispatch order; default 1
 *   NWM_PARAM_DP_HOT_PERCENT      DP strips of pairs whose dependency chain is
 *                                 at least this percent of the longest one run
 *                                 at raised wave priority (0 = never; default 50)
 *   NWM_PARAM_SCORE_COMPACT       1 = the contraction of each 64 x 64 tile runs
 *                                 over the words of its 64 target sentences
 *                                 only (the other words have a zero Y factor);
 *                                 0 = over the whole vocabulary.  Default 1.
 *                                 The FP32 sums are taken in another order, so
 *                                 S may differ in the last bits.
 *   NWM_PARAM_DP_SPIN_LIMIT       polls of the row above before a DP wave gives
 *                                 up (0 = the default, 2^22; at most 2^30)
 *   NWM_PARAM_DP_TEST_HOLD        testing only: 1 = the first strip of every
 *                                 pair taller than one strip publishes nothing,
 *                                 so the strips below it give up (exercises the
 *                                 failure report of nwm_align_check); default 0
 *   NWM_PARAM_SCORE_KGROUP        K width of one round of the compacted
 *                                 contraction: 1 = one 32-word chunk per round,
 *                                 2 = two chunks (64 words) scattered before one
 *                                 barrier; the same sums in the same order, so
 *                                 the results are identical.  Default 1.
 *   NWM_PARAM_FILL_STAGING        how the NW fill stages S: 0 = a two-group LDS
 *                                 ring per wave filled by LDS-direct loads (64
 *                                 rows x 64 steps per group), four waves per
 *                                 workgroup sweeping four strips, consecutive
 *                                 strips of a pair handing their boundary row
 *                                 on through LDS; 2 = the same ring, one strip
 *                                 per workgroup (every hand-off through
 *                                 memory); 1 = 16 cells per lane in registers,
 *                                 two 16-step chunks ahead (no LDS: more waves
 *                                 per compute unit).  The same cells in the
 *                                 same order: identical results.  Default 0.
 *   NWM_PARAM_EXPAND_FUSED        1 = the source-side merge and row-tile list
 *                                 build run as one kernel per row tile (merged
 *                                 rows stay on chip), for plans whose
 *                                 sentences have at most 48 tokens and whose
 *                                 dictionary rows at most 4 entries (other
 *                                 plans take the two-kernel path); 0 = always
 *                                 the two kernels.  Default 1.  The fused path
 *                                 keeps list entries the two-kernel path
 *                                 drops (words outside the pair's target
 *                                 vocabulary, which no tile's contraction
 *                                 reads): identical results.
 * Out-of-range values give NWM_EINVAL.  Setting DP_HOT_PERCENT uploads the
 * plan's work list (synchronous).  A graph captured by nwm_mine is captured
 * again after any change. */
typedef enum {
  NWM_PARAM_FILL_WAVES_PER_CU = 0,
  NWM_PARAM_MERGE_WAVES_PER_CU = 1,
  NWM_PARAM_SCORE_XCD_MAP = 2,
  NWM_PARAM_DP_HOT_PERCENT = 3,
  NWM_PARAM_SCORE_COMPACT = 4,
  NWM_PARAM_DP_SPIN_LIMIT = 5,
  NWM_PARAM_DP_TEST_HOLD = 6,
  NWM_PARAM_SCORE_KGROUP = 7,
  NWM_PARAM_FILL_STAGING = 8,
  NWM_PARAM_EXPAND_FUSED = 9,
  NWM_N_PARAMS = 10
} nwm_param;
nwm_status nwm_plan_set_param(nwm_plan *plan, nwm_param param, int32_t value);
nwm_status nwm_plan_get_param(const nwm_plan *plan, nwm_param param, int32_t *value);

/* --- measurement ------------------------------------------------------------ */

/* Kernel classes of the per-kernel timing. */
typedef enum {
  NWM_K_MERGE = 0,     /* merged dictionary rows of the source sentences */
  NWM_K_BUILD_A = 1,   /* source-side (row-tile) operand lists */
  NWM_K_BUILD_B = 2,   /* target-side (column-tile) operand lists and vocabularies */
  NWM_K_SCORE = 3,     /* contraction + logistic scorer */
  NWM_K_FILL = 4,      /* NW fill (with the reset of its hand-off rows) */
  NWM_K_WALK = 5,      /* traceback */
  NWM_K_KEEP = 6,      /* threshold filter */
  NWM_K_BACKWARD = 7,  /* nwm_align_backward */
  NWM_K_EXPAND_A = 8,  /* fused merge + row-tile lists (NWM_PARAM_EXPAND_FUSED) */
  NWM_N_KCLASSES = 9
} nwm_kclass;

/* Record HIP events around every kernel the plan launches (0 = off).  While
 * on, nwm_mine runs its kernels one at a time on the caller's stream (the
 * target-side lists on a second stream, as in nwm_score_pairs), and
 * nwm_plan_kernel_ms returns the summed device time per kernel class
 * (nwm_kclass) of all launches since the last reset, each measured on the
 * stream that launched it.  `counts` (nullable) receives launches per class.
 * Reading waits for the events. */
nwm_status nwm_plan_set_timing(nwm_plan *plan, int on);
nwm_status nwm_plan_kernel_ms(nwm_plan *plan, double ms[NWM_N_KCLASSES], int32_t counts[NWM_N_KCLASSES],
                              int reset);

#ifdef __cplusplus
}
#endif
#endif /* LIBNWMINE_H */
