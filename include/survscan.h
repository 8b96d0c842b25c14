/*
 * survscan -- Cox and Fine-Gray coordinate gradient / Hessian by fused
 * single-pass scans, for AMD Instinct MI355X (gfx950).
 *
 * Method: Yang, Schuemie, Ji & Suchard, "Massive Parallelization of
 * Massive Sample-size Survival Analysis" (arXiv 2204.08183).  With the
 * subjects arranged by decreasing observed time the risk-set sums of the
 * Cox log partial likelihood become prefix sums and the Fine-Gray ones a
 * prefix plus a weighted suffix sum (Sec. 2.7, eqs. cox_g, cox_h, fg_g,
 * fg_h); one coordinate's g' and g'' are a scan, an element-wise transform
 * and a reduction, fused into one pass over the data (Sec. 2.7, Fig. 2),
 * inside cyclic coordinate descent (Sec. 2.4, Fig. 3).
 *
 * Conventions for every entry point
 *  - All array pointers are DEVICE pointers (hipMalloc'd or torch CUDA
 *    tensors) unless the comment says [host].  The caller owns every buffer;
 *    the library never allocates or frees device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call is asynchronous on that stream, launches kernels only (no
 *    host synchronisation, no memset nodes) and may be captured in a
 *    hipGraph.  Outputs are valid once the stream has synchronised.
 *  - Arguments are checked on the host before any launch; an invalid call
 *    returns a negative status and launches nothing.  No C++ exception
 *    crosses this interface.  NaN or Inf in the data propagate into the
 *    outputs (they are not checked on the hot path).
 *  - "Sorted order" is the order of decreasing observed time produced by
 *    ss_prepare: position k holds subject perm[k]; equal times keep
 *    increasing original index.
 *  - Sizes: 1 <= n < 2^31, 1 <= p < 2^31, 0 <= nnz < 2^31.
 *  - Alignment: e, w_comp and g_end must be 16-byte aligned and d8 8-byte
 *    aligned (any torch CUDA allocation is); the fused kernels read them
 *    with vector loads.  A misaligned pointer is rejected with SS_EINVAL.
 *  - A workspace `ws` belongs to one stream at a time: two calls that use
 *    the same workspace must not run concurrently.
 */
#ifndef SURVSCAN_H
#define SURVSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status */
#define SS_OK            0
#define SS_EINVAL       (-1)   /* null pointer, bad size, index out of range */
#define SS_EWORKSPACE   (-2)   /* workspace too small or misaligned          */
#define SS_EUNSUPPORTED (-3)   /* unknown model / penalty                    */
#define SS_EDEVICE      (-4)   /* a HIP runtime call failed                  */

/* ------------------------------------------------------------ enums */
#define SS_COX        0        /* Sec. 2.1: events are status != 0          */
#define SS_FINE_GRAY  1        /* Sec. 2.2: events are status == 1,
                                  competing events status == 2             */

#define SS_PENALTY_NONE 0
#define SS_PENALTY_L1   1      /* pi = -gamma |beta_j|        (Sec. 2.3)   */
#define SS_PENALTY_L2   2      /* pi = -beta_j^2 / (2 tau)    (Sec. 2.3)   */

/* accumulation of the FP32-storage path (ss_grad_hess_mixed) */
#define SS_ACC_F32       0     /* plain FP32 sums                          */
#define SS_ACC_F32_COMP  1     /* compensated FP32: hi + lo by two-sum     */
#define SS_ACC_F64       2     /* FP64 sums of the FP32 inputs             */
#define SS_ACC_F32_C64   3     /* FP32 inside a tile, FP64 carry between
                                  tiles and FP64 sum of the tile partials  */

/* Granularity (in sorted positions) of the per-column chunk index built by
 * ss_prepare; tiles of the fused kernels are whole multiples of it. */
#define SS_CHUNK 1024

/* Human-readable text for a status code (static storage, never NULL).  For
 * SS_EDEVICE it names the last HIP error seen by the library. */
const char *ss_status_string(int32_t code);

/* Number of chunks ceil(n / SS_CHUNK); the chunk index of ss_prepare holds
 * p * (ss_chunk_count(n) + 1) int32 entries. */
int64_t ss_chunk_count(int64_t n);

/* ------------------------------------------------------------ a0: prepare
 * One-time preparation of a data set (Sec. 2.7: arrangement by decreasing
 * observed time; Sec. 2.2: Kaplan-Meier censoring weights).
 *
 * Inputs (device, original subject order):
 *   y[n]        observed times Y_i = min(T_i, C_i); finite, not NaN.
 *   status[n]   0 censored, 1 event (Fine-Gray: primary event), 2 competing
 *               event (Fine-Gray only; the Cox model counts it as an event).
 *   col_ptr[p+1] int64 CSC column pointers (col_ptr[0] = 0, non-decreasing,
 *               col_ptr[p] = nnz), rows[nnz] int32 subject indices in [0, n)
 *               with no duplicate inside a column (any order),
 *   vals[nnz]   covariate values, or NULL for a 0/1 indicator design.
 * Outputs (device, caller-allocated):
 *   perm[n]      int32, perm[k] = subject at sorted position k.
 *   inv_perm[n]  int32, inverse of perm.
 *   d8[n]        uint8, at the last position of each tie run: number of
 *                events in the run, saturated at 255; 0 elsewhere.
 *   d32[n]       int32, the same counts unsaturated (read only where d8 is
 *                255).
 *   c[p]         c_j = sum over events of x_ij (Sec. 2.7, the constant term
 *                delta' X_j of g'; Fine-Gray: over status == 1).
 *   rows_sorted[nnz] int32, the design re-labelled to sorted positions and
 *                ascending inside each column (same col_ptr).
 *   vals_sorted[nnz] the values in that order (ignored when vals == NULL).
 *   chunk_ptr[p*(ss_chunk_count(n)+1)] int32: entry j*(C+1)+t is the offset
 *                inside column j of its first non-zero at sorted position
 *                >= t*SS_CHUNK (C = ss_chunk_count(n)).
 *   w_comp[n]    Fine-Gray only (else may be NULL): I(status=2)/G(y_k), the
 *                censoring weight of a competing event at sorted position k.
 *   g_end[n]     Fine-Gray only (else may be NULL): G(y_k), the Kaplan-Meier
 *                estimate of Pr(C > y_k), right-continuous.
 * ws/ws_bytes   device scratch of at least ss_prepare_workspace_bytes().
 * The integer outputs are bit-exact and deterministic.
 * Unlike the other calls, ss_prepare synchronises `stream`: it reads col_ptr
 * on the host first, and it reports data errors found on the device (a row
 * index outside [0, n), a duplicate row in a column, a status outside
 * {0, 1, 2}, invalid column pointers) as SS_EINVAL before returning. */
size_t ss_prepare_workspace_bytes(int64_t n, int64_t p, int64_t nnz);
int32_t ss_prepare(int32_t model, int64_t n, int64_t p, int64_t nnz,
                   const double *y, const int8_t *status,
                   const int64_t *col_ptr, const int32_t *rows,
                   const double *vals,
                   int32_t *perm, int32_t *inv_perm, uint8_t *d8,
                   int32_t *d32, double *c, int32_t *rows_sorted,
                   double *vals_sorted, int32_t *chunk_ptr,
                   double *w_comp, double *g_end,
                   void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ workspace
 * Scratch of the fused kernels: tile look-back states, per-tile partial
 * sums and the launch counters.  It must be cleared once with
 * ss_workspace_init before its first use; afterwards every call leaves it
 * ready for the next one (no per-call clearing). */
size_t ss_workspace_bytes(int32_t model, int64_t n);
int32_t ss_workspace_init(void *ws, size_t ws_bytes, void *stream);

/* Device status word kept in the workspace: 0 while every bounded wait of
 * the fused kernels has finished in time, non-zero once one gave up (the
 * results of that call are then not valid).  Copies it to *flag [host]
 * after synchronising `stream`. */
int32_t ss_workspace_error(const void *ws, int32_t *flag, void *stream);

/* ------------------------------------------------------------ a2 / a4
 * Gradient and Hessian of the log partial likelihood (Cox, Sec. 2.7 eqs.
 * cox_g/cox_h) or log pseudo-likelihood (Fine-Gray, eqs. fg_g/fg_h) along
 * coordinate j, for the current e = exp(X beta):
 *   g'  = c_j - sum_k d_k G_k,    g'' = -sum_k d_k (H_k - G_k^2),
 *   G_k = S1_k / S0_k,  H_k = S2_k / S0_k  at the last position k of every
 *   tie run (ties as the risk set y_r >= Y_i is written), where
 *   Cox:        S_m,k = sum_{r <= k} e_r x_rj^m
 *   Fine-Gray:  S_m,k = sum_{r <= k} e_r x_rj^m
 *                       + g_end_k * sum_{r after k's run} e_r x_rj^m w_comp_r
 * One fused pass: tuple scan with decoupled look-back, transform,
 * reduction; the last tile finishes the reduction (Fig. 2).  The partial
 * sums are added in a fixed order, but a tile's prefix combines whichever
 * predecessor values the look-back finds visible first, so repeated calls
 * can differ in the last bits (far inside the 1e-10 parity bound).
 * Inputs: e[n] in sorted order; the ss_prepare outputs; j in [0, p).
 * Output out[3] (device): g', g'', and sum_k d_k log S0_k. */
int32_t ss_grad_hess(int32_t model, int64_t n, int64_t p, int64_t j,
                     const double *e, const uint8_t *d8, const int32_t *d32,
                     const double *w_comp, const double *g_end,
                     const int64_t *col_ptr, const int32_t *rows_sorted,
                     const double *vals_sorted, const int32_t *chunk_ptr,
                     const double *c, double *out,
                     void *ws, size_t ws_bytes, void *stream);

/* Log partial (pseudo-) likelihood l = beta' c - sum_k d_k log S0_k
 * (Sec. 2.7, the prefix-sum form of eq. cox_l; eq. fg_l for Fine-Gray),
 * with beta[p] on the device.  Output out[1] (device). */
int32_t ss_loglik(int32_t model, int64_t n, int64_t p,
                  const double *e, const uint8_t *d8, const int32_t *d32,
                  const double *w_comp, const double *g_end,
                  const double *beta, const double *c, double *out,
                  void *ws, size_t ws_bytes, void *stream);

/* Penalised objective g = l + pi (Secs. 2.3-2.4: CCD maximises the log
 * (pseudo-) likelihood plus the log prior), at beta[p] (device) and the
 * e = exp(X beta) that goes with it: l as ss_loglik computes it, and
 *   pi = -gamma sum_j |beta_j|           (SS_PENALTY_L1, lambda = gamma)
 *   pi = -sum_j beta_j^2 / (2 tau)       (SS_PENALTY_L2, lambda = tau)
 *   pi = 0                               (SS_PENALTY_NONE, lambda ignored)
 * Output out[3] (device): l + pi, l, pi.  One fused launch, the penalty
 * summed by the last tile.  Errors as ss_loglik, plus SS_EUNSUPPORTED for an
 * unknown penalty and SS_EINVAL for a penalty with lambda <= 0. */
int32_t ss_objective(int32_t model, int32_t penalty, double lambda, int64_t n,
                     int64_t p, const double *e, const uint8_t *d8,
                     const int32_t *d32, const double *w_comp,
                     const double *g_end, const double *beta, const double *c,
                     double *out, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ a3 (+ a1)
 * One coordinate update (Secs. 2.3-2.4): from g12[0..1] = (g', g'') of the
 * unpenalised likelihood (device, e.g. the out of ss_grad_hess), take the
 * penalised Newton step (l1 directional rule at beta_j = 0, an l1 step that
 * would cross zero stops at zero), clip it to the trust region,
 *   beta_j += sgn(s) min(|s|, delta_j),  delta_j <- max(2|s|, delta_j/2),
 * store the applied step in *step, and if it is non-zero update
 * eta_k += x_kj * step and e_k = exp(eta_k) at the non-zeros of column j
 * (Sec. 2.7 step (1); Fig. 3's conditional kernel).  lambda is gamma (l1)
 * or tau (l2), ignored for no penalty.  A penalised second derivative that
 * is not strictly negative gives a zero step. */
int32_t ss_ccd_update(int32_t penalty, double lambda, int64_t n, int64_t p,
                      int64_t j, const double *g12, double *beta,
                      double *delta, double *step, double *eta, double *e,
                      const int64_t *col_ptr, const int32_t *rows_sorted,
                      const double *vals_sorted, void *stream);

/* ------------------------------------------------------------ fused sweep
 * Cyclic coordinate descent over coordinates j_begin..j_end-1 (Fig. 3)
 * without any host round trip: per coordinate one fused launch (Fine-Gray:
 * two) that applies the previous coordinate's update to eta and e (step
 * (1)), computes g', g'' (steps (2)-(4)) and, in its last tile, the update
 * of beta_j, delta_j and steps[j] (a3).  The last coordinate's update of
 * eta/e is applied before returning, so eta, e, beta and delta are
 * consistent afterwards.  g12_out[3*p] (optional, may be NULL) receives
 * (g', g'', sum d log S0) of every visited coordinate. */
int32_t ss_ccd_sweep(int32_t model, int32_t penalty, double lambda,
                     int64_t n, int64_t p, int64_t j_begin, int64_t j_end,
                     double *eta, double *e, const uint8_t *d8,
                     const int32_t *d32, const double *w_comp,
                     const double *g_end, const int64_t *col_ptr,
                     const int32_t *rows_sorted, const double *vals_sorted,
                     const int32_t *chunk_ptr, const double *c,
                     double *beta, double *delta, double *steps,
                     double *g12_out, void *ws, size_t ws_bytes,
                     void *stream);

/* e_k = exp(eta_k) for k < n (sorted order; used to initialise e). */
int32_t ss_exp(int64_t n, const double *eta, double *e, void *stream);

/* dst[k] = src[perm[k]] for k < n: brings a per-subject vector into sorted
 * order (dst and src must not overlap). */
int32_t ss_gather(int64_t n, const int32_t *perm, const double *src,
                  double *dst, void *stream);

/* ---------------------------------------------- FP32 storage of e
 * The paper stores the per-subject quantities in FP64 (Sec. 2.7); these two
 * calls keep e = exp(X beta) in FP32 instead, to measure what that costs in
 * accuracy with three ways of accumulating the scans and sums.
 *
 * ss_exp_f32: e32_k = (float) exp(eta_k - m) for k < n with m = max_k eta_k
 * written to *shift (device, one double).  The shift keeps exp inside the
 * FP32 range (it overflows from about 88); g' and g'' do not depend on it
 * and sum_k d_k log S0_k moves by m sum_k d_k.  Uses `ws` (a workspace of
 * ss_workspace_bytes(model, n) bytes for any model) as scratch.
 *
 * ss_grad_hess_mixed: out[3] = g', g'', sum_k d_k log S0_k as ss_grad_hess,
 * from e32 (sorted order, FP32; S0 as e32 gives it, i.e. shifted) with every
 * prefix sum, transform and reduction carried out in the precision `acc`
 * selects (SS_ACC_*).  Other arguments as for ss_grad_hess; e32 needs no
 * particular alignment.  A reduce-then-scan in a fixed order (per-tile
 * aggregates, one scan, the tile pass, the final sum): results are
 * deterministic.  Errors: SS_EINVAL for a bad argument or an unknown `acc`,
 * SS_EWORKSPACE as ss_grad_hess. */
int32_t ss_exp_f32(int64_t n, const double *eta, float *e32, double *shift,
                   void *ws, size_t ws_bytes, void *stream);

/* ss_grad_hess_f32: FP32 storage of e inside the single-pass fused kernel
 * of ss_grad_hess (Sec. 2.7, Fig. 2: one pass with decoupled look-back), so
 * that a coordinate streams 4 instead of 8 bytes of e per subject.  Same
 * outputs as ss_grad_hess_mixed (S0 as e32 gives it, i.e. shifted), with
 * `acc`:
 *   SS_ACC_F64      every sum, the transform and the reduction in FP64
 *                   (only the storage of e is FP32);
 *   SS_ACC_F32_C64  the sums inside a tile (thread-serial and wave scans),
 *                   the transform and each thread's share of the reduction
 *                   in FP32; the tile aggregates, the look-back prefix each
 *                   tile starts from (its carry), the Fine-Gray totals and
 *                   the sum of the tile partials in FP64 (Sec. 2.7 step (4)
 *                   accumulates in double; the paper fixes no other
 *                   precision).
 * Other modes: SS_EINVAL (see ss_grad_hess_mixed).  e32 must be 16-byte
 * aligned (SS_EINVAL otherwise); other arguments, the workspace and the
 * non-determinism in the last bits as for ss_grad_hess. */
int32_t ss_grad_hess_f32(int32_t model, int32_t acc, int64_t n, int64_t p,
                         int64_t j, const float *e32, const uint8_t *d8,
                         const int32_t *d32, const double *w_comp,
                         const double *g_end, const int64_t *col_ptr,
                         const int32_t *rows_sorted, const double *vals_sorted,
                         const int32_t *chunk_ptr, const double *c,
                         double *out, void *ws, size_t ws_bytes, void *stream);
int32_t ss_grad_hess_mixed(int32_t model, int32_t acc, int64_t n, int64_t p,
                           int64_t j, const float *e32, const uint8_t *d8,
                           const int32_t *d32, const double *w_comp,
                           const double *g_end, const int64_t *col_ptr,
                           const int32_t *rows_sorted,
                           const double *vals_sorted,
                           const int32_t *chunk_ptr, const double *c,
                           double *out, void *ws, size_t ws_bytes,
                           void *stream);

/* ss_eta_gradient: the gradient of the log (pseudo-)likelihood with respect
 * to the linear predictor, for every subject at once -- the vector
 * delta - P delta of Sec. 2.9 (Cox, Sec. 2.1 eq. for l(beta)) and its
 * Fine-Gray analogue (Sec. 2.2, IPCW weights), whose product with X' is the
 * full gradient in beta a proximal-gradient method needs.  O(N) by prefix
 * and suffix sums in decreasing-time order, the Sec. 2.7 form that Sec. 2.9
 * points to, with Breslow ties:
 *
 *   dl/deta_m = delta_m - e_m * ( sum over run ends k at or after m of
 *               d_k / S0_k  [+ w_comp_m * sum over run ends k before m of
 *               d_k G(Y_k) / S0_k, Fine-Gray] )
 *
 * and *loglik = sum_m delta_m eta_m - sum_k d_k log S0_k (the value whose
 * gradient this is).  delta_m = 1 for an event of interest (Cox: status
 * != 0; Fine-Gray: status == 1).
 *
 * Arguments (device memory): inv_perm, d8, d32, w_comp, g_end as
 * ss_prepare wrote them; status_sorted[n] int8 in SORTED order
 * (status[perm[k]], as ss_gather_u8 produces it once per data set); eta[n]
 * and e[n] = exp(eta) in SORTED order (as ss_gather / ss_exp produce them;
 * e is not recomputed from eta, so the pair must agree); grad[n] is written
 * in ORIGINAL subject order (gathered through inv_perm); *loglik one
 * double.  The
 * workspace (any 256-byte-aligned device buffer of
 * ss_eta_gradient_workspace_bytes(n) bytes, caller-owned, no
 * initialisation) holds four N-vectors of partial results, the block sums
 * of l and the scan carries; it is distinct from the ss_grad_hess
 * workspace.  All sums are taken in a fixed order: results are
 * deterministic.  Errors: SS_EINVAL for an unknown-size or null argument,
 * SS_EUNSUPPORTED for an unknown model, SS_EWORKSPACE for a short or
 * misaligned workspace.
 *
 * ss_gather_u8: dst[k] = src[perm[k]] for k < n (bytes; e.g. the status
 * vector into sorted order).  SS_EINVAL for a bad size or null pointer. */
size_t ss_eta_gradient_workspace_bytes(int64_t n);
int32_t ss_eta_gradient(int32_t model, int64_t n, const int32_t *inv_perm,
                        const int8_t *status_sorted, const double *eta,
                        const double *e, const uint8_t *d8,
                        const int32_t *d32, const double *w_comp,
                        const double *g_end, double *grad, double *loglik,
                        void *ws, size_t ws_bytes, void *stream);
int32_t ss_gather_u8(int64_t n, const int32_t *perm, const uint8_t *src,
                     uint8_t *dst, void *stream);

/* ss_beta_gradient: the full gradient of l in beta, X' (dl/deta) (Sec. 2.9:
 * the gradient a proximal-gradient method takes is X' times the vector
 * ss_eta_gradient computes), formed from the gradient in eta in SORTED
 * order and the sorted-position design of ss_prepare (col_ptr,
 * rows_sorted, vals_sorted or NULL for 0/1, chunk_ptr), so no permutation
 * of the subjects is involved: grad_beta[j] = sum over column j's
 * non-zeros of x * (dl/deta at that position).  The positions are cut into
 * spans of whole chunks; each (column, span) piece is summed by one
 * wavefront, then each column's pieces in span order: every sum in a fixed
 * order (deterministic).  Also l in *loglik, and, if grad_eta is not NULL,
 * dl/deta in subject order as ss_eta_gradient writes it (then inv_perm is
 * needed; otherwise it may be NULL).  The workspace is
 * ss_beta_gradient_workspace_bytes(n, p) bytes (at most
 * ss_eta_gradient_workspace_bytes(n) plus 16 (n + p) + 256); other
 * arguments and errors as ss_eta_gradient, plus SS_EINVAL for p < 1 or a
 * null column array. */
size_t ss_beta_gradient_workspace_bytes(int64_t n, int64_t p);
int32_t ss_beta_gradient(int32_t model, int64_t n, int64_t p,
                         const int32_t *inv_perm, const int8_t *status_sorted,
                         const double *eta, const double *e,
                         const uint8_t *d8, const int32_t *d32,
                         const double *w_comp, const double *g_end,
                         const int64_t *col_ptr, const int32_t *rows_sorted,
                         const double *vals_sorted, const int32_t *chunk_ptr,
                         double *grad_beta, double *grad_eta, double *loglik,
                         void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Cross-validation replicates in one launch (Sec. 2.8; the single larger
 * kernel for many k-fold repetitions proposed in the paper's concluding
 * discussion).  R replicates share the prepared problem (order, tie runs,
 * design) and each is CCD on its own training subjects: held-out subjects
 * carry e = 0 and drop out of every risk set, event counts and c_j count
 * training events only, and eta = X beta is kept for every subject so the
 * held-out log-likelihood can be scored at the fitted beta.  Cox and
 * Fine-Gray models, 0/1 designs (the designs of Sec. 3.2); SS_EUNSUPPORTED
 * for valued designs.  Fine-Gray: each replicate's competing-event weights
 * use the Kaplan-Meier estimate of its own training subjects (Sec. 2.2, the
 * weight after eq. fg_l, on the replicate's data set), and its held-out
 * likelihood that of its held-out subjects.
 *
 * Per-replicate vectors are in SORTED order, replicate r starting at
 * r * ss_cv_stride(n) elements (the stride is a multiple of 16384; the
 * positions from n to the stride are padding the library keeps at
 * e = 0).  Sizes the caller allocates (device memory, caller-owned):
 *   train_s, d8_r: R * stride bytes; d32_r: R * stride int32 (read only
 *   where d8_r = 255, no initialisation needed); eta, e: R * stride
 *   doubles; xbits: P * stride / 8 bytes (Fine-Gray: (P + 1) * stride / 8,
 *   the last column marking competing events); c_r, beta, delta: R * P doubles
 *   (replicate-major); g12_out: R * P * 3 doubles or NULL; Fine-Gray only
 *   (NULL for Cox): w_r, g_r, g_h: R * stride doubles each; out of
 *   ss_cv_loglik: 2 R doubles; ws of ss_cv_prepare:
 *   ss_cv_prepare_workspace_bytes(n, R) bytes.
 *
 * ss_cv_prepare: from ss_prepare's perm and d8, the ORIGINAL-order status
 * and training masks train[R][n] (1 = training subject, subject order,
 * replicate-major): the sorted training flags train_s, the training events
 * per run end d8_r / d32_r (same encoding as ss_prepare), the column
 * bitmask xbits (bit k of column j, word k/32 of the column's stride/32
 * 32-bit words; Fine-Gray adds column P, bit k set where the subject at
 * sorted position k had a competing event) and c_r[r][j] = the training
 * events with x_kj = 1.
 * vals_sorted must be NULL (0/1 design).  Fine-Gray also takes the
 * ORIGINAL-order times y (for the tie runs of the Kaplan-Meier estimates)
 * and writes, per replicate and sorted position k, g_r = G of the training
 * subjects at y_k, g_h = G of the held-out subjects at y_k (G(t) = product
 * over censoring times c <= t of 1 - m_c / n_c within the subset) and
 * w_r = 1 / g_r for training subjects with status 2, else 0.
 *
 * ss_cv_exp: e = exp(eta) at training positions, 0 elsewhere (all R).
 *
 * ss_cv_sweep: for every replicate at once, the coordinates j_begin ..
 * j_end - 1 in order, each: a1 (the previous step at its column's rows,
 * e multiplied by exp(step)), the Sec. 2.7 scan and reduction giving g' and
 * g'' of the replicate's training data, and the a3 update of Sec. 2.4 on
 * beta[r][j], delta[r][j]; g12_out[r][j] = (g', g'', applied step) if not
 * NULL.  At the end eta holds X beta and e = exp(eta) (masked) afresh.
 * One workgroup per replicate, or two (each half of the positions, one
 * exchange per coordinate, cooperative launch) when all of them fit on
 * the device at once; Fine-Gray carries the weighted totals sum e w and
 * sum e w x_j over the replicate from one coordinate to the next in closed
 * form (a pass before the first coordinate sums them); fixed summation
 * order either way (deterministic for a given device).  ws: ss_cv_workspace_bytes(R) bytes, 256-byte aligned,
 * zero-filled before first use (ss_workspace_init), kept between calls; a
 * bounded wait that gives up sets its error word (ss_workspace_error),
 * after which it must be zero-filled again.  Errors: SS_EINVAL for bad
 * sizes or ranges or a null pointer, SS_EWORKSPACE for a short or
 * misaligned workspace, SS_EUNSUPPORTED for an unknown model.
 *
 * ss_cv_loglik: out[2r] = the training log partial (Fine-Gray: pseudo-)
 * likelihood of replicate r at its current eta, out[2r+1] = the held-out
 * one: the held-out subjects as a data set of their own (their risk sets,
 * their events, for Fine-Gray their own Kaplan-Meier weights g_h), the
 * predictive log-likelihood of the fold (Sec. 2.8).  d8, d32: ss_prepare's
 * full-data counts. */
int64_t ss_cv_stride(int64_t n);
size_t ss_cv_prepare_workspace_bytes(int64_t n, int32_t reps);
int32_t ss_cv_prepare(int32_t model, int64_t n, int64_t p, int32_t reps,
                      const int32_t *perm, const int8_t *status,
                      const double *y, const uint8_t *d8, const uint8_t *train,
                      const int64_t *col_ptr, const int32_t *rows_sorted,
                      const double *vals_sorted, uint8_t *train_s,
                      uint8_t *d8_r, int32_t *d32_r, uint32_t *xbits,
                      double *c_r, double *w_r, double *g_r, double *g_h,
                      void *ws, size_t ws_bytes, void *stream);
int32_t ss_cv_exp(int64_t n, int32_t reps, const double *eta,
                  const uint8_t *train_s, double *e, void *stream);
size_t ss_cv_workspace_bytes(int32_t reps);
int32_t ss_cv_sweep(int32_t model, int32_t penalty, double lambda, int64_t n,
                    int64_t p, int32_t reps, int64_t j_begin, int64_t j_end,
                    double *eta, double *e, const uint8_t *d8_r,
                    const int32_t *d32_r, const uint8_t *train_s,
                    const uint32_t *xbits, const double *c_r,
                    const double *w_r, const double *g_r, double *beta,
                    double *delta, double *g12_out, void *ws, size_t ws_bytes,
                    void *stream);
int32_t ss_cv_loglik(int32_t model, int64_t n, int32_t reps,
                     const int32_t *perm, const int8_t *status,
                     const double *eta, const double *e,
                     const uint8_t *train_s, const uint8_t *d8,
                     const int32_t *d32, const uint8_t *d8_r,
                     const int32_t *d32_r, const double *w_r,
                     const double *g_r, const double *g_h, double *out,
                     void *stream);

/* ss_cv_select: the choice of the penalty strength by cross-validation
 * (Sec. 2.8, and the largest mean predictive log-likelihood as the reading
 * of "best").  scores (device) holds n_gamma rows of 2 * reps doubles, row g
 * as ss_cv_loglik wrote it for the fits at strength g (out[2r+1] = the
 * held-out log-likelihood of replicate r).  Writes mean[g] (device,
 * n_gamma doubles) = the mean held-out log-likelihood over the replicates,
 * summed in replicate order, and *best (device, one int32) = the first g
 * with the largest mean (a NaN mean never wins; -1 if every mean is NaN).
 * One small launch; deterministic.  SS_EINVAL for n_gamma < 1, reps outside
 * [1, 65535] or a null pointer. */
int32_t ss_cv_select(int32_t n_gamma, int32_t reps, const double *scores,
                     double *mean, int32_t *best, void *stream);

/* ---------------------------------------------------------------------
 * Launch shapes and their autotuning.  Sec. 2.7 leaves the block size and
 * the items per thread of the fused scan kernel as tunable constants; here
 * two choices are tuned:
 *   SS_TUNE_GRAD_HESS  positions per thread of the single-pass fused kernel
 *                      of ss_grad_hess, ss_loglik, ss_objective,
 *                      ss_grad_hess_f32 and ss_grad_hess_noalloc: 4, 8, 16
 *                      or 32 (tiles of 1024 ... 8192 positions; the
 *                      per-coordinate launches inside ss_ccd_sweep use 8
 *                      or 16 only);
 *   SS_TUNE_SWEEP      segment shape of the persistent sweep of
 *                      ss_ccd_sweep, block * 100 + positions per thread:
 *                      25608, 25616, 51208 or 51216 (Cox only).
 * A choice is kept per (kind, model, storage of e, valued design or not,
 * size bucket ceil(log2 n)) in a process-wide table that every launch
 * consults; without an entry a launch uses the built-in rule (tiles of
 * 2048 positions up to 1.5 M positions, 4096 above; the first sweep shape
 * whose workgroups all fit on the device).
 *   storage: SS_STORAGE_F64 (FP64 e), SS_STORAGE_F32 (FP32 e, FP64 sums),
 *   SS_STORAGE_F32_SUMS32 (FP32 e, FP32 in-tile sums); the sweep is FP64.
 * ss_tune_get: the choice a launch would use now (the built-in rule's IPT
 * for SS_TUNE_GRAD_HESS, 0 for an untuned sweep); ss_tune_has: 1 if the
 * table holds an entry for the key, else 0.  ss_tune_set: pins a
 * choice (0 removes the entry; SS_EINVAL for an impossible one).
 * ss_tune_clear: empties the table.  ss_tune_save / ss_tune_load [host
 * path]: write the table to a text file / add the entries of a file that
 * were measured on the current device's GPU architecture (*loaded [host]
 * receives their number); SS_EINVAL if the file cannot be opened.  These
 * calls take a mutex and launch nothing. */
#define SS_TUNE_GRAD_HESS       0
#define SS_TUNE_SWEEP           1
#define SS_STORAGE_F64          0
#define SS_STORAGE_F32          1
#define SS_STORAGE_F32_SUMS32   2
int32_t ss_tune_get(int32_t kind, int32_t model, int32_t storage,
                    int32_t valued, int64_t n);
int32_t ss_tune_has(int32_t kind, int32_t model, int32_t storage,
                    int32_t valued, int64_t n);
int32_t ss_tune_set(int32_t kind, int32_t model, int32_t storage,
                    int32_t valued, int64_t n, int32_t choice);
int32_t ss_tune_clear(void);
int32_t ss_tune_save(const char *path);
int32_t ss_tune_load(const char *path, int32_t *loaded);

/* ss_autotune_grad_hess: times every SS_TUNE_GRAD_HESS candidate on the
 * caller's prepared problem and coordinate j (arguments as ss_grad_hess, or
 * as ss_grad_hess_f32 for FP32 storage, with e pointing at the FP64 or FP32
 * vector), `reps` back-to-back launches each between two HIP events on
 * `stream` (synchronises it), and stores the fastest in the table.
 * *choice [host] receives it; us [host, 4 floats, may be NULL] the average
 * microseconds per call of IPT 4, 8, 16, 32.  `out` is overwritten.
 *
 * ss_autotune_sweep: the same for the persistent sweep's segment shapes,
 * over coordinates [j_begin, j_end) of the caller's problem.  The state
 * (eta, e, beta, delta) is only read: before every timed sweep it is copied
 * into the caller's scratch vectors (eta_s, e_s: n doubles; beta_s,
 * delta_s, steps_s: p doubles), which the sweep then updates.  Shapes whose
 * workgroups do not all fit on the device are skipped (us = -1); with none
 * left, SS_EUNSUPPORTED.  us [host, 4 floats, may be NULL]: 25616, 51208,
 * 25608, 51216 in that order.
 * Errors as the calls they time; reps outside [1, 1000]: SS_EINVAL. */
int32_t ss_autotune_grad_hess(int32_t model, int32_t storage, int64_t n,
                              int64_t p, int64_t j, const void *e,
                              const uint8_t *d8, const int32_t *d32,
                              const double *w_comp, const double *g_end,
                              const int64_t *col_ptr,
                              const int32_t *rows_sorted,
                              const double *vals_sorted,
                              const int32_t *chunk_ptr, const double *c,
                              double *out, void *ws, size_t ws_bytes,
                              int32_t reps, int32_t *choice, float *us,
                              void *stream);
int32_t ss_autotune_sweep(int32_t model, int32_t penalty, double lambda,
                          int64_t n, int64_t p, int64_t j_begin, int64_t j_end,
                          const double *eta, const double *e,
                          const uint8_t *d8, const int32_t *d32,
                          const double *w_comp, const double *g_end,
                          const int64_t *col_ptr, const int32_t *rows_sorted,
                          const double *vals_sorted, const int32_t *chunk_ptr,
                          const double *c, const double *beta,
                          const double *delta, double *eta_s, double *e_s,
                          double *beta_s, double *delta_s, double *steps_s,
                          void *ws, size_t ws_bytes, int32_t reps,
                          int32_t *choice, float *us, void *stream);

/* ---------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as ss_grad_hess, with the fused kernels' scratch (look-back
 * pairs, per-tile partial sums, launch counters) in a file-scope device
 * array of ss_noalloc_scratch_bytes() bytes instead of a caller workspace.
 * Each GPU the library runs on holds its own copy until the process ends;
 * the first call on a device looks up its address and clears it (a fill
 * kernel on `stream`).  No allocation happens in any call.
 *   n at most SS_NOALLOC_MAX_N (larger: SS_EINVAL); `stream` must belong
 *   to the current device (else SS_EINVAL); other arguments and out[0..2]
 *   as ss_grad_hess; out[3] (device) = 1.0 if a bounded wait of this call
 *   gave up (results invalid), else 0.0.
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents: calls that overlap on one GPU (several streams, several
 * host threads) race and must be serialised by the caller. */
#define SS_NOALLOC_MAX_N ((int64_t)1 << 25)
size_t ss_noalloc_scratch_bytes(void);
int32_t ss_grad_hess_noalloc(int32_t model, int64_t n, int64_t p, int64_t j,
                             const double *e, const uint8_t *d8,
                             const int32_t *d32, const double *w_comp,
                             const double *g_end, const int64_t *col_ptr,
                             const int32_t *rows_sorted,
                             const double *vals_sorted,
                             const int32_t *chunk_ptr, const double *c,
                             double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SURVSCAN_H */
