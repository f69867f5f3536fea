/*
 * tda.h -- C ABI of libtda: exact time-domain Gaussian log-likelihood on one
 * AMD Instinct MI355X (gfx950).
 *
 * What is computed (paper Sec. II):
 *   For a detector with data d and a waveform template h, both real vectors
 *   of N samples, and stationary Gaussian noise with autocorrelation function
 *   (ACF) rho, the noise covariance is the symmetric Toeplitz matrix
 *   C_ij = rho(|i-j|) (Sec. II, Toeplitz definition).  The log-likelihood is
 *   the exact Gaussian one (eqn:lik, no Whittle approximation):
 *       logL(h) = -1/2 (d-h)^T C^-1 (d-h) - 1/2 log det C - (N_eff/2) log 2 pi.
 *   C is factored once, C = L L^T (Sec. II.A), and each template is scored
 *   through the whitened residual w = L^-1 (d-h), logL = -1/2 w^T w + const
 *   (eq:td_like_whitened).
 *   Time segments (Sec. II.B item 1): C is block-diagonal over disjoint
 *   segments, each block the Toeplitz matrix of the ACF truncated to the
 *   segment length.  Data gaps (Sec. II.B item 2): excluded samples are
 *   marginalised out, i.e. each block is C[keep, keep] over the retained
 *   samples; values of d and h at excluded samples are never read.
 *   N_eff is the number of retained samples over all segments.
 *   Several detectors (Sec. II.B item 3): per-detector logL are summed;
 *   tda_loglik_multi sums items that share an output array.
 *
 * Precision:
 *   TDA_PREC_FP64  -- every step in FP64 (Cholesky, blocked triangular solve
 *                     on FP64 matrix cores, reductions).
 *   TDA_PREC_MIXED -- factorisation, log det and every reduction in FP64; the
 *                     bulk whitening products run on BF16 matrix cores with a
 *                     hi/lo split of both operands (three products, FP32
 *                     accumulation) against the explicit whitening operator
 *                     W = L^-1, followed by an FP64 refinement whose residual
 *                     uses an FP64 FFT Toeplitz product (eq:toeplitz_fft).
 *                     The refined quadratic form is never larger than the
 *                     exact one (variational bound) and its error is
 *                     quadratic in the BF16 product error.  Its FP64 FFT
 *                     product rounds at about u lambda_max ||C^-1 h||^2, which
 *                     keeps |dlogL| <= 1e-3 up to kappa(C) of about 1e7 (3e7
 *                     for the two-detector N = 16384 bank) and exceeds it from
 *                     about 1e8; beyond that use TDA_PREC_FP64.
 *   TDA_PREC_GS    -- FP64 evaluation through the Gohberg-Semencul form of the
 *                     Toeplitz inverse (Sec. III.A.3): x = C^-1 e_1 and log det C
 *                     by Levinson-Durbin once per segment, then per template
 *                     q = (||L(x)^T r||^2 - ||L(z)^T r||^2) / x_0 with
 *                     z = (0, x_{n-1}, .., x_1) and L(v) the lower-triangular
 *                     Toeplitz matrix of v, both products by FFT (O(n log n) per
 *                     template, no factorisation).  Only for segments without
 *                     excluded samples and of at most 65536 samples; a GS handle
 *                     evaluates only in TDA_PREC_GS.
 *   TDA_PREC_CDO   -- an evaluation precision of mixed handles (not a handle
 *                     precision): FP64 through the explicit inverse, the
 *                     paper's CDO form (Sec. III.A.2: w = W (d - h) with
 *                     W = L^-1 precomputed), as one FP64 matrix-core product
 *                     per block instead of the forward substitution of
 *                     TDA_PREC_FP64.  It uses the FP64 W = L^-1 that a mixed
 *                     handle keeps for its data whitening; the explicit
 *                     inverse is less stable than the substitution (its
 *                     forward error grows with kappa(L)).
 *
 * Conventions for every entry point:
 *   - Returns a tda_status; nothing is thrown across the ABI.  On failure a
 *     message is available from tda_last_error() (thread-local).
 *   - "host" pointers are read during the call only; "device" pointers are
 *     HIP device memory of the handle's device and must stay valid until the
 *     work enqueued on the given stream has finished.
 *   - Calls on one handle must not run concurrently from several host
 *     threads.  Different handles are independent.
 *   - Enqueued work is asynchronous with respect to the host unless stated.
 */
#ifndef TDA_H
#define TDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tda_ctx *tda_handle;

typedef enum {
  TDA_OK = 0,
  TDA_EINVAL = 1,    /* invalid argument (sizes, pointers, segments, ACF) */
  TDA_ENOTSPD = 2,   /* a Cholesky pivot was <= 0 or not finite */
  TDA_ENOMEM = 3,    /* device allocation failed or the HBM budget is exceeded */
  TDA_ESTATE = 4,    /* call out of order (e.g. tda_loglik before tda_factor) */
  TDA_ENODEV = 5,    /* no usable HIP device */
  TDA_EHIP = 6,      /* a HIP runtime call failed */
  TDA_EINTERNAL = 7, /* internal consistency check failed */
  TDA_EAGAIN = 8     /* serving: request not admitted now, retry later */
} tda_status;

typedef enum { TDA_PREC_FP64 = 0, TDA_PREC_MIXED = 1, TDA_PREC_GS = 2, TDA_PREC_CDO = 3 } tda_precision;

/* TDA_FLAG_COMPACT (mixed handles): once tda_set_data has cached the whitened
 * data, release the FP64 solve panels and the FP64 whitening operator, keeping
 * only the BF16 hi/lo operator copies (2 N_eff^2 bytes each for W and W^T) and
 * the cached data.  Afterwards FP64 and explicit-inverse evaluation, tda_set_data,
 * and evaluations that pass another data pointer return TDA_ESTATE; if the cached
 * data vector's retained samples change in place, the handle cannot whiten them
 * again and every result (logL and <d,h>) comes back NaN until the original
 * values are restored.  For large resident datasets (serving). */
enum { TDA_FLAG_COMPACT = 1 };

/* Half-open sample range [offset, offset + length) of the N-sample series. */
typedef struct {
  int64_t offset;
  int64_t length;
} tda_segment;

/* Device-memory provider for a handle's buffers (covariance blocks, factor, operator
 * copies, cached data, workspaces), so that the caller's allocator owns that memory
 * (e.g. PyTorch's caching allocator).
 *   alloc(bytes, ctx) returns device memory of the handle's device, at least 256-byte
 *     aligned, or NULL (the call then fails with TDA_ENOMEM);
 *   free(ptr, ctx) releases a pointer returned by alloc.  The library calls it only
 *     after the work that used the buffer has finished (it synchronises first).
 * Both are called on the thread that makes the library call.  The struct is copied by
 * tda_cov_build; the functions and ctx must stay valid until tda_destroy returns.
 * Per-call descriptor rings and pinned staging (a few hundred KB) still come from
 * hipMalloc / hipHostMalloc. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} tda_allocator;

typedef struct {
  uint32_t struct_size;   /* sizeof(tda_options); the size without `allocator` is accepted */
  int32_t precision;      /* tda_precision */
  int32_t device;         /* HIP device ordinal; -1 = current device */
  int32_t flags;          /* TDA_FLAG_* bits; 0 = default */
  size_t hbm_budget_bytes;/* cap on this handle's device memory; 0 = none */
  const tda_allocator *allocator; /* NULL: hipMalloc / hipFree */
} tda_options;

typedef struct {
  int64_t n;            /* N given to tda_cov_build */
  int64_t n_eff;        /* retained samples over all segments */
  int64_t n_pad;        /* padded row count used on the device */
  int64_t n_segments;
  double logdet;        /* log det C (valid once factored) */
  int64_t fail_row;     /* ENOTSPD: retained-sample row (0-based, within the segment); else -1 */
  int32_t fail_segment; /* ENOTSPD: segment index; else -1 */
  int32_t factored;     /* 1 once tda_factor succeeded */
  int32_t precision;
  int32_t data_set;     /* mixed: 1 once whitened data is cached */
  size_t device_bytes;  /* device memory held by the handle */
} tda_info_t;

/*
 * tda_cov_build -- describe one detector's noise model and assemble its
 * covariance blocks on the device (paper Sec. II Toeplitz definition,
 * Sec. II.B items 1-2).
 *   acf      host, float64[acf_len]: rho(0..acf_len-1); acf[0] > 0 and finite.
 *            acf_len must be >= the longest segment.  No regularisation is
 *            added: a numerically singular ACF is reported by tda_factor.
 *   N        total sample count, >= 1.
 *   gap_mask host, uint8[N] or NULL: nonzero = excluded sample.
 *   segments host, tda_segment[n_segments], sorted, disjoint, inside [0, N);
 *            NULL with n_segments == 0 means one segment [0, N).  Samples
 *            outside every segment are excluded.
 *   opt      host, may be NULL (FP64, current device, no budget).
 *   out      receives the handle.  All inputs are copied; the caller may free
 *            them on return.
 * Errors: EINVAL (N < 1, acf_len too short, acf[0] <= 0 or non-finite,
 *   bad segments, no retained sample; for TDA_PREC_GS also an excluded sample
 *   inside a segment or a segment longer than 65536), ENOMEM, ENODEV, EHIP.
 * Synchronous: returns after assembly finished (GS handles assemble nothing).
 */
tda_status tda_cov_build(const double *acf, int64_t acf_len, int64_t N, const uint8_t *gap_mask,
                         const tda_segment *segments, int64_t n_segments, const tda_options *opt,
                         tda_handle *out);

/*
 * tda_factor -- FP64 blocked Cholesky of every block, C = L L^T, and
 * log det C = 2 sum log L_ii (Sec. II.A; one-time cost, Sec. III.A.2).
 * Builds the packed triangular-solve panels; for TDA_PREC_MIXED also the
 * FP64 whitening operator W = L^-1 and its BF16 hi/lo copies.  For TDA_PREC_GS
 * instead: Levinson-Durbin per segment (x = C^-1 e_1, log det C = sum of log
 * prediction-error energies) and the two correlation spectra (Sec. III.A.3).
 * Errors: ENOTSPD (tda_info gives fail_row / fail_segment; for GS the first
 *   order whose prediction-error energy is not positive; the handle stays
 *   destroyable), ENOMEM, EHIP.  Idempotent after success.  Synchronous.
 */
tda_status tda_factor(tda_handle h);

/*
 * tda_set_data -- cache the whitened data of a mixed-precision handle:
 * dbar = W d, y_d = W^T dbar = C^-1 d and q_dd = dbar^T dbar, all FP64
 * (Sec. III.A: cache L and the whitened data once).  d is device
 * float64[N]; only retained samples are read.  FP64 handles accept and
 * ignore the call.  Enqueued on hip_stream (NULL = default stream).
 * The cache is keyed by a fingerprint of d's retained samples (a 64-bit sum of
 * mixed sample bits and positions, computed on the device): every mixed
 * evaluation recomputes it (O(N)) and re-whitens only when it differs, so
 * calling this first is optional; it forces the whitening now (and, with
 * TDA_FLAG_COMPACT, releases the FP64 operator afterwards, synchronously).
 * Errors: ESTATE (not factored; compact handle already compacted), EINVAL.
 */
tda_status tda_set_data(tda_handle h, const double *d, void *hip_stream);

/*
 * tda_loglik -- logL for B templates against one detector, constants
 * included (eq:td_like_whitened plus -1/2 log det C - N_eff/2 log 2 pi).
 *   d    device float64[N]: data.  Mixed handles use their cached whitened
 *        data when the fingerprint of d's retained samples matches the cached
 *        one (new contents, in place or at another address, are re-whitened
 *        within the call, at O(N_eff^2) cost; see tda_set_data).
 *   H    device float64, B rows of length >= N, row stride ldh (>= N).
 *   out  device float64[B], written (not accumulated).
 *   B = 0 is a no-op.  NaN/Inf in a template affects only its own out[b].
 * Errors: ESTATE (not factored), EINVAL (B < 0, ldh < N, NULL pointers).
 * Asynchronous on hip_stream (NULL = default stream).
 */
tda_status tda_loglik(tda_handle h, const double *d, const double *H, int64_t B, int64_t ldh,
                      double *out, void *hip_stream);

/* As tda_loglik, with the precision chosen per call: a mixed handle may
 * also be evaluated in TDA_PREC_FP64 and TDA_PREC_CDO; an FP64 handle
 * rejects TDA_PREC_MIXED and TDA_PREC_CDO with ESTATE. */
tda_status tda_loglik_ex(tda_handle h, const double *d, const double *H, int64_t B, int64_t ldh,
                         double *out, int32_t precision, void *hip_stream);

/*
 * tda_loglik_terms -- logL together with the two noise-weighted inner products
 * behind the paper's time-domain SNRs (Sec. II.B item 7: the matched-filter
 * SNR rho_mf = <d,h>/sqrt(<h,h>) and the effective SNR rho_eff^2 =
 * <d,d> - <r,r>, r = d - h), where <a,b> = a^T C^-1 b over the retained
 * samples of this detector:
 *   out[b]    = logL, exactly as tda_loglik_ex with the same precision,
 *   out_dh[b] = <d, h_b>      (may be NULL: not computed),
 *   out_hh[b] = <h_b, h_b>    (may be NULL: not computed).
 * <d,d> = q + 2 <d,h> - <h,h> follows with q = -2 (logL + 1/2 log det C +
 * N_eff/2 log 2 pi), and <r,r> = q.  All arrays are device float64[B] and
 * distinct.
 * Mixed precision computes <d,h> in FP64 from the cached C^-1 d and <h,h> as
 * the refined (FP64-residual) form plus the correction, in the same launches
 * as logL.  FP64 and Gohberg-Semencul evaluations obtain <h,h> from a second
 * evaluation against zero data and <d,d> from one of the data against a zero
 * template (about twice the cost of tda_loglik_ex when out_hh or out_dh is
 * requested).  NaN/Inf in a template gives NaN in its three outputs.
 * Errors and asynchrony as tda_loglik_ex.
 */
tda_status tda_loglik_terms(tda_handle h, const double *d, const double *H, int64_t B,
                            int64_t ldh, double *out, double *out_dh, double *out_hh,
                            int32_t precision, void *hip_stream);

/*
 * tda_snr -- logL and the paper's time-domain SNRs per template (Sec. II.B item 7),
 * finished on the device from the two inner products of tda_loglik_terms:
 *   out[b]      = logL, exactly as tda_loglik_terms computes it,
 *   rho_mf[b]   = <d,h_b> / sqrt(<h_b,h_b>)    (matched-filter SNR),
 *   rho_opt[b]  = sqrt(<h_b,h_b>)               (optimal SNR),
 *   rho_eff2[b] = <d,d> - <r_b,r_b> = 2 <d,h_b> - <h_b,h_b>, r_b = d - h_b
 *                 (squared effective SNR),
 * each device float64[B], distinct; any of the three may be NULL (not written).
 * A zero template gives rho_mf = NaN (0/0), rho_opt = 0 and rho_eff2 = 0.  Cost as
 * tda_loglik_terms with both inner products requested, plus one O(B) kernel.
 * Errors and asynchrony as tda_loglik_ex.
 */
tda_status tda_snr(tda_handle h, const double *d, const double *H, int64_t B, int64_t ldh,
                   double *out, double *rho_mf, double *rho_opt, double *rho_eff2,
                   int32_t precision, void *hip_stream);

/*
 * tda_loglik_fp64_noalloc -- tda_loglik_ex with TDA_PREC_FP64, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same kernel, same results bit for bit; the solve's scratch
 * (the solution rows of each 32-template column tile) is a fixed device array of
 * 64 MiB held by every GPU the library runs on until the process ends, instead of the
 * handle's workspace, and the call allocates nothing.  Needs
 * ceil(B / 32) * 32 * n_pad * 8 bytes <= 64 MiB (n_pad from tda_info: at N = 16384 up to
 * 512 templates per call); larger calls fail with EINVAL and a message giving the limit.
 * Every call on one GPU shares that array: calls that overlap on one GPU (several
 * streams or host threads, or several handles at once) race and must be serialised by
 * the caller.  On a capturing stream the call neither waits for nor records the
 * handle's earlier work (the caller orders it); otherwise as tda_loglik_ex.
 * Errors: as tda_loglik_ex; ESTATE for handles without the FP64 factor (compact mixed,
 * Gohberg-Semencul).
 */
tda_status tda_loglik_fp64_noalloc(tda_handle h, const double *d, const double *H, int64_t B,
                                   int64_t ldh, double *out, void *hip_stream);

/*
 * tda_whitened_residual -- the whitened residual of every template, the vector
 * whose squared norm is the quadratic form of logL (eq:td_like_whitened):
 *   wres[b * ldw + j] = (L^-1 (d - h_b))_j,  j < n_eff,
 * over the retained samples, segments concatenated in order and each in sample
 * order (L the FP64 Cholesky factor of the segment's block of C[mask,mask]);
 * residual diagnostics of the fit (Sec. II.B item 7) read them.  out[b] is logL
 * exactly as tda_loglik_ex with TDA_PREC_FP64 computes it, from the same solve.
 *   d, H, ldh, out  as tda_loglik (d is read directly, not from a cache).
 *   wres  device float64, caller-owned, at least (B - 1) ldw + n_eff elements;
 *         ldw >= n_eff (tda_info's n_eff).  Entries beyond n_eff are untouched.
 * Runs the FP64 triangular solve, then copies its solution rows out (N_eff B
 * doubles written).  B = 0 is a no-op.  NaN/Inf in a template stays in its row.
 * Errors: ESTATE (not factored; handles without the FP64 factor: Gohberg-Semencul
 * and compact mixed handles), EINVAL (B < 0, ldh < N, ldw < n_eff, NULL
 * pointers), EHIP (more than 2^31 - 1 blocks of 32 templates x 64 rows).
 * Asynchronous on hip_stream (NULL = default stream); not capturable in a graph.
 */
tda_status tda_whitened_residual(tda_handle h, const double *d, const double *H, int64_t B,
                                 int64_t ldh, double *out, double *wres, int64_t ldw,
                                 void *hip_stream);

/*
 * tda_acf_estimate -- autocovariance of a stretch of strain, for building the
 * covariance (Sec. II.B item 6: correlate the data directly, or take a Welch
 * PSD and its inverse Fourier transform, then truncate to the lags needed).
 *   x        device float64[n]: the strain (no signal in it).
 *   n_lags   lags written to acf[0 .. n_lags).
 *   method   TDA_ACF_DIRECT: acf[k] = (1/n) sum_{t < n-k} x_t x_{t+k}
 *            (biased sample autocovariance; n_lags <= n).
 *            TDA_ACF_WELCH: segments of seg_len samples, half overlapping
 *            (K = (n - seg_len) / (seg_len/2) + 1 of them), each with its mean
 *            removed and multiplied by the periodic Hann window w; then
 *            acf[k] = (1/K) sum_s sum_j y_s[j] y_s[(j+k) mod seg_len] / sum_j w_j^2,
 *            which equals the inverse DFT of the two-sided, mean-averaged Welch
 *            PSD (density scaling) times the sampling rate.  seg_len even and
 *            >= 2, n >= seg_len, n_lags <= seg_len / 2.
 *   seg_len  Welch segment length (ignored by TDA_ACF_DIRECT).
 *   acf      device float64[n_lags], written.
 * Units are those of x squared, as tda_cov_build takes them (a prefix of the
 * result serves a shorter segment).  Sums run in a fixed
 * order (reproducible).  The workspace is stream-ordered device memory
 * released on the stream.  Asynchronous on hip_stream.
 * Errors: EINVAL (sizes, method), ENOMEM, EHIP, ESTATE (capturing stream).
 */
typedef enum { TDA_ACF_DIRECT = 0, TDA_ACF_WELCH = 1 } tda_acf_method;
tda_status tda_acf_estimate(const double *x, int64_t n, int64_t n_lags, int32_t method,
                            int64_t seg_len, double *acf, void *hip_stream);

/*
 * tda_loglik_multi -- one batched evaluation over many (handle, data,
 * templates) items, e.g. all detectors of all instances (Sec. II.B item 3).
 * Items whose `out` pointers are equal are summed into that array in item
 * order (network logL); otherwise each out is written.  All handles must be
 * factored, live on one device and be evaluated in `precision` (FP64, MIXED
 * or GS; TDA_PREC_CDO is per handle only and gives EINVAL here).  The work of
 * all items of one precision runs in the same kernel launches.
 * Asynchronous on hip_stream.
 */
typedef struct {
  tda_handle h;
  const double *d; /* device float64[N of h] */
  const double *H; /* device, B rows, stride ldh */
  int64_t B;
  int64_t ldh;
  double *out;     /* device float64[B] */
} tda_work;

tda_status tda_loglik_multi(const tda_work *items, int64_t n_items, int32_t precision,
                            void *hip_stream);

/*
 * tda_release_workspaces -- tda_loglik_multi keeps its device workspaces (sized for
 * the largest batch seen so far) between calls on a device, so a steady stream of
 * batches allocates nothing.  This call frees them after waiting for the device to
 * finish; the next batched call allocates again.  For callers that move from one
 * workload to another and want the memory back (a server, say, after a large
 * batched evaluation).  Handles, plans and servers keep their own workspaces.
 * device: a device index, or -1 for the current device.  Errors: TDA_EINVAL for a
 * bad index, TDA_EHIP if the synchronization fails.  Must not overlap a
 * tda_loglik_multi call on the same device (it takes the same lock, so a
 * concurrent call waits).
 */
tda_status tda_release_workspaces(int32_t device);

/*
 * Plans: a batched evaluation frozen once (items, precision, workspace, kernel
 * variants) and then replayed.  tda_plan_create copies the item list (the
 * pointers inside must stay valid for the plan's lifetime), runs the evaluation
 * once synchronously (allocating every workspace and settling the autotuner),
 * and keeps a private workspace.  tda_plan_execute enqueues the evaluation on
 * hip_stream; with use_graph != 0 the first call captures the launch sequence
 * into a HIP graph on that stream and every call launches the graph (one
 * submission per step, no allocation, no descriptor upload).  Once captured, a
 * plan always replays its graph.  Results overwrite the items' outputs as in
 * tda_loglik_multi.  Calls on one plan must be serialised by the caller.  Each
 * replay re-checks the fingerprint of every mixed item's data, so changed data
 * (in place, or after tda_set_data with another vector on a handle of the plan)
 * is re-whitened inside the replay.
 * tda_loglik, tda_loglik_ex and tda_loglik_multi refuse a capturing stream
 * (TDA_ESTATE); plans are the way to put an evaluation into a graph.
 */
typedef struct tda_plan *tda_plan_t;
tda_status tda_plan_create(const tda_work *items, int64_t n_items, int32_t precision,
                           tda_plan_t *out);
tda_status tda_plan_execute(tda_plan_t p, void *hip_stream, int32_t use_graph);
tda_status tda_plan_destroy(tda_plan_t p);

tda_status tda_info(tda_handle h, tda_info_t *info);

/*
 * Request server: continuous batching of likelihood requests from many
 * concurrent sampler walkers (the paper's proposal pool, Sec. III.B.2, where
 * many proposals are evaluated while the sampler waits) against datasets kept
 * resident in HBM.
 *
 * A dataset is one factored handle plus its data vector.  tda_server_submit
 * enqueues a request of B templates against one dataset and returns at once.
 * A scheduler thread repeatedly takes, for every dataset with pending work,
 * the queued requests in arrival order (up to max_batch templates per dataset),
 * gathers their template rows into one block so a single sweep over the
 * dataset's operator serves all of them, evaluates all datasets in one
 * tda_loglik_multi-style launch sequence, and scatters the results.  Up to
 * n_slots such launches are in flight on separate streams, so requests that
 * arrive while others run are admitted as soon as a slot and staging memory
 * free up, and their work overlaps on the device.  A template's result does not
 * depend on which other templates share its launch.
 *
 * Admission: submit returns TDA_EAGAIN when max_queue requests are pending or
 * when a request alone would exceed a slot's staging memory
 * (staging_bytes / n_slots); datasets are admitted by tda_server_add_dataset
 * only while the sum of their handles' device memory stays within
 * dataset_budget_bytes (0 = no limit), else TDA_ENOMEM.  The scheduler also stops
 * coalescing where the launch's evaluation workspace would exceed the device memory
 * free at that moment plus what the slot's workspace already holds, less 1 GiB
 * (the first request of a launch is always taken); a launch that still fails to
 * allocate is halved, the later half going back to the front of the queue, down to
 * a single request, which then fails with the allocation error.
 * Latency of a request = completion observed by the server minus submit time.
 */
typedef struct tda_server *tda_server_t;

typedef struct {
  uint32_t struct_size;       /* sizeof(tda_server_options) */
  int32_t device;             /* -1 = current device */
  int32_t precision;          /* evaluation precision (datasets must support it) */
  int32_t n_slots;            /* launches in flight, >= 1 */
  int32_t max_batch;          /* max templates per dataset per launch, >= 1 */
  int32_t max_queue;          /* max pending requests before TDA_EAGAIN */
  size_t staging_bytes;       /* device staging for gathered templates, all slots */
  size_t dataset_budget_bytes;/* admission cap on resident datasets; 0 = none */
} tda_server_options;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t launches, templates;
  int64_t max_queue_depth;
  double p50_ms, p99_ms, mean_ms, max_ms; /* request latency */
  double mean_templates_per_launch;
  double busy_s;                          /* wall time with work in flight */
} tda_server_stats_t;

tda_status tda_server_create(const tda_server_options *opt, tda_server_t *out);
/* h: factored handle (not destroyed by the server); d: device float64[N of h],
 * kept alive by the caller while the server runs.  *dataset receives the id. */
tda_status tda_server_add_dataset(tda_server_t s, tda_handle h, const double *d, int32_t *dataset);
/* H: device, B rows (stride ldh >= N); out: device float64[B].  Both stay
 * owned by the caller and must stay valid until the request completes.
 * *ticket identifies the request.  Thread-safe. */
tda_status tda_server_submit(tda_server_t s, int32_t dataset, const double *H, int64_t B,
                             int64_t ldh, double *out, uint64_t *ticket);
/* *done = 1 once the request's results are in `out` (device writes finished). */
tda_status tda_server_poll(tda_server_t s, uint64_t ticket, int32_t *done);
/* Blocks until the request completed or timeout_s elapsed (TDA_EAGAIN). */
tda_status tda_server_wait(tda_server_t s, uint64_t ticket, double timeout_s);
tda_status tda_server_stats(tda_server_t s, tda_server_stats_t *st, int32_t reset);
/* Drains in-flight work, stops the threads, frees server memory (not the datasets). */
tda_status tda_server_destroy(tda_server_t s);

/*
 * Kernel timing (tracing aid).  When enabled, every kernel launch made by the
 * library is bracketed by two HIP events recorded on the launch's stream, so the
 * measured interval is that kernel's own execution in stream order.
 * tda_timing_read synchronises the recorded events and returns, per kernel
 * name, the number of launches and their summed duration in milliseconds
 * (at most `max` entries, count in *n); reset != 0 clears the totals.
 * Process-wide; not intended for concurrent use from several host threads.
 */
typedef struct {
  char name[32];
  int64_t count;
  double total_ms;
} tda_kernel_time;

tda_status tda_timing_enable(int32_t on);
tda_status tda_timing_read(tda_kernel_time *out, int32_t max, int32_t *n, int32_t reset);

/* Releases all device memory of the handle.  Waits for the device first.
 * NULL is accepted. */
tda_status tda_destroy(tda_handle h);

const char *tda_status_str(tda_status s);
const char *tda_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TDA_H */
