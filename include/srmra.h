/*
 * srmra.h -- C ABI of the MI355X (gfx950) EM step for 2-D super-resolution
 * multi-reference alignment (SR-MRA).
 *
 * Method: Shani, Tirer, Giryes, Bendory, "Denoiser-based projections for 2D
 * super-resolution MRA".  One call performs one *unprojected* EM step from
 * theta_t = (x, rho1, rho2):
 *
 *   model          y_i[n] = x[(n1 K - s1) mod Lh, (n2 K - s2) mod Lh] + eps  (Sec. 1, eq. model_1)
 *   log-likelihood l(theta_t) = sum_i log sum_s rho[s] exp(-||y_i - P R_s x||^2 / 2 sigma^2)
 *                                                                (Sec. 2, eq. likelihood_EM)
 *   posterior      w^{i,s} proportional to rho[s] exp(-||y_i - P R_s x||^2 / 2 sigma^2),
 *                  sum_s w^{i,s} = 1                              (Sec. 2, eq. weights_EM)
 *   M-step         A x_new = b                                    (Sec. 2, eq. x_EM)
 *                  rho_new[s] = sum_i w^{i,s} / sum_i sum_s' w^{i,s'}  (Sec. 2, eq. rho_EM)
 *
 * Conventions fixed by this library (the paper leaves them open):
 *  - shifts are 0-based and taken mod L_high; s1 / rho1 act on axis 0 (rows)
 *    of the row-major image, s2 / rho2 on axis 1; (R_s x)[m] = x[m - s];
 *  - P^{-1} in eq. x_EM is P^T, so A is diagonal and x_new = b / A per pixel;
 *    a pixel with zero posterior mass keeps its input value;
 *  - rho = rho1 rho2^T; the rho M-step returns the two marginals of the
 *    numerator of eq. rho_EM over its denominator;
 *  - loglik is eq. likelihood_EM literally (no Gaussian normalising constant)
 *    evaluated at the INPUT theta_t;
 *  - log_rho is used as given (need not be normalised; -inf allowed, but each
 *    row needs at least one finite entry).
 *
 * Memory and execution model:
 *  - every pointer argument except `probs` / `plan` / `workspace_bytes` of the
 *    plan calls is a DEVICE pointer; the caller owns every buffer;
 *  - the library never allocates or frees device memory and never copies
 *    device data to the host, and never synchronises a stream (a plan waits for
 *    its own earlier descriptor upload before rewriting the pinned host buffer
 *    that upload reads);
 *  - arguments are validated on the host before anything is enqueued; on an
 *    error return nothing has been enqueued;
 *  - on success all work is enqueued asynchronously on `stream`; execution
 *    errors surface through the stream (or as SRMRA_EDEVICE from the launch);
 *  - the library keeps no global mutable state: concurrent calls on different
 *    streams with disjoint buffers are safe.
 *
 * Layouts (all row-major, contiguous):
 *  y        float [N][L_low][L_low], 16-byte aligned
 *  x, x_new float [L_high][L_high],  L_high = K * L_low
 *  log_rho  float [2][L_high]   row 0 = log rho1 (axis 0), row 1 = log rho2 (axis 1)
 *  rho_new  float [2][L_high]   probabilities, each row sums to 1
 *  loglik   double [1]
 *
 * Supported shapes: L_low in {8, 12, 16, 24, 32, 48, 64}, K >= 1,
 * L_high = K * L_low <= 4096, 1 <= N <= 2^31 - 1.  Other L_low return
 * SRMRA_EUNSUPPORTED.
 */
#ifndef SRMRA_H
#define SRMRA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SRMRA_OK = 0,
    SRMRA_EINVAL = -1,        /* bad argument (null pointer, size, sigma, aliasing) */
    SRMRA_EUNSUPPORTED = -2,  /* shape or precision not built into this library   */
    SRMRA_EWORKSPACE = -3,    /* workspace / prepared buffer too small              */
    SRMRA_EDEVICE = -4,       /* a HIP launch reported an error                     */
    SRMRA_ESCRATCH = -5       /* srmra_em_step_noalloc: the shape needs more than
                                 SRMRA_SCRATCH_BYTES of workspace                   */
} srmra_status;

/* Arithmetic of the two dense contractions (score and back-projection).
 * Every form accumulates in FP32 and reduces across observations in FP64. */
typedef enum {
    SRMRA_FP32_PLAIN = 0,     /* FP32 FMAs on the vector ALUs                       */
    SRMRA_FP32_MFMA = 1,      /* FP32 matrix cores (v_mfma_f32_32x32x2 / 16x16x4)   */
    SRMRA_BF16_SPLIT3 = 2,    /* BF16 matrix cores, operands split v = hi + lo,
                                 products hi*hi + hi*lo + lo*hi, FP32 accumulate;
                                 every supported L_low (at 8 and 12 the score
                                 maps of 8 observations and 4 or 8 components
                                 are packed into 32x32 tiles)                       */
    SRMRA_BF16_SPLIT4 = 3,    /* as SRMRA_BF16_SPLIT3 plus the lo*lo product        */
    SRMRA_FP32_FFT = 4        /* FFT route: both contractions as products of 2-D
                                 DFTs of the L_low grid (FP32 transforms, FP64 sums
                                 and inverse); L_low in {8, 12, 16, 24, 32, 48, 64}
                                 (powers of two; 3 * 2^m with a radix-3 step);
                                 single-problem calls, and the classes of a plan
                                 a tuning entry sends here (not a plan's own
                                 precision)                                         */
} srmra_precision;

/* Human-readable text of a status code (static storage). */
const char* srmra_status_string(int status);

/* Library version string (static storage). */
const char* srmra_version(void);

/* Bytes of device workspace srmra_em_step needs for this shape/precision
 * (0 if the shape is unsupported).  Workspace content need not be initialised
 * and is not preserved between calls. */
size_t srmra_em_step_workspace_bytes(int64_t N, int L_low, int K, int precision);

/* Passes over the observation stack that one step makes for this shape and
 * precision: 2 (score / log-sum-exp pass, then the posterior / back-projection
 * pass that recomputes the scores) or 1 (SRMRA_FP32_MFMA when all K^2
 * polyphase components of an observation fit in one workgroup: the
 * log-sum-exp of eq. weights_EM completes inside the workgroup and the scores
 * are computed once).  Returns a negative srmra_status for an unsupported
 * shape or precision.  Host-only; enqueues nothing. */
int srmra_em_step_passes(int64_t N, int L_low, int K, int precision);

/* One EM step (see top of file).  y, x, log_rho are read; x_new, rho_new,
 * loglik are written.  x_new must not alias x; outputs must not alias inputs.
 * sigma > 0 and finite (the known noise standard deviation, Sec. 1).
 * `workspace` must be 256-byte aligned and hold
 * srmra_em_step_workspace_bytes(N, L_low, K, precision) bytes.  The per-job
 * preparation (below, with centring) runs inside the call.
 * Returns SRMRA_OK or an error code; see the execution model above. */
int srmra_em_step(const float* y, int64_t N, int L_low, int K,
                  const float* x, const float* log_rho, float sigma,
                  float* x_new, float* rho_new, double* loglik,
                  int precision, void* workspace, size_t workspace_bytes,
                  hipStream_t stream);

/* Allocation-free form of srmra_em_step, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as srmra_em_step
 * without the workspace: the step's workspace is a fixed array of
 * SRMRA_SCRATCH_BYTES bytes of device memory inside the library, one per GPU,
 * held until the process ends.  Returns SRMRA_ESCRATCH, with nothing
 * enqueued, when srmra_em_step_workspace_bytes(N, L_low, K, precision)
 * exceeds SRMRA_SCRATCH_BYTES (every FP32 form up to N = 200000 at
 * L_low 32, K 4; the BF16 split and FFT forms, whose workspace holds the
 * prepared observations, up to a few thousand observations at L_low 32).
 * All calls on one GPU share its single array: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.  The
 * step writes every part of the array it later reads, so nothing carries over
 * between calls.  The first call on a device resolves that device's address
 * of the array.  Results are bitwise those of srmra_em_step. */
#define SRMRA_SCRATCH_BYTES ((size_t)64 << 20)
int srmra_em_step_noalloc(const float* y, int64_t N, int L_low, int K,
                          const float* x, const float* log_rho, float sigma,
                          float* x_new, float* rho_new, double* loglik,
                          int precision, hipStream_t stream);

/* Per-job work that does not depend on theta: the intensity offset mu (the
 * mean of all observation pixels, FP64, rounded to FP32), the per-observation
 * squared norms ||y_i - mu||^2 in FP64, and for the BF16 split forms the hi/lo
 * BF16 planes of y - mu.  The step then works on (y - mu, x - mu) and adds mu
 * back to x': the model of eq. model_1 is invariant under a common offset of
 * y and x (x' shifts by mu; rho', the posterior and the log-likelihood of
 * eq. likelihood_EM are unchanged), and centring keeps the score magnitudes,
 * hence the rounding of the contractions, small for data with a large mean
 * (images in [0, 1]).
 * `prep` (256-byte aligned) must hold srmra_prepared_bytes(...) bytes; it is
 * then passed unchanged to srmra_em_step_prepared for every iteration of the
 * job.  y must stay alive and unchanged while `prep` is used.
 * srmra_prepare_observations centres; srmra_prepare_observations_ex takes
 * `centre` = 1 (centre) or 0 (mu = 0: the step works on y and x as given). */
size_t srmra_prepared_bytes(int64_t N, int L_low, int K, int precision);
int srmra_prepare_observations(const float* y, int64_t N, int L_low, int K,
                               int precision, void* prep, size_t prep_bytes,
                               hipStream_t stream);
int srmra_prepare_observations_ex(const float* y, int64_t N, int L_low, int K,
                                  int precision, int centre, void* prep,
                                  size_t prep_bytes, hipStream_t stream);

/* Same as srmra_em_step, with the per-job work taken from `prep` (made by
 * srmra_prepare_observations for the same y, N, L_low, K and precision).
 * If log_rho_new is not NULL it receives log(rho_new) (float [2][L_high]), the
 * log-prior input of the next iteration. */
int srmra_em_step_prepared(const float* y, const void* prep, size_t prep_bytes,
                           int64_t N, int L_low, int K,
                           const float* x, const float* log_rho, float sigma,
                           float* x_new, float* rho_new, float* log_rho_new, double* loglik,
                           int precision, void* workspace, size_t workspace_bytes,
                           hipStream_t stream);

/* Diagnostics for parity tests (prep may be NULL): per-observation log-likelihood terms
 * ll_i = log sum_s rho[s] exp(-||y_i - P R_s x||^2 / 2 sigma^2)  (float [N]),
 * and the FP64 sufficient statistics of the M-step: b [L_high][L_high] (the
 * right-hand side of eq. x_EM) and c [L_high][L_high] (c[s1][s2] =
 * sum_i w^{i,s}).  Any of the three output pointers may be NULL.  Same
 * argument rules as srmra_em_step_prepared; the step's regular outputs are
 * also written. */
int srmra_em_step_debug(const float* y, const void* prep, size_t prep_bytes,
                        int64_t N, int L_low, int K,
                        const float* x, const float* log_rho, float sigma,
                        float* x_new, float* rho_new, float* log_rho_new, double* loglik,
                        float* ll_obs, double* b_out, double* c_out,
                        int precision, void* workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* Same as srmra_em_step_prepared, and records six caller-created HIP events on
 * `stream` at the phase boundaries of the step: events[0] before the packing
 * of x, [1] before the score / log-sum-exp pass, [2] after it, [3] before the
 * posterior / back-projection pass, [4] after it, [5] after the M-step
 * finalisation.  For measurement (hipEventElapsedTime between them). */
int srmra_em_step_profiled(const float* y, const void* prep, size_t prep_bytes,
                           int64_t N, int L_low, int K,
                           const float* x, const float* log_rho, float sigma,
                           float* x_new, float* rho_new, float* log_rho_new, double* loglik,
                           int precision, void* workspace, size_t workspace_bytes,
                           hipStream_t stream, hipEvent_t* events);

/* ---------------------------------------------------------------------------
 * Batched form: many independent instances of uneven (L_high, K, N, sigma),
 * one EM step of every instance per execution, with one persistent launch per
 * pass over a work list of (instance, observation chunk, component group)
 * items sorted by cost and handed out by an atomic counter.  Each instance is
 * partitioned by a rule that depends only on its own shape and runs the same
 * device code as when it is alone in a plan, so its result is bitwise the
 * same alone and in any mix.  (The partition differs from srmra_em_step's, so
 * plan and single-step results agree to rounding, not bitwise.)
 *
 * Iterates ping-pong: execution number e (0-based since the last upload or
 * srmra_plan_set_iterate) reads (x, log_rho) and writes (x_new, log_rho_new)
 * when e is even, and the reverse when e is odd; rho_new and loglik are
 * written every time.  After an even number of executions the newest iterate
 * is in x / log_rho.
 */
typedef struct srmra_problem {
    const float* y;          /* device [N][L_low][L_low], 16-byte aligned           */
    const void* prep;        /* device, srmra_prepare_observations(y, ...) made with
                                srmra_plan_form(precision, L_low)                  */
    size_t prep_bytes;
    int64_t N;
    int L_low, K;
    const float* x;          /* device [L_high][L_high]  (iterate buffer A)         */
    const float* log_rho;    /* device [2][L_high]       (iterate buffer A)         */
    float sigma;
    float* x_new;            /* device [L_high][L_high]  (iterate buffer B)         */
    float* rho_new;          /* device [2][L_high]       (output)                   */
    float* log_rho_new;      /* device [2][L_high]       (iterate buffer B, required) */
    double* loglik;          /* device [1]               (output)                   */
} srmra_problem;

typedef struct srmra_plan srmra_plan;

/* The precision an instance of this L_low runs in within a plan of the given
 * precision (without a tuning entry: the plan's own; SRMRA_FP32_FFT is not a
 * plan precision).  Returns -1 for unsupported arguments. */
int srmra_plan_form(int precision, int L_low);

/* Build a plan (host only, no device work).  `probs` is copied.  On success
 * *plan is set and *workspace_bytes receives the device workspace size that
 * srmra_plan_upload / srmra_plan_execute need.  Returns SRMRA_OK or an error.
 * A plan with more than one (form, L_low) class also owns two helper streams
 * (default priority, non-blocking) and six events, created here on the
 * current device and released by srmra_plan_destroy: srmra_plan_execute forks
 * the classes of each pass onto them and joins them back to the caller's
 * stream (graph-capturable), so the plan must be executed on that device.
 * If they cannot be created the classes run one after another instead.
 * srmra_plan_upload also gives the plan one event and a pinned host staging
 * buffer (hipHostMalloc, host memory), released by srmra_plan_destroy. */
int srmra_plan_create(const srmra_problem* probs, int count, int precision,
                      srmra_plan** plan, size_t* workspace_bytes);

/* Block layouts a tuning entry may ask for (`tile`; 0 keeps the default of
 * the form and shape):
 * - BF16 split, L_low 8 and 12: SRMRA_TILE_TWO_PASS (scores recomputed by a
 *   second pass; the default is the single pass while the K^2 components fit
 *   in four blocks of 4 (L_low 8) or 8 (L_low 12));
 * - BF16 split, L_low 16: 1, 2 or 4 -- the component slots WC of a workgroup
 *   (32 / WC observations x 4 WC components; the default takes WC from K^2);
 * - BF16 split, L_low 24 and 32: SRMRA_TILE_FUSED_8OBS (single pass, 8
 *   observations x 4 components per 256-thread workgroup, K^2 <= 4; the
 *   default there), SRMRA_TILE_FUSED_4OBS (single pass, 4 observations x 16
 *   components per 512-thread workgroup, K^2 <= 16; the default for
 *   4 < K^2 <= 16), SRMRA_TILE_TWO_PASS (one 32x32 tile per score map, the
 *   scores recomputed by a second pass);
 * - BF16 split, L_low 48: SRMRA_TILE_16X16 (single pass on 3 x 3 tiles of
 *   16x16 per score map, K^2 <= 4; the default there), SRMRA_TILE_TWO_PASS
 *   (2 x 2 tiles of 32x32, two passes);
 * - FP32 MFMA where its default is the single pass: SRMRA_TILE_TWO_PASS.
 * Any other (form, L_low, K, tile) is SRMRA_EINVAL. */
#define SRMRA_TILE_TWO_PASS 8
#define SRMRA_TILE_FUSED_8OBS 16
#define SRMRA_TILE_FUSED_4OBS 32
#define SRMRA_TILE_16X16 64

/* One entry of a tuning table for srmra_plan_create_tuned (the project's
 * autotuner, paper_2204_04754_amd/autotune.py, measures and writes these).
 * Problems with this (L_low, K) in a plan of precision `precision` run in
 * precision `form` -- the plan's own precision, SRMRA_FP32_MFMA in a BF16
 * split plan, or SRMRA_FP32_FFT (the FFT route, any plan, at the L_low it
 * covers) -- with `item_obs` observations per work item
 * (rounded up to the form's observation tile; 0 keeps the default of about
 * 2^28 multiply-adds per item -- for the FFT route about 2^28 flop of its
 * transforms -- smaller, down to 2^24, where that leaves the problem fewer
 * than 128 items per component group), and with the block layout `tile` (see
 * SRMRA_TILE_* above; 0 keeps the default).  Entries of another precision are
 * ignored; the first matching entry wins.  A problem's result depends on its
 * own entry only (form, partition and tile), never on the rest of the plan. */
typedef struct srmra_tuning {
    int precision;
    int L_low, K;
    int form;
    int64_t item_obs;
    int tile;
} srmra_tuning;

/* srmra_plan_create with a tuning table (`table` may be NULL when n_table is
 * 0, which is srmra_plan_create).  SRMRA_EINVAL for a negative item_obs, a
 * tile the entry's form, L_low and K do not offer, or a form the plan's
 * precision does not allow;
 * SRMRA_EUNSUPPORTED for an FFT entry at an L_low the FFT route does not
 * cover.  The prepared buffer
 * of every problem must suit the form it runs in (a BF16 split preparation
 * also serves SRMRA_FP32_MFMA; the FFT route needs an SRMRA_FP32_FFT
 * preparation, which holds the observations' DFTs); SRMRA_EWORKSPACE if it is
 * smaller than that form's preparation. */
int srmra_plan_create_tuned(const srmra_problem* probs, int count, int precision,
                            const srmra_tuning* table, int n_table,
                            srmra_plan** plan, size_t* workspace_bytes);

/* Default observations per work item of a problem run in `form_precision`
 * (the base the autotuner scales); negative srmra_status on error. */
int64_t srmra_plan_default_item_obs(int64_t N, int L_low, int K, int form_precision);

/* Replace the iterate pointers of problem `index` (shape fields unchanged);
 * resets the ping-pong parity and requires a new upload. */
int srmra_plan_set_iterate(srmra_plan* plan, int index, const float* x,
                           const float* log_rho, float* x_new, float* rho_new,
                           float* log_rho_new);

/* Copy the plan's device descriptors and work lists into `workspace`: they are
 * written into a pinned host staging buffer that the plan owns and copied with
 * hipMemcpyAsync on `stream`; the call does not wait for the copies (a later
 * upload of the same plan, or srmra_plan_destroy, waits for them before
 * reusing or freeing the staging buffer).  Call it outside graph capture.
 * Resets the ping-pong parity. */
int srmra_plan_upload(srmra_plan* plan, void* workspace, size_t workspace_bytes,
                      hipStream_t stream);

/* Enqueue one EM step of every instance on `stream` (kernels only once the
 * plan is uploaded to this workspace; otherwise it uploads first).  After an
 * upload it is graph-capturable: a captured sequence of T executions replays
 * T EM iterations with the ping-pong order fixed at capture time. */
int srmra_plan_execute(srmra_plan* plan, void* workspace, size_t workspace_bytes,
                       hipStream_t stream);

/* ------------------------------------------------------------------------
 * Projection step of the projected EM (Alg. 2): x_out = D(x_in, s) with s
 * read from the device scalar *sigma_state, then *sigma_state = s * decay in
 * FP32 (eq. decaying_function: sigma_1 = 1, decay = 2^(-1/10)).  The
 * denoiser D (BM3D in the paper) is a circular Gaussian blur of standard
 * deviation s pixels of the L_high x L_high grid: taps k in [-R, R] with
 * R = min(floor(4 s + 1/2), L_high), weights exp(-k^2 / 2 s^2) normalised to
 * sum 1, applied along axis 0 and then axis 1 with circular boundary; s below
 * 1/8, not positive or not finite gives R = 0 (the identity).
 * x_in, x_out: device [L_high][L_high] (x_out may equal x_in); sigma_state:
 * device float, read and updated in stream order; workspace: 256-byte
 * aligned, srmra_project_workspace_bytes(L_high) bytes, content not
 * preserved.  L_high in [1, 4096], decay > 0 and finite, else SRMRA_EINVAL.
 * Three kernel launches, no host synchronisation: graph-capturable. */
size_t srmra_project_workspace_bytes(int L_high);
int srmra_project_gaussian(const float* x_in, float* x_out, int L_high,
                           float* sigma_state, float decay, void* workspace,
                           size_t workspace_bytes, hipStream_t stream);

/* Batched forward 2-D DFT of real L x L images (the FFT route's transform):
 * out[i][k1][k2] = sum_n in[i][n1][n2] exp(-2 pi i (k1 n1 + k2 n2) / L), FP32
 * complex (interleaved re, im).  in: device [count][L][L] float; out: device
 * [count][L][L] float2.  L in {8, 12, 16, 24, 32, 48, 64}, count >= 1, else
 * SRMRA_EINVAL. */
int srmra_dft2(const float* in, int64_t count, int L, void* out, hipStream_t stream);

/* Empirical moments of the observations (eq. empiric_MOM, the method of
 * moments' summary of the data): m1[l] = (1/N) sum_i y_i[l] and
 * m2[l][l'] = (1/N) sum_i y_i[l] y_i[l'] with l = n1 L_low + n2 (row-major
 * pixel index), m2 symmetric of size L_low^2 x L_low^2.  One pass over y on
 * FP32 matrix cores, per-chunk FP32 partials summed in FP64 in a fixed order
 * (deterministic).  y: device [N][L_low][L_low], 16-byte aligned; m1, m2:
 * device doubles; workspace: srmra_moments_workspace_bytes(N, L_low) bytes,
 * 256-byte aligned.  L_low even in [2, 64], N >= 1, else SRMRA_EINVAL. */
size_t srmra_moments_workspace_bytes(int64_t N, int L_low);
int srmra_moments(const float* y, int64_t N, int L_low, double* m1, double* m2,
                  void* workspace, size_t workspace_bytes, hipStream_t stream);

/* The paper's reconstruction error (Sec. 5): *err = min over circular 2-D
 * translations s of ||R_s x_hat - x_ref||_F / ||x_ref||_F, (R_s v)[m] =
 * v[m - s], every distance summed directly in FP64; best_shift (device int[2],
 * may be NULL) receives the minimising (s1, s2), the lowest s1 * L_high + s2
 * on ties.  x_hat, x_ref: device [L_high][L_high]; err: device double;
 * workspace: srmra_shift_error_workspace_bytes(L_high) bytes, 256-byte
 * aligned.  L_high in [1, 512] (the work grows as L_high^4). */
size_t srmra_shift_error_workspace_bytes(int L_high);
int srmra_shift_error(const float* x_hat, const float* x_ref, int L_high, double* err,
                      int* best_shift, void* workspace, size_t workspace_bytes,
                      hipStream_t stream);

/* Parity of the next execution (0: reads x/log_rho), -1 for NULL. */
int srmra_plan_parity(const srmra_plan* plan);

void srmra_plan_destroy(srmra_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* SRMRA_H */
