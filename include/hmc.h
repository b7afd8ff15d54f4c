/*
 * hmc.h - C-ABI of the GPU-resident Hamiltonian Monte Carlo library for Bayesian
 * multinomial (softmax) regression on AMD Instinct MI355X (gfx950).
 *
 * Model (Beam, Ghosh and Doyle, "Fast Hamiltonian Monte Carlo Using GPU Computing",
 * Section 2.1): observations x_i in R^p with labels y_i in {0..K-1}; coefficients
 * B = [beta_1 .. beta_K] (p x K); class probabilities psi_ik = softmax_k(x_i^T B)
 * (equation (softmax)); log-posterior kernel
 *     log K(B) = sum_i log psi_{i,y_i} + sum_{free jk} log prior(beta_jk)
 * (equations (loglike), (logkernel), (logkernelGPU)); its gradient
 *     X^T (Y - psi(X B)) + prior'(B), masked on the pinned class
 * (equation (gradient); Appendix equations (lastline), (fullgrad) and the mask M).
 * The sampler is the leapfrog integrator of Section 1.1 (equations (hmc1)-(hmc3)) and
 * the Metropolis test of equation (accept), with the kinetic energy taken as
 * 0.5 * eta.eta and the optional annealed acceptance of Section 3.2.
 *
 * Conventions shared by every entry point:
 *  - Every data pointer is a DEVICE pointer, owned by the caller and never freed or
 *    retained by the library beyond the call's stream work.
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL = the
 *    default stream) and never synchronise the host. Scalars the library produces are
 *    written to device memory.
 *  - The library allocates no device memory. Scratch space is the caller's workspace
 *    `ws` of at least hmc_workspace_bytes() bytes (256-byte aligned).
 *  - Argument, shape and format errors are detected on the host before anything is
 *    enqueued; the call then returns a negative hmc_status and hmc_last_error() holds a
 *    thread-local message. A HIP launch failure returns HMC_ERR_HIP.
 *  - Numerical failure is not an API error: a non-finite proposal energy counts as a
 *    rejected, divergent transition.
 *  - Calls that share a workspace must not overlap in time (same stream, or ordered).
 */
#ifndef HMC_MI355X_H
#define HMC_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HMC_OK = 0,
  HMC_ERR_ARG = -1,         /* null pointer, non-finite or out-of-range scalar        */
  HMC_ERR_SHAPE = -2,       /* n, p, K, ldx inconsistent or beyond the supported range */
  HMC_ERR_DTYPE = -3,       /* unknown X format or prior                               */
  HMC_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed              */
  HMC_ERR_WORKSPACE = -5,   /* workspace missing, too small or misaligned              */
  HMC_ERR_UNSUPPORTED = -6  /* valid request this build does not implement             */
} hmc_status;

/* Storage format of X. The state (B, eta, G, samples) is float64 for HMC_X_F64 and
 * float32 for every other format.
 *
 * The two bfloat16 formats are the split-precision form: X is held as hi = bf16(X) and
 * lo = bf16(X - hi) (round to nearest even, see hmc_split_bf16), and every product of X
 * with an FP32 operand A = A_hi + A_lo (the coefficients, the residuals Y - P) is taken
 * as hi*A_hi + hi*A_lo + lo*A_hi on the BF16 matrix cores with FP32 accumulation; the
 * log-sum-exp, the log-likelihood and the Hamiltonian are formed in FP64. The paper
 * computes in one precision; this form trades about 1e-5 relative gradient error for
 * half the bytes of FP32 X per element pair (hi + lo = 4 bytes, hi only = 2 bytes). */
typedef enum {
  HMC_X_F64 = 0,            /* X float64, row-major n x p, row pitch ldx elements      */
  HMC_X_F32 = 1,            /* X float32, row-major n x p, row pitch ldx elements      */
  HMC_X_BF16_HILO = 2,      /* X = hi plane, X_lo = lo plane: bf16 row-major n x p,
                               row pitch ldx elements (a multiple of 8; a multiple of
                               64 streams fastest), both planes 16-byte aligned       */
  HMC_X_BF16 = 3            /* hi plane only (X_lo NULL); the device then sees
                               X = hi exactly                                         */
} hmc_xfmt;

typedef enum {
  HMC_PRIOR_GAUSS = 0,      /* beta ~ N(0, s^2): log prior -beta^2/(2 s^2)             */
  HMC_PRIOR_CAUCHY = 1      /* beta ~ Cauchy(0, s): log prior -log(1 + (beta/s)^2);
                               s = 1 is the paper's choice (Section 2.1)               */
} hmc_prior;

/* The per-row likelihood. The paper's model is the multinomial logit; its Discussion
 * notes that the approach carries over to any model whose likelihood and gradient are
 * matrix products, and the Poisson and probit regressions take the same two contractions
 * with a different per-row term:
 *   HMC_LINK_SOFTMAX  multinomial logit (Section 2.1): y_i in [0, K) is a class label,
 *                     log-likelihood sum_i z_{i,y_i} - log sum_k exp z_ik, residual
 *                     Y - softmax(Z); 2 <= K <= 64
 *   HMC_LINK_POISSON  y_i >= 0 is a count, y_i ~ Poisson(exp(z_i)) with z = X beta:
 *                     K = 1, pin_last_class = 0, log-likelihood sum_i y_i z_i - exp(z_i)
 *                     (the constant -log y_i! dropped), residual y - exp(z); FP64 and
 *                     FP32 X only (HMC_ERR_UNSUPPORTED for the bfloat16 formats and the
 *                     batched calls)
 *   HMC_LINK_PROBIT   binary response, P(y_i = 1) = Phi(z_i) with Phi the standard normal
 *                     distribution function; y_i = 1 is a success and any other label a
 *                     failure; with s_i = +1 for a success and -1 otherwise:
 *                     log-likelihood sum_i log Phi(s_i z_i), residual s phi(z) / Phi(s z)
 *                     (phi the normal density); K = 1, pin_last_class = 0, FP64 and FP32
 *                     X only, as for the Poisson link */
typedef enum {
  HMC_LINK_SOFTMAX = 0,
  HMC_LINK_POISSON = 1,
  HMC_LINK_PROBIT = 2
} hmc_link;

/* Launch decomposition of the single-problem gradient pass. All zero (the default) selects
 * the library's built-in rule; hmc_autotune measures candidates on the device and returns
 * the fastest. The workspace size depends on it (hmc_workspace_bytes reads it from the
 * problem), so a workspace is sized for the tuning it is used with.
 *   path            0: the rule; 1: row tile (X streamed once; FP32/FP64 X with p within
 *                   the tile variants' width); 2: wide-p (column-chunked logits, then a
 *                   column-owner gradient; FP32/FP64 X); 3: split-precision pass (bf16 X;
 *                   the only path for the bfloat16 formats)
 *   waves, mb       row tile: waves per workgroup (8 or 16) and 16-column blocks per wave;
 *                   waves * mb * 16 >= p; both 0 for the rule's variant
 *   grid            row tile: workgroups (1..4096; one partial gradient each); wide-p: row
 *                   tiles of the logits grid (1..65535); split-precision: logits workgroups
 *                   (1..65536); 0 for the rule
 *   rows_per_slice  wide-p: rows per gradient row slice, a multiple of 64 (one slice when
 *                   >= n; the gradient kernel then applies the leapfrog update itself);
 *                   split-precision: a multiple of 32; 0 for the rule
 * With path 0 the other fields must be 0. Invalid values give HMC_ERR_ARG; a path that
 * cannot run the problem gives HMC_ERR_UNSUPPORTED. */
typedef struct {
  int32_t path;
  int32_t waves, mb;
  int32_t grid;
  int32_t rows_per_slice;
} hmc_tuning;

/* One regression problem: the persistent device objects of Section 2.1 (X and the
 * labels; Y is their one-hot expansion, never materialised). */
typedef struct {
  int64_t n;                /* observations, n >= 1                                    */
  int64_t p;                /* predictors, 1 <= p <= hmc_max_p(xfmt, K)                */
  int32_t K;                /* classes, 2 <= K <= 64 (1 for the Poisson and probit
                               links)                                                 */
  int32_t xfmt;             /* hmc_xfmt                                                */
  const void* X;            /* device, n x p row-major, element (i, j) at X[i*ldx + j];
                               the padding elements (columns p .. ldx-1) are never used,
                               whatever they hold. FP32/FP64: (n-1)*ldx + p elements
                               are read; bf16 planes must hold n*ldx elements (the
                               kernels read whole 16-byte pieces up to the pitch)      */
  const void* X_lo;         /* HMC_X_BF16_HILO: device lo plane (layout of X); NULL
                               for every other format                                 */
  int64_t ldx;              /* row pitch in elements, ldx >= p; at most 2^23 - 1
                               (FP64), 2^24 - 1 (FP32) or 2^23 - 8 (bf16), the pitch
                               whose in-kernel 32-bit byte offsets cannot wrap
                               (HMC_ERR_UNSUPPORTED beyond)                           */
  const int32_t* y;         /* device, n labels in [0, K) (counts >= 0 for the Poisson
                               link, 1 = success for the probit link); other values
                               are undefined                                          */
  int32_t prior;            /* hmc_prior                                               */
  double prior_scale;       /* s > 0: Gaussian standard deviation or Cauchy scale      */
  int32_t pin_last_class;   /* 1: beta_K = 0 for identifiability (Section 2.1,
                               Appendix): column K-1 of B, eta and G stays zero and its
                               logit is the constant 0. The kernels read that column of
                               a caller's B as zero whatever it holds, so log K and G
                               are those of the pinned model. 0: all K columns free   */
  int32_t link;             /* hmc_link; 0 (the multinomial logit) when zero-filled     */
  hmc_tuning tuning;        /* launch decomposition; all zero for the built-in rule     */
} hmc_problem;

/* Largest p this build handles for a format and class count (0 for an unknown format
 * or K outside [1, 64]; K = 1 is the single coefficient column of the Poisson and probit
 * links): min(2^30 / K, the largest ldx of the format). Independently of p, n is bounded
 * where per-row work buffers are addressed with 32-bit offsets: on the wide-p path
 * (p beyond the row tile) n * 16 * ceil(K / 16) * (state bytes) < 2^32, and for the
 * bfloat16 formats (n + 128) * 64 * ceil(K / 16) < 2^32 (with `chains` in place of
 * ceil(K / 16) in the batched calls); larger n gives HMC_ERR_UNSUPPORTED. */
int64_t hmc_max_p(int32_t xfmt, int32_t K);

/* Workspace bytes needed by every call below on `prob` (with its tuning). Writes *bytes. */
hmc_status hmc_workspace_bytes(const hmc_problem* prob, size_t* bytes);

/* Autotuner of the single-problem gradient pass: the candidate decompositions of `prob`'s
 * format and shape (row-tile variants and workgroup counts, the wide-p path with its logits
 * grid and row slices, for FP32/FP64 X; logits workgroups and gradient row slices of the
 * split-precision pass), each timed over repeated gradient evaluations at B with HIP events
 * on `stream`; writes the fastest to *out and its mean time per evaluation in microseconds
 * to *best_us (nullable). prob->tuning is ignored. ws must hold
 * hmc_autotune_workspace_bytes(prob) bytes (the largest candidate's workspace); G and
 * logpost receive the gradient and log K at B. Waits for the stream (host-synchronous). */
hmc_status hmc_autotune_workspace_bytes(const hmc_problem* prob, size_t* bytes);
hmc_status hmc_autotune(const hmc_problem* prob, const void* B, double* logpost, void* G, void* ws,
                        size_t ws_bytes, void* stream, hmc_tuning* out, double* best_us);

/* log K(B) and its gradient at B (equations (logkernel) and (gradient)).
 *   B        device, p x K row-major, state dtype; with pin_last_class = 1 column K-1 is
 *            read as zero (beta_K = 0), whatever the buffer holds there
 *   logpost  device, one double: log K(B) without additive constants
 *   G        device, p x K row-major, state dtype: the masked gradient
 * On the row-tile path one fused pass streams X once (the wide-p and split-precision
 * paths read it twice: logits, then the gradient); the gradient is reduced in a fixed
 * order, so repeated calls give bit-identical results. */
hmc_status hmc_logpost_grad(const hmc_problem* prob, const void* B, double* logpost, void* G,
                            void* ws, size_t ws_bytes, void* stream);

/* hmc_logpost_grad without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation). Same kernels, same results bit for bit. The workspace is a built-in device
 * array of 32 MiB that each GPU the library runs on holds from module load until the
 * process ends; this call allocates and frees nothing. Its first call on a device looks up
 * that device's copy of the array (hipGetSymbolAddress). A problem whose workspace
 * (hmc_workspace_bytes) exceeds 32 MiB is refused with HMC_ERR_WORKSPACE. All calls on one
 * GPU share the array: calls that may overlap in time on one GPU (different streams or
 * threads without ordering) race and must not be issued. */
hmc_status hmc_logpost_grad_noalloc(const hmc_problem* prob, const void* B, double* logpost,
                                    void* G, void* stream);

/* L leapfrog updates in place (Section 1.1, equations (hmc1)-(hmc3), applied L times in
 * the printed order: half kick, full position step, gradient, half kick).
 *   B, eta   device, p x K state dtype, updated in place (pinned columns must be zero)
 *   G        device, p x K: on entry the gradient at B, on exit the gradient at the
 *            final B
 *   logpost  device double: on exit log K at the final B
 *   eps      step size (finite, non-zero); L >= 1 gradient evaluations */
hmc_status hmc_leapfrog(const hmc_problem* prob, void* B, void* eta, void* G, double* logpost,
                        double eps, int32_t L, void* ws, size_t ws_bytes, void* stream);

/* Sampler arguments. Iteration t of this call has global index first_iter + t. */
typedef struct {
  double eps;                       /* leapfrog step size                              */
  int32_t L;                        /* leapfrog steps per iteration, >= 1              */
  int32_t n_iter;                   /* iterations, >= 1                                */
  int32_t first_iter;               /* global index of the first iteration (resume)    */
  int32_t chain;                    /* chain id (Philox stream selector)               */
  uint64_t seed;                    /* Philox4x32-10 key                               */
  const double* replay_normals;     /* device [n_iter][p][K] standard normals, or NULL
                                       to draw momenta from Philox4x32-10              */
  const double* replay_uniforms;    /* device [n_iter] uniforms in (0,1), or NULL for
                                       Philox                                          */
  const double* inv_temperature;    /* device [n_iter] values 1/T_t of the annealed
                                       acceptance (Section 3.2), or NULL for 1         */
  void* samples;                    /* device [n_iter][p][K] state dtype, or NULL      */
  int32_t* accepted;                /* device [n_iter], or NULL                        */
  double* H;                        /* device [n_iter][2] = (H0, H1), or NULL          */
  int32_t* divergent;               /* device [n_iter], or NULL                        */
} hmc_sample_args;

/* n_iter HMC transitions from the state (B, G, *logpost), which must hold a position,
 * the gradient there and log K there (as left by hmc_logpost_grad or by an earlier
 * hmc_sample call). Each transition draws eta = M * xi, runs L leapfrog updates, and
 * accepts iff H1 is finite and log u < (H0 - H1) / T (equation (accept) in the log
 * domain; H = -log K + 0.5 eta.eta). On accept B, G and *logpost take the proposal.
 * Nothing returns to the host; records go to the optional device arrays. */
hmc_status hmc_sample(const hmc_problem* prob, void* B, void* G, double* logpost,
                      const hmc_sample_args* args, void* ws, size_t ws_bytes, void* stream);

/* Graph plans: one HMC iteration of hmc_sample (momentum draw, L leapfrog updates,
 * Metropolis test, records) captured once as a HIP graph and replayed, so a run of many
 * iterations costs one graph launch per iteration instead of one launch per kernel. The
 * state, arguments and workspace given at creation are baked into the graph and must stay
 * valid until hmc_plan_destroy. The iteration index and the record slot come from a
 * counter in the workspace, set to args->first_iter before the plan's first launch and
 * advanced by every replay, so consecutive hmc_plan_launch calls continue one chain (the
 * draws equal those of a single hmc_sample call of the combined length). When replay
 * inputs, annealing temperatures or records are given, the total launched iterations may
 * not exceed args->n_iter. A plan must not be launched concurrently from two threads, and
 * nothing else may use its workspace while it runs. */
typedef struct hmc_plan hmc_plan;
hmc_status hmc_plan_create(hmc_plan** plan, const hmc_problem* prob, void* B, void* G,
                           double* logpost, const hmc_sample_args* args, void* ws,
                           size_t ws_bytes, void* stream);
hmc_status hmc_plan_launch(hmc_plan* plan, int32_t n_iter, void* stream);
hmc_status hmc_plan_destroy(hmc_plan* plan);

/* ------------------------------------------------------------------------------------
 * Batched form: many independent problems (bf16 X formats, 2 <= K <= 64) with `chains`
 * chains each (1, 2 or 4), every phase of every leapfrog update run for all of them in one
 * persistent launch. The chains of a problem share each pass over its X: their
 * coefficient blocks are stacked as separate groups of 16-class blocks of one contraction,
 * with one softmax per row and chain. Every chain of a batch takes ceil(K_max / 16) blocks
 * (K_max the batch's largest K), and chains x blocks may not exceed 4 (K_max <= 16 with
 * up to 4 chains, <= 32 with up to 2, <= 64 with 1; HMC_ERR_SHAPE beyond). Per-chain
 * arithmetic is that of the single-problem bf16 path.
 *
 * State layout: B[b] and G[b] (host arrays of n_prob device pointers) point to
 * [chains][p_b][K_b] float32 blocks; logpost is a device array [n_prob][chains] of
 * doubles. Chain c of problem b has global index b * chains + c: its Philox stream and
 * its column in the record arrays.
 * ------------------------------------------------------------------------------------ */

/* Work decomposition of the batched kernels: rows per gradient row slice (a multiple of
 * 32, >= 1024) and persistent workgroups of the logits and gradient kernels (64..65536);
 * 0 selects the default (4096 rows, 2048 workgroups). hmc_batch_autotune measures a set
 * of candidates on the device and returns the fastest. */
typedef struct {
  int32_t rows_per_slice;
  int32_t grid;
} hmc_batch_tuning;

typedef struct {
  const double* eps;                /* host [n_prob] leapfrog step sizes               */
  int32_t L;                        /* leapfrog steps per iteration, >= 1              */
  int32_t n_iter;                   /* iterations, >= 1                                */
  int32_t first_iter;               /* global index of the first iteration             */
  uint64_t seed;                    /* Philox4x32-10 key (momenta and uniforms)        */
  hmc_batch_tuning tuning;          /* {0, 0} for the defaults                         */
  void* const* samples;             /* host [n_prob] of device [n_iter][chains][p][K]
                                       float32 (entries may be NULL), or NULL          */
  double* const* moments;           /* host [n_prob] of device [2][chains][p][K]:
                                       running sum and sum of squares of the chain
                                       states after each iteration, added to (caller
                                       zeroes them), or NULL                           */
  int32_t* accepted;                /* device [n_iter][n_prob * chains], or NULL       */
  double* H;                        /* device [n_iter][n_prob * chains][2], or NULL    */
  int32_t* divergent;               /* device [n_iter][n_prob * chains], or NULL       */
  const double* const* replay_normals;  /* host [n_prob] of device [n_iter][chains][p][K]
                                       standard normals (momenta), or NULL to draw them
                                       from Philox4x32-10                              */
  const double* const* replay_uniforms; /* host [n_prob] of device [n_iter][chains]
                                       uniforms in (0,1) of the accept test, or NULL;
                                       set together with replay_normals                */
  const double* inv_temperature;    /* device [n_iter] values 1/T_t of the annealed
                                       acceptance (Section 3.2), shared by every chain,
                                       or NULL for 1                                   */
} hmc_batch_args;

/* Workspace bytes for a batch (independent of the tuning). */
hmc_status hmc_batch_workspace_bytes(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                                     size_t* bytes);

/* log K and its gradient at every chain's B (equations (logkernel) and (gradient)). */
hmc_status hmc_logpost_grad_batched(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                                    void* const* B, double* logpost, void* const* G,
                                    const hmc_batch_tuning* tune, void* ws, size_t ws_bytes,
                                    void* stream);

/* n_iter HMC transitions of every chain (as hmc_sample: Philox draws, or the replayed
 * normals and uniforms of args; the annealed acceptance of Section 3.2 when
 * args->inv_temperature is set), from states that hold B, the gradient there and log K
 * there. The problem table is uploaded with a host-to-device copy on `stream`. */
hmc_status hmc_sample_batched(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                              void* const* B, void* const* G, double* logpost,
                              const hmc_batch_args* args, void* ws, size_t ws_bytes, void* stream);

/* A graph plan of one batched iteration (see hmc_plan_create); launch and destroy it with
 * hmc_plan_launch / hmc_plan_destroy. */
hmc_status hmc_plan_create_batched(hmc_plan** plan, const hmc_problem* probs, int32_t n_prob,
                                   int32_t chains, void* const* B, void* const* G,
                                   double* logpost, const hmc_batch_args* args, void* ws,
                                   size_t ws_bytes, void* stream);

/* Autotuner: times batched gradient evaluations at the current B for each candidate
 * decomposition (rows per slice 1024..8192, 1024..16384 workgroups) and writes the
 * fastest to *out. Leaves G and logpost holding the gradient and log K at B. Waits for
 * the stream (host-synchronous). */
hmc_status hmc_batch_autotune(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                              void* const* B, void* const* G, double* logpost, void* ws,
                              size_t ws_bytes, void* stream, hmc_batch_tuning* out);

/* Split-precision encoding of X (the precision form's one-time preparation):
 *   X       device, n x p row-major, row pitch ldx, float64 (src_fmt HMC_X_F64) or
 *           float32 (HMC_X_F32)
 *   X_hi    device, n x ld_out bf16 (uint16 encodings): bf16(X), each element rounded
 *           once from its exact value to nearest even (8 significant bits, the exponent
 *           range of binary32, +-inf beyond the largest finite value)
 *   X_lo    device, same layout: bf16(X - hi), or NULL to write the hi plane only
 *   ld_out  row pitch of the planes, >= p and a multiple of 8; columns [p, ld_out) are
 *           written as zero. Both planes must be 16-byte aligned. A multiple of 64 (rows
 *           starting on 128-byte cache lines) streams fastest: the gradient pass reads each
 *           row in 256-byte column blocks, and rows that start mid-line split every block
 *           over three lines instead of two.
 * The planes can then be passed as X / X_lo of an hmc_problem with format
 * HMC_X_BF16_HILO (or HMC_X_BF16 for the hi plane alone). */
hmc_status hmc_split_bf16(const void* X, int32_t src_fmt, int64_t n, int64_t p, int64_t ldx,
                          void* X_hi, void* X_lo, int64_t ld_out, void* stream);

/* Posterior-predictive classification (Section 3.2: the class of each observation is the
 * one of highest posterior-mean probability over the recorded samples). For every row x_i
 * of prob's X:
 *   mean_prob[i][k] = (1 / n_samples) sum_s softmax_k(x_i^T B_s), accumulated in float64
 *   classes[i]      = argmax_k mean_prob[i][k] (the lowest k among exactly equal values)
 *   samples    device [n_samples][p][K], state dtype (float64 for HMC_X_F64, float32 for
 *              HMC_X_F32); with pin_last_class = 1 column K-1 is read as zero
 *   mean_prob  device [n][K] float64, or NULL; classes device [n] int32, or NULL (not both)
 * Only X, ldx, n, p, K, xfmt, pin_last_class and link of prob are used (labels may be NULL).
 * Logits and per-sample probabilities are formed in the X precision. FP64 and FP32 X with
 * the multinomial logit; a 16-row tile of X and one sample (16 p + p K elements) must fit
 * the 160 KB LDS (p <= 1575 at K = 10 in FP32), else HMC_ERR_UNSUPPORTED. */
hmc_status hmc_posterior_predictive(const hmc_problem* prob, const void* samples, int32_t n_samples,
                                    double* mean_prob, int32_t* classes, void* stream);

/* Bandwidth reference for benchmarks (not part of the sampler): `reps` passes that each
 * read every byte of `buf` once with 16-byte vector loads (2048 workgroups of 256 threads,
 * four loads in flight per thread), enqueued on `stream`; time them with events to get the
 * attainable read bandwidth of the device for a buffer of that size.
 *   buf    device, 16-byte aligned, `bytes` a positive multiple of 16
 *   sink   device array of 2048 unsigned ints, or NULL: written only on a data-dependent
 *          condition that makes the loads observable (practically never) */
hmc_status hmc_stream_read(const void* buf, size_t bytes, int32_t reps, void* sink, void* stream);

/* Kernel timing for benchmarks. Between hmc_profile_begin and hmc_profile_end, every
 * launch of the gradient pass over X (the fused pass; the split-precision, wide-p and
 * batched passes likewise) is bracketed by a pair of HIP events recorded on the launch's
 * stream, from a pool of `capacity` pairs the library creates (host-side event objects; no
 * device memory). A pass that only overwrites workspace runs `repeat` times (1..64) back to
 * back inside its pair, which spreads the cost of recording the events; the wide-p pass
 * with one row slice updates the chain state itself and always runs once. Launches beyond
 * the capacity are not timed. hmc_profile_end waits for the recorded events, writes the
 * number of timed pairs and the mean / min / max duration of one launch in microseconds
 * (each pair's time over its launches), and releases the pool. A timed run with
 * repeat > 1 does extra work, so its wall-clock time is not a throughput figure.
 * Not thread-safe: profile from one host thread. */
hmc_status hmc_profile_begin(int32_t capacity, int32_t repeat);
hmc_status hmc_profile_end(int64_t* launches, double* mean_us, double* min_us, double* max_us);

const char* hmc_status_string(hmc_status s);
const char* hmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HMC_MI355X_H */
