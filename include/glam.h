/*
 * glam.h -- C ABI of the MI355X (gfx950) l1-penalised GLAM solver.
 *
 * Model (Lund, Vincent & Hansen, arXiv:1510.03298):
 *   design X = X_3 (x) X_2 (x) X_1 (Sec. 2, eq. fivenew), X_j is n_j x p_j;
 *   linear predictor eta = H(<X_j>, Theta) = rho(X_3, rho(X_2, rho(X_1, Theta)))
 *   (Sec. 6.1, eq. eighteen; rho of App. A); gradient maps use
 *   G(<X_j>, U) = rho(X_3^T, rho(X_2^T, rho(X_1^T, U))) (eq. nineteen);
 *   PMLE theta* = argmin -l(eta(theta))/n + lambda sum_m w_m |theta_m| (eq. five,
 *   with the 1/n scale of eqs. eleven and twentyfour carried to the objective).
 *
 * Conventions shared by every entry point
 *   - Arrays are column-major, i.e. the paper's vec (App. A, eq. index): the
 *     first index runs fastest.  X_j is n_j x p_j with leading dimension n_j;
 *     Theta is p_1 x p_2 x p_3; Eta, U, Y and observation weights are
 *     n_1 x n_2 x n_3.
 *   - d = 2 and d = 3 (where an entry point takes d; the NLL entry points are
 *     d = 3).  A d = 2 model X_2 (x) X_1 runs as the d = 3 model X_2 (x) [1] (x) X_1,
 *     which keeps every array's vec layout.  Sizes are int64_t; every n_j and p_j
 *     must be >= 1.
 *   - Array pointers are DEVICE pointers owned by the caller unless stated
 *     otherwise.  The library never frees or retains them after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Return value: a glam_status code.  Size and option errors (GLAM_EINVAL) are
 *     returned before any work is enqueued; the fits' data checks (Y, obs_w,
 *     pen_w) run on the device and also return GLAM_EINVAL.  glam_last_error()
 *     then gives a message for the calling thread.
 *   - The rho and NLL entry points are asynchronous on `stream`; glam_fit_path
 *     and glam_fit_batched are synchronous (they need host control flow) and
 *     return when their results are in place.
 */
#ifndef GLAM_H
#define GLAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GLAM_OK = 0,
  GLAM_EINVAL = 1,      /* invalid argument (sizes, pointers, values, limits)      */
  GLAM_ENOMEM = 2,      /* device allocation failed                                */
  GLAM_EDEVICE = 3,     /* a HIP runtime call failed                               */
  GLAM_ENOCONV = 4,     /* a fit hit its iteration limit (path truncated)          */
  GLAM_ENONFINITE = 5   /* a non-finite gradient or objective was produced         */
} glam_status;

/* Exponential families of App. B with the links the paper's package supports (Sec. 6.4).
 * Response ranges (checked on the device, GLAM_EINVAL otherwise): Gaussian any finite y;
 * Poisson y >= 0; Binomial proportions 0 <= y <= 1 (counts out of m trials: y = count/m with
 * prior weight a = m); Gamma y > 0 (dispersion 1).  IRLS weights (eq. nine): 1, mu,
 * mu (1 - mu) and 1 respectively (Gamma-log is a non-canonical link: Fisher scoring). */
typedef enum { GLAM_GAUSSIAN = 0, GLAM_POISSON = 1, GLAM_BINOMIAL = 2, GLAM_GAMMA = 3 } glam_family;

/* Penalty J of the PMLE (Sec. 2 eq. five; Sec. 6.3, 6.4).  GLAM_PENALTY_RIDGE: J = sum_m w_m
 * theta_m^2, whose prox is the multiplicative shrinkage z / (1 + 2 delta lambda w_m) (Sec. 6.3); it has
 * no zero solution, so its lambda grid and KKT scale are the lasso's lambda_max, and the KKT
 * residual is |g_m + 2 lambda w_m theta_m|; alpha must be 0 with it. */
typedef enum { GLAM_PENALTY_LASSO = 0, GLAM_PENALTY_SCAD = 1, GLAM_PENALTY_RIDGE = 2 } glam_penalty;

/* Element type of the rho products.  F64: all FP64.  F32: FP32 inputs and
 * outputs, FP32 accumulation.  BF16: bfloat16 inputs (stored as uint16_t),
 * FP32 accumulation and FP32 outputs. */
typedef enum { GLAM_F64 = 0, GLAM_F32 = 1, GLAM_BF16 = 2 } glam_dtype;

/* Text of a status code (static storage). */
const char* glam_status_string(int status);
/* Detail message of the last failing call on this thread ("" if none). */
const char* glam_last_error(void);
/* Library version string, e.g. "glam-mi355x 0.1.0 (gfx950)". */
const char* glam_version(void);

/* Limits of the fused slab kernels: the two modes they contract in registers/LDS (modes 1
 * and 2 of the order that runs) must satisfy p_j <= GLAM_MAX_INNER_P and n_j <=
 * GLAM_MAX_INNER_N (the third is unrestricted).  The rho entry points and both fits run a
 * problem whose own order does not fit in an order that does, when one exists.
 * d = 2 (Sec. 6.4: the package fits d = 2 and d = 3): X_2 (x) X_1 is taken as the d = 3 model
 * X_2 (x) [1] (x) X_1 with a 1 x 1 middle factor, which keeps every array's vec layout; then
 * mode 1 has the limits above and mode 2 is unrestricted. */
#define GLAM_MAX_INNER_P 32
#define GLAM_MAX_INNER_N 256

/* ---------------------------------------------------------------------------
 * rho transforms (App. A; Sec. 6.1 eqs. eighteen and nineteen, c = 1)
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace the rho entry points need for these sizes/dtype (0: the sizes are
 * refused; glam_last_error says why).  When modes 1-2 of the caller's order do not fit the slab
 * kernels, the transforms run in a mode order that does (the largest remaining n last) and the
 * workspace also holds the permuted input and output (n + p elements of 8 bytes). */
size_t glam_rho_workspace_size(int d, const int64_t* n, const int64_t* p, int dtype);

/* Eta = H(<X_j>, Theta) = rho(X_3, rho(X_2, rho(X_1, Theta)))  (eq. eighteen).
 *   n, p     : host arrays of length d (d == 2 or 3).
 *   X        : host array of d device pointers; X[j] -> n_j x p_j of `dtype`.
 *   Theta    : device, p_1 x ... x p_d of `dtype`.
 *   Eta      : device, n_1 x ... x n_d; FP64 for GLAM_F64, FP32 otherwise.
 *   workspace: device, >= glam_rho_workspace_size(...) bytes, 256-byte aligned.
 * The mode products commute, so a reordered run (see glam_rho_workspace_size) gives the
 * same transform; Theta is permuted into the workspace and Eta back out of it.  When no order
 * of the modes fits the slab kernels (p_j > n_j designs, large p_j), the transform runs as three
 * tiled matrix-core GEMMs in the caller's cyclic mode order, with the intermediates in dtype
 * (the workspace holds X_j^T and two intermediates).
 * Errors: GLAM_EINVAL for d not 2 or 3, sizes < 1, NULL pointers, a bad dtype or a
 * too-small workspace; GLAM_EDEVICE for a mode with more than about 2 million entries on the
 * generic chain (its launch grid). */
int glam_rho_forward(int d, const int64_t* n, const int64_t* p, const void* const* X,
                     const void* Theta, void* Eta, int dtype, void* workspace,
                     size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): glam_rho_forward with its workspace taken from a static
 * device array of the library, GLAM_STATIC_SCRATCH_BYTES on every GPU it runs on (held until the
 * process ends); the call itself allocates nothing.  Arguments, results and the mode reordering are
 * those of glam_rho_forward; the caller still provides Theta and Eta.
 * Sharing: every call on one GPU uses that GPU's one array, so calls on a GPU must not overlap
 * (two streams, or two host threads, in flight at once race on it); calls queued one after another
 * on one stream are fine.  Nothing in the array needs to start at any value.
 * Errors: those of glam_rho_forward, GLAM_EINVAL when glam_rho_workspace_size(d, n, p, dtype)
 * exceeds GLAM_STATIC_SCRATCH_BYTES (glam_last_error says how much the sizes need), and
 * GLAM_EDEVICE if the array's device address cannot be looked up. */
#define GLAM_STATIC_SCRATCH_BYTES (32u << 20)
int glam_rho_forward_static(int d, const int64_t* n, const int64_t* p, const void* const* X,
                            const void* Theta, void* Eta, int dtype, void* stream);

/* Out = G(<X_j>, U) = rho(X_3^T, rho(X_2^T, rho(X_1^T, U)))  (eq. nineteen),
 * i.e. vec(Out) = X^T vec(U).
 *   U   : device, n_1 x n_2 x n_3 of `dtype`.
 *   Out : device, p_1 x p_2 x p_3; FP64 for GLAM_F64, FP32 otherwise.
 * Other arguments, reordering (U permuted in, Out back) and errors as glam_rho_forward. */
int glam_rho_adjoint(int d, const int64_t* n, const int64_t* p, const void* const* X,
                     const void* U, void* Out, int dtype, void* workspace,
                     size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * lambda path of the GD-PG algorithm (Sec. 3, Algorithm 1; Sec. 6.4)
 * ------------------------------------------------------------------------- */
typedef struct {
  int d;                  /* 2 or 3 (entries d.. of n, p, X are ignored)            */
  int64_t n[3], p[3];     /* mode sizes                                             */
  const double* X[3];     /* device, FP64, X[j] is n_j x p_j column-major           */
  const double* Y;        /* device, FP64 response array n_1 x n_2 x n_3            */
  const double* obs_w;    /* device, FP64 prior weights a_i >= 0 (App. B), or NULL  */
  int family;             /* glam_family                                            */
  const double* pen_w;    /* device, FP64 penalty weights w_m > 0 (length p), or NULL = 1 */
} glam_problem;

typedef struct {
  const double* lambda;   /* HOST array of nlambda strictly decreasing values, or NULL:
                             log grid lambda_max * ratio^(l/(nlambda-1))           */
  int nlambda;            /* number of models (>= 1)                                */
  double lambda_min_ratio;/* ratio of the log grid (0 < ratio <= 1)                 */
  int dtype;              /* glam_dtype of the inner rho chain (FP64 anchors always) */
  double kkt_tol;         /* target FP64 KKT residual (relative to lambda_max), e.g. 1e-6 */
  double nu;              /* step control (Sec. 6.4): 1 = delta = 1/Lhat, no backtracking;
                             0 < nu < 1: delta = 1/(nu Lhat), halved (never below 1/Lhat)
                             whenever the sufficient-decrease test of a step fails
                             (host-checked every inner iteration, no graph replay);
                             nu = 0: delta starts at 1 and the same test runs at every
                             iteration (halving never below 1/Lhat)                  */
  int max_outer;          /* outer (Alg. 1) iterations per lambda, e.g. 100         */
  int max_inner;          /* inner PG iterations per outer iteration, e.g. 100000   */
  int check_every;        /* inner iterations between host convergence checks (>= 1) */
  const double* theta0;   /* device, FP64 p-array warm start for the first lambda, or NULL */
  void* stream;           /* hipStream_t (NULL = default stream)                    */
  int profile_every;      /* > 0: in one inner iteration in every profile_every, time the
                             iteration, then the fused slab kernel re-run 8 times back to
                             back on that iteration's own input, with HIP events on the
                             fit's stream (0 = off; the re-runs rewrite identical values);
                             for BF16/FP32 chains with nu = 1 the mode-3 forward kernel and
                             the adjoint + proximal-step kernel are re-run the same way (the
                             latter writes into scratch buffers of the fit)          */
  int graph_mode;         /* 0: replay each block of check_every inner iterations as a
                             captured HIP graph (default); 1: plain stream launches */
  int inner_mode;         /* glam_inner: how the inner loop evaluates grad h (the FP64
                             outer steps always use the rho chain)                  */
  double alpha;           /* elastic-net weight (Sec. 6.3), >= 0: the penalty becomes
                             J(theta) = sum_m w_m (|theta_m| + alpha theta_m^2); 0 = lasso.
                             The prox is the soft threshold divided by 1 + 2 alpha delta
                             lambda w_m; lambda_max is unchanged (the quadratic term has
                             zero slope at theta = 0)                               */
  int penalty;            /* glam_penalty: GLAM_PENALTY_LASSO, or GLAM_PENALTY_SCAD solved by
                             the multi-step adaptive lasso (Sec. 6.4): at each lambda, step 1
                             is the (pen_w-weighted) lasso, and each of msa_steps - 1 further
                             steps the weighted lasso with w_m = pen_w_m p'(|theta_m|)/lambda
                             at the previous step's estimate (Fan and Li's SCAD slope, zero
                             for |theta_m| >= scad_a lambda).  lambda_max and the KKT scale
                             are the lasso's; kkt and objective report the last step's
                             weighted lasso.  Not combinable with alpha != 0.        */
  double scad_a;          /* SCAD shape a > 2 (0 = 3.7)                               */
  int msa_steps;          /* MSA steps per lambda (>= 1; 1 = the lasso)               */
  int extrapolation;      /* the inner loop's extrapolation sequence (Sec. 3.2 leaves it to the
                             implementation: any omega_l in [0, 1)):
                             0 (default): omega_l = (l' - 1)/(l' + 2) with l' counted from the
                             last restart; at each convergence check a positive
                             (y - x^{l+1})^T (x^{l+1} - x^l) restarts it (omega = 0 next; the
                             gradient restart test of O'Donoghue and Candes); applies to the
                             rho-chain loop with nu = 1, the other forms keep 1;
                             1: omega_l = (l - 1)/(l + 2), l counted from the start of each
                             inner loop (the paper's example sequence)                */
  int kron_step;          /* GLAM_INNER_KRON only: 0 (default): delta from Proposition 1 with
                             max V-hat; 1: delta from the exact Lipschitz constant of the
                             tensor-product model, (1/n) prod_j rho(X_j^T W_j X_j) (Sec. 5),
                             the radii by the power method each outer step (Proposition 1
                             where it does not converge).  The longer step shortens the inner
                             loops but, with V-hat's approximate curvature, can lengthen the
                             outer loop (Poisson n = (64, 64, 365): it stalls; see the notes) */
} glam_options;

/* Inner-gradient evaluation.  GLAM_INNER_CHAIN: G(X, V .* H(X, x - theta_ref)) / n through the
 * n-sized rho chain (Sec. 6.1).  GLAM_INNER_GRAM: (S_3 (x) S_2 (x) S_1) vec(x - theta_ref) / n
 * with the Gram factors S_j = X_j^T X_j (Sec. 6.2, tensor-product weights with W = I), i.e.
 * p-sized products only; exact for the families with unit IRLS weights (Gaussian, Gamma-log)
 * without prior weights, and only there (GLAM_EINVAL for Poisson, Binomial, obs_w != NULL or
 * nu < 1).  The Gram products run in the
 * accumulation type of the dtype (FP32 for BF16/F32, FP64 for F64), the mode-3 product on
 * the matrix cores in the chain dtype. */
/* GLAM_INNER_KRON: the same p-sized inner loop for any family, with the IRLS weights replaced
 * by their tensor-product approximation V-hat (Sec. 6.2): each outer step forms
 * S_j = X_j^T diag(v_j) X_j from the geometric means of log V over all but one index, and
 * W = V-hat enters through eq. (ten), so the model's gradient at theta^k is exact and only its
 * curvature is approximated (the Armijo rule and the FP64 KKT test are unchanged).  For the
 * unit-weight families it is GLAM_INNER_GRAM.  Needs nu = 1 (GLAM_EINVAL otherwise). */
/* GLAM_INNER_ONE: unit IRLS weights w_i = 1 in the quadratic model of every outer step, for
 * any family (Sec. 5, the remark after the corollary to Theorem 2: the convergence argument holds
 * for any strictly positive continuous
 * weights, and constant ones are the notable special case; the package's iwls = "one").  The
 * inner loop is then the p-sized Gram form above; the model's gradient at theta^k is the exact
 * FP64 one and the Armijo rule and the FP64 KKT test are unchanged, so the fit reaches the same
 * PMLE.  For the unit-weight families it is GLAM_INNER_GRAM.  Needs obs_w = NULL and nu = 1. */
typedef enum { GLAM_INNER_CHAIN = 0, GLAM_INNER_GRAM = 1, GLAM_INNER_KRON = 2, GLAM_INNER_ONE = 3 } glam_inner;

typedef struct {
  double* theta;          /* device, FP64, nlambda x p (model l at offset l*p), caller-allocated */
  double* lambda_out;     /* host, nlambda: the lambda values used                   */
  double* kkt;            /* host, nlambda: FP64 KKT residual / lambda_max at return */
  double* objective;      /* host, nlambda: F = -l/n + lambda J                      */
  int* iters_outer;       /* host, nlambda                                           */
  int* iters_inner;       /* host, nlambda: total inner iterations                   */
  int* status;            /* host, nlambda: glam_status per model                    */
  int n_done;             /* out: number of models fitted (< nlambda on early exit) */
  double lambda_max;      /* out: lambda_max (Sec. 6.4)                              */
  double seconds;         /* out: wall time of the call                              */
  double chain_ms;        /* out: summed per-launch duration of the sampled fused slab kernels */
  int chain_samples;      /* out: number of sampled launches (profile_every > 0)     */
  double iter_ms;         /* out: summed duration of the sampled whole inner iterations */
  long long inner_total;  /* out: inner iterations over the whole path               */
  int escalated_at;       /* out: first model whose fit continued with the FP64 inner chain
                             because the BF16/FP32 chain stopped refining it (three outer
                             steps in a row ending on the chain's rounding floor with less
                             than 10% KKT progress; the rest of the path stays FP64), or -1 */
  double adj_ms;          /* out: summed per-launch duration of the sampled mode-3 adjoint +
                             proximal-step kernel (BF16/FP32 chains, nu = 1; 0 otherwise) */
  double fwd_ms;          /* out: the same for the mode-3 forward kernel                  */
} glam_result;

/* Fit the whole lambda path with warm starts.  Models are fitted in order;
 * on a fit that does not converge (GLAM_ENOCONV) or produces non-finite values
 * (GLAM_ENONFINITE) the path stops and only the preceding models are valid
 * (n_done), as the reference package does (Sec. 6.5).
 * Errors: GLAM_EINVAL for bad sizes/pointers/options, non-finite Y, Y outside the
 * family's range, negative obs_w, non-positive pen_w, or a lambda sequence that is not
 * strictly decreasing and positive.  Sizes: besides the rho limits, the FP64 outer steps
 * hold both orientations of X_1 and X_2 in LDS, so the two slab modes take n_1, n_2 <= 256
 * when p_1, p_2 <= 16, and about n_1 + n_2 <= 256 when max(p_1, p_2) is 17..32.  When the
 * caller's order does not fit, the fit reorders the modes itself (the largest remaining mode
 * last; Y, obs_w, pen_w and theta0 are permuted on the caller's stream into buffers of its own,
 * and theta is returned in the caller's order).  When no order fits (p_j > n_j designs, large
 * p_j), the path runs on the generic-GEMM solver of glam_fit_path_multi (c = 1), which takes
 * the rho-chain and unit-weight inner loops (GLAM_EINVAL for the Gram forms). */
int glam_fit_path(const glam_problem* prob, const glam_options* opt, glam_result* res);

/* ---------------------------------------------------------------------------
 * models of c >= 1 tensor components (Sec. 2, eq. fivenew: X = [X_1 | ... | X_c] with
 * X_r = X_{r,d} (x) ... (x) X_{r,1}; theta = (vec(Theta_1), ..., vec(Theta_c)))
 * ------------------------------------------------------------------------- */
typedef struct {
  int d;                  /* 2 or 3, shared by every component                      */
  int64_t n[3];           /* mode sizes of the response array                       */
  int c;                  /* number of tensor components (>= 1)                     */
  const int64_t* p;       /* HOST, 3 c entries: p[3 r + j] = p_{r,j} (j >= d ignored) */
  const double* const* X; /* HOST, 3 c device pointers: X[3 r + j] -> n_j x p_{r,j},
                             FP64 column-major (j >= d ignored)                      */
  const double* Y;        /* device, FP64 response array n_1 x ... x n_d            */
  const double* obs_w;    /* device, FP64 prior weights a_i >= 0, or NULL           */
  int family;             /* glam_family                                            */
  const double* pen_w;    /* device, FP64 penalty weights w_m > 0, length
                             p = sum_r prod_j p_{r,j}, or NULL = 1                  */
} glam_multi_problem;

/* The lambda path of glam_fit_path for a c-component model: eta = H(<X_rj>, <Theta_r>), the sum
 * over components of the rho chains (eq. eighteen), the gradient the tuple of the components'
 * adjoint chains (eq. nineteen), and delta from Proposition 1 with its sum over components,
 * Lhat = max(w)/n sum_r prod_j rho(X_{r,j}^T X_{r,j}).  Every rho product runs as a tiled
 * matrix-core GEMM in the paper's cyclic mode order, with no limit on the mode sizes beyond
 * device memory; glam_fit_path itself uses this solver (c = 1) when no order of the modes fits
 * its slab kernels (p_j > n_j designs).
 * Options as glam_fit_path, except: inner_mode GLAM_INNER_CHAIN or GLAM_INNER_ONE only
 * (GLAM_EINVAL for the Gram forms); graph_mode, profile_every and kron_step are ignored, and
 * chain_ms, iter_ms, adj_ms, fwd_ms and chain_samples are returned as 0.  res->theta holds
 * nlambda x p values, model l at offset l p in the order of theta above.
 * Errors: those of glam_fit_path, and GLAM_EINVAL for c < 1 or NULL p / X. */
int glam_fit_path_multi(const glam_multi_problem* prob, const glam_options* opt, glam_result* res);

/* ---------------------------------------------------------------------------
 * Many independent GLAMs at once (one lambda each): every inner proximal step of
 * all unconverged problems is three batched launches (mode-3 forward tiles, the
 * slabs, mode-3 adjoint tiles with the proximal step); the FP64 outer steps of
 * Algorithm 1 run per problem.
 * ------------------------------------------------------------------------- */
typedef struct {
  const double* lambda;   /* HOST array of nprob lambdas, or NULL: lambda_ratio * lambda_max_i */
  double lambda_ratio;    /* used when lambda == NULL (0 < ratio <= 1)                   */
  int dtype;              /* glam_dtype of the inner rho chain                           */
  double kkt_tol;         /* FP64 KKT target (relative to each lambda_max_i)             */
  int max_outer;          /* outer iterations per problem                                */
  int max_inner;          /* batched proximal steps per outer round                      */
  int check_every;        /* steps between host convergence checks                       */
  void* stream;           /* hipStream_t (NULL = default stream)                         */
  double alpha;           /* elastic-net weight of every problem, as in glam_options     */
  int tuning;             /* 0: the slab phase's launch choices (run length, kernel width) per
                             shape class picked by timing the variants once on the batch's
                             first block (kept per class signature for the process, and in the
                             file named by GLAM_TUNE_FILE when set); 1: fixed heuristics.  The
                             variants compute the same values (bit for bit)             */
  int graph_mode;         /* 0: each block of check_every batched steps replayed as a captured
                             HIP graph (the work list is read from device memory, so one graph
                             serves until a grid would grow or could shrink to a quarter);
                             1: stream launches                                           */
} glam_batch_options;

typedef struct {
  double* const* theta;   /* HOST array of nprob DEVICE pointers; theta[i] -> p_i FP64 (caller-allocated) */
  double* lambda_out;     /* host, nprob                                                 */
  double* lambda_max;     /* host, nprob                                                 */
  double* kkt;            /* host, nprob: FP64 KKT residual / lambda_max_i               */
  double* objective;      /* host, nprob                                                 */
  int* iters_outer;       /* host, nprob                                                 */
  int* status;            /* host, nprob: glam_status per problem                        */
  long long steps;        /* out: batched proximal-step launches                         */
  long long problem_steps;/* out: proximal steps summed over problems                    */
  double seconds;         /* out: wall time of the call                                  */
  long long graph_replays;/* out: blocks of batched steps run as graph replays               */
  double tune_seconds;    /* out: time spent timing slab-phase variants (0 when cached)      */
} glam_batch_result;

/* Fit nprob independent problems (each as in glam_fit_path with nlambda = 1; nu = 1).
 * Problems may differ in sizes and family.  A problem whose modes do not fit the slab
 * kernels in the caller's order is solved in another order, as in glam_fit_path (its Y,
 * obs_w and pen_w permuted on opt->stream into buffers of its own, theta[i] returned in
 * the caller's order).  Per-problem set-up and outer steps run on a few internal streams
 * ordered after opt->stream; the call returns once all of them are done.  Returns
 * GLAM_ENOCONV if any problem did not converge (its status says which).  Errors:
 * GLAM_EINVAL as glam_fit_path, plus nprob < 1. */
int glam_fit_batched(const glam_problem* probs, int nprob, const glam_batch_options* opt,
                     glam_batch_result* res);

/* ---------------------------------------------------------------------------
 * Poisson negative log-likelihood in beta (eqs. two, three and four with
 * a = 1, log y! dropped): L(beta) = (1/n) sum_i (exp(eta_i) - y_i eta_i),
 * eta = H(<X_j>, beta); grad L = G(<X_j>, exp(eta) - y) / n.
 * ------------------------------------------------------------------------- */
/* Like the rho entry points, a problem whose mode order does not fit the slab kernels runs in
 * one that does: beta, Y (and the gradient) are permuted through the workspace, whose size
 * query then includes them. */
size_t glam_nll_workspace_size(const int64_t* n, const int64_t* p, int dtype);

/* loss (device, one FP64) = L(beta).  X and beta of `dtype`; Y FP64 counts. */
int glam_poisson_nll_forward(const int64_t* n, const int64_t* p, const void* const* X,
                             const void* beta, const double* Y, double* loss, int dtype,
                             void* workspace, size_t ws_bytes, void* stream);

/* grad (device, FP32 for F32/BF16, FP64 for F64, p-array) = gscale * grad L(beta),
 * where gscale is the device FP64 scalar *gscale (the upstream gradient). */
int glam_poisson_nll_backward(const int64_t* n, const int64_t* p, const void* const* X,
                              const void* beta, const double* Y, const double* gscale,
                              void* grad, int dtype, void* workspace, size_t ws_bytes,
                              void* stream);

/* The same loss and gradient with X and Y packed into the workspace once (a fit or a
 * training loop evaluates L at many beta for one design and one response).
 * glam_poisson_nll_pack writes the packed factors and a copy of the counts (FP32,
 * tiled like the slab kernel's tiles, for BF16/FP32 chains with n_1, n_2 <= 128; FP64
 * otherwise) into a workspace of glam_nll_packed_workspace_size bytes, on `stream`.
 * The *_packed calls then take only beta: they read that workspace (which must have
 * been packed for the same n, p and dtype, and not written since) and give the same
 * values as glam_poisson_nll_forward / _backward (bit for bit for integer counts below
 * 2^24).  Y must be integer-valued counts when the FP32 copy is used.  Calls that share
 * a workspace must not overlap (the T1 and partial-sum regions are reused).  Errors:
 * GLAM_EINVAL for bad sizes, NULL pointers or a workspace too small. */
size_t glam_nll_packed_workspace_size(const int64_t* n, const int64_t* p, int dtype);
int glam_poisson_nll_pack(const int64_t* n, const int64_t* p, const void* const* X,
                          const double* Y, int dtype, void* workspace, size_t ws_bytes,
                          void* stream);
int glam_poisson_nll_forward_packed(const int64_t* n, const int64_t* p, const void* beta,
                                    double* loss, int dtype, void* workspace, size_t ws_bytes,
                                    void* stream);
int glam_poisson_nll_backward_packed(const int64_t* n, const int64_t* p, const void* beta,
                                     const double* gscale, void* grad, int dtype,
                                     void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GLAM_H */
