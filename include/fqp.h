/*
 * fqp.h -- C-ABI of the MI355X batched factor-model rebalancing solver.
 *
 * Each account a of a book solves the paper's problem class (Eq. 1, Sec.
 * "Benchmark Problem Class") in this instantiation:
 *
 *   min_w (gamma_a/2)(w - wb_a)^T Sigma (w - wb_a) - eta_a mu_a^T w
 *         + sum_i phi_ai(w_i - w0_ai)
 *   s.t.  1^T w = 1                                  (budget)
 *         lb_ai <= w_i <= ub_ai, w_i = 0 if excluded  (box, exclusion mask)
 *         band_lo_a <= A w <= band_hi_a               (one-hot exposure bands)
 *         half_lo_a <= H w <= half_hi_a               (policy halfspaces)
 *         sum_i |w_i - w0_ai| <= tau_a                (turnover cap)
 *
 *   Sigma  = B diag(f) B^T + diag(d)   (factor risk model shared by the book)
 *   phi_ai(D) = kappa_a |D| + T_ai((-D)_+), T_ai the convex piecewise-linear
 *              tax on the sold amount (four lots, three breakpoints).
 *   H (n_half rows) is shared by the book (the policy halfspaces G_a w <= h_a
 *   of Eq. 1 with G_a = H); each account bounds its rows, either side
 *   possibly infinite.  Without wb / eta the risk is (gamma_a/2) w^T Sigma w
 *   and eta_a = 1.
 *
 * The solver returns weights, a status per account, iteration counts and
 * the external diagnostics of Sec. "External Diagnostics" recomputed in
 * float64 (budget/box/exposure/turnover residuals, nonsmooth stationarity,
 * complementarity) -- the observables of the public evaluation boundary
 * (Sec. "Public Evaluation Boundary").  Status codes follow the status
 * vocabulary of Sec. "Status Vocabulary and Objective Agreement".
 *
 * Memory: every array pointer in fqp_universe, fqp_book and fqp_result is a
 * DEVICE pointer on the handle's device, caller-owned, row-major, densely
 * packed (no strides).  Inputs are never modified.  The handle owns its
 * workspace (grown on demand, freed by fqp_destroy).
 *
 * Errors: call-level problems (null pointers, non-positive sizes, HIP
 * failures, allocation failure) return a negative fqp_error;
 * fqp_last_error() describes the last one.  Argument errors and
 * FQP_ERR_ALLOC (every workspace request precedes the first write) leave the
 * outputs untouched; after FQP_ERR_HIP they are undefined.  Problems of one
 * account (invalid data, provable infeasibility, non-finite values) are
 * reported in status[a] and never fail the batch.
 *
 * Threading: one handle per host thread.  The call is synchronous: it
 * enqueues on `stream` (a hipStream_t, NULL = default stream), synchronises
 * it at convergence checks, and returns once every output is written.
 */
#ifndef FQP_H
#define FQP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define FQP_API __attribute__((visibility("default")))
#else
#define FQP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fqp_handle fqp_handle;

typedef enum {
  FQP_OK = 0,
  FQP_ERR_INVALID_ARG = -1,
  FQP_ERR_ALLOC = -2,
  FQP_ERR_HIP = -3,
  FQP_ERR_UNSUPPORTED = -4
} fqp_error;

/* Per-account status (Sec. "Status Vocabulary and Objective Agreement"). */
typedef enum {
  FQP_SOLVED = 0,               /* certified: float64 KKT residuals <= eps */
  FQP_FEASIBLE_UNCERTIFIED = 1, /* quality gates pass, certificate missing */
  FQP_MAX_ITER = 2,             /* iteration cap reached, gates fail       */
  FQP_TIME_LIMIT = 3,           /* declared time limit reached             */
  FQP_PRIMAL_INFEASIBLE = 4,    /* proven on input: no feasible portfolio  */
  FQP_INVALID_INPUT = 5,        /* malformed data (lb > ub, bad tax lots)   */
  FQP_NUMERICAL_ERROR = 6       /* non-finite input or breakdown           */
} fqp_status;

/* Universe shared by all accounts of a book. */
typedef struct fqp_universe {
  int32_t n;             /* assets, >= 1                                   */
  int32_t k;             /* factors, 1..128                                */
  int32_t n_groups;      /* exposure groups, 0..64 (0 = no bands)          */
  const float *B;        /* [n][k] factor loadings                         */
  const float *f;        /* [k]   factor variances, > 0                    */
  const float *d;        /* [n]   idiosyncratic variances, > 0             */
  const int32_t *group;  /* [n]   labels in [0, n_groups); NULL if none    */
  int32_t n_half;        /* policy halfspace rows, 0..64 - n_groups        */
  const float *half;     /* [n_half][n] rows H of the halfspaces; NULL if
                            n_half = 0                                     */
} fqp_universe;

/* Per-account data of Eq. 1 for m accounts (m * n < 2^31 per call). */
typedef struct fqp_book {
  int32_t m;                 /* accounts, >= 1                              */
  const float *mu;           /* [m][n] expected returns                    */
  const float *w0;           /* [m][n] current weights                     */
  const float *lb, *ub;      /* [m] box bounds lb <= ub of eligible names
                                (excluded names: [0, 0])                    */
  const uint32_t *eligible;  /* [m][ceil(n/32)] bit i%32 of word i/32 set =
                                asset i eligible; NULL = all eligible       */
  const float *gamma;        /* [m] risk aversion, > 0                     */
  const float *kappa;        /* [m] L1 turnover cost, >= 0                 */
  const float *tau;          /* [m] turnover cap; +INF = no cap            */
  const float *band_lo;      /* [m][n_groups] or NULL (no bands)           */
  const float *band_hi;      /* [m][n_groups] or NULL                      */
  const int32_t *tax_ptr;    /* [m+1] CSR of tax lots; NULL = no tax       */
  const int32_t *tax_asset;  /* [nnz] asset of each entry, strictly
                                increasing within an account, w0 > 0 there */
  const float *tax_brk;      /* [nnz][3] cumulative sale breakpoints,
                                0 < b1 < b2 < b3                            */
  const float *tax_slope;    /* [nnz][4] lot slopes, 0 <= s0 <= .. <= s3     */
  const float *warm_state;   /* NULL, or an ADMM state block of
                                fqp_state_floats(m, n, n_groups + n_half)
                                floats that an
                                earlier call wrote to fqp_result.state (the
                                same accounts, any handle or process); used
                                when settings.warm_start = 1 (the cold /
                                repeated / warm lanes of Sec. "Timing
                                Lanes").  Non-finite entries restart from 0 */
  /* The rest of Eq. 1; every pointer may be NULL. */
  const float *lb_asset;     /* [m][n] per-asset lower bounds (replace lb for
                                eligible names); NULL = lb[a] everywhere    */
  const float *ub_asset;     /* [m][n] per-asset upper bounds; NULL = ub[a] */
  const float *half_lo;      /* [m][n_half] lower bounds of H w (-INF: none);
                                required when n_half > 0                    */
  const float *half_hi;      /* [m][n_half] upper bounds of H w (+INF: none) */
  const float *wb;           /* [m][n] benchmark weights w_b; NULL = 0       */
  const float *eta;          /* [m] return scale eta >= 0; NULL = 1          */
} fqp_book;

/* Arithmetic of the factor contractions inside the ADMM iterations (the
 * polish and the certificate are float64 either way). */
typedef enum {
  FQP_PREC_FP32 = 0,    /* float32 MFMA (32x32x2)                           */
  FQP_PREC_BF16X3 = 1   /* bf16 MFMA on hi/lo splits of each float32 operand:
                           hi*hi + hi*lo + lo*hi, float32 accumulation
                           (factor blocks k + n_groups + n_half + 1 <= 96; wider ones
                           run the float32 contraction)                    */
} fqp_precision;

typedef struct fqp_settings {
  double eps_prim;       /* absolute primal residual target (1e-6)        */
  double eps_dual;       /* scaled stationarity target (1e-6)             */
  double eps_comp;       /* scaled complementarity target (1e-6)          */
  int32_t max_iter;      /* ADMM iteration cap per account                 */
  int32_t check_every;   /* iterations between polish / certification     */
  float rho;             /* ADMM penalty on the asset split (<= 0: auto)  */
  float rho_band;        /* ADMM penalty on the band split (<= 0: auto)   */
  float alpha;           /* over-relaxation in (0, 2)                     */
  int32_t polish_rounds; /* active-set refinement rounds per polish       */
  int32_t use_graph;     /* capture a block of check_every iterations in a
                            hipGraph; the handle keeps the executable graph
                            and a later call with the same arguments (same
                            buffers, sizes and schedule) replays it        */
  int32_t profile;       /* bit 0: time every PROJECT-pass launch, bit 1:
                            every CONTRACT-pass launch, bit 2: every PROX-
                            pass launch, with events that the kernel's own
                            start and end stamp (no graphs)                */
  double time_limit_ms;  /* wall-clock limit of the call (<= 0: none)     */
  int32_t precision;     /* fqp_precision of the ADMM contractions        */
  int32_t first_check;   /* iteration of the first polish / certification
                            pass (<= check_every: at check_every); later
                            passes every check_every iterations           */
  int32_t warm_start;    /* 1: start from book.warm_state when given, else
                            from the ADMM state (v, band state, cap
                            multiplier) this handle kept from its last
                            completed solve, when that book had the same m,
                            n and constraint rows (n_groups + n_half; e.g.
                            the same accounts with the
                            next day's returns); otherwise, or 0: cold.  Any
                            start converges to the same optimum            */
  int32_t debug_fail_alloc; /* test hook: > 0 makes the workspace request
                            with that number (1-based, in call order) fail
                            like a device allocation failure; the call then
                            returns FQP_ERR_ALLOC with every output
                            untouched.  0 in production                    */
  int32_t tile_rows;     /* rows of one iteration-pass workgroup, in 128-row
                            chunks (0: sized from the occupancy so that a
                            full batch runs in one round of workgroups)    */
} fqp_settings;

/* Outputs (device pointers, caller-owned).  Any may be NULL except w and
 * status. */
typedef struct fqp_result {
  double *w;          /* [m][n] weights                                    */
  int32_t *status;    /* [m] fqp_status                                    */
  int32_t *iters;     /* [m] ADMM iterations run                           */
  double *r_prim;     /* [m] max(budget, box, exposure, turnover) residual */
  double *r_dual;     /* [m] nonsmooth stationarity / gradient scale       */
  double *r_comp;     /* [m] complementarity / gradient scale              */
  double *obj;        /* [m] objective recomputed in float64               */
  double *nu;         /* [m] budget multiplier                             */
  double *lam_cap;    /* [m] turnover-cap multiplier (>= 0)                */
  double *lam_band;   /* [m][n_groups + n_half] multipliers of the band rows,
                         then of the halfspace rows (> 0: the upper bound
                         binds, < 0: the lower one)                      */
  float *state;       /* NULL, or fqp_state_floats(m, n, n_groups + n_half)
                         floats: the final ADMM state (v [m][n], row z
                         [m][R], row u [m][R], cap multiplier [m], R =
                         n_groups + n_half) for a later warm start through
                         fqp_book.warm_state                             */
} fqp_result;

/* Size in floats of an ADMM state block (fqp_book.warm_state,
 * fqp_result.state): m n + 2 m R + m, R = n_groups + n_half (the third
 * argument). */
static inline size_t fqp_state_floats(int32_t m, int32_t n, int32_t n_groups) {
  return (size_t)m * (size_t)n + 2 * (size_t)m * (size_t)n_groups + (size_t)m;
}

/* Host-side counters of the last fqp_solve_batch call. */
typedef struct fqp_stats {
  int32_t iterations;       /* ADMM iterations run (max over accounts)      */
  int32_t iter_launches;    /* fused iteration kernel launches              */
  int32_t polish_calls;     /* polish / certification kernel launches       */
  int32_t n_solved;         /* accounts with status SOLVED                  */
  double iter_kernel_ms;    /* summed execution time of the PROJECT-pass
                               launches (settings.profile bit 0, else 0)   */
  double account_iters;     /* sum over accounts of iterations run          */
  double total_ms;          /* host wall-clock of the call                  */
  size_t workspace_bytes;   /* device workspace held by the handle          */
  int32_t polish_solves;    /* reduced float64 KKT systems formed (accounts
                               x polish rounds)                            */
  int32_t polish_gated;     /* polish attempts skipped because the iterate's
                               pattern was not yet settled                 */
  double contract_kernel_ms; /* summed execution time of the CONTRACT-pass
                               launches (settings.profile bit 1, else 0)   */
  double phase_ms[4];       /* device lane of the call by phase, from events
                               on the handle's stream: [0] validation, packing
                               and factor-space setup, [1] ADMM iterations,
                               [2] polish / certification passes, [3] final
                               polish of uncertified accounts and outputs   */
  int32_t graph_reused;     /* 1: the blocks replayed the executable graph
                               kept from an earlier call with the same
                               arguments (no capture in this call)         */
  int32_t workspace_requests; /* workspace requests the call made (the range
                               of settings.debug_fail_alloc)               */
  double prox_kernel_ms;    /* summed execution time of the PROX-pass
                               launches (settings.profile bit 2, else 0)   */
} fqp_stats;

FQP_API void fqp_default_settings(fqp_settings *s);

FQP_API fqp_error fqp_create(fqp_handle **h, int device);

FQP_API fqp_error fqp_solve_batch(fqp_handle *h, const fqp_universe *U,
                          const fqp_book *P, const fqp_settings *S,
                          fqp_result *R, void *stream);

/* Gradients of a loss L(w) through the last fqp_solve_batch call on this
 * handle (implicit differentiation of the KKT system at each certified
 * optimum, Eq. 1 with the active pattern held fixed):
 *   dL_dw  [m][n] float64 device, input  (dL/dw)
 *   dL_dmu [m][n] float64 device, output (dL/dmu; zero for accounts that are
 *          not certified and for coordinates fixed at a bound or kink)
 *   dL_dB  [n][k] float64 device, output (dL/dB summed over certified
 *          accounts; the factor loadings are shared by the book)
 * The inputs and outputs of that solve must still be alive and unchanged.
 * Asynchronous on `stream`; FQP_ERR_INVALID_ARG if no solve preceded it. */
FQP_API fqp_error fqp_adjoint_batch(fqp_handle *h, const double *dL_dw,
                                    double *dL_dmu, double *dL_dB,
                                    void *stream);

/* fqp_adjoint_batch without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results as
 * fqp_adjoint_batch; its per-account scratch (m * 2k float64 values) comes
 * from a statically allocated device array of 2 MiB (262,144 float64) that
 * each device the library runs on holds until the process ends.  Books with
 * m * 2k above that return FQP_ERR_UNSUPPORTED and write nothing.  Every
 * call on one device shares that device's array: calls that overlap on one
 * device (several handles or streams at once) race; serialise them.  The
 * array needs no clearing: each call writes every entry it reads. */
FQP_API fqp_error fqp_adjoint_batch_noalloc(fqp_handle *h, const double *dL_dw,
                                            double *dL_dmu, double *dL_dB,
                                            void *stream);

FQP_API fqp_error fqp_get_stats(const fqp_handle *h, fqp_stats *out);

/* Certification passes of the last fqp_solve_batch call (the queue lane of
 * Sec. "Production Queue": an account certified after `iters[a]` ADMM
 * iterations completed at the end of the pass run after that many
 * iterations).  For pass p < *count: iter[p] = ADMM iterations before the
 * pass, ms[p] = host wall-clock from the call's start to the end of the pass
 * (the call synchronises the stream there).  Writes at most `cap` entries
 * into the caller's host arrays; *count gets the number of passes.
 * FQP_ERR_INVALID_ARG for null pointers. */
FQP_API fqp_error fqp_get_pass_times(const fqp_handle *h, int32_t *iter, double *ms,
                                     int32_t cap, int32_t *count);

FQP_API const char *fqp_error_string(int e);
FQP_API const char *fqp_status_string(int s);
FQP_API const char *fqp_last_error(const fqp_handle *h);

FQP_API void fqp_destroy(fqp_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* FQP_H */
