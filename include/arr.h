/*
 * arr.h -- C ABI of the MI355X (gfx950) ARRABIT block eigensolver.
 *
 * Computes the k algebraically largest or smallest eigenpairs of a sparse
 * symmetric matrix A with the block algorithm of Wen & Zhang, "Block
 * algorithms with augmented Rayleigh-Ritz projections for large-scale eigenpair
 * computation" (arXiv 1507.06078): a multi-power subspace update with a
 * Chebyshev-interpolant polynomial accelerator (Sec. 5, Algorithm 7) followed by
 * augmented Rayleigh-Ritz projections (Algorithm 5), driven by the detailed
 * ARRABIT iteration (Algorithm 8) with the heuristics of Sec. 6.
 *
 * Every step runs in hand-written HIP kernels on the GPU; the host only keeps
 * scalars (interval ends, tolerances, degree, block counts) and makes the
 * decisions of Sec. 6.
 *
 * Conventions shared by all entry points
 *  - Return codes: ARR_OK (0) on success; ARR_NOT_CONVERGED / ARR_STAGNATED
 *    (> 0) mean a solve ended by stop rule (i) / (ii) of Sec. 6 and the best
 *    pairs are still retrievable; negative values are errors, with a message
 *    available from arr_last_error (handle API) or arr_last_global_error.
 *  - Dense blocks are ROW-MAJOR: element (i, j) of an n x w block with leading
 *    dimension ld (>= w) is at p[i*ld + j]. This is the one layout of the
 *    library, for device blocks and for the eigenvectors arr_get_eigpairs
 *    returns alike (eigenvector j is column j, entry i at evecs[i*ldv + j]):
 *    a row of the block is what one SpMM gather reads, so results leave the
 *    device without a transpose.
 *  - Residual scalings: the stop rules use eq. resi, ||r||_2 / max(1,
 *    |lambda|); arr_get_residuals also returns ||r||_2 / ||A||_2 (with the
 *    Lanczos estimate of ||A||_2) and ||r||_2. When ||A||_2 >= 1 the first
 *    bounds the second.
 *  - CSR matrices are 0-based with int64 row pointers and int32 column
 *    indices; both triangles are stored (A must be symmetric), duplicates are
 *    not allowed.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory on the handle's (or the current) device.
 *  - A handle is not thread-safe; distinct handles may be used from distinct
 *    threads.
 */
#ifndef ARR_H_
#define ARR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define ARR_OK 0
#define ARR_NOT_CONVERGED 1 /* stop rule (i): maxit outer iterations reached   */
#define ARR_STAGNATED 2     /* stop rule (ii): maxres not reduced 3 times     */
#define ARR_EINVAL (-1)     /* invalid argument (message says which)          */
#define ARR_ENOMEM (-2)     /* device memory could not be allocated           */
#define ARR_EDEVICE (-3)    /* a HIP call failed                              */
#define ARR_ESTATE (-4)     /* call out of order (e.g. results before solve)  */
#define ARR_EBREAKDOWN (-5) /* numerical breakdown that no fallback resolved  */

typedef enum { ARR_LARGEST_ALGEBRAIC = 0, ARR_SMALLEST_ALGEBRAIC = 1 } arr_which_t;

/* Arithmetic of the block iteration. ARR_FP64: every block in FP64.
 * ARR_MIXED: filter SpMMs and blocks in FP32 (FP64 small dense work and
 * FP64 Gram accumulation), then FP64 closing iterations down to tol. */
typedef enum { ARR_FP64 = 0, ARR_MIXED = 1 } arr_precision_t;

/* Inner solver of Algorithm 8 (the subspace update between ARR projections):
 * ARR_INNER_MPM, the multi-power method (Sec. 3: filter, then normalize the
 * columns); ARR_INNER_GN, the Gauss-Newton iteration of Sec. 2.6 with unit step
 * (Y = X (X^T X)^{-1}, Z = rho(A) Y, X = Z - X (Y^T Z - I)/2). */
typedef enum { ARR_INNER_MPM = 0, ARR_INNER_GN = 1 } arr_inner_t;

/* How the filter psi_d (Sec. 5) is applied. ARR_POLY_PRODUCT: as the product
 * lead * prod (A' - r_i I) over psi_d's d real roots (all in [-1, 1)), Leja
 * ordered, with A' the shifted and scaled operator of Algorithm 7: one
 * gathered read and one write of the block per degree. ARR_POLY_HORNER:
 * Algorithm 7's Horner recurrence on the monomial coefficients Gamma_d, which
 * also reads X every degree. The two are the same polynomial.
 * ARR_POLY_CHEBYSHEV: the classic Chebyshev polynomial T_d of eq. cheby-poly
 * on the same mapped operator instead of psi_d (the alternative of Table
 * comp-cheby), by its three-term recursion (reads Y_{j-1} every degree); the
 * degree rule eq. hat-d is then evaluated on T_d. */
typedef enum { ARR_POLY_PRODUCT = 0, ARR_POLY_HORNER = 1, ARR_POLY_CHEBYSHEV = 2 } arr_poly_form_t;

/* Host CSR description (arr_create deep-copies it to the device). */
typedef struct {
  int64_t n;             /* order of A                                   */
  int64_t nnz;           /* stored entries, = rowptr[n]                  */
  const int64_t *rowptr; /* host, [n+1], rowptr[0] = 0, non-decreasing   */
  const int32_t *colind; /* host, [nnz], in [0, n)                       */
  const double *val;     /* host, [nnz]                                  */
} arr_csr_t;

/* Row form of the matrix in the SpMM kernels. Plain: per row the three
 * central entries, up to four other ("far") entries, and an overflow CSR for
 * the rest. Paired: for matrices with a frequent column offset P (a grid
 * operator's neighbour one grid line away), rows i and i + P of each block of
 * 2P rows are processed together and each row's entry in the other's column
 * is served from registers instead of a gather; chosen only when every row
 * then has at most three far entries besides that one. Grid: for matrices
 * whose every entry is a neighbour of its row in a 7-point stencil on a
 * gx x gy x gz grid, or a 5-point stencil on a gx x gz grid, in lexicographic
 * order (x fastest; any values, Dirichlet boundary: no entry wraps from one
 * grid line to the next); a workgroup streams an x-y tile of rows through LDS
 * plane by plane, so each input row is read about once instead of once per
 * stencil entry. ARR_ROW_AUTO takes the grid form for 2D (5-point) grids,
 * else the paired form where it applies (on 3D grids the paired form measured
 * faster); ARR_ROW_GRID takes the grid form wherever it applies, 3D included,
 * else falls back as ARR_ROW_AUTO; ARR_ROW_PAIRED never takes the grid form;
 * ARR_ROW_PLAIN always takes the plain form. All forms compute the same
 * product (the filter SpMM of Algorithm 7's loop body), up to the order of
 * the sums. */
typedef enum { ARR_ROW_AUTO = 0, ARR_ROW_PLAIN = 1, ARR_ROW_PAIRED = 2, ARR_ROW_GRID = 3 } arr_row_form_t;

/* The row form the SpMM kernels use for a host CSR (same checks as
 * arr_create; host only, no device needed): *pair = the pairing offset P (0
 * for the plain and grid forms), *far_slots = far entries gathered per row (4
 * plain; 1 or 3 paired; 0 grid), *overflow = entries in the plain form's
 * overflow CSR. Any output pointer may be NULL, and so may csr->val (the form
 * depends on the pattern only). ARR_EINVAL on a malformed CSR or an unknown
 * form. */
int arr_row_form(const arr_csr_t *csr, int32_t form, int64_t *pair, int32_t *far_slots, int64_t *overflow);

/* Grid dimensions of the grid form for a host CSR: dims[0..2] = (gx, gy, gz)
 * (gy = 1 for a 5-point 2D grid), or zeros when the form `form` selects is
 * not the grid form. Host only; same checks and errors as arr_row_form. */
int arr_row_grid(const arr_csr_t *csr, int32_t form, int64_t *dims);

/* Device CSR description used by the step-level entry points. val is a
 * device array of FP64 (dtype 0) or FP32 (dtype 1) values; column indices
 * strictly increase within each row. Each step call copies the matrix to the
 * host, checks it (ARR_EINVAL on a malformed CSR) and builds, in temporary
 * device memory, the row form its kernels read (arr_row_form_t). */
typedef struct {
  int64_t n, nnz;
  const int64_t *rowptr; /* device [n+1] */
  const int32_t *colind; /* device [nnz] */
  const void *val;       /* device [nnz] */
  int32_t dtype;         /* 0 = FP64, 1 = FP32 */
  int32_t row_form;      /* arr_row_form_t, 0 = ARR_ROW_AUTO */
} arr_dev_csr_t;

/* Parameters of Algorithm 8; arr_options_default fills the defaults of
 * Sec. 6. */
typedef struct {
  int32_t w;             /* block width k+q; 0 -> k + round(0.1 k) (Sec. 6, guard vectors) */
  int32_t p0, p_max;     /* augmentation blocks: initial 1, max 3 (eq. block)              */
  int32_t d0, d_max;     /* polynomial degree: initial 3, max 15 (eq. degree)              */
  int32_t maxit;         /* outer iterations, 30 (stop rule (i))                           */
  int32_t maxit1;        /* inner stop checks, 10                                          */
  int32_t maxit2;        /* inner iterations between checks, 5                             */
  double tol1;           /* first continuation tolerance; 0 -> 1e-6 if tol <= 1e-8 else tol */
  int32_t precision;     /* arr_precision_t                                                */
  int32_t paper_faithful;/* 1: also stop by rule (iii) of Sec. 6                            */
  int32_t lanczos_steps; /* Lanczos steps for the lower interval end, 100                  */
  int32_t device;        /* HIP device ordinal, default 0                                  */
  uint64_t seed;         /* seed of the device Gaussian starting block                     */
  double mixed_switch;   /* ARR_MIXED: leave FP32 once maxres <= this (default 1e-2)       */
  int32_t verbose;       /* 1: one line per outer iteration on stderr; 2: also each inner check */
  int32_t timing;        /* 1: time filter SpMM launches with HIP events (stats)           */
  int32_t keep_vectors;  /* served requests: keep eigenvectors on the host (default 1)    */
  int32_t inner_solver;  /* arr_inner_t, default ARR_INNER_MPM                              */
  int32_t poly_form;     /* arr_poly_form_t, default ARR_POLY_PRODUCT                       */
  int32_t row_form;      /* arr_row_form_t, default ARR_ROW_AUTO                            */
  /* Test hook for the non-finite guard, 0 (off) by default: n > 0 writes a
   * NaN into the iterate right after the n-th filter application of the
   * solve; n < 0 does so after every application from the |n|-th on. */
  int32_t debug_nan_poly;
  /* 1: lean-memory mode. The n x m block A U of the Rayleigh-Ritz step is not
   * kept: H = U^T (A U) is formed from column chunks of 256 (FP64) or 512
   * (FP32) columns, and A X of the new Ritz vectors comes from one more SpMM;
   * the returned eigenvectors stay in a block the solve no longer needs. Saves
   * (p_max + 1) w + k columns of n values per precision (one of the three
   * n x (p_max + 1) w blocks and the output block) for one extra SpMM of the
   * new Ritz vectors per outer iteration. Needs the MPM inner solver. */
  int32_t lean_memory;
  /* ARR_MIXED: at the handover to the FP64 stage, when the FP32 stage's last
   * maxres is at most this, b moves up to that iteration's mu_{k+q}, as a
   * continuation step (eq. contin) moves it; tol_t is unchanged. Default
   * 1e-2 (the default mixed_switch: every handover by the switch); 0 never. */
  double mixed_contin;
  /* Test hook of the FP32 stage's collapse check, 0 (off) by default: 1
   * treats the first FP32-stage iteration as collapsed. */
  int32_t debug_fp32_collapse;
  /* ARR_FP64: the first time maxres is at most this, b moves up to that
   * iteration's mu_{k+q} (the b update of eq. contin, tol_t unchanged),
   * before Sec. 6's continuation would move it at maxres <= tol_t. 0
   * (default): Sec. 6 exactly. The mixed path takes its step at the handover
   * instead (mixed_contin). */
  double early_contin;
} arr_options_t;

/* Counters and timings of the last solve. */
typedef struct {
  int32_t status;        /* return code of arr_solve */
  int32_t outer_iters;
  int32_t arr_calls;
  int32_t poly_calls;
  int32_t final_p, final_d;
  int32_t n_locked;      /* converged pairs held in Q_c at the end */
  int32_t fp32_outer;    /* outer iterations done in FP32 (ARR_MIXED) */
  int64_t spmm_degrees;  /* block SpMM filter degrees                 */
  int64_t spmm_cols;     /* sum over filter degrees of block widths   */
  double a, b;           /* final interval ends (working operator)    */
  double norm_est;       /* |A|_2 estimate (Lanczos Ritz values)       */
  double maxres;         /* final max residual, eq. resi scaling       */
  double t_total;        /* seconds inside arr_solve                    */
  double t_setup;        /* interval estimation                         */
  double t_filter;       /* subspace update (filter, normalize, project, rcond) */
  double t_arr;          /* augmentation + RR + residuals               */
  double t_dense;        /* orthonormalization + Rayleigh-Ritz inside t_arr */
  /* HIP-event timing of the filter SpMM launches of the most time-consuming
   * kernel variant (set when arr_options_t.timing = 1): launch count, summed
   * kernel milliseconds, summed algorithmic bytes (CSR read once, the gathered
   * input block counted once, the recurrence block and the output block). */
  int64_t spmm_launches;
  double spmm_ms;
  double spmm_bytes;
  int32_t spmm_cols_per_lane; /* kernel variant: columns per lane (1, 2, 4, 8, 16) */
  int32_t spmm_fp64;          /* data type of that variant: 1 FP64, 0 FP32 */
  int32_t spmm_vec;           /* columns per lane load: 1, 4 (16-byte FP32 loads) or 2 (16-byte FP64 loads) */
  /* HIP-event timing (timing = 1) of the dense products: Gram products X^T Y
   * (tile kernel plus its split reduction) and block updates X W. Work is
   * counted in algorithmic flops: 2 n mx my, n m (m + 1) for a symmetric
   * product (upper triangle), 2 n m c for an update (n m (m + 1) when W is
   * upper triangular, as in Cholesky QR). "64" = FP64 matrix cores
   * (FP64 data, or FP32 data widened exactly); "32" = FP32 matrix cores. */
  int64_t gram64_launches, gram32_launches, upd64_launches, upd32_launches;
  double gram64_ms, gram64_flops, gram32_ms, gram32_flops;
  double upd64_ms, upd64_flops, upd32_ms, upd32_flops;
  /* the most time-consuming FP32 SpMM variant alone (ARR_MIXED), as above */
  int64_t spmm32_launches;
  double spmm32_ms, spmm32_bytes;
  int32_t spmm32_cols_per_lane, spmm32_vec;
  double fp32_maxres;    /* ARR_MIXED: maxres of the last FP32-stage iteration (eq. resi) */
  /* flags of the SpMM variants above: 1 = recurrence block Z present,
   * 2 = matrix has rows with more than four entries off the central band,
   * 4 = column sums of squares computed, 8 = paired row form (rows i and
   * i + P of a block of 2P rows processed together, P a frequent column
   * offset of the matrix), 16 = paired form with one far entry per row
   * (otherwise three) */
  int32_t spmm_flags, spmm32_flags;
  /* inner loops restarted by the non-finite guard: a filtered block with a
   * NaN or Inf column norm is restored to the start of the outer iteration's
   * filter stage, renormalized, and filtered again at half the degree (once
   * per outer iteration; a second failure ends the solve with
   * ARR_EBREAKDOWN) */
  int32_t nan_retries;
  /* max over the k returned pairs of the explicit FP64 residual, in the eq.
   * resi scaling and as ||A x - lambda x||_2 / ||A||_2 with norm_est */
  double maxres_explicit, maxres_norm_a;
  /* sum over the Rayleigh-Ritz steps of m^2, m the dimension of the projected
   * subspace ((p + 1) w' columns): the dense work of a solve scales with n
   * times this */
  double arr_m2;
  /* ARR_MIXED: 1 if the handover to the FP64 stage took the continuation
   * step of option mixed_contin */
  int32_t handover_contin;
  /* ARR_MIXED: 1 if the FP32 stage's Ritz values collapsed (all w within
   * 1e-6 (b - a) of each other: the block driven onto one isolated dominant
   * eigenvector below FP32 resolution) and the FP64 stage restarted from the
   * starting block */
  int32_t fp32_collapsed;
  /* the outer iteration that took option early_contin's step, 0 if none */
  int32_t early_contin;
} arr_stats_t;

typedef struct arr_solver *arr_handle_t;

/* Fill *o with the defaults of Sec. 6 and Algorithm 8. */
void arr_options_default(arr_options_t *o);

/* Problem setup: the k extreme eigenpairs of A with residual tolerance tol
 * (eq. out-stop, eq. resi). Validates on the host (row pointers, column
 * bounds and order, finite values, symmetry, 0 < k <= w, (p_max+1) w < n as
 * required by Algorithm 8, tol > 0) and keeps a host copy of the matrix in
 * the SpMM's row form. Device memory (about (p_max+3) n w values plus the
 * matrix; arr_footprint gives the exact size) is allocated and the matrix
 * uploaded by the first arr_solve, or on admission when the handle is
 * served. The caller keeps ownership of csr's arrays and may free them on
 * return. n must equal csr->n. On success *out is a new handle that the
 * caller releases with arr_destroy. */
int arr_create(const arr_csr_t *csr, int64_t n, int32_t k, arr_which_t which, double tol,
               arr_handle_t *out);
int arr_create_ex(const arr_csr_t *csr, int64_t n, int32_t k, arr_which_t which, double tol,
                  const arr_options_t *opts, arr_handle_t *out);

/* Optional: use X0 (host, n x w row-major with leading dimension ld >= w,
 * FP64) as the starting block instead of the device Gaussian draw (Algorithm 8
 * initializes X as an i.i.d. Gaussian matrix; its first column also starts
 * the Lanczos estimate of the lower interval end). Copied; must be called
 * before arr_solve. */
int arr_set_initial_block(arr_handle_t h, const double *X0, int64_t ld);

/* Run Algorithm 8 to completion on the handle's stream (blocking). Returns
 * ARR_OK, ARR_NOT_CONVERGED, ARR_STAGNATED or an error code. */
int arr_solve(arr_handle_t h);

/* Copy results to caller-owned host buffers (any pointer may be NULL):
 * evals [k] (descending for LARGEST, ascending for SMALLEST), evecs n x k
 * ROW-MAJOR with leading dimension ldv >= k (column j is eigenvector j; unit
 * columns, sign chosen so the entry of largest magnitude is positive; the
 * library's one layout for blocks, see the conventions above), resid [k] =
 * ||A x - lambda x||_2 / max(1, |lambda|) (eq. resi, the scaling of the stop
 * rule eq. out-stop). Residuals are recomputed for the returned vectors with
 * an explicit FP64 SpMM; ARR_OK is returned by arr_solve only if every one of
 * them meets the accepting rule (tol, or (1 + 9h/k) tol under rule (iii)). */
int arr_get_eigpairs(arr_handle_t h, double *evals, double *evecs, int64_t ldv, double *resid);

/* The residuals of the returned pairs in every scaling (host buffers of k
 * values, any may be NULL): resid = ||r||_2 / max(1, |lambda|) (eq. resi),
 * resid_norm_a = ||r||_2 / ||A||_2 with ||A||_2 estimated by the extreme
 * Lanczos Ritz values of the interval setup (a lower bound of ||A||_2, so
 * this is an upper bound of the exact scaled residual), rnorm = ||r||_2,
 * r = A x - lambda x. ARR_ESTATE before a solve. */
int arr_get_residuals(arr_handle_t h, double *resid, double *resid_norm_a, double *rnorm);

/* ARR_MIXED: the k wanted Ritz values of the last FP32-stage outer iteration
 * (the values handed to the FP64 stage, in the order of arr_get_eigpairs),
 * into a host buffer of k values: what the FP32 filter stage of the mixed
 * path alone reaches. ARR_ESTATE before a solve or when the solve had no FP32
 * stage (ARR_FP64). */
int arr_get_fp32_stage_values(arr_handle_t h, double *evals);

int arr_get_stats(arr_handle_t h, arr_stats_t *s);
const char *arr_last_error(arr_handle_t h);
const char *arr_last_global_error(void);
void arr_destroy(arr_handle_t h);

/* ---- serving: continuous batching of many solves on one GPU -------------
 *
 * A server owns a device arena of hbm_budget_bytes. Submitted requests (each a
 * handle made by arr_create / arr_create_ex, not yet solved) wait in a FIFO
 * queue; the head is admitted as soon as fewer than max_slots requests run and
 * a contiguous block of its footprint (arr_footprint) is free in the arena.
 * An admitted request runs Algorithm 8 with all its state resident in its
 * block, on its own stream, concurrently with the other admitted requests;
 * when it finishes its results are copied to host memory (eigenvalues and
 * residuals always, eigenvectors if keep_vectors) and its block is returned.
 * The caller keeps ownership of the handle and must not use or destroy it
 * until arr_wait (or arr_poll) reports the request done; arr_get_eigpairs and
 * arr_get_stats then work as after arr_solve. A request's results do not
 * depend on which other requests ran beside it. */
typedef struct arr_server *arr_server_t;
typedef struct {
  uint64_t hbm_budget_bytes; /* device arena; 0 -> 80% of the free device memory */
  int32_t max_slots;         /* requests solved concurrently; 0 -> 4             */
  int32_t device;            /* HIP device ordinal                               */
  int32_t batch_spmm;        /* 1: the running requests' filter SpMMs run
                                together in multi-request launches (the kernel
                                of arr_filter_step_batch), gathered by a broker
                                thread; 0 (default): each request launches its
                                own on its stream                           */
  int32_t reserved;          /* must be 0                                        */
} arr_server_opts_t;

void arr_server_opts_default(arr_server_opts_t *o);
int arr_server_create(const arr_server_opts_t *o, arr_server_t *out);
/* Device bytes a solve of h reserves (matrix, blocks, work). */
int arr_footprint(arr_handle_t h, uint64_t *bytes);
/* Queue h; non-blocking. ARR_ENOMEM if its footprint exceeds the budget. */
int arr_submit(arr_server_t s, arr_handle_t h, uint64_t *ticket);
/* *done = 1 once the request has finished (successfully or not). */
int arr_poll(arr_server_t s, uint64_t ticket, int *done);
/* Block until the request finishes; returns its arr_solve status. */
int arr_wait(arr_server_t s, uint64_t ticket);
/* Seconds since server creation at submission, admission and completion. */
int arr_request_times(arr_server_t s, uint64_t ticket, double *t_submit, double *t_admit, double *t_done);
/* With batch_spmm: the broker's rounds so far (each round takes every SpMM
 * call the running requests had handed in) and the plain- and paired-form
 * launches those rounds ran inside multi-request launches (grid-form
 * launches run as launches of their own and are not counted); zeros without
 * batch_spmm. */
int arr_server_batch_stats(arr_server_t s, int64_t *batches, int64_t *launches);
/* Waits for the running requests; queued ones are cancelled (status
 * ARR_ESTATE). */
void arr_server_destroy(arr_server_t s);

/* ---- step-level entry points (device pointers, for composing and testing
 * the steps of Algorithm 8). All run on `stream` (a hipStream_t, NULL for
 * the default stream) and return after the work is enqueued unless stated. */

/* One fused filter degree (the body of the loop of Algorithm 7):
 *   Yout = alpha * A * Yin + beta * Yin + gamma * Z
 * on w columns. Yin, Z, Yout are device blocks of A's dtype (n x w, row-major,
 * leading dimensions ldy, ldz, ldo). Z may equal Yin or be NULL (gamma
 * ignored). Yout must not overlap Yin; it may equal Z. If colsumsq (device,
 * FP64 [w]) is non-NULL it receives the squared 2-norms of Yout's columns.
 * Synchronous. */
int arr_filter_step(const arr_dev_csr_t *A, int64_t w, const void *Yin, int64_t ldy, const void *Z,
                    int64_t ldz, void *Yout, int64_t ldo, double alpha, double beta, double gamma,
                    double *colsumsq, void *stream);

/* `count` independent filter degrees (arr_filter_step's operation on each
 * item i: A[i], w[i], Yin[i], ldy[i], Z[i] (may be NULL), ldz[i], Yout[i],
 * ldo[i], alpha[i], beta[i], gamma[i], colsumsq[i] (may be NULL; the array
 * itself may be NULL)), as the multi-request kernel of the serving loop runs
 * them: the plain- and paired-form launches of all items share one
 * persistent launch per kernel variant, whose workgroups take the items'
 * workgroups from a device task table (grid-form items run as their own
 * launches). Each item's result is bitwise what arr_filter_step returns for
 * it. Items may mix dtypes and sizes; their outputs must not overlap any
 * item's inputs or outputs. ARR_EINVAL for count < 1 or an invalid item.
 * Synchronous. */
int arr_filter_step_batch(int32_t count, const arr_dev_csr_t *const *A, const int64_t *w, const void *const *Yin,
                          const int64_t *ldy, const void *const *Z, const int64_t *ldz, void *const *Yout,
                          const int64_t *ldo, const double *alpha, const double *beta, const double *gamma,
                          double *const *colsumsq, void *stream);

/* Algorithm 7 on the shifted operator, as called by Algorithm 8:
 * X <- poly(A - shift I, X, lo, hi, Gamma_d), with Gamma_d (host, d+1 values,
 * leading coefficient first). X is a device block n x w (ld), overwritten.
 * Temporary device memory is allocated internally. Synchronous. */
int arr_poly(const arr_dev_csr_t *A, int64_t w, void *X, int64_t ld, double shift, double lo,
             double hi, const double *gamma, int32_t d, void *stream);

/* Real roots of psi_d (Sec. 5), in the Leja order the product form applies
 * them, and its leading monomial coefficient: psi_d(t) = lead * prod (t -
 * roots[i]). roots: host, d doubles. 1 <= d <= 64. */
int arr_filter_roots(int32_t d, double *roots, double *lead);

/* Apply the library's filter psi_d of Sec. 5 as Algorithm 8 does:
 * X <- psi_d(c0 I + c1 (A - shift I)) X with c0 = (lo + hi)/(lo - hi),
 * c1 = 2/(hi - lo), in the given arr_poly_form_t (ARR_POLY_CHEBYSHEV: T_d of
 * eq. cheby-poly in place of psi_d). X is a device block n x w
 * (ld, A's dtype), overwritten. Temporary device memory is allocated
 * internally. Synchronous. */
int arr_filter(const arr_dev_csr_t *A, int64_t w, void *X, int64_t ld, double shift, double lo, double hi,
               int32_t d, int32_t form, void *stream);

/* One Gauss-Newton inner iteration (Sec. 2.6 with unit step, the GN branch of
 * Algorithm 8) with rho = poly(A - shift I, ., lo, hi, Gamma_d):
 *   Y = X (X^T X)^{-1},  Z = rho(A) Y,  X <- Z - X (Y^T Z - I) / 2.
 * X is a device block n x w (ld, A's dtype), overwritten; w >= 1. X^T X is
 * formed with FP64 sums and inverted through its FP64 Cholesky factor;
 * ARR_EBREAKDOWN if it is not numerically positive definite. Temporary
 * device memory (4 n x w blocks) is allocated internally. Synchronous. */
int arr_gn_step(const arr_dev_csr_t *A, int64_t w, void *X, int64_t ld, double shift, double lo,
                double hi, const double *gamma, int32_t d, void *stream);

/* Chebyshev-interpolant coefficients Gamma_d of Sec. 5 (eq. chebfun-f),
 * computed by the library: out[0..d] leading first. 1 <= d <= 32. */
int arr_filter_coefficients(int32_t d, double *out);

/* Gram product G = X^T Y (FP64 result, device, mx x my row-major, ld my) of
 * device blocks X (n x mx, ldx) and Y (n x my, ldy), accumulated in FP64 with
 * a deterministic split reduction; when X == Y (same pointer, ld and width)
 * only the upper triangle is formed and G is exactly symmetric. dtype: 0 FP64;
 * 1 FP32 data with FP64 products and sums; 2 FP32 data on the FP32 matrix
 * cores, each 32-row slice summed in FP32 (for well-conditioned products, as
 * the Rayleigh quotient of the FP32 stage). Other dtype: ARR_EINVAL.
 * Synchronous. */
int arr_gram(int32_t dtype, int64_t n, const void *X, int64_t ldx, int32_t mx, const void *Y,
             int64_t ldy, int32_t my, double *G, void *stream);

/* arr_gram without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same product G = X^T Y with the same arguments, but
 * its split partial tiles live in a fixed 32 MiB device array of the library
 * (2^22 doubles, one per device, held until the process ends) instead of a
 * buffer allocated per call. Calls no hipMalloc/hipFree and does not
 * synchronize: the work is enqueued on `stream` and G is ready when the
 * stream reaches it. Every partial the reduction reads is written by the same
 * call, so nothing needs clearing between calls. Requires mx * my <= 2^22
 * (ARR_EINVAL otherwise, before anything is launched); larger products take
 * fewer split partials than arr_gram, so the two agree to rounding, not
 * bitwise. Calls that overlap on one device (several streams or host
 * threads) share the array and race: serialize them. */
int arr_gram_noalloc(int32_t dtype, int64_t n, const void *X, int64_t ldx, int32_t mx, const void *Y,
                     int64_t ldy, int32_t my, double *G, void *stream);

/* Block update Y = beta * Y + alpha * X W with X device n x m (ldx, dtype),
 * W device FP64 m x c row-major (ldw), Y device n x c (ldy, dtype). dtype: 0
 * FP64; 1 FP32 data with FP64 products and sums; 2 FP32 data with W rounded to
 * FP32 on the FP32 matrix cores (for a well-conditioned W, as the Ritz
 * rotation). Other dtype: ARR_EINVAL. Y must not alias X. Asynchronous on
 * stream. */
int arr_block_update(int32_t dtype, int64_t n, int32_t m, int32_t c, double alpha, const void *X,
                     int64_t ldx, const double *W, int64_t ldw, double beta, void *Y, int64_t ldy,
                     void *stream);

/* rcond(X^T X) (eq. inn-stop): 1/(||G||_1 ||G^-1||_1) for G = X^T X, or 0 if
 * G is not numerically positive definite. X device n x w (ld, dtype).
 * Synchronous; result in *rc (host). */
int arr_rcond_gram(int32_t dtype, int64_t n, int32_t w, const void *X, int64_t ld, double *rc,
                   void *stream);

/* Orthonormalize the columns of the FP64 device block Z (n x m, ld) in place
 * by Cholesky QR with a shifted first pass when needed (the orth(Z) step of
 * Algorithm 1). Synchronous. */
int arr_orthonormalize(int64_t n, int32_t m, double *Z, int64_t ld, void *stream);

/* Symmetric eigendecomposition of a small FP64 matrix H (device, m x m
 * row-major, read only; its symmetric part is used): evals (device [m]) in
 * descending order and unit eigenvectors as the COLUMNS of V (device, m x m
 * row-major): H = V diag(evals) V^T. Parallel cyclic Jacobi (the eigensolve of
 * Algorithm 1). Synchronous. */
int arr_syev(int32_t m, double *H, double *evals, double *V, void *stream);

/* One augmented Rayleigh-Ritz projection (Algorithm 5 with the deflation
 * projection of Sec. 6) on the FP64 device block X (n x w, ld): builds
 * [X, AX, ..., A^p X], projects out Qc (device n x nc, ldq; nc may be 0),
 * orthonormalizes, projects A, and writes the w leading Ritz values (host,
 * descending) to ritz_vals and the Ritz vectors to Y (device n x w, ldy).
 * Temporary device memory is allocated internally. Synchronous. */
int arr_augmented_rr(const arr_dev_csr_t *A, int64_t w, const double *X, int64_t ld, int32_t p,
                     const double *Qc, int64_t ldq, int32_t nc, double *Y, int64_t ldy,
                     double *ritz_vals, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ARR_H_ */
