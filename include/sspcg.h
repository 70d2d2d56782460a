/* sspcg.h - C ABI of the MI355X (gfx950) s-step PCG library (libsspcg.so).
 *
 * The library solves A x = b for a sparse symmetric positive definite A in
 * CSR form with the s-step preconditioned conjugate gradient method of
 * D'Ambra, Bernaschi, Carrozzo and Thomas, "Scalable s-step Preconditioned
 * Conjugate Gradient with Chebyshev Basis and Gauss-Seidel Gram Solve"
 * (arXiv 2603.09790): Algorithm 1 (outer iteration), Algorithm 2 (matrix
 * powers kernel, MPK, for the Chebyshev basis) and the Forward Gauss-Seidel
 * (FGS) iteration of Sec. 3.1 for the two reduced s x s Gram systems.  The
 * preconditioner is Jacobi, M = diag(A).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named in a "device" argument are HIP device addresses; all
 *   others are host addresses.  Device buffers are owned by the caller and
 *   must stay alive until the work that uses them has finished on `stream`.
 * - The library allocates no memory on the device and no pinned host memory:
 *   the matrix copy (`aux`), solver workspaces, kernel scratch and the
 *   polling buffer of the solvers all come from the caller, sized by the
 *   *_bytes query functions.
 * - `stream` is a hipStream_t passed as a plain pointer; NULL selects the
 *   default stream.  Kernel-level calls only enqueue work and return; the
 *   solve calls block until the solve has finished.
 * - Indices are int32 (n and nnz below 2^31).  Floating point is IEEE binary64
 *   unless a call says otherwise.  Device pointers must be aligned to their
 *   element size (256 bytes recommended); workspaces to 256 bytes.
 * - Blocks of vectors are column-major with leading dimension `ld` >= n,
 *   counted in elements: column j starts at base + j*ld.
 * - Small s x s matrices (W, B2, beta) live in device memory, row-major:
 *   entry (i, j) at i*s + j.
 * - Every call returns an sspcg_status.  On an argument error nothing is
 *   enqueued and no output is touched.  HIP failures return SSPCG_ERR_HIP;
 *   sspcg_last_error() then holds the HIP message (per thread).  No C++
 *   exception crosses this interface.
 * - Results are deterministic: every reduction runs in a fixed order, so
 *   repeated calls with equal inputs give bitwise equal outputs.
 */
#ifndef SSPCG_H
#define SSPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSPCG_ABI_VERSION 3
#define SSPCG_MAX_S 16          /* largest supported step size s */

typedef void* sspcg_stream;     /* hipStream_t */

typedef enum {
    SSPCG_OK = 0,
    SSPCG_NOT_CONVERGED = 1,    /* iteration limit reached; x holds the last iterate */
    SSPCG_ERR_ARG = -1,         /* invalid argument; nothing was done */
    SSPCG_ERR_HIP = -2,         /* a HIP runtime call failed */
    SSPCG_ERR_BREAKDOWN = -3,   /* non-positive Gram or matrix diagonal (A not SPD) */
    SSPCG_ERR_WORKSPACE = -4,   /* workspace smaller than sspcg_workspace_bytes() */
    SSPCG_ERR_NONFINITE = -5,   /* NaN or Inf in the data or the iteration */
    SSPCG_ERR_UNSUPPORTED = -6  /* option not available for this matrix */
} sspcg_status;

typedef enum {
    SSPCG_FP64 = 0,             /* everything in binary64 */
    SSPCG_MIXED = 1             /* FP32 inner solves inside FP64 iterative refinement */
} sspcg_precision;

typedef enum {
    SSPCG_GRAM_FGS = 0,         /* `sweeps` FGS sweeps from zero (Sec. 3.1) */
    SSPCG_GRAM_CHOLESKY = 1     /* exact solve by Cholesky (the paper's comparison) */
} sspcg_gram_solver;

typedef enum {
    SSPCG_BASIS_CHEBYSHEV = 0,  /* z_j = T_{j-1}(alpha M^{-1}A - sigma I) M^{-1} r (Sec. 2) */
    SSPCG_BASIS_MONOMIAL = 1    /* z_j = (M^{-1}A)^{j-1} M^{-1} r, the ill-conditioned contrast */
} sspcg_basis;

/* Element type of vector arguments of the kernel-level calls. */
typedef enum { SSPCG_F64 = 0, SSPCG_F32 = 1 } sspcg_dtype;

/* Flags of sspcg_matrix_create. */
#define SSPCG_MATRIX_FP32 1     /* also keep FP32 values (needed by SSPCG_MIXED) */
#define SSPCG_MATRIX_FULL_STORAGE 2  /* store both triangles even when A is symmetric */

/* Parameters of a solve (the requirements of Algorithm 1 plus the basis
 * interval of Sec. 2).  Use sspcg_default_params() and change fields. */
typedef struct {
    int32_t s;                  /* step size, 1..SSPCG_MAX_S */
    int32_t sweeps;             /* FGS sweeps nu, 1..1000 */
    double lambda_min;          /* Chebyshev interval of M^{-1}A, 0 <= lambda_min < lambda_max */
    double lambda_max;
    double tol;                 /* stop when ||r|| <= tol ||b|| (recursive r; FP64 true r in MIXED) */
    int32_t max_outer;          /* outer-iteration limit (FP64) / per inner solve limit (MIXED) */
    int32_t precision;          /* sspcg_precision */
    double inner_tol;           /* MIXED: inner solves reduce their residual by inner_tol, or
                                   only to half the outer target once that is closer */
    int32_t max_refine;         /* MIXED: limit on FP64 residual corrections */
    int32_t gram;               /* sspcg_gram_solver */
    int32_t check_every;        /* outer iterations enqueued between host polls (>= 1) */
    int32_t profile;            /* 1: time every phase with HIP events (profile output) */
    double sweep_tol;           /* 0: exactly `sweeps` FGS sweeps.  > 0: each right-hand side
                                   stops sweeping once ||m - W a|| <= sweep_tol ||m|| (the
                                   accuracy criterion of Sec. 3), after at most `sweeps` */
    int32_t basis;              /* sspcg_basis of the Krylov block */
    int32_t use_graph;          /* 1: capture `check_every` outer iterations into one HIP
                                   graph and replay it (fewer launches; ignored with profile,
                                   or on the NULL stream, which cannot be captured) */
} sspcg_params;

/* Outcome of a solve (host struct filled by the solve calls). */
typedef struct {
    int32_t status;             /* sspcg_status */
    int32_t outer_iters;        /* x updates taken (FP64) / inner iterations summed (MIXED) */
    int32_t refinements;        /* MIXED: FP64 corrections applied */
    int32_t inner_iters_total;  /* MIXED: inner outer-iterations summed over the refinements;
                                   FP64 and PCG: equal to outer_iters */
    double relres;              /* ||r|| / ||b|| of the residual the stop test used (the
                                   recursive r in FP64 and PCG, the FP64 true r in MIXED) */
    double relres_true;         /* ||b - A x|| / ||b|| of the returned x, recomputed in FP64
                                   on the device after the solve (one more SpMV) */
    double device_ms;           /* GPU time of the solve, from HIP events */
} sspcg_result;

/* Host buffer the solvers poll the device through: pinned host memory
 * (hipHostMalloc, or a torch tensor with pin_memory=True), at least this
 * many bytes, 64-byte aligned.  One per concurrently running solve. */
#define SSPCG_POLL_BYTES 256

/* Phases of the s-step solve, as timed by the profile. */
enum {
    SSPCG_PHASE_SPMV = 0,       /* matrix powers kernel: s SpMV launches with fused epilogue */
    SSPCG_PHASE_GRAM_UPDATE,    /* block update fused with the W, b1 reduction */
    SSPCG_PHASE_GRAM_RECT,      /* B2 = -Q^T AZ reduction */
    SSPCG_PHASE_FGS,            /* finishing of a reduction + FGS solve (alpha or beta) */
    SSPCG_PHASE_NORM,           /* residual norm, stop test */
    SSPCG_PHASE_XR,             /* x, r update with ||r||^2 and z_1 */
    SSPCG_NUM_PHASES
};

/* Per-phase GPU time of a profiled solve, counted over the phases that did
 * work (the launches enqueued after the stop test passed, which return at
 * once, are excluded). */
typedef struct {
    int64_t launches[SSPCG_NUM_PHASES];   /* kernel launches that did work */
    double ms[SSPCG_NUM_PHASES];          /* GPU time between the bracketing events */
    int64_t outer_iters;                  /* outer iterations covered */
} sspcg_profile;

typedef struct sspcg_matrix sspcg_matrix;   /* opaque */

/* ---------------------------------------------------------------- misc */
int sspcg_abi_version(void);
const char* sspcg_status_string(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char* sspcg_last_error(void);
void sspcg_default_params(sspcg_params* p);

/* ---------------------------------------------------------------- matrix */
/* The library keeps its own layout of A (below) in a caller-provided device
 * buffer `aux`.  Its size depends on the sparsity pattern, so it is found in
 * two steps:
 *   1. sspcg_matrix_scratch_bytes(n): device scratch for the analysis;
 *   2. sspcg_matrix_aux_bytes(...): checks the CSR on the device, chooses
 *      the layout, and returns the exact size of `aux`;
 * then sspcg_matrix_create builds the layout in `aux`.  The scratch can be
 * released once step 2 has returned. */
size_t sspcg_matrix_scratch_bytes(int32_t n);

/* CSR input of both calls below:
 *   row_ptr (device, int32[n+1]), col (device, int32[nnz]), val (device,
 *   double[nnz]): row_ptr[0] = 0, increasing row pointers, columns in [0, n)
 *   and every diagonal entry stored.  Column order inside a row fixes the
 *   summation order of the SpMV.
 * scratch (device, >= sspcg_matrix_scratch_bytes(n), 256-byte aligned).
 * aux_bytes (host, required): the device bytes sspcg_matrix_create needs in
 * `aux` for this pattern, these values (whether A is symmetric bit for bit
 * decides the layout) and these flags.  Synchronizes `stream`.
 * Errors as for sspcg_matrix_create. */
int sspcg_matrix_aux_bytes(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col,
                           const double* val, int32_t flags, void* scratch, size_t scratch_bytes,
                           sspcg_stream stream, size_t* aux_bytes);

/* Builds the library's copy of a CSR matrix (arguments as above) in `aux`
 * (device, >= the aux_bytes reported for the same pattern, values and
 * flags; 256-byte aligned; owned by the caller and kept alive, unmoved,
 * until sspcg_matrix_destroy).  `aux` receives the sliced layout, the Jacobi
 * scaling 1/diag(A) and, with SSPCG_MATRIX_FP32, FP32 copies of both.  The
 * handle itself is a small host struct.  The call synchronizes `stream`.
 * Layout: 64-row slices, one row per lane.  A slice whose rows share one
 * list of at most 32 column offsets (col - row) stores that list once and
 * no column indices; other slices keep explicit columns, padded to their
 * longest row.  When one list fits every row (structured-grid stencils) the
 * whole matrix is stored against it; if A is then also symmetric bit for bit,
 * only its diagonal and upper triangle are stored, which halves the values
 * the SpMV streams.  Every layout sums each row's entries in CSR order, so
 * the product does not depend on the layout.  SSPCG_MATRIX_FULL_STORAGE
 * keeps both triangles (for later non-symmetric value updates).
 * Solves use only the copy in `aux`, but sspcg_matrix_update_values,
 * sspcg_csr_value_grad and the diffusion calls read the caller's row_ptr and
 * col again: keep them alive as long as the handle is used with those calls.
 * Returns SSPCG_ERR_ARG for a malformed pattern (checked on the device),
 * SSPCG_ERR_BREAKDOWN when a diagonal entry is missing or not positive,
 * SSPCG_ERR_NONFINITE for a NaN/Inf value and SSPCG_ERR_WORKSPACE when
 * aux_bytes is too small. */
int sspcg_matrix_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col,
                        const double* val, int32_t flags, void* aux, size_t aux_bytes,
                        sspcg_stream stream, sspcg_matrix** out);
/* Replaces the values (same pattern): val is device double[nnz] in CSR
 * order.  Synchronizes `stream`.  The values are checked before anything is
 * changed: SSPCG_ERR_NONFINITE / SSPCG_ERR_BREAKDOWN as for create, and
 * SSPCG_ERR_UNSUPPORTED for values that are not symmetric when the matrix
 * stores one triangle; on an error the matrix keeps its old values. */
int sspcg_matrix_update_values(sspcg_matrix* A, const double* val, sspcg_stream stream);
/* Frees the host handle; `aux` stays the caller's. */
int sspcg_matrix_destroy(sspcg_matrix* A);
/* Size of the library's copy (host outputs, each may be NULL): n, nnz, the
 * stored slots of the sliced layout (nnz plus zero padding; with the
 * symmetric half storage one triangle and the diagonal), the number of
 * 64-row slices and how many of them use a shared offset list (no column
 * indices), the bytes of `aux` in use, and 1 if only one triangle is stored. */
int sspcg_matrix_info(const sspcg_matrix* A, int64_t* n, int64_t* nnz, int64_t* slots,
                      int64_t* slices, int64_t* shared_slices, int64_t* device_bytes,
                      int64_t* symmetric);

/* ---------------------------------------------------------------- solvers */
/* Workspace (device bytes) that sspcg_solve / sspcg_pcg_solve need. */
int sspcg_workspace_bytes(const sspcg_matrix* A, const sspcg_params* p, size_t* bytes);

/* s-step PCG, Algorithm 1 with Algorithm 2 and FGS Gram solves.
 *   b (device, double[n]); x (device, double[n]): x0 on entry, the solution
 *   on exit - the iterate at the first passing stop test.
 *   work (device, >= sspcg_workspace_bytes, 256-byte aligned): scratch,
 *   contents undefined after.
 *   poll (host, pinned, >= SSPCG_POLL_BYTES): the buffer the host reads the
 *   device's stop flag through; contents undefined after.
 *   res (host, required).
 *   history (host, optional): per outer iteration k, 4 doubles {relative
 *   residual after the x update, eta_alpha, eta_beta, conjugacy defect}:
 *   eta_alpha = ||b1 - W alpha|| / ||b1|| and eta_beta = ||B2 - W beta||_F /
 *   ||B2||_F are the reduced-system residuals of Sec. 3.4, and the defect is
 *   ||B2 - W beta||_F, which equals ||Q_{k+1}^T A Q_k||_F in exact
 *   arithmetic (B2 = -Q_k^T A Z and Q_{k+1} = Z + Q_k beta, Sec. 2); 0 where
 *   not formed.  Room for 4*max_outer doubles.  MIXED: per refinement the
 *   FP64 true relative residual, room for max_refine+1 doubles.
 *   profile (host, optional): with p->profile = 1 the per-phase GPU time.
 * If ||b|| = 0 the result is x = 0 after no iteration; if the starting
 * residual already passes the test, x is returned unchanged.
 * On SSPCG_ERR_BREAKDOWN / SSPCG_ERR_NONFINITE, x holds the last iterate
 * before the failing Gram solve.  Blocks until done.  The matrix handle is
 * only read, so solves on one matrix with their own workspace and poll
 * buffer may run at the same time. */
int sspcg_solve(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                void* work, size_t work_bytes, void* poll, sspcg_stream stream,
                sspcg_result* res, double* history, sspcg_profile* profile);

/* For callers that cannot allocate (code that must not call hipMalloc, such
 * as tight serving loops or harnesses that forbid it): sspcg_solve without the
 * workspace argument.  Its workspace is a static device array of
 * SSPCG_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (its address is looked up once per device, at the
 * first call there); it allocates no device or pinned memory and creates no
 * HIP events or graphs after that first call.  Solves whose workspace
 * (sspcg_workspace_bytes) exceeds the array return SSPCG_ERR_WORKSPACE with
 * nothing enqueued; p->profile and p->use_graph return SSPCG_ERR_UNSUPPORTED.
 * All calls on one GPU share its array, and the contents of one call are left
 * for the next: calls that overlap on one GPU (from several threads or
 * streams) race and must not be made.  The current device must be the
 * matrix's.  Otherwise as sspcg_solve (poll: the caller's pinned buffer;
 * blocking; no history or profile output). */
#define SSPCG_STATIC_SCRATCH_BYTES (64 * 1024 * 1024)
int sspcg_solve_static(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                       void* poll, sspcg_stream stream, sspcg_result* res);

/* Classical Jacobi PCG (the method s-step PCG replaces), same stop test.
 * Uses p->tol, p->max_outer (as the iteration limit) and p->check_every;
 * work and poll as for sspcg_solve.
 * history (host, optional): relative residual per iteration. */
int sspcg_pcg_solve(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                    void* work, size_t work_bytes, void* poll, sspcg_stream stream,
                    sspcg_result* res, double* history);

/* ---------------------------------------------------------------- basis interval */
/* The Chebyshev basis needs an interval [lambda_min, lambda_max] holding the
 * spectrum of M^{-1}A (Sec. 2, the s-step PCG method with Chebyshev Krylov
 * basis).  Two device estimates: */
typedef enum {
    SSPCG_INTERVAL_LANCZOS = 0, /* extreme Ritz values of `steps` Lanczos steps on
                                   D^{-1/2} A D^{-1/2} (no reorthogonalisation, no margin) */
    SSPCG_INTERVAL_POWER = 1    /* lambda_min = 0, lambda_max from the power method on M^{-1}A:
                                   ||M^{-1}A v|| for unit v, stopping when successive estimates
                                   differ by less than rtol relative, or after `steps` steps */
} sspcg_interval_method;
#define SSPCG_MAX_INTERVAL_STEPS 1000

/* Device bytes of the `work` argument of sspcg_interval. */
int sspcg_interval_work_bytes(const sspcg_matrix* A, int32_t steps, size_t* bytes);

/* Estimates the basis interval on the device.
 *   method: sspcg_interval_method; steps: 1..SSPCG_MAX_INTERVAL_STEPS (Lanczos
 *   takes at most n steps and stops early on an invariant subspace, beta = 0);
 *   rtol: finite, >= 0 (power method only; the paper uses 1e-3 and 50 steps).
 *   v0 (device, double[n]): start vector, any non-zero scaling; the caller
 *   draws it (for instance uniform in [-1, 1]).
 *   work (device, >= sspcg_interval_work_bytes, 256-byte aligned): scratch.
 *   lambda_min, lambda_max (host, required); steps_taken (host, optional).
 * A start vector with zero norm or non-finite entries gives SSPCG_ERR_ARG,
 * after the device has checked it; a non-finite step SSPCG_ERR_NONFINITE.
 * Blocks until done. */
int sspcg_interval(const sspcg_matrix* A, int32_t method, int32_t steps, double rtol,
                   const double* v0, void* work, size_t work_bytes, sspcg_stream stream,
                   double* lambda_min, double* lambda_max, int32_t* steps_taken);

/* ---------------------------------------------------------------- kernels */
/* The kernels the solvers are built from, for step-by-step checking.  All
 * enqueue on `stream` and return at once.  `work` is device scratch of at
 * least sspcg_kernel_work_bytes(); its contents are undefined afterwards. */
size_t sspcg_kernel_work_bytes(int32_t s);

/* y = A x (x, y device, dtype elements; F32 needs SSPCG_MATRIX_FP32: values
 * and x in FP32, products and sum in FP64, one rounding to FP32).  x should
 * be finite: the offset-list layouts multiply stored zeros by neighbouring
 * elements of x, so a NaN or Inf in x can also reach rows without an entry
 * in its column (the solvers stop with SSPCG_ERR_NONFINITE either way). */
int sspcg_spmv(const sspcg_matrix* A, int32_t dtype, const void* x, void* y, sspcg_stream stream);

/* Algorithm 2 for the residual r: Z = [z_1..z_s] and P = [p_1..p_{s+1}]
 * (device, n x s and n x (s+1), leading dimension ld, dtype elements) with
 * z_1 = M^{-1} r, z_{q+1} the Chebyshev three-term recurrence in
 * alpha M^{-1}A - sigma I (first step the T_1 one), p_1 = r, p_{q+1} = A z_q;
 * alpha = 2/(lmax-lmin), sigma = (lmax+lmin)/(lmax-lmin), gamma = 1.  With
 * basis = SSPCG_BASIS_MONOMIAL, z_{q+1} = M^{-1} p_{q+1} (interval unused). */
int sspcg_mpk(const sspcg_matrix* A, int32_t dtype, const void* r, int32_t s, double lmin,
              double lmax, int32_t basis, void* Z, void* P, int64_t ld, sspcg_stream stream);

/* Block update fused with the Gram reduction of Algorithm 1:
 *   if beta != NULL: Q <- Z + Q beta and AQ <- AZ + AQ beta (in place);
 *   else:            Q <- Z and AQ <- AZ (the first block);
 * then W = Q^T AQ (lower triangle i >= j computed, mirrored) and b1 = Q^T r.
 * Q, AQ, Z, AZ: device n x s, ld; r: device n; dtype elements.  beta, W:
 * device double s*s; b1: device double s.  Gram sums are FP64. */
int sspcg_block_update_gram(int64_t n, int32_t s, int32_t dtype, const void* Z, void* Q,
                            const void* AZ, void* AQ, const double* beta, const void* r,
                            int64_t ld, double* W, double* b1, void* work, size_t work_bytes,
                            sspcg_stream stream);

/* B2 = -Q^T AZ (all s*s entries; device double, row-major), Algorithm 1's
 * right-hand side of the beta system.  FP64 sums. */
int sspcg_gram_rect(int64_t n, int32_t s, int32_t dtype, const void* Q, const void* AZ,
                    int64_t ld, double* B2, void* work, size_t work_bytes, sspcg_stream stream);

/* FGS (or Cholesky) solve of W X = B for nrhs right-hand sides: B, X device
 * double s x nrhs row-major, W device double s x s (lower triangle read).
 * `sweeps` sweeps of (D + L_W) x_new = b - L_W^T x_old from x = 0; with
 * sweep_tol > 0 a column stops early once ||b - W x|| <= sweep_tol ||b||.
 * status (device int32): set to SSPCG_ERR_BREAKDOWN for W_ii <= 0 and to
 * SSPCG_ERR_NONFINITE for NaN/Inf in W or B, else SSPCG_OK. */
int sspcg_fgs(int32_t s, int32_t nrhs, const double* W, const double* B, int32_t sweeps,
              double sweep_tol, int32_t gram_solver, double* X, int32_t* status,
              sspcg_stream stream);

/* x += Q alpha; r -= AQ alpha; rr = ||r||^2 (device double, FP64 sum);
 * when z1 != NULL also z1 = M^{-1} r.  alpha: device double s. */
int sspcg_xr_update(const sspcg_matrix* A, int32_t s, int32_t dtype, const void* Q,
                    const void* AQ, const double* alpha, int64_t ld, void* x, void* r,
                    void* z1, double* rr, void* work, size_t work_bytes, sspcg_stream stream);

/* ---------------------------------------------------------- differentiation */
/* gval_e = -lambda_i x_j for every stored entry e = (i, j) (device double
 * arrays; gval in CSR order): the gradient of a loss L(x) with respect to the
 * matrix values when A x = b and A lambda = dL/dx. */
int sspcg_csr_value_grad(const sspcg_matrix* A, const double* lambda, const double* x,
                         double* gval, sspcg_stream stream);

/* Values of the 7-point variable-coefficient diffusion operator on the
 * matrix's pattern: k = exp(theta) per cell, off-diagonal -w_ij with
 * w_ij = 2 k_i k_j/(k_i + k_j), diagonal sum_j w_ij + (6 - deg_i) k_i.
 * theta (device double[n]), val (device double[nnz], CSR order). */
int sspcg_diffusion7_assemble(const sspcg_matrix* A, const double* theta, double* val,
                              sspcg_stream stream);

/* Vector-Jacobian product of sspcg_diffusion7_assemble:
 * gtheta_c = sum_e gval_e d(val_e)/d(theta_c) (device double arrays). */
int sspcg_diffusion7_theta_grad(const sspcg_matrix* A, const double* theta, const double* gval,
                                double* gtheta, sspcg_stream stream);

/* ------------------------------------------------------------ measurement */
/* STREAM-style triad a = b + q c over n doubles (device arrays, 16-byte
 * aligned; a must not overlap b or c), asynchronous on `stream`.  It moves
 * 24 n bytes with non-temporal 16-byte loads and stores over per-die
 * contiguous ranges, in the fastest launch shape measured for this pattern:
 * the achievable HBM bandwidth that the kernels' byte rates are set against,
 * next to the published peak.  Not a step of the method.  n = 0 does
 * nothing. */
int sspcg_stream_triad(int64_t n, const double* b, const double* c, double q, double* a,
                       sspcg_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* SSPCG_H */
