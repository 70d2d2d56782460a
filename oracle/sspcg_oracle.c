/* CPU oracle for the Chebyshev-basis s-step PCG method with Forward
 * Gauss-Seidel (FGS) Gram solves.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load it; the solver library never does,
 * and the two share no code.
 *
 * Everything is FP64 unless a function says otherwise, written as plain
 * loops in the order the paper states the operations.  Dot products are
 * taken sequentially with Neumaier's compensated summation (A. Neumaier,
 * ZAMM 54, 1974) so that the oracle's own rounding error stays far below the
 * tolerances the GPU is held to.  Loops over independent rows, and the
 * independent dot products of one Gram matrix (each still summed
 * sequentially), may run in parallel (OpenMP); that never changes a result.
 *
 * Blocks of vectors are column-major: column j of an n x m block B is
 * B + j*ld.  Small s x s matrices are row-major: W[i*s + j].
 *
 * Method references (sections, algorithms and equations of the paper):
 *   basis_info and Chebyshev recurrence ... Sec. 2 (s-step PCG with
 *                                           Chebyshev Krylov basis)
 *   MPK .................................... Algorithm 2
 *   outer iteration ........................ Algorithm 1
 *   FGS, direct form, zero start ........... Sec. 3.1, eq. (fgs-iteration)
 *   Gram residuals eta_alpha, eta_beta ..... Sec. 3.4 (numerical experiments)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops over fewer rows than this run on one thread (threads cost more
 * than they save there, and compete with other work on the host). */
#define OR_PAR_MIN 32768

enum {
    OR_OK = 0, OR_NOT_CONVERGED = 1, OR_ERR_ARG = -1, OR_BREAKDOWN = -3,
    OR_NONFINITE = -5
};

typedef struct {
    int32_t status;
    int32_t iters;          /* outer iterations (x updates) of the last solve */
    int32_t refinements;    /* mixed precision: FP64 residual corrections */
    int32_t inner_total;    /* mixed precision: inner outer-iterations, summed */
    double relres;          /* recursive ||r|| / ||b|| at exit */
    double relres_true;     /* ||b - A x|| / ||b|| at exit */
} or_result;

int or_version(void) { return 1; }

/* Sets the number of threads the row loops may use (k >= 1). */
void or_set_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* vector primitives                                                   */
/* ------------------------------------------------------------------ */

/* Compensated sequential dot product (Neumaier). */
double or_dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double p = a[i] * b[i];
        const double t = s + p;
        if (fabs(s) >= fabs(p)) c += (s - t) + p;
        else c += (p - t) + s;
        s = t;
    }
    return s + c;
}

double or_nrm2(int64_t n, const double* a) { return sqrt(or_dot(n, a, a)); }

/* y = A x for CSR A (row sums in column order). */
void or_spmv(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
             const double* x, double* y)
{
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) acc += val[e] * x[col[e]];
        y[i] = acc;
    }
}

/* FP32 storage, FP64 arithmetic: y = fl32( sum_e v_e x_col ) with the
 * products of FP32 numbers formed exactly in FP64, summed in FP64 and
 * rounded once. */
void or_spmv_f32(int64_t n, const int32_t* rp, const int32_t* col, const float* val,
                 const float* x, float* y)
{
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            acc += (double)val[e] * (double)x[col[e]];
        y[i] = (float)acc;
    }
}

/* d[i] = A_ii; returns the number of rows whose diagonal is missing or <= 0. */
int64_t or_diagonal(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                    double* d)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        double di = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] == i) di = val[e];
        d[i] = di;
        if (!(di > 0.0)) ++bad;
    }
    return bad;
}

/* Chebyshev scaling of M^{-1}A onto [-1, 1]:
 * alpha = 2/(lmax - lmin), sigma = (lmax + lmin)/(lmax - lmin), gamma = 1. */
static void basis_info(double lmin, double lmax, double* a, double* sg, double* gm)
{
    *a = 2.0 / (lmax - lmin);
    *sg = (lmax + lmin) / (lmax - lmin);
    *gm = 1.0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2: matrix powers kernel for the Chebyshev basis            */
/* ------------------------------------------------------------------ */

/* Z (n x s, ld) and P (n x (s+1), ld) from r.  zp_q is stored literally; the
 * preconditioner is M = diag(A), applied as z = dinv .* zp.
 *   p_1 = r, zp_1 = p_1, z_1 = M^{-1} zp_1
 *   p_2 = A z_1, zp_2 = alpha p_2 - sigma zp_1                (T_1 step)
 *   p_{q+1} = A z_q, zp_{q+1} = 2 alpha p_{q+1} - 2 sigma zp_q - gamma zp_{q-1}
 *   z_{q+1} = M^{-1} zp_{q+1};  finally p_{s+1} = A z_s. */
void or_mpk_basis(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                  const double* dinv, const double* r, int s, double lmin, double lmax,
                  int basis, double* Z, double* P, int64_t ld);

void or_mpk(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
            const double* dinv, const double* r, int s, double lmin, double lmax,
            double* Z, double* P, int64_t ld)
{
    or_mpk_basis(n, rp, col, val, dinv, r, s, lmin, lmax, 0, Z, P, ld);
}

/* basis = 0: the Chebyshev recurrence above.  basis = 1: the monomial block
 * of the paper's introduction, z_{q+1} = M^{-1} A z_q, i.e. zp_{q+1} =
 * p_{q+1} (the contrast the Chebyshev basis is chosen against). */
void or_mpk_basis(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                  const double* dinv, const double* r, int s, double lmin, double lmax,
                  int basis, double* Z, double* P, int64_t ld)
{
    double al, sg, gm;
    basis_info(lmin, lmax, &al, &sg, &gm);
    double* zp = (double*)malloc(sizeof(double) * (size_t)n * (size_t)s);
    #define ZP(q) (zp + (int64_t)((q) - 1) * n)
    #define ZC(q) (Z + (int64_t)((q) - 1) * ld)
    #define PC(q) (P + (int64_t)((q) - 1) * ld)
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        PC(1)[i] = r[i];
        ZP(1)[i] = PC(1)[i];
        ZC(1)[i] = dinv[i] * ZP(1)[i];
    }
    if (basis == 1) {
        for (int q = 1; q <= s - 1; ++q) {
            or_spmv(n, rp, col, val, ZC(q), PC(q + 1));
            #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) {
                ZP(q + 1)[i] = PC(q + 1)[i];
                ZC(q + 1)[i] = dinv[i] * ZP(q + 1)[i];
            }
        }
    } else if (s > 1) {
        or_spmv(n, rp, col, val, ZC(1), PC(2));
        #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
        for (int64_t i = 0; i < n; ++i) {
            ZP(2)[i] = al * PC(2)[i] - sg * ZP(1)[i];
            ZC(2)[i] = dinv[i] * ZP(2)[i];
        }
        for (int q = 2; q <= s - 1; ++q) {
            or_spmv(n, rp, col, val, ZC(q), PC(q + 1));
            #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) {
                ZP(q + 1)[i] = 2.0 * al * PC(q + 1)[i] - 2.0 * sg * ZP(q)[i] - gm * ZP(q - 1)[i];
                ZC(q + 1)[i] = dinv[i] * ZP(q + 1)[i];
            }
        }
    }
    or_spmv(n, rp, col, val, ZC(s), PC(s + 1));
    #undef ZP
    #undef ZC
    #undef PC
    free(zp);
}

/* ------------------------------------------------------------------ */
/* Gram matrices and right-hand sides (Algorithm 1, lines for W, b1, b2) */
/* ------------------------------------------------------------------ */

/* W = Q^T AQ (lower triangle i >= j computed, then mirrored) and b1 = Q^T r. */
void or_gram(int64_t n, int s, const double* Q, const double* AQ, const double* r,
             int64_t ld, double* W, double* b1)
{
    /* task t < s(s+1)/2: entry (i, j), i >= j, in row order; then b1_i */
    const int nw = s * (s + 1) / 2;
    #pragma omp parallel for schedule(dynamic, 1) if (n >= OR_PAR_MIN)
    for (int t = 0; t < nw + s; ++t) {
        if (t >= nw) {
            const int i = t - nw;
            b1[i] = or_dot(n, Q + (int64_t)i * ld, r);
            continue;
        }
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        const int j = t - i * (i + 1) / 2;
        const double w = or_dot(n, Q + (int64_t)i * ld, AQ + (int64_t)j * ld);
        W[i * s + j] = w;
        W[j * s + i] = w;
    }
}

/* B2 = -Q^T AZ, all s*s entries: B2[i*s+j] = -Q_i . AZ_j. */
void or_gram_rect(int64_t n, int s, const double* Q, const double* AZ, int64_t ld,
                  double* B2)
{
    #pragma omp parallel for schedule(dynamic, 1) if (n >= OR_PAR_MIN)
    for (int t = 0; t < s * s; ++t) {
        const int i = t / s, j = t % s;
        B2[i * s + j] = -or_dot(n, Q + (int64_t)i * ld, AZ + (int64_t)j * ld);
    }
}

/* ------------------------------------------------------------------ */
/* Forward Gauss-Seidel on the s x s Gram system                        */
/* ------------------------------------------------------------------ */

/* nu sweeps of (D + L_W) a_new = m - L_W^T a_old from a = 0, for every column
 * of the s x nrhs right-hand side B (row-major, B[i*nrhs + c]); the result
 * goes to X with the same layout.  W is read as symmetric from its lower
 * triangle.  Returns OR_BREAKDOWN if a diagonal entry is not positive and
 * OR_NONFINITE if W or B holds a non-finite value. */
int or_fgs_tol(int s, int nrhs, const double* W, const double* B, int sweeps, double delta,
               double* X);

int or_fgs(int s, int nrhs, const double* W, const double* B, int sweeps, double* X)
{
    return or_fgs_tol(s, nrhs, W, B, sweeps, 0.0, X);
}

/* As or_fgs, but with delta > 0 a column stops sweeping as soon as its
 * residual satisfies ||m - W a||_2 <= delta ||m||_2 (the practical accuracy
 * criterion of Sec. 3, eq. cond:inexactKrylov1), checked before every sweep
 * after the first; at most `sweeps` sweeps. */
int or_fgs_tol(int s, int nrhs, const double* W, const double* B, int sweeps, double delta,
               double* X)
{
    for (int i = 0; i < s; ++i) {
        for (int j = 0; j <= i; ++j)
            if (!isfinite(W[i * s + j])) return OR_NONFINITE;
        for (int c = 0; c < nrhs; ++c)
            if (!isfinite(B[i * nrhs + c])) return OR_NONFINITE;
        if (!(W[i * s + i] > 0.0)) return OR_BREAKDOWN;
    }
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < s; ++i) X[i * nrhs + c] = 0.0;
        double mn = 0.0;
        for (int i = 0; i < s; ++i) mn += B[i * nrhs + c] * B[i * nrhs + c];
        mn = sqrt(mn);
        for (int v = 0; v < sweeps; ++v) {
            if (delta > 0.0 && v > 0) {
                double r2 = 0.0;
                for (int i = 0; i < s; ++i) {
                    double t = B[i * nrhs + c];
                    for (int j = 0; j < s; ++j)
                        t -= (j <= i ? W[i * s + j] : W[j * s + i]) * X[j * nrhs + c];
                    r2 += t * t;
                }
                if (sqrt(r2) <= delta * mn) break;
            }
            for (int i = 0; i < s; ++i) {
                double t = B[i * nrhs + c];
                for (int j = 0; j < i; ++j) t -= W[i * s + j] * X[j * nrhs + c];
                for (int j = i + 1; j < s; ++j) t -= W[j * s + i] * X[j * nrhs + c];
                X[i * nrhs + c] = t / W[i * s + i];
            }
        }
    }
    return OR_OK;
}

/* Exact solve of W X = B by Cholesky (W = L L^T), the reference the paper
 * compares FGS against.  Same layouts and status rules as or_fgs. */
int or_chol_solve(int s, int nrhs, const double* W, const double* B, double* X)
{
    double L[64 * 64];
    if (s < 1 || s > 64) return OR_ERR_ARG;
    for (int i = 0; i < s; ++i) {
        for (int j = 0; j <= i; ++j)
            if (!isfinite(W[i * s + j])) return OR_NONFINITE;
        for (int c = 0; c < nrhs; ++c)
            if (!isfinite(B[i * nrhs + c])) return OR_NONFINITE;
    }
    for (int i = 0; i < s; ++i)
        for (int j = 0; j <= i; ++j) {
            double t = W[i * s + j];
            for (int k = 0; k < j; ++k) t -= L[i * s + k] * L[j * s + k];
            if (i == j) {
                if (!(t > 0.0)) return OR_BREAKDOWN;
                L[i * s + i] = sqrt(t);
            } else {
                L[i * s + j] = t / L[j * s + j];
            }
        }
    for (int c = 0; c < nrhs; ++c) {
        double y[64];
        for (int i = 0; i < s; ++i) {
            double t = B[i * nrhs + c];
            for (int k = 0; k < i; ++k) t -= L[i * s + k] * y[k];
            y[i] = t / L[i * s + i];
        }
        for (int i = s - 1; i >= 0; --i) {
            double t = y[i];
            for (int k = i + 1; k < s; ++k) t -= L[k * s + i] * X[k * nrhs + c];
            X[i * nrhs + c] = t / L[i * s + i];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Block updates                                                        */
/* ------------------------------------------------------------------ */

/* x += Q alpha;  r -= AQ alpha. */
void or_xr_update(int64_t n, int s, const double* Q, const double* AQ,
                  const double* alpha, int64_t ld, double* x, double* r)
{
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        double qa = 0.0, aqa = 0.0;
        for (int j = 0; j < s; ++j) {
            qa += Q[(int64_t)j * ld + i] * alpha[j];
            aqa += AQ[(int64_t)j * ld + i] * alpha[j];
        }
        x[i] += qa;
        r[i] -= aqa;
    }
}

/* Q <- Z + Q beta;  AQ <- AZ + AQ beta  (beta row-major s x s). */
void or_block_update(int64_t n, int s, const double* Z, double* Q, const double* AZ,
                     double* AQ, const double* beta, int64_t ld)
{
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        double q[64], aq[64];
        for (int j = 0; j < s; ++j) {
            q[j] = Q[(int64_t)j * ld + i];
            aq[j] = AQ[(int64_t)j * ld + i];
        }
        for (int j = 0; j < s; ++j) {
            double tq = 0.0, taq = 0.0;
            for (int l = 0; l < s; ++l) {
                tq += q[l] * beta[l * s + j];
                taq += aq[l] * beta[l * s + j];
            }
            Q[(int64_t)j * ld + i] = Z[(int64_t)j * ld + i] + tq;
            AQ[(int64_t)j * ld + i] = AZ[(int64_t)j * ld + i] + taq;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Diagnostics: relative residuals of the two reduced systems           */
/* ------------------------------------------------------------------ */

/* ||B - W X||_F, the absolute residual of the reduced system.  For the beta
 * system it is the size of Q_{k+1}^T A Q_k: with B2 = -Q_k^T AZ and
 * Q_{k+1} = Z + Q_k beta, Q_k^T A Q_{k+1} = -B2 + W beta (Sec. 2). */
double or_gram_resnorm(int s, int nrhs, const double* W, const double* B, const double* X)
{
    double num = 0.0;
    for (int c = 0; c < nrhs; ++c)
        for (int i = 0; i < s; ++i) {
            double t = B[i * nrhs + c];
            for (int j = 0; j < s; ++j) t -= W[i * s + j] * X[j * nrhs + c];
            num += t * t;
        }
    return sqrt(num);
}

/* ||m - W a||_2 / ||m||_2 for every column, combined in the Frobenius norm. */
double or_gram_relres(int s, int nrhs, const double* W, const double* B, const double* X)
{
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nrhs; ++c)
        for (int i = 0; i < s; ++i) {
            double t = B[i * nrhs + c];
            for (int j = 0; j < s; ++j) t -= W[i * s + j] * X[j * nrhs + c];
            num += t * t;
            den += B[i * nrhs + c] * B[i * nrhs + c];
        }
    return den > 0.0 ? sqrt(num / den) : 0.0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: s-step PCG with Chebyshev basis and FGS Gram solves     */
/* ------------------------------------------------------------------ */

/* Solves A x = b from x (in: x0, out: x).  gram = 0: FGS with `sweeps`
 * sweeps (or fewer once a column meets sweep_tol > 0, see or_fgs_tol);
 * gram = 1: Cholesky.  basis: 0 Chebyshev, 1 monomial (or_mpk_basis).
 * hist (optional, 4*max_outer doubles) receives per outer iteration k: the
 * relative residual after the x update, eta_alpha, eta_beta and the
 * conjugacy defect ||B2 - W beta||_F (the last two 0 where no beta system
 * was solved).
 * Stops when ||r|| <= tol ||b|| on the recursively updated residual.  If
 * ||b|| = 0 the solution is x = 0; if the starting residual already meets the
 * test no iteration is taken. */
int or_sspcg_perturbed(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                       const double* b, double* x, int s, int sweeps, double lmin,
                       double lmax, double tol, int max_outer, int gram, double sweep_tol,
                       int basis, uint64_t perturb_seed, double* hist, or_result* res);

int or_sspcg(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
             const double* b, double* x, int s, int sweeps, double lmin, double lmax,
             double tol, int max_outer, int gram, double sweep_tol, int basis, double* hist,
             or_result* res)
{
    return or_sspcg_perturbed(n, rp, col, val, b, x, s, sweeps, lmin, lmax, tol, max_outer,
                              gram, sweep_tol, basis, 0, hist, res);
}

/* SplitMix64 (G. Steele, D. Lea, C. Flood, OOPSLA 2014): a counter-based
 * generator for the Gram perturbations below. */
static uint64_t splitmix64(uint64_t* state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Moves every entry of an m-entry Gram block one unit in the last place up
 * or down, at random.  A symmetric W is perturbed in its lower triangle and
 * mirrored, so it stays symmetric. */
static void ulp_perturb(double* v, int rows, int cols, int symmetric, uint64_t* state)
{
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < (symmetric ? i + 1 : cols); ++j) {
            const double up = (splitmix64(state) & 1) ? INFINITY : -INFINITY;
            v[i * cols + j] = nextafter(v[i * cols + j], up);
            if (symmetric) v[j * cols + i] = v[i * cols + j];
        }
}

/* As or_sspcg; with perturb_seed != 0 each W, b1 and B2 the solve forms is
 * moved by one unit in the last place per entry (a seeded random direction)
 * before it is solved: repeated runs then show how far rounding alone moves
 * the iteration count and the solution. */
int or_sspcg_perturbed(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                       const double* b, double* x, int s, int sweeps, double lmin,
                       double lmax, double tol, int max_outer, int gram, double sweep_tol,
                       int basis, uint64_t perturb_seed, double* hist, or_result* res)
{
    memset(res, 0, sizeof(*res));
    uint64_t rng = perturb_seed;
    if (n < 1 || s < 1 || s > 64 || (gram == 0 && sweeps < 1) || !(lmax > lmin)
        || !(lmin >= 0.0) || !(tol > 0.0) || max_outer < 1) {
        res->status = OR_ERR_ARG;
        return OR_ERR_ARG;
    }
    const int64_t ld = n;
    const double nb = or_nrm2(n, b);
    if (!isfinite(nb)) { res->status = OR_NONFINITE; return OR_NONFINITE; }
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        res->status = OR_OK;
        return OR_OK;
    }
    double* dinv = (double*)malloc(sizeof(double) * n);
    if (or_diagonal(n, rp, col, val, dinv) != 0) {
        free(dinv);
        res->status = OR_BREAKDOWN;
        return OR_BREAKDOWN;
    }
    for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];

    double* r = (double*)malloc(sizeof(double) * n);
    double* Z = (double*)malloc(sizeof(double) * n * s);
    double* P = (double*)malloc(sizeof(double) * n * (s + 1));
    double* Q = (double*)malloc(sizeof(double) * n * s);
    double* AQ = (double*)malloc(sizeof(double) * n * s);
    double W[64 * 64], b1[64], al[64], B2[64 * 64], be[64 * 64];

    /* r0 = b - A x0 */
    or_spmv(n, rp, col, val, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double relres = or_nrm2(n, r) / nb;
    int status = OR_NOT_CONVERGED, k = 0;
    if (relres <= tol) { status = OR_OK; goto done; }

    or_mpk_basis(n, rp, col, val, dinv, r, s, lmin, lmax, basis, Z, P, ld);
    memcpy(Q, Z, sizeof(double) * n * s);
    memcpy(AQ, P + ld, sizeof(double) * n * s);
    for (k = 0; k < max_outer; ++k) {
        or_gram(n, s, Q, AQ, P, ld, W, b1);        /* P(:,1) = r */
        if (perturb_seed) {
            ulp_perturb(W, s, s, 1, &rng);
            ulp_perturb(b1, s, 1, 0, &rng);
        }
        int st = gram ? or_chol_solve(s, 1, W, b1, al)
                      : or_fgs_tol(s, 1, W, b1, sweeps, sweep_tol, al);
        if (st != OR_OK) { status = st; break; }
        or_xr_update(n, s, Q, AQ, al, ld, x, r);
        relres = or_nrm2(n, r) / nb;
        if (hist) {
            hist[4 * k] = relres;
            hist[4 * k + 1] = or_gram_relres(s, 1, W, b1, al);
            hist[4 * k + 2] = 0.0;
            hist[4 * k + 3] = 0.0;
        }
        if (!isfinite(relres)) { status = OR_NONFINITE; k += 1; break; }
        if (relres <= tol) { status = OR_OK; k += 1; break; }
        or_mpk_basis(n, rp, col, val, dinv, r, s, lmin, lmax, basis, Z, P, ld);
        /* AQ_new = P(:, 2:s+1) */
        or_gram_rect(n, s, Q, P + ld, ld, B2);
        if (perturb_seed) ulp_perturb(B2, s, s, 0, &rng);
        st = gram ? or_chol_solve(s, s, W, B2, be)
                  : or_fgs_tol(s, s, W, B2, sweeps, sweep_tol, be);
        if (hist) {
            hist[4 * k + 2] = or_gram_relres(s, s, W, B2, be);
            hist[4 * k + 3] = or_gram_resnorm(s, s, W, B2, be);
        }
        if (st != OR_OK) { status = st; k += 1; break; }
        or_block_update(n, s, Z, Q, P + ld, AQ, be, ld);
    }
done:
    res->status = status;
    res->iters = k;
    res->relres = relres;
    {
        double* t = (double*)malloc(sizeof(double) * n);
        or_spmv(n, rp, col, val, x, t);
        for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
        res->relres_true = or_nrm2(n, t) / nb;
        free(t);
    }
    free(dinv); free(r); free(Z); free(P); free(Q); free(AQ);
    return status;
}

/* ------------------------------------------------------------------ */
/* Classical Jacobi PCG (the comparator)                                */
/* ------------------------------------------------------------------ */

/* hist (optional, max_iter doubles): relative residual after each step. */
int or_pcg(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
           const double* b, double* x, double tol, int max_iter, double* hist,
           or_result* res)
{
    memset(res, 0, sizeof(*res));
    if (n < 1 || !(tol > 0.0) || max_iter < 1) { res->status = OR_ERR_ARG; return OR_ERR_ARG; }
    const double nb = or_nrm2(n, b);
    if (!isfinite(nb)) { res->status = OR_NONFINITE; return OR_NONFINITE; }
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        return OR_OK;
    }
    double* dinv = (double*)malloc(sizeof(double) * n);
    if (or_diagonal(n, rp, col, val, dinv) != 0) {
        free(dinv);
        res->status = OR_BREAKDOWN;
        return OR_BREAKDOWN;
    }
    for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];
    double* r = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    or_spmv(n, rp, col, val, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double relres = or_nrm2(n, r) / nb;
    int status = OR_NOT_CONVERGED, k = 0;
    if (relres <= tol) { status = OR_OK; goto done; }
    for (int64_t i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rho = or_dot(n, r, z);
    for (k = 0; k < max_iter; ++k) {
        or_spmv(n, rp, col, val, p, q);
        const double pq = or_dot(n, p, q);
        if (!(pq > 0.0)) { status = isfinite(pq) ? OR_BREAKDOWN : OR_NONFINITE; break; }
        const double a = rho / pq;
        for (int64_t i = 0; i < n; ++i) { x[i] += a * p[i]; r[i] -= a * q[i]; }
        relres = or_nrm2(n, r) / nb;
        if (hist) hist[k] = relres;
        if (!isfinite(relres)) { status = OR_NONFINITE; k += 1; break; }
        if (relres <= tol) { status = OR_OK; k += 1; break; }
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        const double rho_new = or_dot(n, r, z);
        const double bt = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + bt * p[i];
        rho = rho_new;
    }
done:
    res->status = status;
    res->iters = k;
    res->relres = relres;
    {
        or_spmv(n, rp, col, val, x, q);
        for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
        res->relres_true = or_nrm2(n, q) / nb;
    }
    free(dinv); free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Mixed precision: FP32 inner s-step PCG inside FP64 refinement        */
/* ------------------------------------------------------------------ */
/* Storage of matrix values, Jacobi scaling, basis vectors, directions and
 * the inner residual/correction is FP32.  Every arithmetic step forms its
 * result in FP64 from the (exactly converted) FP32 inputs and rounds once
 * when it stores to FP32.  Gram entries, FGS solves, norms and the true
 * residual b - A x of the outer loop are FP64. */

static double dot_f32(int64_t n, const float* a, const float* b)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double p = (double)a[i] * (double)b[i];
        const double t = s + p;
        if (fabs(s) >= fabs(p)) c += (s - t) + p;
        else c += (p - t) + s;
        s = t;
    }
    return s + c;
}

/* Algorithm 2 in FP32 storage (zp stored, z = dinv .* zp). */
void or_mpk_f32(int64_t n, const int32_t* rp, const int32_t* col, const float* val,
                const float* dinv, const float* r, int s, double lmin, double lmax,
                float* Z, float* P, int64_t ld)
{
    double al, sg, gm;
    basis_info(lmin, lmax, &al, &sg, &gm);
    float* zp = (float*)malloc(sizeof(float) * (size_t)n * (size_t)s);
    #define ZP(q) (zp + (int64_t)((q) - 1) * n)
    #define ZC(q) (Z + (int64_t)((q) - 1) * ld)
    #define PC(q) (P + (int64_t)((q) - 1) * ld)
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        PC(1)[i] = r[i];
        ZP(1)[i] = PC(1)[i];
        ZC(1)[i] = (float)((double)dinv[i] * (double)ZP(1)[i]);
    }
    if (s > 1) {
        or_spmv_f32(n, rp, col, val, ZC(1), PC(2));
        #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
        for (int64_t i = 0; i < n; ++i) {
            ZP(2)[i] = (float)(al * (double)PC(2)[i] - sg * (double)ZP(1)[i]);
            ZC(2)[i] = (float)((double)dinv[i] * (double)ZP(2)[i]);
        }
        for (int q = 2; q <= s - 1; ++q) {
            or_spmv_f32(n, rp, col, val, ZC(q), PC(q + 1));
            #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) {
                ZP(q + 1)[i] = (float)(2.0 * al * (double)PC(q + 1)[i] - 2.0 * sg * (double)ZP(q)[i]
                                       - gm * (double)ZP(q - 1)[i]);
                ZC(q + 1)[i] = (float)((double)dinv[i] * (double)ZP(q + 1)[i]);
            }
        }
    }
    or_spmv_f32(n, rp, col, val, ZC(s), PC(s + 1));
    #undef ZP
    #undef ZC
    #undef PC
    free(zp);
}

void or_gram_f32(int64_t n, int s, const float* Q, const float* AQ, const float* r,
                 int64_t ld, double* W, double* b1)
{
    /* the tasks of or_gram */
    const int nw = s * (s + 1) / 2;
    #pragma omp parallel for schedule(dynamic, 1) if (n >= OR_PAR_MIN)
    for (int t = 0; t < nw + s; ++t) {
        if (t >= nw) {
            const int i = t - nw;
            b1[i] = dot_f32(n, Q + (int64_t)i * ld, r);
            continue;
        }
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        const int j = t - i * (i + 1) / 2;
        const double w = dot_f32(n, Q + (int64_t)i * ld, AQ + (int64_t)j * ld);
        W[i * s + j] = w;
        W[j * s + i] = w;
    }
}

void or_gram_rect_f32(int64_t n, int s, const float* Q, const float* AZ, int64_t ld,
                      double* B2)
{
    #pragma omp parallel for schedule(dynamic, 1) if (n >= OR_PAR_MIN)
    for (int t = 0; t < s * s; ++t) {
        const int i = t / s, j = t % s;
        B2[i * s + j] = -dot_f32(n, Q + (int64_t)i * ld, AZ + (int64_t)j * ld);
    }
}

void or_xr_update_f32(int64_t n, int s, const float* Q, const float* AQ,
                      const double* alpha, int64_t ld, float* x, float* r)
{
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        double qa = 0.0, aqa = 0.0;
        for (int j = 0; j < s; ++j) {
            qa += (double)Q[(int64_t)j * ld + i] * alpha[j];
            aqa += (double)AQ[(int64_t)j * ld + i] * alpha[j];
        }
        x[i] = (float)((double)x[i] + qa);
        r[i] = (float)((double)r[i] - aqa);
    }
}

void or_block_update_f32(int64_t n, int s, const float* Z, float* Q, const float* AZ,
                         float* AQ, const double* beta, int64_t ld)
{
    #pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        double q[64], aq[64];
        for (int j = 0; j < s; ++j) {
            q[j] = Q[(int64_t)j * ld + i];
            aq[j] = AQ[(int64_t)j * ld + i];
        }
        for (int j = 0; j < s; ++j) {
            double tq = 0.0, taq = 0.0;
            for (int l = 0; l < s; ++l) {
                tq += q[l] * beta[l * s + j];
                taq += aq[l] * beta[l * s + j];
            }
            Q[(int64_t)j * ld + i] = (float)((double)Z[(int64_t)j * ld + i] + tq);
            AQ[(int64_t)j * ld + i] = (float)((double)AZ[(int64_t)j * ld + i] + taq);
        }
    }
}

/* Inner FP32 s-step PCG for A d = r32 from d = 0; stops when the recursive
 * inner residual satisfies ||r_in|| <= inner_tol * ||r32|| or after
 * max_inner outer iterations.  Returns a status; *iters gets the count.
 * Exported so that tests can pin it directly. */
int or_inner_sspcg_f32(int64_t n, const int32_t* rp, const int32_t* col,
                           const float* val, const float* dinv, const float* r32,
                           float* d, int s, int sweeps, double lmin, double lmax,
                           double inner_tol, int max_inner, int* iters)
{
    const int64_t ld = n;
    float* r = (float*)malloc(sizeof(float) * n);
    float* Z = (float*)malloc(sizeof(float) * n * s);
    float* P = (float*)malloc(sizeof(float) * n * (s + 1));
    float* Q = (float*)malloc(sizeof(float) * n * s);
    float* AQ = (float*)malloc(sizeof(float) * n * s);
    double W[64 * 64], b1[64], al[64], B2[64 * 64], be[64 * 64];
    const double n0 = sqrt(dot_f32(n, r32, r32));
    int status = OR_NOT_CONVERGED, k = 0;
    for (int64_t i = 0; i < n; ++i) { d[i] = 0.0f; r[i] = r32[i]; }
    or_mpk_f32(n, rp, col, val, dinv, r, s, lmin, lmax, Z, P, ld);
    memcpy(Q, Z, sizeof(float) * n * s);
    memcpy(AQ, P + ld, sizeof(float) * n * s);
    for (k = 0; k < max_inner; ++k) {
        or_gram_f32(n, s, Q, AQ, P, ld, W, b1);
        int st = or_fgs(s, 1, W, b1, sweeps, al);
        if (st != OR_OK) { status = st; break; }
        or_xr_update_f32(n, s, Q, AQ, al, ld, d, r);
        const double nr = sqrt(dot_f32(n, r, r));
        if (!isfinite(nr)) { status = OR_NONFINITE; k += 1; break; }
        if (nr <= inner_tol * n0) { status = OR_OK; k += 1; break; }
        or_mpk_f32(n, rp, col, val, dinv, r, s, lmin, lmax, Z, P, ld);
        or_gram_rect_f32(n, s, Q, P + ld, ld, B2);
        st = or_fgs(s, s, W, B2, sweeps, be);
        if (st != OR_OK) { status = st; k += 1; break; }
        or_block_update_f32(n, s, Z, Q, P + ld, AQ, be, ld);
    }
    *iters = k;
    free(r); free(Z); free(P); free(Q); free(AQ);
    return status;
}

/* Iterative refinement: r = b - A x in FP64; stop when ||r|| <= tol ||b||;
 * else solve A d = fl32(r) with the FP32 inner method and set x += d.  The
 * inner solve of a refinement reduces its residual by inner_tol, or only to
 * half the outer target when that is less work:
 * its relative tolerance is min(max(inner_tol, tol / (2 relres)), 1/2).
 * hist (optional, max_refine+1 doubles): true relative residual before each
 * correction.  An inner NOT_CONVERGED is accepted (the correction is still
 * applied); inner breakdowns end the solve. */
int or_sspcg_mixed(int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                   const double* b, double* x, int s, int sweeps, double lmin, double lmax,
                   double tol, double inner_tol, int max_inner, int max_refine,
                   double* hist, or_result* res)
{
    memset(res, 0, sizeof(*res));
    if (n < 1 || s < 1 || s > 64 || sweeps < 1 || !(lmax > lmin) || !(lmin >= 0.0)
        || !(tol > 0.0) || !(inner_tol > 0.0) || max_inner < 1 || max_refine < 0) {
        res->status = OR_ERR_ARG;
        return OR_ERR_ARG;
    }
    const double nb = or_nrm2(n, b);
    if (!isfinite(nb)) { res->status = OR_NONFINITE; return OR_NONFINITE; }
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        return OR_OK;
    }
    double* dg = (double*)malloc(sizeof(double) * n);
    if (or_diagonal(n, rp, col, val, dg) != 0) {
        free(dg);
        res->status = OR_BREAKDOWN;
        return OR_BREAKDOWN;
    }
    const int64_t nnz = rp[n];
    float* val32 = (float*)malloc(sizeof(float) * (nnz > 0 ? nnz : 1));
    float* dinv32 = (float*)malloc(sizeof(float) * n);
    for (int64_t e = 0; e < nnz; ++e) val32[e] = (float)val[e];
    for (int64_t i = 0; i < n; ++i) dinv32[i] = (float)(1.0 / dg[i]);
    double* r = (double*)malloc(sizeof(double) * n);
    float* r32 = (float*)malloc(sizeof(float) * n);
    float* d32 = (float*)malloc(sizeof(float) * n);
    int status = OR_NOT_CONVERGED, inner_total = 0, nref = 0;
    double relres = 0.0;
    for (;;) {
        or_spmv(n, rp, col, val, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        relres = or_nrm2(n, r) / nb;
        if (hist) hist[nref] = relres;
        if (!isfinite(relres)) { status = OR_NONFINITE; break; }
        if (relres <= tol) { status = OR_OK; break; }
        if (nref >= max_refine) { status = OR_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) r32[i] = (float)r[i];
        double itol = 0.5 * tol / relres;
        if (itol < inner_tol) itol = inner_tol;
        if (itol > 0.5) itol = 0.5;
        int it = 0;
        const int st = or_inner_sspcg_f32(n, rp, col, val32, dinv32, r32, d32, s, sweeps,
                                       lmin, lmax, itol, max_inner, &it);
        inner_total += it;
        if (st != OR_OK && st != OR_NOT_CONVERGED) { status = st; break; }
        for (int64_t i = 0; i < n; ++i) x[i] += (double)d32[i];
        ++nref;
    }
    res->status = status;
    res->iters = inner_total;
    res->refinements = nref;
    res->inner_total = inner_total;
    res->relres = relres;
    res->relres_true = relres;
    free(dg); free(val32); free(dinv32); free(r); free(r32); free(d32);
    return status;
}

/* ------------------------------------------------------------------ */
/* Differentiable solve on the 7-point diffusion operator               */
/* ------------------------------------------------------------------ */
/* A(theta): k = exp(theta) per cell; off-diagonal -w_ij with
 * w_ij = 2 k_i k_j / (k_i + k_j); diagonal sum_j w_ij + (6 - deg_i) k_i.
 * The CSR structure (row_ptr, col) is given; values are written to val. */
void or_diffusion7_assemble(int64_t n, const int32_t* rp, const int32_t* col,
                            const double* theta, double* val)
{
    for (int64_t i = 0; i < n; ++i) {
        const double ki = exp(theta[i]);
        double diag = 0.0;
        int deg = 0;
        int64_t dpos = -1;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t j = col[e];
            if (j == i) { dpos = e; continue; }
            const double kj = exp(theta[j]);
            const double w = 2.0 * ki * kj / (ki + kj);
            val[e] = -w;
            diag += w;
            ++deg;
        }
        diag += (double)(6 - deg) * ki;
        if (dpos >= 0) val[dpos] = diag;
    }
}

/* dL/dA_ij = -lambda_i x_j over the sparsity pattern (the gradient of
 * L(x(A)) when A x = b and A lambda = dL/dx). */
void or_csr_value_grad(int64_t n, const int32_t* rp, const int32_t* col,
                       const double* lambda, const double* x, double* gval)
{
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) gval[e] = -lambda[i] * x[col[e]];
}

/* Chain rule through the assembly: gtheta_c = sum_e gval_e d(val_e)/d(theta_c).
 * dw_ij/dtheta_i = w_ij k_j/(k_i + k_j); d((6-deg_i) k_i)/dtheta_i = (6-deg_i) k_i.
 * Written as a scatter over the nonzeros. */
void or_diffusion7_theta_grad(int64_t n, const int32_t* rp, const int32_t* col,
                              const double* theta, const double* gval, double* gtheta)
{
    for (int64_t i = 0; i < n; ++i) gtheta[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double ki = exp(theta[i]);
        int deg = 0;
        int64_t dpos = -1;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] == i) dpos = e; else ++deg;
        const double gd = dpos >= 0 ? gval[dpos] : 0.0;
        gtheta[i] += gd * (double)(6 - deg) * ki;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t j = col[e];
            if (j == i) continue;
            const double kj = exp(theta[j]);
            const double w = 2.0 * ki * kj / (ki + kj);
            const double dwi = w * kj / (ki + kj);   /* dw/dtheta_i */
            const double dwj = w * ki / (ki + kj);   /* dw/dtheta_j */
            /* off-diagonal entry (i,j) = -w */
            gtheta[i] -= gval[e] * dwi;
            gtheta[j] -= gval[e] * dwj;
            /* diagonal entry (i,i) contains +w */
            gtheta[i] += gd * dwi;
            gtheta[j] += gd * dwj;
        }
    }
}
