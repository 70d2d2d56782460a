// Single-block kernels that end each reduction and solve the reduced
// systems of the outer iteration (Algorithm 1):
//  - the alpha system W a = b1 and the beta system W B = B2 = -Q^T AZ,
//    solved by `sweeps` Forward Gauss-Seidel sweeps from zero, the direct
//    form (D + L_W) a_new = m - L_W^T a_old of Sec. 3.1, or by Cholesky;
//  - the residual norm, the relative residual and the stop test.
// A block of 1024 threads first sums the per-block partials in a fixed order
// (16 wavefronts, one entry per wavefront at a time); the s x s solve itself
// is a few hundred flops, done by one thread per right-hand side.  No host
// round trip: the results stay in device memory for the next kernel.

#include "launch.h"

namespace sspcg {

namespace {

// Checks W (lower triangle) and B; returns a status.
template <int S>
__device__ inline int check_system(const double (&W)[S][S], const double (&B)[S][S], int nrhs)
{
    int st = SSPCG_OK;
    for (int i = 0; i < S; ++i) {
        for (int j = 0; j <= i; ++j)
            if (!isfinite(W[i][j])) st = SSPCG_ERR_NONFINITE;
        for (int c = 0; c < nrhs; ++c)
            if (!isfinite(B[i][c])) st = SSPCG_ERR_NONFINITE;
    }
    if (st == SSPCG_OK)
        for (int i = 0; i < S; ++i)
            if (!(W[i][i] > 0.0)) st = SSPCG_ERR_BREAKDOWN;
    return st;
}

// Cholesky factor L of W into L (lower); returns a status.
template <int S>
__device__ inline int cholesky(const double (&W)[S][S], double (&L)[S][S])
{
    for (int i = 0; i < S; ++i)
        for (int j = 0; j <= i; ++j) {
            double t = W[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(t > 0.0)) return SSPCG_ERR_BREAKDOWN;
                L[i][i] = sqrt(t);
            } else {
                L[i][j] = t / L[j][j];
            }
        }
    return SSPCG_OK;
}

// ||b - W x||_2 for column c (W mirrored from its lower triangle).
template <int S>
__device__ inline double column_residual(const double (&W)[S][S], const double (&B)[S][S], int c,
                                         const double (&x)[S])
{
    double r2 = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        double t = B[i][c];
#pragma unroll
        for (int j = 0; j < S; ++j) t -= (j <= i ? W[i][j] : W[j][i]) * x[j];
        r2 += t * t;
    }
    return sqrt(r2);
}

// Column c of X from column c of B: FGS sweeps (at most `sweeps`; with
// delta > 0 stopping once ||b - W x|| <= delta ||b||) or the Cholesky solve.
template <int S>
__device__ inline void solve_column(const double (&W)[S][S], const double (&L)[S][S],
                                    const double (&B)[S][S], int c, int sweeps, double delta,
                                    int solver, double (&X)[S][S])
{
    double x[S];
    if (solver == SSPCG_GRAM_CHOLESKY) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double t = B[i][c];
#pragma unroll
            for (int k = 0; k < i; ++k) t -= L[i][k] * x[k];
            x[i] = t / L[i][i];
        }
#pragma unroll
        for (int i = S - 1; i >= 0; --i) {
            double t = x[i];
#pragma unroll
            for (int k = i + 1; k < S; ++k) t -= L[k][i] * x[k];
            x[i] = t / L[i][i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < S; ++i) x[i] = 0.0;
        double bn = 0.0;
        if (delta > 0.0) {
#pragma unroll
            for (int i = 0; i < S; ++i) bn += B[i][c] * B[i][c];
            bn = sqrt(bn);
        }
        for (int v = 0; v < sweeps; ++v) {
            if (delta > 0.0 && v > 0 && column_residual<S>(W, B, c, x) <= delta * bn) break;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                double t = B[i][c];
#pragma unroll
                for (int j = 0; j < i; ++j) t -= W[i][j] * x[j];
#pragma unroll
                for (int j = i + 1; j < S; ++j) t -= W[j][i] * x[j];
                x[i] = t / W[i][i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < S; ++i) X[i][c] = x[i];
}

// ||B - W X||_F and ||B||_F over nrhs columns (W mirrored from its lower part).
template <int S>
__device__ inline void reduced_residual(const double (&W)[S][S], const double (&B)[S][S],
                                        const double (&X)[S][S], int nrhs, double* res,
                                        double* rhs)
{
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nrhs; ++c)
        for (int i = 0; i < S; ++i) {
            double t = B[i][c];
            for (int j = 0; j < S; ++j) t -= (j <= i ? W[i][j] : W[j][i]) * X[j][c];
            num += t * t;
            den += B[i][c] * B[i][c];
        }
    *res = sqrt(num);
    *rhs = sqrt(den);
}

// which = 0: alpha system.  Partials: W lower (row-major, i >= j) then b1.
// which = 1: beta system.   Partials: Q^T AZ (row-major); W from Wbuf.
template <int S>
__global__ __launch_bounds__(kFinBlock) void k_fgs_step(int which, const double* __restrict__ partials,
                                                        int G, double* __restrict__ Wbuf,
                                                        double* __restrict__ out, int sweeps,
                                                        double delta, int solver,
                                                        Ctrl* __restrict__ ctrl,
                                                        double* __restrict__ hist)
{
    if (ctrl->done) return;
    // the alpha system follows the block update, which has applied any
    // pending x += Q alpha with the previous alpha before this overwrites it
    if (which == 0 && threadIdx.x == 0) ctrl->x_pending = 0;
    const int K = which == 0 ? S * (S + 1) / 2 + S : S * S;
    __shared__ double sv[S * S + S];
    __shared__ double W[S][S], L[S][S], B[S][S], X[S][S];
    __shared__ int st;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int e = wave; e < K; e += kFinBlock / kWave) {
        const double v = wave_finish(partials, e, G);
        if (lane == 0) sv[e] = v;
    }
    __syncthreads();
    const int nrhs = which == 0 ? 1 : S;
    if (threadIdx.x == 0) {
        if (which == 0) {
            int e = 0;
            for (int i = 0; i < S; ++i)
                for (int j = 0; j <= i; ++j) {
                    W[i][j] = sv[e];
                    W[j][i] = sv[e];
                    ++e;
                }
            for (int i = 0; i < S; ++i) B[i][0] = sv[e + i];
        } else {
            for (int i = 0; i < S; ++i)
                for (int j = 0; j < S; ++j) {
                    W[i][j] = Wbuf[i * S + j];
                    B[i][j] = -sv[i * S + j];
                }
        }
        int s0 = check_system<S>(W, B, nrhs);
        if (s0 == SSPCG_OK && solver == SSPCG_GRAM_CHOLESKY) s0 = cholesky<S>(W, L);
        st = s0;
    }
    __syncthreads();
    if (st == SSPCG_OK && (int)threadIdx.x < nrhs)
        solve_column<S>(W, L, B, threadIdx.x, sweeps, delta, solver, X);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (st != SSPCG_OK) {
            ctrl->status = st;
            ctrl->done = 1;
            return;
        }
        if (which == 0) {
            for (int i = 0; i < S; ++i) {
                out[i] = X[i][0];
                for (int j = 0; j < S; ++j) Wbuf[i * S + j] = W[i][j];
            }
            if (hist) {
                double res, rhs;
                reduced_residual<S>(W, B, X, 1, &res, &rhs);
                hist[kHistStride * ctrl->iter + 1] = rhs > 0.0 ? res / rhs : 0.0;
            }
        } else {
            for (int i = 0; i < S; ++i)
                for (int j = 0; j < S; ++j) out[i * S + j] = X[i][j];
            if (hist && ctrl->iter > 0) {
                // eta_beta and the conjugacy defect: Q_{k+1}^T A Q_k = -(B2 - W beta)^T
                double res, rhs;
                reduced_residual<S>(W, B, X, S, &res, &rhs);
                hist[kHistStride * (ctrl->iter - 1) + 2] = rhs > 0.0 ? res / rhs : 0.0;
                hist[kHistStride * (ctrl->iter - 1) + 3] = res;
            }
        }
    }
}

template <int S>
__global__ __launch_bounds__(kWave) void k_fgs_direct(int nrhs, const double* __restrict__ Wd,
                                                      const double* __restrict__ Bd, int sweeps,
                                                      double delta, int solver,
                                                      double* __restrict__ Xd,
                                                      int32_t* __restrict__ status)
{
    __shared__ double W[S][S], L[S][S], B[S][S], X[S][S];
    __shared__ int st;
    const int chunk = S;   // right-hand sides handled per pass
    if (threadIdx.x == 0) {
        for (int i = 0; i < S; ++i)
            for (int j = 0; j <= i; ++j) {
                W[i][j] = Wd[i * S + j];
                W[j][i] = Wd[i * S + j];
            }
        st = SSPCG_OK;
    }
    __syncthreads();
    for (int c0 = 0; c0 < nrhs; c0 += chunk) {
        const int nc = min(chunk, nrhs - c0);
        if (threadIdx.x == 0) {
            for (int i = 0; i < S; ++i)
                for (int c = 0; c < nc; ++c) B[i][c] = Bd[i * nrhs + c0 + c];
            int s0 = check_system<S>(W, B, nc);
            if (s0 == SSPCG_OK && solver == SSPCG_GRAM_CHOLESKY) s0 = cholesky<S>(W, L);
            if (st == SSPCG_OK) st = s0;
        }
        __syncthreads();
        if (st == SSPCG_OK && (int)threadIdx.x < nc)
            solve_column<S>(W, L, B, threadIdx.x, sweeps, delta, solver, X);
        __syncthreads();
        if (st == SSPCG_OK && threadIdx.x == 0)
            for (int i = 0; i < S; ++i)
                for (int c = 0; c < nc; ++c) Xd[i * nrhs + c0 + c] = X[i][c];
        __syncthreads();
    }
    if (threadIdx.x == 0) *status = st;
}

// The outer iteration k is ctrl->iter (the x updates taken so far), so a
// sequence of iterations has no per-iteration launch argument and can be
// replayed from a HIP graph.
__global__ __launch_bounds__(kWave) void k_norm_step(const double* __restrict__ partials, int G,
                                                     Ctrl* __restrict__ ctrl,
                                                     double* __restrict__ hist)
{
    if (ctrl->done) return;
    const double rr = wave_finish(partials, 0, G);
    if (threadIdx.x != 0) return;
    // the x/r update before this step changed r only: x += Q alpha is
    // applied by the next block update (or at the end of the solve)
    ctrl->x_pending = 1;
    const int64_t k = ctrl->iter;
    const double relres = sqrt(rr) / ctrl->nb;
    ctrl->relres = relres;
    ctrl->iter = (int32_t)(k + 1);
    if (hist) {
        hist[kHistStride * k] = relres;
        hist[kHistStride * k + 2] = 0.0;
        hist[kHistStride * k + 3] = 0.0;
    }
    if (!isfinite(relres)) {
        ctrl->status = SSPCG_ERR_NONFINITE;
        ctrl->done = 1;
    } else if (relres <= ctrl->tol) {
        ctrl->status = SSPCG_OK;
        ctrl->done = 1;
    } else if (k + 1 >= ctrl->max_iter) {
        ctrl->status = SSPCG_NOT_CONVERGED;
        ctrl->done = 1;
    }
}

__global__ __launch_bounds__(kFinBlock) void k_finish(const double* __restrict__ partials, int K,
                                                      int G, double* __restrict__ out)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int e = wave; e < K; e += kFinBlock / kWave) {
        const double v = wave_finish(partials, e, G);
        if (lane == 0) out[e] = v;
    }
}

__global__ __launch_bounds__(kFinBlock) void k_gram_out(int s, int which,
                                                        const double* __restrict__ partials, int G,
                                                        double* __restrict__ W,
                                                        double* __restrict__ b1)
{
    const int K = which == 0 ? s * (s + 1) / 2 + s : s * s;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int e = wave; e < K; e += kFinBlock / kWave) {
        const double v = wave_finish(partials, e, G);
        if (lane != 0) continue;
        if (which == 1) {
            W[e] = -v;
        } else if (e < s * (s + 1) / 2) {
            int i = 0;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            const int j = e - i * (i + 1) / 2;
            W[i * s + j] = v;
            W[j * s + i] = v;
        } else {
            b1[e - s * (s + 1) / 2] = v;
        }
    }
}

}  // namespace

#define SSPCG_S_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

int launch_fgs_step(int s, int which, const double* partials, int G, double* Wbuf, double* out,
                    int sweeps, double delta, int solver, Ctrl* ctrl, double* hist, hipStream_t st)
{
    switch (s) {
#define X(S)                                                                                   \
    case S:                                                                                    \
        hipLaunchKernelGGL((k_fgs_step<S>), dim3(1), dim3(kFinBlock), 0, st, which, partials, \
                           G, Wbuf, out, sweeps, delta, solver, ctrl, hist);                   \
        break;
        SSPCG_S_CASES(X)
#undef X
    default:
        set_error("s out of range");
        return SSPCG_ERR_ARG;
    }
    SSPCG_LAUNCHED("k_fgs_step");
    return SSPCG_OK;
}

int launch_fgs_direct(int s, int nrhs, const double* W, const double* B, int sweeps, double delta,
                      int solver, double* X, int32_t* status, hipStream_t st)
{
    switch (s) {
#define X(S)                                                                                  \
    case S:                                                                                   \
        hipLaunchKernelGGL((k_fgs_direct<S>), dim3(1), dim3(kWave), 0, st, nrhs, W, B, sweeps, \
                           delta, solver, X, status);                                         \
        break;
        SSPCG_S_CASES(X)
#undef X
    default:
        set_error("s out of range");
        return SSPCG_ERR_ARG;
    }
    SSPCG_LAUNCHED("k_fgs_direct");
    return SSPCG_OK;
}

int launch_norm_step(const double* partials, int G, Ctrl* ctrl, double* hist, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm_step, dim3(1), dim3(kWave), 0, st, partials, G, ctrl, hist);
    SSPCG_LAUNCHED("k_norm_step");
    return SSPCG_OK;
}

int launch_finish(const double* partials, int K, int G, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinBlock), 0, st, partials, K, G, out);
    SSPCG_LAUNCHED("k_finish");
    return SSPCG_OK;
}

int launch_gram_out(int s, int which, const double* partials, int G, double* W, double* b1,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_gram_out, dim3(1), dim3(kFinBlock), 0, st, s, which, partials, G, W, b1);
    SSPCG_LAUNCHED("k_gram_out");
    return SSPCG_OK;
}

}  // namespace sspcg
