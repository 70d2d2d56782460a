// Device estimates of the basis interval [lambda_min, lambda_max].
//
// The Chebyshev basis is scaled by an interval that holds the spectrum of the
// Jacobi-preconditioned operator M^{-1}A, M = diag(A) (Sec. "The s-step PCG
// method with Chebyshev Krylov basis").  Two estimates, both run entirely on
// the device:
//   power   : lambda_min = 0 and the power method's lambda_max, stopping once
//             successive estimates differ by less than rtol relative to the
//             newer one or after `steps` steps (the paper's choice);
//   Lanczos : the extreme eigenvalues of the tridiagonal matrix of `steps`
//             Lanczos steps on C = D^{-1/2} A D^{-1/2}, which is similar to
//             M^{-1}A, without reorthogonalisation or safety margin.
// Lanczos runs in the variables y = D^{-1/2} v: then C v = D^{1/2} (dinv .* A y)
// and ||v||^2 = sum(y_i^2 / dinv_i), so the recurrence needs the existing
// SpMV and dinv only.  Every step is three launches; the host enqueues all
// steps at once and kernels return on entry once the device sets the stop
// flag.  The tridiagonal eigenvalues come from Sturm-count bisection in one
// lane.
#include <cfloat>
#include <cmath>
#include <cstring>

#include <algorithm>

#include "launch.h"

namespace sspcg {
namespace {

// ||v0||^2 partials.
__global__ __launch_bounds__(kRowBlock) void k_iv_norm0(int64_t n, const double* __restrict__ v0,
                                                        double* __restrict__ partials)
{
    double acc[1] = {0.0};
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        zero_acc(acc);
        const TileRange tr = vblock_tiles(ntiles, VB, v);
        for (int64_t t = tr.first; t < tr.end; t += tr.step) {
            const int64_t i = t * kRowBlock + threadIdx.x;
            if (i < n) acc[0] = fma(v0[i], v0[i], acc[0]);
        }
        block_partials<1, kRowBlock>(acc, partials, v, VB);
    }
}

// First vector: v_1 = v0 / ||v0|| (power) or y_1 = D^{-1/2} v_1 (Lanczos,
// with y_0 = 0).  A zero or non-finite start vector ends the estimate.
__global__ __launch_bounds__(kRowBlock) void k_iv_start(int64_t n, int lanczos,
                                                        const double* __restrict__ v0,
                                                        const double* __restrict__ dinv,
                                                        const double* __restrict__ partials, int G,
                                                        double* __restrict__ y,
                                                        double* __restrict__ yp,
                                                        Ctrl* __restrict__ ctrl)
{
    __shared__ double s_nv;
    if (threadIdx.x < kWave) {
        const double ss = wave_finish(partials, 0, G);
        if (threadIdx.x == 0) s_nv = sqrt(ss);
    }
    __syncthreads();
    const double nv = s_nv;
    if (!(nv > 0.0) || !isfinite(nv)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctrl->status = SSPCG_ERR_ARG;
            ctrl->done = 1;
        }
        return;
    }
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i < n) {
            const double v = v0[i] / nv;
            if (lanczos) {
                y[i] = sqrt(dinv[i]) * v;
                yp[i] = 0.0;
            } else {
                y[i] = v;
            }
        }
    }
}

// Lanczos step j, after q = A y_j with partials of y_j^T q:
//   alpha_j = y_j^T A y_j  (= v_j^T C v_j)
//   w = dinv .* q - alpha_j y_j - beta_{j-1} y_{j-1}, stored over y_{j-1}
// with partials of w^T D w = ||C v_j - alpha_j v_j - beta_{j-1} v_{j-1}||^2.
__global__ __launch_bounds__(kRowBlock) void k_lz_orth(int64_t n, int j, int steps,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ yp,
                                                       const double* __restrict__ q,
                                                       const double* __restrict__ dinv,
                                                       const double* __restrict__ yq_part, int Gq,
                                                       double* __restrict__ partials,
                                                       double* __restrict__ coef,
                                                       const Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    __shared__ double s_a;
    if (threadIdx.x < kWave) {
        const double a = wave_finish(yq_part, 0, Gq);
        if (threadIdx.x == 0) s_a = a;
    }
    __syncthreads();
    const double a = s_a;
    // coef[0..steps) holds alpha, coef[steps..2 steps) beta; block 0 writes
    // alpha_j, every block reads beta_{j-1} (written by the previous step)
    if (blockIdx.x == 0 && threadIdx.x == 0) coef[j] = a;
    const double bp = j > 0 ? coef[steps + j - 1] : 0.0;
    double acc[1] = {0.0};
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        zero_acc(acc);
        const TileRange tr = vblock_tiles(ntiles, VB, v);
        for (int64_t t = tr.first; t < tr.end; t += tr.step) {
            const int64_t i = t * kRowBlock + threadIdx.x;
            if (i < n) {
                const double di = dinv[i];
                const double w = di * q[i] - a * y[i] - bp * yp[i];
                yp[i] = w;
                acc[0] = fma(w, w / di, acc[0]);
            }
        }
        block_partials<1, kRowBlock>(acc, partials, v, VB);
    }
}

// beta_j = ||w||; y_{j+1} = w / beta_j in place.  Block 0 records the step
// and sets the stop flag on an invariant subspace (beta_j = 0), a
// non-finite coefficient or the last step.
__global__ __launch_bounds__(kRowBlock) void k_lz_next(int64_t n, int j, int steps,
                                                       double* __restrict__ w,
                                                       const double* __restrict__ partials, int G,
                                                       double* __restrict__ coef,
                                                       Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    __shared__ double s_b;
    if (threadIdx.x < kWave) {
        const double ss = wave_finish(partials, 0, G);
        if (threadIdx.x == 0) s_b = sqrt(ss);
    }
    __syncthreads();
    const double b = s_b;
    const double a = coef[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        coef[steps + j] = b;
        ctrl->iter = j + 1;
        if (!isfinite(a) || !isfinite(b)) {
            ctrl->status = SSPCG_ERR_NONFINITE;
            ctrl->done = 1;
        } else if (b == 0.0 || j + 1 >= ctrl->max_iter) {
            ctrl->status = SSPCG_OK;
            ctrl->done = 1;
        }
    }
    if (!(b > 0.0) || !isfinite(b) || !isfinite(a)) return;
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i < n) w[i] = w[i] / b;
    }
}

// Power step, after q = A v: w = dinv .* q in place, partials of ||w||^2.
__global__ __launch_bounds__(kRowBlock) void k_pw_apply(int64_t n, double* __restrict__ q,
                                                        const double* __restrict__ dinv,
                                                        double* __restrict__ partials,
                                                        const Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    double acc[1] = {0.0};
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        zero_acc(acc);
        const TileRange tr = vblock_tiles(ntiles, VB, v);
        for (int64_t t = tr.first; t < tr.end; t += tr.step) {
            const int64_t i = t * kRowBlock + threadIdx.x;
            if (i < n) {
                const double w = dinv[i] * q[i];
                q[i] = w;
                acc[0] = fma(w, w, acc[0]);
            }
        }
        block_partials<1, kRowBlock>(acc, partials, v, VB);
    }
}

// Power step j: lambda_j = ||w||, v = w / lambda_j.  Block 0 keeps the
// previous estimate in sums[1] and applies the stop rule.
__global__ __launch_bounds__(kRowBlock) void k_pw_next(int64_t n, int j, double rtol,
                                                       double* __restrict__ v,
                                                       const double* __restrict__ w,
                                                       const double* __restrict__ partials, int G,
                                                       Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    __shared__ double s_l;
    if (threadIdx.x < kWave) {
        const double ss = wave_finish(partials, 0, G);
        if (threadIdx.x == 0) s_l = sqrt(ss);
    }
    __syncthreads();
    const double lam = s_l;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double old = ctrl->sums[1];
        ctrl->sums[1] = lam;
        ctrl->iter = j + 1;
        if (!(lam > 0.0) || !isfinite(lam)) {
            ctrl->status = SSPCG_ERR_NONFINITE;
            ctrl->done = 1;
        } else if (fabs(lam - old) < rtol * fabs(lam) || j + 1 >= ctrl->max_iter) {
            ctrl->status = SSPCG_OK;
            ctrl->done = 1;
        }
    }
    if (!(lam > 0.0) || !isfinite(lam)) return;
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i < n) v[i] = w[i] / lam;
    }
}

// Eigenvalues of the k x k tridiagonal T (diagonal a, off-diagonal b) below
// x: the number of negative pivots of T - x I = L D L^T (Sylvester's law of
// inertia); tiny pivots are replaced by -pivmin.
__device__ int sturm_below(const double* a, const double* b, int k, double x, double pivmin)
{
    int cnt = 0;
    double d = a[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    cnt += d < 0.0;
    for (int i = 1; i < k; ++i) {
        d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        cnt += d < 0.0;
    }
    return cnt;
}

// Bisection for the point where the count of eigenvalues below x first
// reaches `target`, inside the Gershgorin interval [lo, hi].
__device__ double bisect(const double* a, const double* b, int k, int target, double lo, double hi,
                         double pivmin)
{
    for (int it = 0; it < 2100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;   // adjacent doubles
        if (sturm_below(a, b, k, mid, pivmin) >= target)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Extreme eigenvalues of T_k, k = ctrl->iter, into sums[0] and sums[1].
__global__ void k_lz_extremes(const double* __restrict__ coef, int steps, Ctrl* __restrict__ ctrl)
{
    if (threadIdx.x != 0 || ctrl->status != SSPCG_OK) return;
    const int k = ctrl->iter;
    const double* a = coef;
    const double* b = coef + steps;
    if (k == 1) {
        ctrl->sums[0] = ctrl->sums[1] = a[0];
        return;
    }
    double lo = INFINITY, hi = -INFINITY, bmax = 0.0;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
        if (i + 1 < k) bmax = fmax(bmax, b[i] * b[i]);
    }
    const double scale = fmax(fabs(lo), fabs(hi));
    lo -= 4.0 * DBL_EPSILON * scale;
    hi += 4.0 * DBL_EPSILON * scale;
    const double pivmin = DBL_MIN * fmax(1.0, bmax);
    ctrl->sums[0] = bisect(a, b, k, 1, lo, hi, pivmin);
    ctrl->sums[1] = bisect(a, b, k, k, lo, hi, pivmin);
}

struct IntervalLayout {
    size_t ctrl = 0, coef = 0, part = 0, part2 = 0, vec = 0, total = 0;
    int64_t ld = 0;
};

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

IntervalLayout layout_interval(int64_t n, int steps)
{
    IntervalLayout L;
    L.ld = (n + kSlice - 1) / kSlice * kSlice;
    size_t off = 0;
    L.ctrl = off;
    off += 256;
    L.coef = off;
    off += round256(sizeof(double) * 2 * (size_t)steps);
    L.part = off;
    off += round256(sizeof(double) * kMaxGrid);
    L.part2 = off;
    off += round256(sizeof(double) * kMaxGrid);
    L.vec = off;
    off += round256(sizeof(double) * 3 * (size_t)L.ld);   // y, y_prev / w, q
    L.total = off;
    return L;
}

}  // namespace

size_t interval_work_bytes(int64_t n, int steps) { return layout_interval(n, steps).total; }

int run_interval(const sspcg_matrix* A, int method, int steps, double rtol, const double* v0,
                 void* work, hipStream_t st, double* lmin, double* lmax, int* steps_taken)
{
    const int64_t n = A->n;
    const IntervalLayout L = layout_interval(n, steps);
    char* base = static_cast<char*>(work);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + L.ctrl);
    double* coef = reinterpret_cast<double*>(base + L.coef);
    double* part = reinterpret_cast<double*>(base + L.part);
    double* part2 = reinterpret_cast<double*>(base + L.part2);
    double* y = reinterpret_cast<double*>(base + L.vec);
    double* yp = y + L.ld;
    double* q = yp + L.ld;
    const bool lanczos = method == SSPCG_INTERVAL_LANCZOS;
    const int max_iter = lanczos ? (int)std::min<int64_t>(steps, n) : steps;

    Ctrl c;
    std::memset(&c, 0, sizeof(c));
    c.status = SSPCG_NOT_CONVERGED;
    c.max_iter = max_iter;
    // `c` lives on this stack frame: wait for the copy before anything can return
    SSPCG_HIP(hipMemcpyAsync(ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, st));
    SSPCG_HIP(hipStreamSynchronize(st));

    // reductions over the rows write one partial per virtual block (common.h)
    const int VBr = virtual_blocks((n + kRowBlock - 1) / kRowBlock);
    const int Gr = std::min(row_grid(n), VBr);
    hipLaunchKernelGGL(k_iv_norm0, dim3(Gr), dim3(kRowBlock), 0, st, n, v0, part2);
    SSPCG_LAUNCHED("k_iv_norm0");
    hipLaunchKernelGGL(k_iv_start, dim3(Gr), dim3(kRowBlock), 0, st, n, lanczos ? 1 : 0, v0,
                       A->dinv, part2, VBr, y, yp, ctrl);
    SSPCG_LAUNCHED("k_iv_start");
    for (int j = 0; j < max_iter; ++j) {
        int G = 0;
        int rc = launch_pcg_spmv(A, y, q, part, &G, ctrl, st);
        if (rc != SSPCG_OK) return rc;
        if (lanczos) {
            hipLaunchKernelGGL(k_lz_orth, dim3(Gr), dim3(kRowBlock), 0, st, n, j, steps, y, yp, q,
                               A->dinv, part, G, part2, coef, ctrl);
            SSPCG_LAUNCHED("k_lz_orth");
            hipLaunchKernelGGL(k_lz_next, dim3(Gr), dim3(kRowBlock), 0, st, n, j, steps, yp, part2,
                               VBr, coef, ctrl);
            SSPCG_LAUNCHED("k_lz_next");
            std::swap(y, yp);
        } else {
            hipLaunchKernelGGL(k_pw_apply, dim3(Gr), dim3(kRowBlock), 0, st, n, q, A->dinv, part2,
                               ctrl);
            SSPCG_LAUNCHED("k_pw_apply");
            hipLaunchKernelGGL(k_pw_next, dim3(Gr), dim3(kRowBlock), 0, st, n, j, rtol, y, q, part2,
                               VBr, ctrl);
            SSPCG_LAUNCHED("k_pw_next");
        }
    }
    if (lanczos) {
        hipLaunchKernelGGL(k_lz_extremes, dim3(1), dim3(kWave), 0, st, coef, steps, ctrl);
        SSPCG_LAUNCHED("k_lz_extremes");
    }
    SSPCG_HIP(hipMemcpyAsync(&c, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipStreamSynchronize(st));
    if (steps_taken) *steps_taken = c.iter;
    if (c.status == SSPCG_ERR_ARG) {
        set_error("start vector has zero norm or non-finite entries");
        return SSPCG_ERR_ARG;
    }
    if (c.status != SSPCG_OK) {
        set_error("non-finite value in the interval estimate");
        return c.status;
    }
    *lmin = lanczos ? c.sums[0] : 0.0;
    *lmax = c.sums[1];
    return SSPCG_OK;
}

}  // namespace sspcg
