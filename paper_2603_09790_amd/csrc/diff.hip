// Kernels of the differentiable solve x = A(theta)^{-1} b on the 7-point
// variable-coefficient diffusion operator:
//   assembly   k = exp(theta); a_ij = -w_ij, w_ij = 2 k_i k_j / (k_i + k_j);
//              a_ii = sum_j w_ij + (6 - deg_i) k_i  (Dirichlet ghost cells)
//   value grad dL/da_ij = -lambda_i x_j with A lambda = dL/dx
//   theta grad vector-Jacobian product of the assembly, gathered per cell:
//              g_c = G_cc (6 - deg_c) k_c
//                    + sum_j (G_cc + G_jj - G_cj - G_jc) w_cj k_j / (k_c + k_j)
// One thread per row; rows of the stencil have at most 7 entries.

#include "launch.h"

namespace sspcg {

namespace {

__global__ __launch_bounds__(kRowBlock) void k_value_grad(int32_t n, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ lambda,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ gval)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (i >= n) return;
    const double li = lambda[i];
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) gval[e] = -li * x[col[e]];
}

__global__ __launch_bounds__(kRowBlock) void k_assemble7(int32_t n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ theta,
                                                         double* __restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (i >= n) return;
    const double ki = exp(theta[i]);
    double diag = 0.0;
    int deg = 0;
    int32_t dpos = -1;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = col[e];
        if (j == i) {
            dpos = e;
            continue;
        }
        const double kj = exp(theta[j]);
        const double w = 2.0 * ki * kj / (ki + kj);
        val[e] = -w;
        diag += w;
        ++deg;
    }
    diag += (double)(6 - deg) * ki;
    if (dpos >= 0) val[dpos] = diag;
}

__device__ inline int32_t find_entry(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                     int32_t row, int32_t c)
{
    for (int32_t e = rp[row]; e < rp[row + 1]; ++e)
        if (col[e] == c) return e;
    return -1;
}

__global__ __launch_bounds__(kRowBlock) void k_theta_grad7(int32_t n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ theta,
                                                           const double* __restrict__ gval,
                                                           double* __restrict__ gtheta)
{
    const int64_t c = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (c >= n) return;
    const double kc = exp(theta[c]);
    const int32_t ecc = find_entry(rp, col, (int32_t)c, (int32_t)c);
    const double gcc = ecc >= 0 ? gval[ecc] : 0.0;
    int deg = 0;
    double g = 0.0;
    for (int32_t e = rp[c]; e < rp[c + 1]; ++e) {
        const int32_t j = col[e];
        if (j == c) continue;
        ++deg;
        const double kj = exp(theta[j]);
        const double w = 2.0 * kc * kj / (kc + kj);
        const double dw = w * kj / (kc + kj);   // d w_cj / d theta_c
        const int32_t ejc = find_entry(rp, col, j, (int32_t)c);
        const int32_t ejj = find_entry(rp, col, j, j);
        const double gjc = ejc >= 0 ? gval[ejc] : 0.0;
        const double gjj = ejj >= 0 ? gval[ejj] : 0.0;
        g += (gcc + gjj - gval[e] - gjc) * dw;
    }
    g += gcc * (double)(6 - deg) * kc;
    gtheta[c] = g;
}

inline int blocks_for(int64_t n) { return (int)((n + kRowBlock - 1) / kRowBlock); }

}  // namespace

int launch_value_grad(const sspcg_matrix* A, const double* lambda, const double* x, double* gval,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_value_grad, dim3(blocks_for(A->n)), dim3(kRowBlock), 0, st, A->n,
                       A->row_ptr, A->col, lambda, x, gval);
    SSPCG_LAUNCHED("k_value_grad");
    return SSPCG_OK;
}

int launch_diffusion7_assemble(const sspcg_matrix* A, const double* theta, double* val,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_assemble7, dim3(blocks_for(A->n)), dim3(kRowBlock), 0, st, A->n,
                       A->row_ptr, A->col, theta, val);
    SSPCG_LAUNCHED("k_assemble7");
    return SSPCG_OK;
}

int launch_diffusion7_theta_grad(const sspcg_matrix* A, const double* theta, const double* gval,
                                 double* gtheta, hipStream_t st)
{
    hipLaunchKernelGGL(k_theta_grad7, dim3(blocks_for(A->n)), dim3(kRowBlock), 0, st, A->n,
                       A->row_ptr, A->col, theta, gval, gtheta);
    SSPCG_LAUNCHED("k_theta_grad7");
    return SSPCG_OK;
}

}  // namespace sspcg
