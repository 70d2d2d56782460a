// Host-side launchers of the kernels, shared by the HIP sources.
#pragma once

#include <vector>

#include "common.h"

struct sspcg_matrix {
    int32_t n = 0, nnz = 0, flags = 0, device = 0;
    const int32_t* row_ptr = nullptr;   // caller's CSR (device, not owned)
    const int32_t* col = nullptr;
    int64_t nslices = 0, slots = 0, nshared = 0;
    // Every device array below lives in the caller's `aux` buffer.
    int64_t* slice_ptr = nullptr;
    int64_t* slice_aux = nullptr;
    int32_t* scol = nullptr;
    int32_t* soff = nullptr;
    int32_t uniform = 0, uw = 0;        // uniform layout: global offset list length
    int32_t usym = 0;                   // uniform layout: symmetric half storage
    int32_t* uoff = nullptr;
    int32_t uoff_host[32] = {};         // the same list, copied into kernel arguments
    int32_t lds_n = 0, ncl = 0, lds_self = 0;   // LDS staging of x (see Sell)
    int32_t cl_lo[12] = {}, cl_len[12] = {}, cl_base[12] = {}, lds_k[32] = {};
    double* sval = nullptr;
    float* sval32 = nullptr;
    double* dinv = nullptr;
    float* dinv32 = nullptr;
    // analysis area (the first bytes of `aux`): check flags, per-slice
    // longest row, per-slice offset union and its length
    int32_t* dflags = nullptr;
    int32_t* a_width = nullptr;
    int32_t* a_ulen = nullptr;
    int32_t* a_union = nullptr;
    void* aux = nullptr;                // the caller's buffer
    size_t aux_used = 0;                // bytes of it in use
};

namespace sspcg {

template <typename T>
Sell<T> sell_view(const sspcg_matrix* A);

// Matrix layout (sell.hip).  inspect validates the CSR input on the device
// and writes dinv; with a plan it also chooses the kind of every slice (the
// per-slice offset unions stay in the analysis area, A->a_union, for
// matrix_pack).  pack copies the chosen offset lists; fill writes the
// sliced values (and explicit columns).  None of them allocates: the
// analysis area and every output array are set in A beforehand.
struct LayoutPlan {
    std::vector<int64_t> slice_ptr, slice_aux;
    int64_t slots = 0, ncol = 0, nsoff = 0, nshared = 0;
    std::vector<int32_t> uoff;          // non-empty: use the uniform layout with these offsets
    bool usym = false;                  // uniform: A is symmetric, store one triangle
};
// write_dinv = false checks the values without touching the matrix.  With a
// plan, allow_sym lets the uniform layout use the symmetric half storage.
int matrix_inspect(sspcg_matrix* A, const double* val, bool values_only, LayoutPlan* plan,
                   hipStream_t st, bool write_dinv = true, bool allow_sym = true);
// Bytes of the analysis area for n rows (also the scratch of the size query).
size_t analysis_bytes(int64_t n);
// Points A->dflags, a_width, a_ulen, a_union into the area at `base`.
void bind_analysis(sspcg_matrix* A, void* base);
// Whether the CSR values val (the matrix's pattern) are symmetric bit for
// bit: a(i, j) equals a(j, i), an absent entry counting as +0.
int matrix_check_symmetric(const sspcg_matrix* A, const double* val, bool* sym, hipStream_t st);
int matrix_pack(sspcg_matrix* A, hipStream_t st);
int matrix_fill(sspcg_matrix* A, const double* val, bool values_only, hipStream_t st);
// Windows of the LDS staging of x for the uniform offset list (host only).
void plan_lds(sspcg_matrix* A);
template <typename T>
int launch_mpk_start(int64_t n, const T* r, const T* dinv, T* z1, T* p1, hipStream_t st);

// SpMV with the MPK epilogue (sell.hip).
//   mode 0: y = A x
//   mode 1: y = A x;  znext = c1 * dinv .* y - c2 * x
//   mode 2: y = A x;  znext = c1 * dinv .* y - c2 * x - c3 * zprev
template <typename T>
int launch_spmv(const sspcg_matrix* A, int mode, const T* x, T* y, const T* zprev, T* znext,
                double c1, double c2, double c3, const Ctrl* ctrl, hipStream_t st);

// FP64 residual: r = b - A x stored as TR; z1 = dinv_T .* r when z1 != null;
// partials of {||b - Ax||^2 (FP64), ||r_stored||^2, ||b||^2, r_stored^T z1}.
template <typename TR>
int launch_residual(const sspcg_matrix* A, const double* x, const double* b, TR* r, TR* z1,
                    double* partials, int* G_out, hipStream_t st);

// Classical PCG: q = A p with partials of p^T q.
int launch_pcg_spmv(const sspcg_matrix* A, const double* p, double* q, double* partials,
                    int* G_out, const Ctrl* ctrl, hipStream_t st);
int launch_pcg_update(const sspcg_matrix* A, int64_t k, double* x, double* r, double* z,
                      const double* p, const double* q, const double* pq_partials, int Gpq,
                      double* partials, int* G_out, Ctrl* ctrl, hipStream_t st);
int launch_pcg_pupdate(int64_t n, int64_t k, const double* z, double* p, const double* partials,
                       int G, Ctrl* ctrl, double* hist, hipStream_t st);

// Block kernels (block.hip).
int row_grid(int64_t n);
// beta == nullptr: the first update (Q = Z, AQ = AZ).  x != nullptr: also
// x += Q alpha with the incoming Q when ctrl->x_pending is set.
template <typename T>
int launch_update_gram(int64_t n, int s, const T* Z, T* Q, const T* AZ, T* AQ,
                       const double* beta, const T* r, T* x, const double* alpha, int64_t ld,
                       double* partials, int* G_out, const Ctrl* ctrl, hipStream_t st);
template <typename T>
int launch_gram_rect(int64_t n, int s, const T* Q, const T* AZ, int64_t ld, double* partials,
                     int* G_out, const Ctrl* ctrl, hipStream_t st);
template <typename T>
int launch_xr(int64_t n, int s, const T* Q, const T* AQ, const double* alpha, int64_t ld,
              T* x, T* r, const T* dinv, T* z1, double* partials, int* G_out,
              const Ctrl* ctrl, hipStream_t st);
template <typename T>
int launch_axpy_up(int64_t n, double* x, const T* d, const Ctrl* ctrl, hipStream_t st);
// x += Q alpha if ctrl->x_pending (the end of a solve).
template <typename T>
int launch_x_pending(int64_t n, int s, const T* Q, const double* alpha, int64_t ld, T* x,
                     const Ctrl* ctrl, hipStream_t st);
template <typename T>
int launch_fill(int64_t n, T* x, T v, hipStream_t st);

// Small kernels (fgs.hip).
//   which = 0: alpha system (partials hold W lower + b1; W is also stored)
//   which = 1: beta system (partials hold Q^T AZ; W from Wbuf)
int launch_fgs_step(int s, int which, const double* partials, int G, double* Wbuf, double* out,
                    int sweeps, double delta, int solver, Ctrl* ctrl, double* hist,
                    hipStream_t st);
int launch_fgs_direct(int s, int nrhs, const double* W, const double* B, int sweeps, double delta,
                      int solver, double* X, int32_t* status, hipStream_t st);
// Finishes ||r||^2 of outer iteration ctrl->iter: relres, stop test, history.
int launch_norm_step(const double* partials, int G, Ctrl* ctrl, double* hist, hipStream_t st);
// Finishes K partial sums into out[0..K).
int launch_finish(const double* partials, int K, int G, double* out, hipStream_t st);
// Kernel-level Gram output: W (mirrored) and b1, or B2 = -sums.
int launch_gram_out(int s, int which, const double* partials, int G, double* W, double* b1,
                    hipStream_t st);

// Basis interval estimates (interval.hip): Lanczos or power method on the
// device; blocks until the host outputs are written.
size_t interval_work_bytes(int64_t n, int steps);
int run_interval(const sspcg_matrix* A, int method, int steps, double rtol, const double* v0,
                 void* work, hipStream_t st, double* lmin, double* lmax, int* steps_taken);

// Differentiation (diff.hip).
int launch_value_grad(const sspcg_matrix* A, const double* lambda, const double* x,
                      double* gval, hipStream_t st);
int launch_diffusion7_assemble(const sspcg_matrix* A, const double* theta, double* val,
                               hipStream_t st);
int launch_diffusion7_theta_grad(const sspcg_matrix* A, const double* theta, const double* gval,
                                 double* gtheta, hipStream_t st);

// STREAM triad a = b + q c (stream.hip): the achievable-bandwidth reference.
int launch_triad(int64_t n, const double* b, const double* c, double q, double* a,
                 hipStream_t st);

}  // namespace sspcg
