// Tall-skinny block kernels of the outer iteration (Algorithm 1): the fused
// block update + Gram reduction, the right-hand side of the beta system,
// and the x / r update with the residual norm and the first basis vector.
//
// All are row-parallel and stream every input once: thread i owns row i of
// every column (columns are ld apart, so a wave's load of one column is 512
// contiguous bytes).  Gram sums are FP64 per thread, then reduced over the
// block in a fixed order into per-block partials; a single-block kernel
// finishes them (fgs.hip).  The step size s is a template parameter so the
// s(s+1)/2 + s accumulators live in registers.

#include "launch.h"

namespace sspcg {

namespace {

// The blocks are hundreds of MB, far larger than L2 and the Infinity Cache,
// and no kernel re-reads them before they would have been evicted: read
// them (and write z_1) with non-temporal accesses so the streams do not
// allocate in the caches and evict each other.  Measured on the x/r update
// and the B2 reduction at 192^3: 4.97 -> 6.05 and 5.57 -> 6.42 TB/s; the
// in-place update of Q and AQ needs non-temporal stores too (4.95 -> 5.21;
// with non-temporal loads but cached stores it is slower than without).
template <typename T>
__device__ inline T ldnt(const T* p)
{
    return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ inline void stnt(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}

template <int S, typename T, bool FIRST>
__global__ __launch_bounds__(kRowBlock) void k_update_gram(int64_t n, int64_t ld,
                                                           const T* __restrict__ Z,
                                                           T* __restrict__ Q,
                                                           const T* __restrict__ AZ,
                                                           T* __restrict__ AQ,
                                                           const double* __restrict__ beta,
                                                           const T* __restrict__ r,
                                                           double* __restrict__ partials,
                                                           const Ctrl* __restrict__ ctrl)
{
    if (ctrl && ctrl->done) return;
    constexpr int K = S * (S + 1) / 2 + S;
    double acc[K];
#pragma unroll
    for (int e = 0; e < K; ++e) acc[e] = 0.0;
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i >= n) break;
        double q[S], aq[S];
        if (FIRST) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const T zj = ldnt(Z + j * ld + i), azj = ldnt(AZ + j * ld + i);
                stnt(Q + j * ld + i, zj);
                stnt(AQ + j * ld + i, azj);
                q[j] = (double)zj;
                aq[j] = (double)azj;
            }
        } else {
            double qo[S], aqo[S];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                qo[j] = (double)ldnt(Q + j * ld + i);
                aqo[j] = (double)ldnt(AQ + j * ld + i);
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double tq = 0.0, taq = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    tq = fma(qo[l], beta[l * S + j], tq);
                    taq = fma(aqo[l], beta[l * S + j], taq);
                }
                const T qn = (T)((double)ldnt(Z + j * ld + i) + tq);
                const T aqn = (T)((double)ldnt(AZ + j * ld + i) + taq);
                stnt(Q + j * ld + i, qn);
                stnt(AQ + j * ld + i, aqn);
                q[j] = (double)qn;
                aq[j] = (double)aqn;
            }
        }
        const double ri = (double)ldnt(r + i);
        int e = 0;
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                acc[e] = fma(q[a], aq[b], acc[e]);
                ++e;
            }
#pragma unroll
        for (int a = 0; a < S; ++a) acc[K - S + a] = fma(q[a], ri, acc[K - S + a]);
    }
    block_partials<K, kRowBlock>(acc, partials);
}

// R consecutive rows per thread, read as one R-wide vector per column (the
// FP32 blocks use R = 4: a 4-byte load per row and column leaves the kernel
// limited by load instructions rather than bytes).  Rows are summed in order
// within a thread.
template <int S, typename T, int R>
__global__ __launch_bounds__(kRowBlock) void k_gram_rect(int64_t n, int64_t ld,
                                                         const T* __restrict__ Q,
                                                         const T* __restrict__ AZ,
                                                         double* __restrict__ partials,
                                                         const Ctrl* __restrict__ ctrl)
{
    if (ctrl && ctrl->done) return;
    constexpr int K = S * S;
    double acc[K];
#pragma unroll
    for (int e = 0; e < K; ++e) acc[e] = 0.0;
    auto add_row = [&](const double (&q)[S], const double (&az)[S]) {
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b < S; ++b) acc[a * S + b] = fma(q[a], az[b], acc[a * S + b]);
    };
    constexpr int64_t kRows = (int64_t)kRowBlock * R;
    const int64_t ntiles = (n + kRows - 1) / kRows;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRows + (int64_t)threadIdx.x * R;
        if (i >= n) break;
        if constexpr (R > 1) {
            if (i + R <= n) {
                typedef T VT __attribute__((ext_vector_type(R)));
                VT qv[S], azv[S];
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    qv[j] = ldnt(reinterpret_cast<const VT*>(Q + j * ld + i));
                    azv[j] = ldnt(reinterpret_cast<const VT*>(AZ + j * ld + i));
                }
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    double q[S], az[S];
#pragma unroll
                    for (int j = 0; j < S; ++j) {
                        q[j] = (double)qv[j][e];
                        az[j] = (double)azv[j][e];
                    }
                    add_row(q, az);
                }
                continue;
            }
        }
        for (int e = 0; e < R && i + e < n; ++e) {
            double q[S], az[S];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                q[j] = (double)ldnt(Q + j * ld + i + e);
                az[j] = (double)ldnt(AZ + j * ld + i + e);
            }
            add_row(q, az);
        }
    }
    block_partials<K, kRowBlock>(acc, partials);
}

// R consecutive rows per thread as R-wide vectors (R = 16 bytes / element
// when every column is 16-byte aligned), each row computed as with R = 1.
template <int S, typename T, int R>
__global__ __launch_bounds__(kRowBlock) void k_xr(int64_t n, int64_t ld, const T* __restrict__ Q,
                                                  const T* __restrict__ AQ,
                                                  const double* __restrict__ alpha,
                                                  T* __restrict__ x, T* __restrict__ r,
                                                  const T* __restrict__ dinv, T* __restrict__ z1,
                                                  double* __restrict__ partials,
                                                  const Ctrl* __restrict__ ctrl)
{
    if (ctrl && ctrl->done) return;
    double al[S];
#pragma unroll
    for (int j = 0; j < S; ++j) al[j] = alpha[j];
    double acc[1] = {0.0};
    constexpr int64_t kRows = (int64_t)kRowBlock * R;
    const int64_t ntiles = (n + kRows - 1) / kRows;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRows + (int64_t)threadIdx.x * R;
        if (i >= n) break;
        if constexpr (R > 1) {
            if (i + R <= n) {
                typedef T VT __attribute__((ext_vector_type(R)));
                double qa[R], aqa[R];
#pragma unroll
                for (int e = 0; e < R; ++e) qa[e] = aqa[e] = 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    const VT q = ldnt(reinterpret_cast<const VT*>(Q + j * ld + i));
                    const VT aq = ldnt(reinterpret_cast<const VT*>(AQ + j * ld + i));
#pragma unroll
                    for (int e = 0; e < R; ++e) {
                        qa[e] = fma((double)q[e], al[j], qa[e]);
                        aqa[e] = fma((double)aq[e], al[j], aqa[e]);
                    }
                }
                VT xv = *reinterpret_cast<const VT*>(x + i);
                VT rv = *reinterpret_cast<const VT*>(r + i);
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    xv[e] = (T)((double)xv[e] + qa[e]);
                    rv[e] = (T)((double)rv[e] - aqa[e]);
                }
                *reinterpret_cast<VT*>(x + i) = xv;
                *reinterpret_cast<VT*>(r + i) = rv;
                if (z1) {
                    const VT dv = ldnt(reinterpret_cast<const VT*>(dinv + i));
                    VT zv;
#pragma unroll
                    for (int e = 0; e < R; ++e) zv[e] = (T)((double)dv[e] * (double)rv[e]);
                    stnt(reinterpret_cast<VT*>(z1 + i), zv);
                }
#pragma unroll
                for (int e = 0; e < R; ++e) acc[0] = fma((double)rv[e], (double)rv[e], acc[0]);
                continue;
            }
        }
        for (int e = 0; e < R && i + e < n; ++e) {
            const int64_t k = i + e;
            double qa = 0.0, aqa = 0.0;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                qa = fma((double)ldnt(Q + j * ld + k), al[j], qa);
                aqa = fma((double)ldnt(AQ + j * ld + k), al[j], aqa);
            }
            x[k] = (T)((double)x[k] + qa);
            const T rk = (T)((double)r[k] - aqa);
            r[k] = rk;
            if (z1) stnt(z1 + k, (T)((double)ldnt(dinv + k) * (double)rk));
            acc[0] = fma((double)rk, (double)rk, acc[0]);
        }
    }
    block_partials<1, kRowBlock>(acc, partials);
}

template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_axpy_up(int64_t n, double* __restrict__ x,
                                                       const T* __restrict__ d,
                                                       const Ctrl* __restrict__ ctrl)
{
    if (ctrl && ctrl->done) return;
    const int64_t stride = (int64_t)gridDim.x * kRowBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n; i += stride)
        x[i] += (double)d[i];
}

template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_fill(int64_t n, T* __restrict__ x, T v)
{
    const int64_t stride = (int64_t)gridDim.x * kRowBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n; i += stride) x[i] = v;
}

}  // namespace

int row_grid(int64_t n)
{
    return persistent_grid((n + kRowBlock - 1) / kRowBlock, 4);
}

// Persistent grid of a block kernel: up to 8 workgroups per CU, no more than
// fit at once.
template <typename K>
static int block_grid(int64_t n, K kernel)
{
    const int resident = resident_blocks(reinterpret_cast<const void*>(kernel), kRowBlock);
    return persistent_grid((n + kRowBlock - 1) / kRowBlock, 8, resident);
}

#define SSPCG_S_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <typename T>
int launch_update_gram(int64_t n, int s, const T* Z, T* Q, const T* AZ, T* AQ, const double* beta,
                       const T* r, int64_t ld, double* partials, int* G_out, const Ctrl* ctrl,
                       hipStream_t st)
{
    int G = 0;
    switch (s) {
#define X(S)                                                                                     \
    case S:                                                                                      \
        if (beta) {                                                                              \
            G = block_grid(n, k_update_gram<S, T, false>);                                       \
            hipLaunchKernelGGL((k_update_gram<S, T, false>), dim3(G), dim3(kRowBlock), 0, st, n, \
                               ld, Z, Q, AZ, AQ, beta, r, partials, ctrl);                       \
        } else {                                                                                 \
            G = block_grid(n, k_update_gram<S, T, true>);                                        \
            hipLaunchKernelGGL((k_update_gram<S, T, true>), dim3(G), dim3(kRowBlock), 0, st, n,  \
                               ld, Z, Q, AZ, AQ, beta, r, partials, ctrl);                       \
        }                                                                                        \
        break;
        SSPCG_S_CASES(X)
#undef X
    default:
        set_error("s out of range");
        return SSPCG_ERR_ARG;
    }
    SSPCG_LAUNCHED("k_update_gram");
    *G_out = G;
    return SSPCG_OK;
}

template <typename T>
int launch_gram_rect(int64_t n, int s, const T* Q, const T* AZ, int64_t ld, double* partials,
                     int* G_out, const Ctrl* ctrl, hipStream_t st)
{
    // FP32 columns whose elements 4i.. are 16-byte aligned go 4 rows per
    // thread; anything else one row per thread
    constexpr int RV = sizeof(T) == 4 ? 4 : 1;
    const bool vec = RV > 1 && ld % RV == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(AZ) % 16 == 0;
    const int64_t units = vec ? (n + RV - 1) / RV : n;
    int G = 0;
    switch (s) {
#define X(S)                                                                                   \
    case S:                                                                                    \
        if (vec) {                                                                             \
            G = block_grid(units, k_gram_rect<S, T, RV>);                                      \
            hipLaunchKernelGGL((k_gram_rect<S, T, RV>), dim3(G), dim3(kRowBlock), 0, st, n, ld, \
                               Q, AZ, partials, ctrl);                                         \
        } else {                                                                               \
            G = block_grid(units, k_gram_rect<S, T, 1>);                                       \
            hipLaunchKernelGGL((k_gram_rect<S, T, 1>), dim3(G), dim3(kRowBlock), 0, st, n, ld, \
                               Q, AZ, partials, ctrl);                                         \
        }                                                                                      \
        break;
        SSPCG_S_CASES(X)
#undef X
    default:
        set_error("s out of range");
        return SSPCG_ERR_ARG;
    }
    SSPCG_LAUNCHED("k_gram_rect");
    *G_out = G;
    return SSPCG_OK;
}

template <typename T>
int launch_xr(int64_t n, int s, const T* Q, const T* AQ, const double* alpha, int64_t ld, T* x,
              T* r, const T* dinv, T* z1, double* partials, int* G_out, const Ctrl* ctrl,
              hipStream_t st)
{
    constexpr int RV = 16 / (int)sizeof(T);
    auto a16 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    const bool vec = ld % RV == 0 && a16(Q) && a16(AQ) && a16(x) && a16(r) && a16(dinv) && a16(z1);
    const int64_t units = vec ? (n + RV - 1) / RV : n;
    int G = 0;
    switch (s) {
#define X(S)                                                                                   \
    case S:                                                                                    \
        if (vec) {                                                                             \
            G = block_grid(units, k_xr<S, T, RV>);                                             \
            hipLaunchKernelGGL((k_xr<S, T, RV>), dim3(G), dim3(kRowBlock), 0, st, n, ld, Q, AQ, \
                               alpha, x, r, dinv, z1, partials, ctrl);                         \
        } else {                                                                               \
            G = block_grid(units, k_xr<S, T, 1>);                                              \
            hipLaunchKernelGGL((k_xr<S, T, 1>), dim3(G), dim3(kRowBlock), 0, st, n, ld, Q, AQ, \
                               alpha, x, r, dinv, z1, partials, ctrl);                         \
        }                                                                                      \
        break;
        SSPCG_S_CASES(X)
#undef X
    default:
        set_error("s out of range");
        return SSPCG_ERR_ARG;
    }
    SSPCG_LAUNCHED("k_xr");
    *G_out = G;
    return SSPCG_OK;
}

template <typename T>
int launch_axpy_up(int64_t n, double* x, const T* d, const Ctrl* ctrl, hipStream_t st)
{
    hipLaunchKernelGGL((k_axpy_up<T>), dim3(row_grid(n)), dim3(kRowBlock), 0, st, n, x, d, ctrl);
    SSPCG_LAUNCHED("k_axpy_up");
    return SSPCG_OK;
}

template <typename T>
int launch_fill(int64_t n, T* x, T v, hipStream_t st)
{
    hipLaunchKernelGGL((k_fill<T>), dim3(row_grid(n)), dim3(kRowBlock), 0, st, n, x, v);
    SSPCG_LAUNCHED("k_fill");
    return SSPCG_OK;
}

#define SSPCG_INST(T)                                                                            \
    template int launch_update_gram<T>(int64_t, int, const T*, T*, const T*, T*, const double*, \
                                       const T*, int64_t, double*, int*, const Ctrl*,           \
                                       hipStream_t);                                             \
    template int launch_gram_rect<T>(int64_t, int, const T*, const T*, int64_t, double*, int*,  \
                                     const Ctrl*, hipStream_t);                                  \
    template int launch_xr<T>(int64_t, int, const T*, const T*, const double*, int64_t, T*, T*, \
                              const T*, T*, double*, int*, const Ctrl*, hipStream_t);           \
    template int launch_axpy_up<T>(int64_t, double*, const T*, const Ctrl*, hipStream_t);       \
    template int launch_fill<T>(int64_t, T*, T, hipStream_t);
SSPCG_INST(double)
SSPCG_INST(float)
#undef SSPCG_INST

}  // namespace sspcg
