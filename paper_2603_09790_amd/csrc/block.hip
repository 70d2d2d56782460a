// Tall-skinny block kernels of the outer iteration (Algorithm 1): the fused
// block update + Gram reduction, the right-hand side of the beta system,
// and the x / r update with the residual norm and the first basis vector.
//
// All are row-parallel and stream every input once: a thread owns one row
// (or R consecutive rows, read as 16-byte vectors) of every column (columns
// are ld apart, so a wave's load of one column is contiguous).  Gram sums are
// FP64 per thread, then reduced over the block in a fixed order into
// per-block partials; a single-block kernel finishes them (fgs.hip).  The
// step size s is a template parameter so the s(s+1)/2 + s accumulators live
// in registers.  In the solve, x += Q alpha of an outer iteration is applied
// by the next block update, which reads that Q anyway (k_update_gram MODE 2),
// or after the loop (k_x_pending).

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

// MODE 0: the first update (Q = Z, AQ = AZ).  MODE 1: Q = Z + Q beta,
// AQ = AZ + AQ beta.  MODE 2: MODE 1 and, if ctrl->x_pending, the x update of
// the previous outer iteration, x += Q alpha with the old Q streamed here
// anyway, in the same arithmetic as k_xr; the solve's x/r update then
// leaves x alone and never reads Q.  x is loaded with the row's other
// operands, so its latency overlaps theirs.
template <int S, typename T, int MODE>
__global__ __launch_bounds__(kRowBlock) void k_update_gram(int64_t n, int64_t ld,
                                                           const T* __restrict__ Z,
                                                           T* __restrict__ Q,
                                                           const T* __restrict__ AZ,
                                                           T* __restrict__ AQ,
                                                           const double* __restrict__ beta,
                                                           const T* __restrict__ r,
                                                           T* __restrict__ x,
                                                           const double* __restrict__ alpha,
                                                           double* __restrict__ partials,
                                                           const Ctrl* __restrict__ ctrl)
{
    if (ctrl && ctrl->done) return;
    constexpr int K = S * (S + 1) / 2 + S;
    double acc[K];
#pragma unroll
    for (int e = 0; e < K; ++e) acc[e] = 0.0;
    constexpr bool FIRST = MODE == 0;
    bool pend = false;
    double al[S];
    if constexpr (MODE == 2) {
        pend = ctrl->x_pending != 0;
#pragma unroll
        for (int j = 0; j < S; ++j) al[j] = alpha[j];
    }
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i >= n) break;
        // Every load of the row is issued before its first store (the wait
        // counter is shared by loads and stores, so a load queued behind a
        // store also waits for the store): 271 -> 217 us per FP32 update at
        // 192^3, 420 -> 407 us per FP64 update (all operands held at once
        // cost a wave per SIMD, but the loads are in flight together).
        constexpr bool kPreload = true;
        double q[S], aq[S];
        T zv[S], azv[S];
        T rv = (T)0;
        if constexpr (kPreload) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                zv[j] = ldnt(Z + j * ld + i);
                azv[j] = ldnt(AZ + j * ld + i);
            }
            rv = ldnt(r + i);
        }
        if constexpr (FIRST) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const T zj = kPreload ? zv[j] : ldnt(Z + j * ld + i);
                const T azj = kPreload ? azv[j] : ldnt(AZ + j * ld + i);
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
            T xi = (T)0;
            if constexpr (MODE == 2) xi = ldnt(x + i);
            T qn[S], aqn[S];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double tq = 0.0, taq = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    tq = fma(qo[l], beta[l * S + j], tq);
                    taq = fma(aqo[l], beta[l * S + j], taq);
                }
                const T zj = kPreload ? zv[j] : ldnt(Z + j * ld + i);
                const T azj = kPreload ? azv[j] : ldnt(AZ + j * ld + i);
                qn[j] = (T)((double)zj + tq);
                aqn[j] = (T)((double)azj + taq);
                q[j] = (double)qn[j];
                aq[j] = (double)aqn[j];
                if constexpr (!kPreload) {
                    stnt(Q + j * ld + i, qn[j]);
                    stnt(AQ + j * ld + i, aqn[j]);
                }
            }
            if constexpr (kPreload) {
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    stnt(Q + j * ld + i, qn[j]);
                    stnt(AQ + j * ld + i, aqn[j]);
                }
            }
            if constexpr (MODE == 2) {
                // a select, not a branch, so the load of x stays with the
                // others; without a pending update x is written back as read
                double qa = 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) qa = fma(qo[j], al[j], qa);
                stnt(x + i, pend ? (T)((double)xi + qa) : xi);
            }
        }
        const double ri = (double)(kPreload ? rv : ldnt(r + i));
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
// x == nullptr: r, z1 and ||r||^2 only (the solve defers x += Q alpha to the
// next block update).
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
                double aqa[R];
#pragma unroll
                for (int e = 0; e < R; ++e) aqa[e] = 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    const VT aq = ldnt(reinterpret_cast<const VT*>(AQ + j * ld + i));
#pragma unroll
                    for (int e = 0; e < R; ++e) aqa[e] = fma((double)aq[e], al[j], aqa[e]);
                }
                if (x) {
                    double qa[R];
#pragma unroll
                    for (int e = 0; e < R; ++e) qa[e] = 0.0;
#pragma unroll
                    for (int j = 0; j < S; ++j) {
                        const VT q = ldnt(reinterpret_cast<const VT*>(Q + j * ld + i));
#pragma unroll
                        for (int e = 0; e < R; ++e) qa[e] = fma((double)q[e], al[j], qa[e]);
                    }
                    VT xv = *reinterpret_cast<const VT*>(x + i);
#pragma unroll
                    for (int e = 0; e < R; ++e) xv[e] = (T)((double)xv[e] + qa[e]);
                    *reinterpret_cast<VT*>(x + i) = xv;
                }
                VT rv = *reinterpret_cast<const VT*>(r + i);
#pragma unroll
                for (int e = 0; e < R; ++e) rv[e] = (T)((double)rv[e] - aqa[e]);
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
            double aqa = 0.0;
#pragma unroll
            for (int j = 0; j < S; ++j) aqa = fma((double)ldnt(AQ + j * ld + k), al[j], aqa);
            if (x) {
                double qa = 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) qa = fma((double)ldnt(Q + j * ld + k), al[j], qa);
                x[k] = (T)((double)x[k] + qa);
            }
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

// x += Q alpha if the solve ended with that update still pending (the
// arithmetic of k_xr, row by row).
template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_x_pending(int64_t n, int s, int64_t ld,
                                                         const T* __restrict__ Q,
                                                         const double* __restrict__ alpha,
                                                         T* __restrict__ x,
                                                         const Ctrl* __restrict__ ctrl)
{
    if (!ctrl->x_pending) return;
    const int64_t stride = (int64_t)gridDim.x * kRowBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n; i += stride) {
        double qa = 0.0;
        for (int j = 0; j < s; ++j) qa = fma((double)Q[j * ld + i], alpha[j], qa);
        x[i] = (T)((double)x[i] + qa);
    }
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
static int block_grid(int64_t n, K kernel, int blocks_per_cu = 8)
{
    const int resident = resident_blocks(reinterpret_cast<const void*>(kernel), kRowBlock);
    return persistent_grid((n + kRowBlock - 1) / kRowBlock, blocks_per_cu, resident);
}

#define SSPCG_S_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <typename T>
int launch_update_gram(int64_t n, int s, const T* Z, T* Q, const T* AZ, T* AQ, const double* beta,
                       const T* r, T* x, const double* alpha, int64_t ld, double* partials,
                       int* G_out, const Ctrl* ctrl, hipStream_t st)
{
    int G = 0;
    switch (s) {
#define X(S)                                                                                    \
    case S:                                                                                     \
        if (!beta) {                                                                            \
            G = block_grid(n, k_update_gram<S, T, 0>);                                          \
            hipLaunchKernelGGL((k_update_gram<S, T, 0>), dim3(G), dim3(kRowBlock), 0, st, n, ld, \
                               Z, Q, AZ, AQ, beta, r, x, alpha, partials, ctrl);                \
        } else if (!x || !ctrl) {                                                               \
            G = block_grid(n, k_update_gram<S, T, 1>);                                          \
            hipLaunchKernelGGL((k_update_gram<S, T, 1>), dim3(G), dim3(kRowBlock), 0, st, n, ld, \
                               Z, Q, AZ, AQ, beta, r, x, alpha, partials, ctrl);                \
        } else {                                                                                \
            G = block_grid(n, k_update_gram<S, T, 2>);                                          \
            hipLaunchKernelGGL((k_update_gram<S, T, 2>), dim3(G), dim3(kRowBlock), 0, st, n, ld, \
                               Z, Q, AZ, AQ, beta, r, x, alpha, partials, ctrl);                \
        }                                                                                       \
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
    // columns whose elements R i.. are 16-byte aligned go R rows per thread
    // as one 16-byte vector per column (4 FP32 or 2 FP64 rows); anything
    // else one row per thread.  FP64 at 192^3: 133 us with one row per thread
    // at 8-byte loads, 110 us with two rows and two workgroups per CU (the
    // read-only stream then runs at 6.1 TB/s)
    constexpr int RV = sizeof(T) == 4 ? 4 : 2;
    constexpr int kBlocksPerCu = sizeof(T) == 4 ? 8 : 2;
    const bool vec = RV > 1 && ld % RV == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(AZ) % 16 == 0;
    const int64_t units = vec ? (n + RV - 1) / RV : n;
    int G = 0;
    switch (s) {
#define X(S)                                                                                   \
    case S:                                                                                    \
        if (vec) {                                                                             \
            G = block_grid(units, k_gram_rect<S, T, RV>, kBlocksPerCu);                        \
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
int launch_x_pending(int64_t n, int s, const T* Q, const double* alpha, int64_t ld, T* x,
                     const Ctrl* ctrl, hipStream_t st)
{
    hipLaunchKernelGGL((k_x_pending<T>), dim3(row_grid(n)), dim3(kRowBlock), 0, st, n, s, ld, Q,
                       alpha, x, ctrl);
    SSPCG_LAUNCHED("k_x_pending");
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
                                       const T*, T*, const double*, int64_t, double*, int*,     \
                                       const Ctrl*, hipStream_t);                                \
    template int launch_gram_rect<T>(int64_t, int, const T*, const T*, int64_t, double*, int*,  \
                                     const Ctrl*, hipStream_t);                                  \
    template int launch_xr<T>(int64_t, int, const T*, const T*, const double*, int64_t, T*, T*, \
                              const T*, T*, double*, int*, const Ctrl*, hipStream_t);           \
    template int launch_axpy_up<T>(int64_t, double*, const T*, const Ctrl*, hipStream_t);       \
    template int launch_x_pending<T>(int64_t, int, const T*, const double*, int64_t, T*,        \
                                     const Ctrl*, hipStream_t);                                  \
    template int launch_fill<T>(int64_t, T*, T, hipStream_t);
SSPCG_INST(double)
SSPCG_INST(float)
#undef SSPCG_INST

}  // namespace sspcg
