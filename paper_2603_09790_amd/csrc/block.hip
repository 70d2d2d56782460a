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

#include <algorithm>

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

// RR consecutive rows of one column: one 16-byte vector when RR > 1.
template <typename T, int RR>
struct Rows {
    T v[RR];
};

template <typename T, int RR>
__device__ inline Rows<T, RR> ld_rows(const T* p)
{
    Rows<T, RR> o;
    if constexpr (RR == 1) {
        o.v[0] = ldnt(p);
    } else {
        typedef T VT __attribute__((ext_vector_type(RR)));
        const VT w = ldnt(reinterpret_cast<const VT*>(p));
#pragma unroll
        for (int e = 0; e < RR; ++e) o.v[e] = w[e];
    }
    return o;
}

template <typename T, int RR>
__device__ inline void st_rows(T* p, const Rows<T, RR>& o)
{
    if constexpr (RR == 1) {
        stnt(p, o.v[0]);
    } else {
        typedef T VT __attribute__((ext_vector_type(RR)));
        VT w;
#pragma unroll
        for (int e = 0; e < RR; ++e) w[e] = o.v[e];
        stnt(reinterpret_cast<VT*>(p), w);
    }
}

// Rows i .. i+RR-1 of the block update and their Gram terms (see
// k_update_gram).  Every load of the rows is issued before the first store
// (the wait counter is shared by loads and stores, so a load queued behind a
// store also waits for the store): 271 -> 217 us per FP32 update at 192^3,
// 420 -> 407 us per FP64 update with one row per thread.  The rows' terms
// are added to acc in row order.
template <int S, typename T, int MODE, int RR, int K>
__device__ inline void update_rows(int64_t i, int64_t ld, const T* __restrict__ Z,
                                   T* __restrict__ Q, const T* __restrict__ AZ,
                                   T* __restrict__ AQ, const double* __restrict__ beta,
                                   const T* __restrict__ r, T* __restrict__ x,
                                   const double (&al)[S], bool pend, double (&acc)[K])
{
    Rows<T, RR> zv[S], azv[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        zv[j] = ld_rows<T, RR>(Z + j * ld + i);
        azv[j] = ld_rows<T, RR>(AZ + j * ld + i);
    }
    const Rows<T, RR> rv = ld_rows<T, RR>(r + i);
    double q[S][RR], aq[S][RR];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            st_rows<T, RR>(Q + j * ld + i, zv[j]);
            st_rows<T, RR>(AQ + j * ld + i, azv[j]);
#pragma unroll
            for (int e = 0; e < RR; ++e) {
                q[j][e] = (double)zv[j].v[e];
                aq[j][e] = (double)azv[j].v[e];
            }
        }
    } else {
        Rows<T, RR> qo[S], aqo[S], xi;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            qo[j] = ld_rows<T, RR>(Q + j * ld + i);
            aqo[j] = ld_rows<T, RR>(AQ + j * ld + i);
        }
        if constexpr (MODE == 2) xi = ld_rows<T, RR>(x + i);
        Rows<T, RR> qn[S], aqn[S];
#pragma unroll
        for (int j = 0; j < S; ++j)
#pragma unroll
            for (int e = 0; e < RR; ++e) {
                double tq = 0.0, taq = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    tq = fma((double)qo[l].v[e], beta[l * S + j], tq);
                    taq = fma((double)aqo[l].v[e], beta[l * S + j], taq);
                }
                qn[j].v[e] = (T)((double)zv[j].v[e] + tq);
                aqn[j].v[e] = (T)((double)azv[j].v[e] + taq);
                q[j][e] = (double)qn[j].v[e];
                aq[j][e] = (double)aqn[j].v[e];
            }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            st_rows<T, RR>(Q + j * ld + i, qn[j]);
            st_rows<T, RR>(AQ + j * ld + i, aqn[j]);
        }
        if constexpr (MODE == 2) {
            // a select, not a branch, so the load of x stays with the
            // others; without a pending update x is written back as read
            Rows<T, RR> xo;
#pragma unroll
            for (int e = 0; e < RR; ++e) {
                double qa = 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) qa = fma((double)qo[j].v[e], al[j], qa);
                xo.v[e] = pend ? (T)((double)xi.v[e] + qa) : xi.v[e];
            }
            st_rows<T, RR>(x + i, xo);
        }
    }
#pragma unroll
    for (int e = 0; e < RR; ++e) {
        int k = 0;
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                acc[k] = fma(q[a][e], aq[b][e], acc[k]);
                ++k;
            }
        const double ri = (double)rv.v[e];
#pragma unroll
        for (int a = 0; a < S; ++a) acc[K - S + a] = fma(q[a][e], ri, acc[K - S + a]);
    }
}

// MODE 0: the first update (Q = Z, AQ = AZ).  MODE 1: Q = Z + Q beta,
// AQ = AZ + AQ beta.  MODE 2: MODE 1 and, if ctrl->x_pending, the x update of
// the previous outer iteration, x += Q alpha with the old Q streamed here
// anyway, in the same arithmetic as k_xr; the solve's x/r update then
// leaves x alone and never reads Q.  x is loaded with the row's other
// operands, so its latency overlaps theirs.  R consecutive rows per thread
// as one 16-byte vector per column when the columns allow it (the rows of
// a ragged tail one by one), else R = 1.
template <int S, typename T, int MODE, int R>
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
    bool pend = false;
    double al[S];
    if constexpr (MODE == 2) {
        pend = ctrl->x_pending != 0;
#pragma unroll
        for (int j = 0; j < S; ++j) al[j] = alpha[j];
    }
    constexpr int64_t kRows = (int64_t)kRowBlock * R;
    const int64_t ntiles = (n + kRows - 1) / kRows;
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        double acc[K];
#pragma unroll
        for (int e = 0; e < K; ++e) acc[e] = 0.0;
        const TileRange tr = vblock_tiles(ntiles, VB, v);
        for (int64_t t = tr.first; t < tr.end; t += tr.step) {
            const int64_t i = t * kRows + (int64_t)threadIdx.x * R;
            if (i >= n) break;
            if (R == 1 || i + R <= n) {
                update_rows<S, T, MODE, R, K>(i, ld, Z, Q, AZ, AQ, beta, r, x, al, pend, acc);
            } else {
                for (int64_t k = i; k < n; ++k)
                    update_rows<S, T, MODE, 1, K>(k, ld, Z, Q, AZ, AQ, beta, r, x, al, pend, acc);
            }
        }
        block_partials<K, kRowBlock>(acc, partials, v, VB);
    }
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
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        zero_acc(acc);
        const TileRange tr = vblock_tiles(ntiles, VB, v);
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
        block_partials<K, kRowBlock>(acc, partials, v, VB);
    }
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
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        zero_acc(acc);
        const TileRange tr = vblock_tiles(ntiles, VB, v);
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
        block_partials<1, kRowBlock>(acc, partials, v, VB);
    }
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
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    return std::min(persistent_grid(ntiles, blocks_per_cu, resident), virtual_blocks(ntiles));
}

// Partial sums a reduction over `units` threads' worth of rows writes: one
// per virtual block (common.h), however many workgroups ran.
static int reduce_slots(int64_t units) { return virtual_blocks((units + kRowBlock - 1) / kRowBlock); }

#define SSPCG_S_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <typename T>
int launch_update_gram(int64_t n, int s, const T* Z, T* Q, const T* AZ, T* AQ, const double* beta,
                       const T* r, T* x, const double* alpha, int64_t ld, double* partials,
                       int* G_out, const Ctrl* ctrl, hipStream_t st)
{
    // FP32: four rows per thread as 16-byte vectors when every column allows
    // it (217 -> 202 us at 192^3).  FP64 keeps one row per thread: two rows
    // as 16-byte vectors measured the same (402-411 vs 407-409 us); the
    // kernel already streams at the rate a copy or triad reaches on these
    // boxes for its mix of reads and writes (12 of 37 columns written).
    constexpr int RV = sizeof(T) == 4 ? 4 : 1;
    auto a16 = [](const void* p) { return p == nullptr || reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    const bool vec = RV > 1 && ld % RV == 0 && a16(Z) && a16(Q) && a16(AZ) && a16(AQ) && a16(r) &&
                     a16(x);
    const int64_t units = vec ? (n + RV - 1) / RV : n;
    const int mode = !beta ? 0 : (!x || !ctrl) ? 1 : 2;
    int G = 0;
    switch (s) {
#define L(S, M, R)                                                                               \
    do {                                                                                         \
        G = block_grid(units, k_update_gram<S, T, M, R>);                                       \
        hipLaunchKernelGGL((k_update_gram<S, T, M, R>), dim3(G), dim3(kRowBlock), 0, st, n, ld,  \
                           Z, Q, AZ, AQ, beta, r, x, alpha, partials, ctrl);                     \
    } while (0)
#define X(S)                                                                                    \
    case S:                                                                                     \
        if (vec) {                                                                              \
            if (mode == 0) L(S, 0, RV); else if (mode == 1) L(S, 1, RV); else L(S, 2, RV);      \
        } else {                                                                                \
            if (mode == 0) L(S, 0, 1); else if (mode == 1) L(S, 1, 1); else L(S, 2, 1);         \
        }                                                                                       \
        break;
        SSPCG_S_CASES(X)
#undef X
#undef L
    default:
        set_error("s out of range");
        return SSPCG_ERR_ARG;
    }
    SSPCG_LAUNCHED("k_update_gram");
    *G_out = reduce_slots(units);
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
    *G_out = reduce_slots(units);
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
    *G_out = reduce_slots(units);
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
