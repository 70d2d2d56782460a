// Sliced layout of the CSR matrix and the kernels that stream it: SpMV with
// the fused matrix-powers epilogue (Algorithm 2), the FP64 residual, and the
// SpMV of classical PCG.
//
// Layout.  Slice c holds rows 64c..64c+63, one per lane of a wavefront.
// Entry k of every row in the slice is stored contiguously (64 values), so
// each load instruction of the wave reads 512 contiguous bytes of values.
// In a stencil matrix the rows of a slice use the same column offsets
// col - row; such a slice stores its sorted offset list once and no column
// indices at all (8 instead of 12 bytes per FP64 entry, 4 instead of 8 in
// FP32), and the gathers x[row + o_k] of a wave are contiguous too.  A row
// without an entry at offset o_k holds an exact zero there and gathers its
// own element instead.  Slices whose offset union is too long keep explicit
// columns (64 indices per entry k), padded to the longest row.  In both
// kinds the entries of a row keep their CSR order, which is the summation
// order, and a zero adds nothing: the sum is the CSR sum.

#include <algorithm>
#include <climits>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "launch.h"

namespace sspcg {

namespace {

constexpr int kFlagPattern = 1, kFlagDiag = 2, kFlagValue = 4;

__global__ __launch_bounds__(kRowBlock) void k_inspect(int32_t n, int32_t nnz, int64_t nslices,
                                                       const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val,
                                                       int32_t* __restrict__ flags,
                                                       int32_t* __restrict__ width,
                                                       double* __restrict__ dinv,
                                                       float* __restrict__ dinv32,
                                                       bool values_only)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    int len = 0;
    if (i < n) {
        const int32_t a = rp[i], b = rp[i + 1];
        int f = 0;
        if (i == 0 && a != 0) f |= kFlagPattern;
        if (i == n - 1 && b != nnz) f |= kFlagPattern;
        if (a < 0 || b < a || b > nnz) {
            f |= kFlagPattern;
        } else {
            len = b - a;
            double d = 0.0;
            bool has = false;
            for (int32_t e = a; e < b; ++e) {
                const int32_t c = col[e];
                const double v = val[e];
                if (!values_only && (c < 0 || c >= n)) f |= kFlagPattern;
                if (!isfinite(v)) f |= kFlagValue;
                if (c == i) {
                    d = v;
                    has = true;
                }
            }
            if (!has || !(d > 0.0)) f |= kFlagDiag;
            const double di = (has && d > 0.0) ? 1.0 / d : 0.0;
            dinv[i] = di;
            if (dinv32) dinv32[i] = (float)di;
        }
        if (f) atomicOr(flags, f);
    }
    int w = len;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) w = max(w, __shfl_xor(w, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int64_t c = i / kSlice;
        if (c < nslices) width[c] = w;
    }
}

__device__ inline int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}

// One wavefront per slice: the sorted union of the offsets col - row of the
// slice's rows (a merge of 64 sorted lists), or -1 in ulen when the union
// exceeds kMaxUnion or a row's columns are not strictly increasing.
__global__ __launch_bounds__(kRowBlock) void k_slice_union(int32_t n, int64_t nslices,
                                                           const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           int32_t* __restrict__ uni,
                                                           int32_t* __restrict__ ulen)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c = (int64_t)blockIdx.x * (kRowBlock / kWave) + threadIdx.x / kWave;
    if (c >= nslices) return;
    const int64_t row = c * kSlice + lane;
    int32_t p = 0, e = 0;
    if (row < n) {
        p = rp[row];
        e = rp[row + 1];
    }
    bool sorted = true;
    int prev = INT_MIN;
    int U = 0;
    for (;;) {
        const int cur = p < e ? col[p] - (int32_t)row : INT_MAX;
        const int m = wave_min(cur);
        if (m == INT_MAX) break;
        if (U < kMaxUnion && lane == 0) uni[c * kMaxUnion + U] = m;
        ++U;
        if (p < e && cur == m) {
            if (cur <= prev) sorted = false;
            prev = cur;
            ++p;
        }
        if (U > kMaxUnion) break;
    }
    const bool all_sorted = __all(sorted);
    if (lane == 0) ulen[c] = (U > kMaxUnion || !all_sorted) ? -1 : U;
}

// Copies the offset lists of the shared-offset slices into soff.
__global__ __launch_bounds__(kRowBlock) void k_pack_union(int64_t nslices,
                                                          const int64_t* __restrict__ slice_ptr,
                                                          const int64_t* __restrict__ slice_aux,
                                                          const int32_t* __restrict__ uni,
                                                          int32_t* __restrict__ soff)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c = (int64_t)blockIdx.x * (kRowBlock / kWave) + threadIdx.x / kWave;
    if (c >= nslices) return;
    const int64_t aux = slice_aux[c];
    if (aux >= 0) return;
    const int w = (int)((slice_ptr[c + 1] - slice_ptr[c]) / kSlice);
    for (int k = lane; k < w; k += kWave) soff[-aux - 1 + k] = uni[c * kMaxUnion + k];
}

// One thread per row: values (and explicit columns) of the sliced layout.
__global__ __launch_bounds__(kRowBlock) void k_fill(int32_t n, int64_t nslices,
                                                    const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const int64_t* __restrict__ slice_ptr,
                                                    const int64_t* __restrict__ slice_aux,
                                                    const int32_t* __restrict__ soff,
                                                    int32_t* __restrict__ scol,
                                                    uint32_t* __restrict__ smask,
                                                    double* __restrict__ sval,
                                                    float* __restrict__ sval32, bool values_only)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    const int64_t c = i / kSlice;
    if (c >= nslices) return;
    const int lane = (int)(i % kSlice);
    const int64_t base = slice_ptr[c], aux = slice_aux[c];
    const int w = (int)((slice_ptr[c + 1] - base) / kSlice);
    int32_t a = 0, len = 0;
    if (i < n) {
        a = rp[i];
        len = rp[i + 1] - a;
    }
    if (aux < 0) {
        const int32_t* off = soff + (-aux - 1);
        int32_t p = 0;
        uint32_t mask = 0;
        for (int k = 0; k < w; ++k) {
            double v = 0.0;
            if (p < len && col[a + p] - (int32_t)i == off[k]) {
                v = val[a + p];
                mask |= 1u << k;
                ++p;
            }
            const int64_t slot = base + (int64_t)k * kSlice + lane;
            sval[slot] = v;
            if (sval32) sval32[slot] = (float)v;
        }
        if (!values_only) smask[i] = mask;
    } else {
        for (int k = 0; k < w; ++k) {
            const int64_t slot = base + (int64_t)k * kSlice + lane;
            double v = 0.0;
            int32_t cc = i < n ? (int32_t)i : 0;
            if (k < len) {
                v = val[a + k];
                cc = col[a + k];
            }
            sval[slot] = v;
            if (sval32) sval32[slot] = (float)v;
            if (!values_only) scol[aux + (int64_t)k * kSlice + lane] = cc;
        }
    }
}

// Uniform layout: one thread per row walks its sorted columns against the
// global offset list; slot of entry k in FP64 (pairs) and FP32 (quads).
__device__ inline int64_t uslot(int64_t c, int k, int lane, int uwv, int V)
{
    return c * kSlice * uwv + (int64_t)(k / V) * (kSlice * V) + lane * V + k % V;
}

__global__ __launch_bounds__(kRowBlock) void k_fill_uniform(int32_t n, int64_t nslices,
                                                            const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ val,
                                                            const int32_t* __restrict__ uoff, int uw,
                                                            int uwv64, int uwv32,
                                                            uint32_t* __restrict__ smask,
                                                            double* __restrict__ sval,
                                                            float* __restrict__ sval32,
                                                            bool values_only)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    const int64_t c = i / kSlice;
    if (c >= nslices) return;
    const int lane = (int)(i % kSlice);
    int32_t a = 0, len = 0;
    if (i < n) {
        a = rp[i];
        len = rp[i + 1] - a;
    }
    double v[kMaxUnion];
    uint32_t mask = 0;
    int32_t p = 0;
    for (int k = 0; k < uw; ++k) {
        v[k] = 0.0;
        if (p < len && col[a + p] - (int32_t)i == uoff[k]) {
            v[k] = val[a + p];
            mask |= 1u << k;
            ++p;
        }
    }
    for (int k = 0; k < uwv64; ++k) sval[uslot(c, k, lane, uwv64, 2)] = k < uw ? v[k] : 0.0;
    if (sval32)
        for (int k = 0; k < uwv32; ++k) sval32[uslot(c, k, lane, uwv32, 4)] = k < uw ? (float)v[k] : 0.0f;
    if (!values_only) smask[i] = mask;
}

// ------------------------------------------------------------------ SpMV

template <typename T>
__device__ inline T ld_stream(const T* p)
{
    return __builtin_nontemporal_load(p);
}

// Sum of one row of an explicit-column slice, entries in CSR order.  FP32
// values and vectors are multiplied exactly in FP64 and summed in FP64.
template <typename T, int U>
__device__ inline double row_explicit(const int32_t* __restrict__ cp, const T* __restrict__ vp, int w,
                                      const T* __restrict__ x)
{
    double acc = 0.0;
    int k = 0;
    for (; k + U <= w; k += U) {
        int32_t cc[U];
        T vv[U], xx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = ld_stream(cp + (int64_t)(k + u) * kSlice);
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u] = ld_stream(vp + (int64_t)(k + u) * kSlice);
#pragma unroll
        for (int u = 0; u < U; ++u) xx[u] = x[cc[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = fma((double)vv[u], (double)xx[u], acc);
    }
    for (; k < w; ++k) {
        const int32_t cc = ld_stream(cp + (int64_t)k * kSlice);
        const T vv = ld_stream(vp + (int64_t)k * kSlice);
        acc = fma((double)vv, (double)x[cc], acc);
    }
    return acc;
}

// Sum of one row of a shared-offset slice: entry k multiplies x[row + o_k],
// or x[self] (with the stored zero: an exact zero term) where bit k of the
// row's mask is clear.  The gather addresses depend only on the mask and the
// offsets, so values and gathers are in flight together.
template <typename T, int U>
__device__ inline double row_shared(const int32_t* __restrict__ off, const T* __restrict__ vp, int w,
                                    uint32_t mask, int32_t row, int32_t self,
                                    const T* __restrict__ x)
{
    double acc = 0.0;
    int k = 0;
    for (; k + U <= w; k += U) {
        T vv[U], xx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u] = ld_stream(vp + (int64_t)(k + u) * kSlice);
#pragma unroll
        for (int u = 0; u < U; ++u) xx[u] = x[(mask >> (k + u)) & 1u ? row + off[k + u] : self];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = fma((double)vv[u], (double)xx[u], acc);
    }
    for (; k < w; ++k) {
        const T vv = ld_stream(vp + (int64_t)k * kSlice);
        acc = fma((double)vv, (double)x[(mask >> k) & 1u ? row + off[k] : self], acc);
    }
    return acc;
}

constexpr int kUnroll = 9;

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};

// Row of the uniform layout: NV 16-byte vectors per lane (NV > 0: known at
// compile time, fully unrolled; NV = 0: runtime count).  The gather index
// depends only on the mask and the offsets, so all loads are independent.
template <typename T, int NV>
__device__ inline double row_uniform(const Sell<T>& A, int64_t c, int lane,
                                     const T* __restrict__ x)
{
    constexpr int V = 16 / sizeof(T);
    typedef typename Vec16<T>::type VT;
    const int64_t row = c * kSlice + lane;
    const int32_t self = (int32_t)(row < A.n ? row : A.n - 1);
    const uint32_t m = A.smask[row];
    const VT* vp = reinterpret_cast<const VT*>(A.val + c * kSlice * A.uwv) + lane;
    const int nv = NV > 0 ? NV : A.uwv / V;
    double acc = 0.0;
#pragma unroll 4
    for (int j = 0; j < nv; ++j) {
        const VT v = __builtin_nontemporal_load(vp + (int64_t)j * kSlice);
#pragma unroll
        for (int h = 0; h < V; ++h) {
            const int k = j * V + h;
            const int32_t idx = (m >> k) & 1u ? (int32_t)row + A.uoff[k] : self;
            acc = fma((double)v[h], (double)x[idx], acc);
        }
    }
    return acc;
}

template <typename T>
__device__ inline double uniform_row(const Sell<T>& A, int64_t c, int lane, const T* __restrict__ x)
{
    constexpr int V = 16 / sizeof(T);
    switch (A.uwv / V) {
    case 2: return row_uniform<T, 2>(A, c, lane, x);     // 5-point (FP32)
    case 3: return row_uniform<T, 3>(A, c, lane, x);     // 5-point (FP64)
    case 4: return row_uniform<T, 4>(A, c, lane, x);     // 7-point (FP64)
    case 7: return row_uniform<T, 7>(A, c, lane, x);     // 27-point (FP32)
    case 14: return row_uniform<T, 14>(A, c, lane, x);   // 27-point (FP64)
    default: return row_uniform<T, 0>(A, c, lane, x);
    }
}

// (A x)_row for the row of this lane in slice c (c < nslices).
template <typename T>
__device__ inline double slice_row(const Sell<T>& A, int64_t c, int lane, const T* __restrict__ x)
{
    if (A.uniform) return uniform_row<T>(A, c, lane, x);
    const int64_t base = A.slice_ptr[c], aux = A.slice_aux[c];
    const int w = (int)((A.slice_ptr[c + 1] - base) / kSlice);
    const int64_t row = c * kSlice + lane;
    if (aux < 0) {
        const int32_t self = (int32_t)(row < A.n ? row : A.n - 1);
        return row_shared<T, kUnroll>(A.soff + (-aux - 1), A.val + base + lane, w, A.smask[row],
                                      (int32_t)row, self, x);
    }
    return row_explicit<T, kUnroll>(A.col + aux + lane, A.val + base + lane, w, x);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kRowBlock) void k_spmv(Sell<T> A, const T* __restrict__ x,
                                                    T* __restrict__ y,
                                                    const T* __restrict__ zprev,
                                                    T* __restrict__ znext, double c1, double c2,
                                                    double c3, const Ctrl* __restrict__ ctrl)
{
    if (ctrl && ctrl->done) return;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr int kSlicesPerTile = kRowBlock / kSlice;
    // one tile (4 slices, one per wavefront) per workgroup
    const int64_t c = xcd_block_tile() * kSlicesPerTile + wave;
    if (c >= A.nslices) return;
    const double acc = slice_row<T>(A, c, lane, x);
    const int64_t row = c * kSlice + lane;
    if (row < A.n) {
        const T p = (T)acc;
        y[row] = p;
        if (MODE >= 1) {
            const double t1 = (double)A.dinv[row] * (double)p;
            double z = c1 * t1 - c2 * (double)x[row];
            if (MODE == 2) z -= c3 * (double)zprev[row];
            znext[row] = (T)z;
        }
    }
}

template <typename TR>
__global__ __launch_bounds__(kRowBlock) void k_residual(Sell<double> A, const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        TR* __restrict__ r, TR* __restrict__ z1,
                                                        const TR* __restrict__ dinvT,
                                                        double* __restrict__ partials)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr int kSlicesPerTile = kRowBlock / kSlice;
    const int64_t ntiles = (A.nslices + kSlicesPerTile - 1) / kSlicesPerTile;
    const TileRange tr = xcd_tiles(ntiles);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t c = t * kSlicesPerTile + wave;
        if (c >= A.nslices) break;
        const double ax = slice_row<double>(A, c, lane, x);
        const int64_t row = c * kSlice + lane;
        if (row < A.n) {
            const double bi = b[row];
            const double ri = bi - ax;
            const TR rs = (TR)ri;
            r[row] = rs;
            acc[0] = fma(ri, ri, acc[0]);
            acc[1] = fma((double)rs, (double)rs, acc[1]);
            acc[2] = fma(bi, bi, acc[2]);
            if (z1) {
                const TR zs = (TR)((double)dinvT[row] * (double)rs);
                z1[row] = zs;
                acc[3] = fma((double)rs, (double)zs, acc[3]);
            }
        }
    }
    block_partials<4, kRowBlock>(acc, partials);
}

__global__ __launch_bounds__(kRowBlock) void k_pcg_spmv(Sell<double> A, const double* __restrict__ p,
                                                        double* __restrict__ q,
                                                        double* __restrict__ partials,
                                                        const Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr int kSlicesPerTile = kRowBlock / kSlice;
    const int64_t ntiles = (A.nslices + kSlicesPerTile - 1) / kSlicesPerTile;
    const TileRange tr = xcd_tiles(ntiles);
    double acc[1] = {0.0};
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t c = t * kSlicesPerTile + wave;
        if (c >= A.nslices) break;
        const double ap = slice_row<double>(A, c, lane, p);
        const int64_t row = c * kSlice + lane;
        if (row < A.n) {
            q[row] = ap;
            acc[0] = fma(p[row], ap, acc[0]);
        }
    }
    block_partials<1, kRowBlock>(acc, partials);
}

// Classical PCG update, iteration k: alpha = rho_k / p^T q (every block sums
// the same partials in the same order); x += alpha p; r -= alpha q;
// z = dinv .* r; partials of r^T z and r^T r.
__global__ __launch_bounds__(kRowBlock) void k_pcg_update(int64_t n, int64_t k, double* __restrict__ x,
                                                          double* __restrict__ r,
                                                          double* __restrict__ z,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ dinv,
                                                          const double* __restrict__ pq_part,
                                                          int Gpq, double* __restrict__ partials,
                                                          const Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    __shared__ double s_alpha;
    if (threadIdx.x < kWave) {
        const double pq = wave_finish(pq_part, 0, Gpq);
        if (threadIdx.x == 0) s_alpha = ctrl->rho[k & 1] / pq;
    }
    __syncthreads();
    const double a = s_alpha;
    double acc[2] = {0.0, 0.0};
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i < n) {
            x[i] = fma(a, p[i], x[i]);
            const double ri = fma(-a, q[i], r[i]);
            r[i] = ri;
            const double zi = dinv[i] * ri;
            z[i] = zi;
            acc[0] = fma(ri, zi, acc[0]);
            acc[1] = fma(ri, ri, acc[1]);
        }
    }
    block_partials<2, kRowBlock>(acc, partials);
}

// p = z + (rho_{k+1} / rho_k) p, after the stop test of iteration k.  Every
// block finishes the same partial sums; block 0 records the bookkeeping.
__global__ __launch_bounds__(kRowBlock) void k_pcg_pupdate(int64_t n, int64_t k,
                                                           const double* __restrict__ z,
                                                           double* __restrict__ p,
                                                           const double* __restrict__ partials,
                                                           int G, Ctrl* __restrict__ ctrl,
                                                           double* __restrict__ hist)
{
    if (ctrl->done) return;
    __shared__ double s_v[2];
    if (threadIdx.x < 2 * kWave) {
        const int e = threadIdx.x / kWave;
        const double v = wave_finish(partials, e, G);
        if ((threadIdx.x & (kWave - 1)) == 0) s_v[e] = v;
    }
    __syncthreads();
    const double rz = s_v[0], rr = s_v[1];
    const double relres = sqrt(rr) / ctrl->nb;
    const bool stop = !isfinite(relres) || relres <= ctrl->tol || k + 1 >= ctrl->max_iter;
    // Block 0 writes only fields no block reads in this launch: rho of the
    // other parity, relres, iter, status and done (read at entry only, by
    // blocks that then have nothing left to do once it is set).
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (hist) hist[k] = relres;
        ctrl->rho[(k + 1) & 1] = rz;
        ctrl->relres = relres;
        ctrl->iter = (int32_t)(k + 1);
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
    if (stop) return;
    const double bt = rz / ctrl->rho[k & 1];
    const int64_t ntiles = (n + kRowBlock - 1) / kRowBlock;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t i = t * kRowBlock + threadIdx.x;
        if (i < n) p[i] = fma(bt, p[i], z[i]);
    }
}

// z_1 = M^{-1} r and p_1 = r: the start of the matrix powers kernel.
template <typename T>
__global__ __launch_bounds__(kRowBlock) void k_mpk_start(int64_t n, const T* __restrict__ r,
                                                         const T* __restrict__ dinv,
                                                         T* __restrict__ z1, T* __restrict__ p1)
{
    const int64_t stride = (int64_t)gridDim.x * kRowBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n; i += stride) {
        const T ri = r[i];
        p1[i] = ri;
        z1[i] = (T)((double)dinv[i] * (double)ri);
    }
}

}  // namespace

// ------------------------------------------------------------------ host

int num_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

int resident_blocks(const void* kernel, int threads)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1)
        nb = 1;
    cache.emplace(kernel, nb);
    return nb;
}

int persistent_grid(int64_t ntiles, int blocks_per_cu, int resident)
{
    int64_t g = (int64_t)num_cus() * std::min(blocks_per_cu, resident);
    g = std::min<int64_t>(g, kMaxGrid);
    g = std::min<int64_t>(g, std::max<int64_t>(ntiles, 1));
    if (g >= kNumXcd) g -= g % kNumXcd;
    return (int)std::max<int64_t>(g, 1);
}

template <typename T>
Sell<T> sell_view(const sspcg_matrix* A);

template <>
Sell<double> sell_view<double>(const sspcg_matrix* A)
{
    return {A->n, A->uniform, A->uw, (A->uw + 1) / 2 * 2, A->uoff, A->nslices, A->slice_ptr,
            A->slice_aux, A->scol, A->soff, A->smask, A->sval, A->dinv};
}

template <>
Sell<float> sell_view<float>(const sspcg_matrix* A)
{
    return {A->n, A->uniform, A->uw, (A->uw + 3) / 4 * 4, A->uoff, A->nslices, A->slice_ptr,
            A->slice_aux, A->scol, A->soff, A->smask, A->sval32, A->dinv32};
}

static int64_t spmv_tiles(const sspcg_matrix* A)
{
    return (A->nslices + kRowBlock / kSlice - 1) / (kRowBlock / kSlice);
}

// Persistent grid for the SpMV kernels that also reduce: all workgroups
// resident at once.
template <typename K>
static int spmv_reduce_grid(const sspcg_matrix* A, K kernel)
{
    const int resident = resident_blocks(reinterpret_cast<const void*>(kernel), kRowBlock);
    return persistent_grid(spmv_tiles(A), 8, resident);
}

int matrix_inspect(sspcg_matrix* A, const double* val, bool values_only, LayoutPlan* plan,
                   int32_t** d_union, hipStream_t st)
{
    const int64_t nrows_padded = A->nslices * kSlice;
    const int blocks = (int)((nrows_padded + kRowBlock - 1) / kRowBlock);
    std::vector<int32_t> width(A->nslices), ulen(A->nslices);
    int32_t* dwidth = nullptr;
    int32_t* dulen = nullptr;
    SSPCG_HIP(hipMallocAsync((void**)&dwidth, sizeof(int32_t) * A->nslices, st));
    SSPCG_HIP(hipMemsetAsync(A->dflags, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_inspect, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nnz, A->nslices,
                       A->row_ptr, A->col, val, A->dflags, dwidth, A->dinv, A->dinv32, values_only);
    SSPCG_LAUNCHED("k_inspect");
    int32_t hflags = 0;
    SSPCG_HIP(hipMemcpyAsync(&hflags, A->dflags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipMemcpyAsync(width.data(), dwidth, sizeof(int32_t) * A->nslices,
                             hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipFreeAsync(dwidth, st));
    SSPCG_HIP(hipStreamSynchronize(st));
    if (hflags & kFlagPattern) {
        set_error("malformed CSR pattern (row pointers or column indices)");
        return SSPCG_ERR_ARG;
    }
    if (hflags & kFlagValue) {
        set_error("non-finite matrix value");
        return SSPCG_ERR_NONFINITE;
    }
    if (hflags & kFlagDiag) {
        set_error("a diagonal entry is missing or not positive: A is not SPD");
        return SSPCG_ERR_BREAKDOWN;
    }
    if (!plan) return SSPCG_OK;
    // the pattern is valid: choose the kind of every slice
    SSPCG_HIP(hipMallocAsync((void**)d_union, sizeof(int32_t) * A->nslices * kMaxUnion, st));
    SSPCG_HIP(hipMallocAsync((void**)&dulen, sizeof(int32_t) * A->nslices, st));
    hipLaunchKernelGGL(k_slice_union, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nslices,
                       A->row_ptr, A->col, *d_union, dulen);
    SSPCG_LAUNCHED("k_slice_union");
    SSPCG_HIP(hipMemcpyAsync(ulen.data(), dulen, sizeof(int32_t) * A->nslices,
                             hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipFreeAsync(dulen, st));
    SSPCG_HIP(hipStreamSynchronize(st));
    plan->slice_ptr.assign(A->nslices + 1, 0);
    plan->slice_aux.assign(A->nslices, 0);
    plan->ncol = plan->nsoff = plan->nshared = 0;
    for (int64_t c = 0; c < A->nslices; ++c) {
        // shared offsets pay off while the value stream grows by less than
        // the column stream it removes: 8 U < 12 w bytes per lane (FP64)
        const bool shared = ulen[c] > 0 && 2 * ulen[c] < 3 * width[c] + 2;
        int64_t w = width[c];
        if (shared) {
            w = ulen[c];
            plan->slice_aux[c] = -(plan->nsoff + 1);
            plan->nsoff += w;
            plan->nshared += 1;
        } else {
            plan->slice_aux[c] = plan->ncol;
            plan->ncol += w * kSlice;
        }
        plan->slice_ptr[c + 1] = plan->slice_ptr[c] + w * kSlice;
    }
    plan->slots = plan->slice_ptr[A->nslices];
    // uniform layout: every slice shared, and the union of all their lists
    // fits one mask and costs at most 2 % more stored entries
    plan->uoff.clear();
    if (plan->nshared == A->nslices) {
        std::vector<int32_t> hun((size_t)A->nslices * kMaxUnion);
        SSPCG_HIP(hipMemcpy(hun.data(), *d_union, sizeof(int32_t) * hun.size(),
                            hipMemcpyDeviceToHost));
        std::vector<int32_t> all;
        all.reserve(64);
        bool fits = true;
        for (int64_t c = 0; c < A->nslices && fits; ++c) {
            for (int k = 0; k < ulen[c]; ++k) {
                const int32_t o = hun[(size_t)c * kMaxUnion + k];
                if (std::find(all.begin(), all.end(), o) == all.end()) {
                    all.push_back(o);
                    if ((int)all.size() > kMaxUnion) {
                        fits = false;
                        break;
                    }
                }
            }
        }
        if (fits && !all.empty() &&
            (double)A->nslices * kSlice * all.size() <= 1.02 * (double)plan->slots) {
            std::sort(all.begin(), all.end());
            plan->uoff = all;
        }
    }
    return SSPCG_OK;
}

int matrix_pack(sspcg_matrix* A, const int32_t* d_union, hipStream_t st)
{
    const int blocks = (int)((A->nslices * kSlice + kRowBlock - 1) / kRowBlock);
    hipLaunchKernelGGL(k_pack_union, dim3(blocks), dim3(kRowBlock), 0, st, A->nslices,
                       A->slice_ptr, A->slice_aux, d_union, A->soff);
    SSPCG_LAUNCHED("k_pack_union");
    return SSPCG_OK;
}

int matrix_fill(sspcg_matrix* A, const double* val, bool values_only, hipStream_t st)
{
    const int64_t nrows_padded = A->nslices * kSlice;
    const int blocks = (int)((nrows_padded + kRowBlock - 1) / kRowBlock);
    if (A->uniform) {
        hipLaunchKernelGGL(k_fill_uniform, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nslices,
                           A->row_ptr, A->col, val, A->uoff, A->uw, (A->uw + 1) / 2 * 2,
                           (A->uw + 3) / 4 * 4, A->smask, A->sval, A->sval32, values_only);
        SSPCG_LAUNCHED("k_fill_uniform");
        SSPCG_HIP(hipStreamSynchronize(st));
        return SSPCG_OK;
    }
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nslices, A->row_ptr,
                       A->col, val, A->slice_ptr, A->slice_aux, A->soff, A->scol, A->smask,
                       A->sval, A->sval32, values_only);
    SSPCG_LAUNCHED("k_fill");
    SSPCG_HIP(hipStreamSynchronize(st));
    return SSPCG_OK;
}

template <typename T>
int launch_mpk_start(int64_t n, const T* r, const T* dinv, T* z1, T* p1, hipStream_t st)
{
    hipLaunchKernelGGL((k_mpk_start<T>), dim3(row_grid(n)), dim3(kRowBlock), 0, st, n, r, dinv,
                       z1, p1);
    SSPCG_LAUNCHED("k_mpk_start");
    return SSPCG_OK;
}

template int launch_mpk_start<double>(int64_t, const double*, const double*, double*, double*,
                                      hipStream_t);
template int launch_mpk_start<float>(int64_t, const float*, const float*, float*, float*,
                                     hipStream_t);

template <typename T>
int launch_spmv(const sspcg_matrix* A, int mode, const T* x, T* y, const T* zprev, T* znext,
                double c1, double c2, double c3, const Ctrl* ctrl, hipStream_t st)
{
    const Sell<T> S = sell_view<T>(A);
    const int64_t G = spmv_tiles(A);
    if (mode == 0)
        hipLaunchKernelGGL((k_spmv<T, 0>), dim3(G), dim3(kRowBlock), 0, st, S, x, y, zprev, znext,
                           c1, c2, c3, ctrl);
    else if (mode == 1)
        hipLaunchKernelGGL((k_spmv<T, 1>), dim3(G), dim3(kRowBlock), 0, st, S, x, y, zprev, znext,
                           c1, c2, c3, ctrl);
    else
        hipLaunchKernelGGL((k_spmv<T, 2>), dim3(G), dim3(kRowBlock), 0, st, S, x, y, zprev, znext,
                           c1, c2, c3, ctrl);
    SSPCG_LAUNCHED("k_spmv");
    return SSPCG_OK;
}

template int launch_spmv<double>(const sspcg_matrix*, int, const double*, double*, const double*,
                                 double*, double, double, double, const Ctrl*, hipStream_t);
template int launch_spmv<float>(const sspcg_matrix*, int, const float*, float*, const float*,
                                float*, double, double, double, const Ctrl*, hipStream_t);

template <typename TR>
int launch_residual(const sspcg_matrix* A, const double* x, const double* b, TR* r, TR* z1,
                    double* partials, int* G_out, hipStream_t st)
{
    const Sell<double> S = sell_view<double>(A);
    const TR* dinvT = sell_view<TR>(A).dinv;
    const int G = spmv_reduce_grid(A, k_residual<TR>);
    hipLaunchKernelGGL((k_residual<TR>), dim3(G), dim3(kRowBlock), 0, st, S, x, b, r, z1, dinvT,
                       partials);
    SSPCG_LAUNCHED("k_residual");
    *G_out = G;
    return SSPCG_OK;
}

template int launch_residual<double>(const sspcg_matrix*, const double*, const double*, double*,
                                     double*, double*, int*, hipStream_t);
template int launch_residual<float>(const sspcg_matrix*, const double*, const double*, float*,
                                    float*, double*, int*, hipStream_t);

int launch_pcg_spmv(const sspcg_matrix* A, const double* p, double* q, double* partials,
                    int* G_out, const Ctrl* ctrl, hipStream_t st)
{
    const int G = spmv_reduce_grid(A, k_pcg_spmv);
    hipLaunchKernelGGL(k_pcg_spmv, dim3(G), dim3(kRowBlock), 0, st, sell_view<double>(A), p, q,
                       partials, ctrl);
    SSPCG_LAUNCHED("k_pcg_spmv");
    *G_out = G;
    return SSPCG_OK;
}

int launch_pcg_update(const sspcg_matrix* A, int64_t k, double* x, double* r, double* z,
                      const double* p, const double* q, const double* pq_partials, int Gpq,
                      double* partials, int* G_out, Ctrl* ctrl, hipStream_t st)
{
    const int G = row_grid(A->n);
    hipLaunchKernelGGL(k_pcg_update, dim3(G), dim3(kRowBlock), 0, st, (int64_t)A->n, k, x, r, z,
                       p, q, A->dinv, pq_partials, Gpq, partials, ctrl);
    SSPCG_LAUNCHED("k_pcg_update");
    *G_out = G;
    return SSPCG_OK;
}

int launch_pcg_pupdate(int64_t n, int64_t k, const double* z, double* p, const double* partials,
                       int G, Ctrl* ctrl, double* hist, hipStream_t st)
{
    const int Gp = row_grid(n);
    hipLaunchKernelGGL(k_pcg_pupdate, dim3(Gp), dim3(kRowBlock), 0, st, n, k, z, p, partials, G,
                       ctrl, hist);
    SSPCG_LAUNCHED("k_pcg_pupdate");
    return SSPCG_OK;
}

}  // namespace sspcg
