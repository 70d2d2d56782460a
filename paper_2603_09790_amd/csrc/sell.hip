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
// without an entry at offset o_k holds an exact zero there, and its gather
// index is clamped into x.  Slices whose offset union is too long keep
// explicit columns (64 indices per entry k), padded to the longest row.
// When one list fits all slices the matrix uses the uniform layout instead
// (one global list, 16-byte value groups, optionally one triangle of a
// symmetric matrix, and in FP64 the gathered parts of x staged in LDS as
// aligned 16-byte vectors, one window per group of nearby offsets; see Sell
// in common.h).  In every kind the entries
// of a row keep their CSR order, which is the summation order, and a zero
// adds nothing (for finite x): the sum is the CSR sum.

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include <cstdlib>

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
            if (dinv) dinv[i] = di;
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
        for (int k = 0; k < w; ++k) {
            double v = 0.0;
            if (p < len && col[a + p] - (int32_t)i == off[k]) {
                v = val[a + p];
                ++p;
            }
            const int64_t slot = base + (int64_t)k * kSlice + lane;
            sval[slot] = v;
            if (sval32) sval32[slot] = (float)v;
        }
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

// Symmetry check, one thread per row of a validated pattern: every stored
// a(i, j) must equal a(j, i) bit for bit, an absent entry counting as +0.
__global__ __launch_bounds__(kRowBlock) void k_check_symmetric(int32_t n,
                                                               const int32_t* __restrict__ rp,
                                                               const int32_t* __restrict__ col,
                                                               const double* __restrict__ val,
                                                               int32_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (i >= n) return;
    bool ok = true;
    const int32_t b = rp[i + 1];
    for (int32_t e = rp[i]; e < b; ++e) {
        const int32_t j = col[e];
        if (j == (int32_t)i) continue;
        double w = 0.0;
        const int32_t fb = rp[j + 1];
        for (int32_t f = rp[j]; f < fb; ++f)
            if (col[f] == (int32_t)i) {
                w = val[f];
                break;
            }
        if (__double_as_longlong(w) != __double_as_longlong(val[e])) ok = false;
    }
    if (!ok) atomicOr(flags, 1);
}

// Uniform layout: one thread per row walks its sorted columns against the
// global offset list; stored entry t = k - h0 (h0 = 0, or uw/2 for the
// symmetric half storage) in groups of v64 FP64 and v32 FP32 values (16
// bytes each, or single values with the symmetric half storage).
__device__ inline int64_t uslot(int64_t c, int k, int lane, int uwv, int V)
{
    return c * kSlice * uwv + (int64_t)(k / V) * (kSlice * V) + lane * V + k % V;
}

__global__ __launch_bounds__(kRowBlock) void k_fill_uniform(int32_t n, int64_t nslices,
                                                            const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ val,
                                                            const int32_t* __restrict__ uoff, int uw,
                                                            int h0, int uwv64, int v64, int uwv32,
                                                            int v32,
                                                            double* __restrict__ sval,
                                                            float* __restrict__ sval32)
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
    int32_t p = 0;
    for (int k = 0; k < uw; ++k) {
        v[k] = 0.0;
        if (p < len && col[a + p] - (int32_t)i == uoff[k]) {
            v[k] = val[a + p];
            ++p;
        }
    }
    for (int t = 0; t < uwv64; ++t)
        sval[uslot(c, t, lane, uwv64, v64)] = h0 + t < uw ? v[h0 + t] : 0.0;
    if (sval32)
        for (int t = 0; t < uwv32; ++t)
            sval32[uslot(c, t, lane, uwv32, v32)] = h0 + t < uw ? (float)v[h0 + t] : 0.0f;
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

// Gather index of entry k of a row: row + o_k clamped into [0, last].  A row
// without an entry at o_k holds a stored zero there, so whatever element the
// clamped index reaches adds an exact zero term (x finite); no mask has to be
// loaded first, and values and gathers are in flight together.
__device__ inline int32_t gather_index(int32_t row, int32_t o, int32_t last)
{
    const int64_t i = (int64_t)row + o;
    return (int32_t)(i < 0 ? 0 : (i > last ? last : i));
}

// Sum of one row of a shared-offset slice: entry k multiplies x[row + o_k].
template <typename T, int U>
__device__ inline double row_shared(const int32_t* __restrict__ off, const T* __restrict__ vp, int w,
                                    int32_t row, int32_t last, const T* __restrict__ x)
{
    double acc = 0.0;
    int k = 0;
    for (; k + U <= w; k += U) {
        T vv[U], xx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u] = ld_stream(vp + (int64_t)(k + u) * kSlice);
#pragma unroll
        for (int u = 0; u < U; ++u) xx[u] = x[gather_index(row, off[k + u], last)];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = fma((double)vv[u], (double)xx[u], acc);
    }
    for (; k < w; ++k) {
        const T vv = ld_stream(vp + (int64_t)k * kSlice);
        acc = fma((double)vv, (double)x[gather_index(row, off[k], last)], acc);
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
// compile time, fully unrolled; NV = 0: runtime count).  The gather indices
// depend only on the row and the offsets, so all loads are independent
// (padding entries past the list hold zeros and gather a valid element).
template <typename T, int NV>
__device__ inline double row_uniform(const Sell<T>& A, int64_t c, int lane,
                                     const T* __restrict__ x)
{
    constexpr int V = 16 / sizeof(T);
    typedef typename Vec16<T>::type VT;
    const int64_t row = c * kSlice + lane;
    const VT* vp = reinterpret_cast<const VT*>(A.val + c * kSlice * A.uwv) + lane;
    const int nv = NV > 0 ? NV : A.uwv / V;
    double acc = 0.0;
#pragma unroll 4
    for (int j = 0; j < nv; ++j) {
        const VT v = __builtin_nontemporal_load(vp + (int64_t)j * kSlice);
#pragma unroll
        for (int h = 0; h < V; ++h) {
            const int k = j * V + h;
            acc = fma((double)v[h], (double)x[gather_index((int32_t)row, A.uo[k], A.n - 1)], acc);
        }
    }
    return acc;
}

// Row of the symmetric half storage (single values per lane in both
// precisions: stored entry t of slice row l at slice base + 64t + l).
// Entries k < H (negative offsets) are read from row r = row + o_k, stored
// entry H - k (an exact zero when r < 0; rows past the boundary otherwise
// hold the stored zero of the missing pair), entries k >= H are the row's own
// NV = H + 1 stored entries; the sum runs in list order like the full
// layout's.  These loads are cached: the value a row reads for a negative
// offset was streamed by row r shortly before.  Grouping a lane's values in
// 16-byte vectors would make every such read touch two (FP64) or four (FP32)
// times the cache lines it uses; measured at 192^3: FP32 112 us single vs
// 160 us quads, FP64 with x staged in LDS 202 us single vs 209 us pairs,
// although single values take 14 instead of 7 loads for the own entries.
// H, NV > 0: known at compile time; 0: from the matrix.
template <typename T, int H, int NV>
__device__ inline double row_uniform_half(const Sell<T>& A, int64_t c, int lane,
                                          const T* __restrict__ x)
{
    const int64_t row = c * kSlice + lane;
    const int h = H > 0 ? H : A.uw / 2;
    const int nv = NV > 0 ? NV : A.uwv;
    const int64_t sw = (int64_t)kSlice * nv;
    auto gather = [&](int k) { return (double)x[gather_index((int32_t)row, A.uo[k], A.n - 1)]; };
    double acc = 0.0;
    auto lower = [&](int k) {
        const int64_t r = row + A.uo[k];
        const int64_t rc = r < 0 ? 0 : r;
        const T v = A.val[(rc >> 6) * sw + (int64_t)(h - k) * kSlice + (rc & 63)];
        acc = fma(r < 0 ? 0.0 : (double)v, gather(k), acc);
    };
    const T* vp = A.val + c * sw + lane;
    auto upper = [&](int j) { acc = fma((double)vp[(int64_t)j * kSlice], gather(h + j), acc); };
    if constexpr (H > 0) {
#pragma unroll
        for (int k = 0; k < H; ++k) lower(k);
#pragma unroll
        for (int j = 0; j < NV; ++j) upper(j);
    } else {
        for (int k = 0; k < h; ++k) lower(k);
        for (int j = 0; j < nv; ++j) upper(j);
    }
    return acc;
}

template <typename T>
__device__ inline double uniform_row(const Sell<T>& A, int64_t c, int lane, const T* __restrict__ x)
{
    constexpr int V = 16 / sizeof(T);
    if (A.usym) {
        // (list length, stored vectors per row) of the 27-, 7- and 5-point stencils
        switch (A.uw * 32 + A.uwv) {
        case 27 * 32 + 14: return row_uniform_half<T, 13, 14>(A, c, lane, x);
        case 7 * 32 + 4: return row_uniform_half<T, 3, 4>(A, c, lane, x);
        case 5 * 32 + 3: return row_uniform_half<T, 2, 3>(A, c, lane, x);
        default: return row_uniform_half<T, 0, 0>(A, c, lane, x);
        }
    }
    switch (A.uwv / V) {
    case 2: return row_uniform<T, 2>(A, c, lane, x);     // 5-point (FP32)
    case 3: return row_uniform<T, 3>(A, c, lane, x);     // 5-point (FP64)
    case 4: return row_uniform<T, 4>(A, c, lane, x);     // 7-point (FP64)
    case 7: return row_uniform<T, 7>(A, c, lane, x);     // 27-point (FP32)
    case 14: return row_uniform<T, 14>(A, c, lane, x);   // 27-point (FP64)
    default: return row_uniform<T, 0>(A, c, lane, x);
    }
}

// ---- uniform layout with x staged in LDS (Sell::lds_n > 0)

// Copies the tile's windows of x to LDS (all threads of the workgroup; the
// caller synchronizes).  Windows start at offsets that are multiples of 4
// and have lengths that are multiples of 4, and tiles start at multiples of
// 256 rows, so every window is a run of 16-byte vectors (2 FP64 or 4 FP32
// elements), aligned in x (when x is) and in LDS: thread t moves vectors
// t and t + 256 of each window.  Windows are taken four at a time, all loads
// of a group issued before its first store (the 27-point stencil has three
// windows, one plane each).  The window index is the same for all lanes, so
// the window bounds stay scalar.  Elements outside [0, n) are staged as 0:
// the entries that would read them are stored zeros.
template <typename T>
__device__ inline void stage_x(const Sell<T>& A, int64_t a, const T* __restrict__ x,
                               T* __restrict__ sx)
{
    constexpr int V = 16 / sizeof(T);
    typedef T TV __attribute__((ext_vector_type(V)));
    constexpr int kGroup = 4;
    const int t = threadIdx.x;
    const bool x16 = reinterpret_cast<uintptr_t>(x) % 16 == 0;
    auto loadv = [&](int64_t g) {
        TV v;
        if (x16 && g >= 0 && g + V <= A.n) {
            v = *reinterpret_cast<const TV*>(x + g);
        } else {
#pragma unroll
            for (int h = 0; h < V; ++h) v[h] = (g + h >= 0 && g + h < A.n) ? x[g + h] : (T)0;
        }
        return v;
    };
    for (int j0 = 0; j0 < A.ncl; j0 += kGroup) {
        TV v[kGroup][kStageRounds];
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
#pragma unroll
            for (int r = 0; r < kStageRounds; ++r) {
                const int j = j0 + g, e = V * (t + r * kRowBlock);
                if (j < A.ncl && e < A.cl_len[j]) v[g][r] = loadv(a + A.cl_lo[j] + e);
            }
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
#pragma unroll
            for (int r = 0; r < kStageRounds; ++r) {
                const int j = j0 + g, e = V * (t + r * kRowBlock);
                if (j < A.ncl && e < A.cl_len[j])
                    *reinterpret_cast<TV*>(sx + A.cl_base[j] + e) = v[g][r];
            }
    }
}

// Full storage, x from LDS: entry k of tile row t multiplies sx[lds_k[k] + t]
// (a row without that neighbour holds a stored zero there; the stored
// padding entries point at a valid element too).
template <typename T, int NV>
__device__ inline double row_uniform_lds(const Sell<T>& A, int64_t c, int lane, int t,
                                         const T* __restrict__ sx)
{
    constexpr int V = 16 / sizeof(T);
    typedef typename Vec16<T>::type VT;
    const VT* vp = reinterpret_cast<const VT*>(A.val + c * kSlice * A.uwv) + lane;
    const int nv = NV > 0 ? NV : A.uwv / V;
    double acc = 0.0;
#pragma unroll 4
    for (int j = 0; j < nv; ++j) {
        const VT v = __builtin_nontemporal_load(vp + (int64_t)j * kSlice);
#pragma unroll
        for (int h = 0; h < V; ++h)
            acc = fma((double)v[h], (double)sx[A.lds_k[j * V + h] + t], acc);
    }
    return acc;
}

// Symmetric half storage, x from LDS (see row_uniform_half).  The row's
// first own entry is its diagonal; it is returned in dg.
template <typename T, int H, int NV>
__device__ inline double row_uniform_half_lds(const Sell<T>& A, int64_t c, int lane, int t,
                                              const T* __restrict__ sx, T& dg)
{
    const int64_t row = c * kSlice + lane;
    const int h = H > 0 ? H : A.uw / 2;
    const int nv = NV > 0 ? NV : A.uwv;
    const int64_t sw = (int64_t)kSlice * nv;
    double acc = 0.0;
    auto lower = [&](int k) {
        const int64_t r = row + A.uo[k];
        const int64_t rc = r < 0 ? 0 : r;
        const T v = A.val[(rc >> 6) * sw + (int64_t)(h - k) * kSlice + (rc & 63)];
        acc = fma(r < 0 ? 0.0 : (double)v, (double)sx[A.lds_k[k] + t], acc);
    };
    const T* vp = A.val + c * sw + lane;
    auto upper = [&](int j) {
        const T v = vp[(int64_t)j * kSlice];
        if (j == 0) dg = v;
        acc = fma((double)v, (double)sx[A.lds_k[h + j] + t], acc);
    };
    if constexpr (H > 0) {
#pragma unroll
        for (int k = 0; k < H; ++k) lower(k);
#pragma unroll
        for (int j = 0; j < NV; ++j) upper(j);
    } else {
        for (int k = 0; k < h; ++k) lower(k);
        for (int j = 0; j < nv; ++j) upper(j);
    }
    return acc;
}

// (A x)_row from LDS-staged x.  dg receives the row's diagonal value with
// the symmetric half storage and is left untouched otherwise.
template <typename T>
__device__ inline double uniform_row_lds(const Sell<T>& A, int64_t c, int lane, int t,
                                         const T* __restrict__ sx, T& dg)
{
    constexpr int V = 16 / sizeof(T);
    if (A.usym) {
        switch (A.uw * 32 + A.uwv) {
        case 27 * 32 + 14: return row_uniform_half_lds<T, 13, 14>(A, c, lane, t, sx, dg);
        case 7 * 32 + 4: return row_uniform_half_lds<T, 3, 4>(A, c, lane, t, sx, dg);
        case 5 * 32 + 3: return row_uniform_half_lds<T, 2, 3>(A, c, lane, t, sx, dg);
        default: return row_uniform_half_lds<T, 0, 0>(A, c, lane, t, sx, dg);
        }
    }
    switch (A.uwv / V) {
    case 2: return row_uniform_lds<T, 2>(A, c, lane, t, sx);
    case 3: return row_uniform_lds<T, 3>(A, c, lane, t, sx);
    case 4: return row_uniform_lds<T, 4>(A, c, lane, t, sx);
    case 7: return row_uniform_lds<T, 7>(A, c, lane, t, sx);
    case 14: return row_uniform_lds<T, 14>(A, c, lane, t, sx);
    default: return row_uniform_lds<T, 0>(A, c, lane, t, sx);
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
    if (aux < 0)
        return row_shared<T, kUnroll>(A.soff + (-aux - 1), A.val + base + lane, w, (int32_t)row,
                                      A.n - 1, x);
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
    const int64_t tile = xcd_block_tile();
    const int64_t c = tile * kSlicesPerTile + wave;
    double acc;
    T xself = (T)0;   // x[row] for the epilogue
    T dg = (T)0;      // the row's diagonal value, if the row function returns it
    bool staged = false;
    if constexpr (sizeof(T) == 8) staged = A.lds_n > 0;   // FP32 views never stage
    if (staged) {
        extern __shared__ __attribute__((aligned(16))) double lds_dyn[];
        T* sx = reinterpret_cast<T*>(lds_dyn);
        stage_x<T>(A, tile * kRowBlock, x, sx);
        __syncthreads();
        if (c >= A.nslices) return;
        acc = uniform_row_lds<T>(A, c, lane, (int)threadIdx.x, sx, dg);
        if (MODE >= 1) xself = sx[A.lds_self + threadIdx.x];   // staged with offset 0
    } else {
        if (c >= A.nslices) return;
        acc = slice_row<T>(A, c, lane, x);
    }
    const int64_t row = c * kSlice + lane;
    if (row < A.n) {
        const T p = (T)acc;
        // y (a column of AZ) is next read by the Gram kernels, long after
        // it has left the caches, and z_{q-1} is dead after this step: both
        // bypass cache allocation; z_{q+1} is read again by the next launch
        __builtin_nontemporal_store(p, y + row);
        if (MODE >= 1) {
            if (!staged) xself = x[row];
            // with the half storage the diagonal came with the row's values:
            // its reciprocal (correctly rounded, as when dinv was formed)
            // equals dinv[row] bit for bit and saves reading dinv
            const double di = (staged && A.usym) ? 1.0 / (double)dg : (double)A.dinv[row];
            const double t1 = di * (double)p;
            double z = c1 * t1 - c2 * (double)xself;
            if (MODE == 2) z -= c3 * (double)__builtin_nontemporal_load(zprev + row);
            znext[row] = (T)z;
        }
    }
}

// STAGED: the uniform layout with x staged in LDS (A.lds_n > 0), the only
// row code the kernel then holds, so the persistent loop keeps few registers.
template <typename TR, bool STAGED>
__global__ __launch_bounds__(kRowBlock) void k_residual(Sell<double> A, const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        TR* __restrict__ r, TR* __restrict__ z1,
                                                        const TR* __restrict__ dinvT,
                                                        double* __restrict__ partials)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr int kSlicesPerTile = kRowBlock / kSlice;
    const int64_t ntiles = (A.nslices + kSlicesPerTile - 1) / kSlicesPerTile;
    const int VB = virtual_blocks(ntiles);
    for (int v = blockIdx.x; v < VB; v += gridDim.x) {
        const TileRange tr = vblock_tiles(ntiles, VB, v);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        extern __shared__ __attribute__((aligned(16))) double lds_dyn[];
        for (int64_t t = tr.first; t < tr.end; t += tr.step) {
            const int64_t c = t * kSlicesPerTile + wave;
            double ax = 0.0;
            if constexpr (STAGED) {
                // every wave of the workgroup reaches both barriers of every tile
                __syncthreads();
                stage_x<double>(A, t * kRowBlock, x, lds_dyn);
                __syncthreads();
                if (c >= A.nslices) continue;
                double dg;
                ax = uniform_row_lds<double>(A, c, lane, (int)threadIdx.x, lds_dyn, dg);
            } else {
                if (c >= A.nslices) break;
                ax = slice_row<double>(A, c, lane, x);
            }
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
        block_partials<4, kRowBlock>(acc, partials, v, VB);
    }
}

template <bool STAGED>
__global__ __launch_bounds__(kRowBlock) void k_pcg_spmv(Sell<double> A, const double* __restrict__ p,
                                                        double* __restrict__ q,
                                                        double* __restrict__ partials,
                                                        const Ctrl* __restrict__ ctrl)
{
    if (ctrl->done) return;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr int kSlicesPerTile = kRowBlock / kSlice;
    const int64_t ntiles = (A.nslices + kSlicesPerTile - 1) / kSlicesPerTile;
    // classical PCG keeps one partial per workgroup: its iteration count
    // does not hinge on rounding the way two FGS sweeps do, and the loop over
    // virtual blocks costs its SpMV registers (127 -> 156) and 10 % of time
    const TileRange tr = xcd_tiles(ntiles);
    double acc[1] = {0.0};
    extern __shared__ __attribute__((aligned(16))) double lds_dyn[];
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t c = t * kSlicesPerTile + wave;
        double ap = 0.0, prow = 0.0;
        if constexpr (STAGED) {
            // every wave of the workgroup reaches both barriers of every tile
            __syncthreads();
            stage_x<double>(A, t * kRowBlock, p, lds_dyn);
            __syncthreads();
            if (c >= A.nslices) continue;
            double dg;
            ap = uniform_row_lds<double>(A, c, lane, (int)threadIdx.x, lds_dyn, dg);
            prow = lds_dyn[A.lds_self + threadIdx.x];   // p[row], staged with offset 0
        } else {
            if (c >= A.nslices) break;
            ap = slice_row<double>(A, c, lane, p);
        }
        const int64_t row = c * kSlice + lane;
        if (row < A.n) {
            if constexpr (!STAGED) prow = p[row];
            q[row] = ap;
            acc[0] = fma(prow, ap, acc[0]);
        }
    }
    block_partials<1, kRowBlock>(acc, partials, blockIdx.x, gridDim.x);
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
    block_partials<2, kRowBlock>(acc, partials, blockIdx.x, gridDim.x);
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
    // initialised once, thread-safe (solves may run from several host threads)
    static const int cus = [] {
        int dev = 0, n = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            n = prop.multiProcessorCount;
        return n > 0 ? n : 256;
    }();
    return cus;
}

int resident_blocks(const void* kernel, int threads, size_t dyn_lds)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, size_t>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(kernel, dyn_lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, dyn_lds) != hipSuccess ||
        nb < 1)
        nb = 1;
    cache.emplace(key, nb);
    return nb;
}

void plan_lds(sspcg_matrix* A)
{
    A->lds_n = A->ncl = 0;
    if (!A->uniform || A->uw < 1) return;
    const int32_t* o = A->uoff_host;
    for (int k = 1; k < A->uw; ++k)
        if (o[k] <= o[k - 1]) return;   // the list is ascending by construction
    // runs of consecutive offsets, merged while the next starts at most one
    // tile after the current window's last offset: one window then costs no
    // more LDS and fewer loads than two (the 27-point stencil's three runs
    // of a plane, N apart, share one window when N <= 256)
    // (a merge that would make a window longer than the copy covers starts a
    // new window instead)
    constexpr int kMaxLen = 2 * kStageRounds * kRowBlock;
    auto span = [](int l, int h) { return ((h + kRowBlock - (l & ~3)) + 3) & ~3; };
    int lo[kMaxUnion], hi[kMaxUnion], win[kMaxUnion];
    int nw = 0;
    for (int k = 0; k < A->uw; ++k) {
        if (nw == 0 || o[k] - hi[nw - 1] > kRowBlock || span(lo[nw - 1], o[k]) > kMaxLen) {
            lo[nw] = hi[nw] = o[k];
            ++nw;
        } else {
            hi[nw - 1] = o[k];
        }
        win[k] = nw - 1;
    }
    if (nw > kMaxWindows) return;   // too many windows: gathers from memory
    int base = 0;
    for (int j = 0; j < nw; ++j) {
        // multiples of 4: windows are copied as aligned 16-byte vectors
        const int l = lo[j] & ~3;
        const int len = span(lo[j], hi[j]);
        if (len > kMaxLen) return;   // one run longer than the FP64 copy covers
        A->cl_lo[j] = l;
        A->cl_len[j] = len;
        A->cl_base[j] = base;
        base += len;
    }
    if (base > kMaxStaged) return;
    A->lds_self = -1;
    for (int k = 0; k < A->uw; ++k) {
        A->lds_k[k] = A->cl_base[win[k]] + (o[k] - A->cl_lo[win[k]]);
        // the element x[row] itself, for the epilogue of the matrix powers kernel
        if (o[k] == 0) A->lds_self = A->lds_k[k];
    }
    for (int k = A->uw; k < kMaxUnion; ++k) A->lds_k[k] = A->lds_k[A->uw - 1];
    if (A->lds_self < 0) return;   // no diagonal offset (cannot happen: the diagonal is stored)
    A->ncl = nw;
    A->lds_n = base;
}

// SSPCG_GRID_BLOCKS_PER_CU=k in the environment (read once per process)
// caps every persistent grid at k workgroups per CU: a debugging aid that
// shows the s-step results do not depend on the grid (virtual blocks).
static int grid_cap_from_env()
{
    static const int cap = [] {
        const char* v = std::getenv("SSPCG_GRID_BLOCKS_PER_CU");
        const int k = v ? std::atoi(v) : 0;
        return k > 0 ? k : 1 << 20;
    }();
    return cap;
}

int persistent_grid(int64_t ntiles, int blocks_per_cu, int resident)
{
    blocks_per_cu = std::min(blocks_per_cu, grid_cap_from_env());
    int64_t g = (int64_t)num_cus() * std::min(blocks_per_cu, resident);
    g = std::min<int64_t>(g, kMaxGrid);
    g = std::min<int64_t>(g, std::max<int64_t>(ntiles, 1));
    if (g >= kNumXcd) g -= g % kNumXcd;
    return (int)std::max<int64_t>(g, 1);
}

template <typename T>
Sell<T> sell_view(const sspcg_matrix* A);

// Stored entries per row of the uniform layout (one triangle plus the
// diagonal with the symmetric half storage).
static int uniform_stored(const sspcg_matrix* A) { return A->uw - (A->usym ? A->uw / 2 : 0); }

template <typename T>
static Sell<T> make_view(const sspcg_matrix* A, int uwv, const T* val, const T* dinv)
{
    Sell<T> S;
    S.n = A->n;
    S.uniform = A->uniform;
    S.uw = A->uw;
    S.uwv = uwv;
    S.usym = A->usym;
    std::copy(A->uoff_host, A->uoff_host + kMaxUnion, S.uo);
    // LDS staging pays in FP64, where the gathers keep the address units
    // busy; FP32 gathers move half the bytes and are faster straight from
    // memory (124 vs 181 us at 192^3, 27 points)
    S.lds_n = sizeof(T) == 8 ? A->lds_n : 0;
    S.ncl = A->ncl;
    S.lds_self = A->lds_self;
    std::copy(A->cl_lo, A->cl_lo + kMaxWindows, S.cl_lo);
    std::copy(A->cl_len, A->cl_len + kMaxWindows, S.cl_len);
    std::copy(A->cl_base, A->cl_base + kMaxWindows, S.cl_base);
    std::copy(A->lds_k, A->lds_k + kMaxUnion, S.lds_k);
    S.nslices = A->nslices;
    S.slice_ptr = A->slice_ptr;
    S.slice_aux = A->slice_aux;
    S.col = A->scol;
    S.soff = A->soff;
    S.val = val;
    S.dinv = dinv;
    return S;
}

template <>
Sell<double> sell_view<double>(const sspcg_matrix* A)
{
    return make_view<double>(A, A->usym ? uniform_stored(A) : (uniform_stored(A) + 1) / 2 * 2,
                             A->sval, A->dinv);
}

template <>
Sell<float> sell_view<float>(const sspcg_matrix* A)
{
    const int stored = uniform_stored(A);
    return make_view<float>(A, A->usym ? stored : (stored + 3) / 4 * 4, A->sval32, A->dinv32);
}

static int64_t spmv_tiles(const sspcg_matrix* A)
{
    return (A->nslices + kRowBlock / kSlice - 1) / (kRowBlock / kSlice);
}

// Persistent grid for the SpMV kernels that also reduce: all workgroups
// resident at once.
template <typename K>
static int spmv_persistent_grid(const sspcg_matrix* A, K kernel, size_t dyn_lds)
{
    const int resident = resident_blocks(reinterpret_cast<const void*>(kernel), kRowBlock, dyn_lds);
    return persistent_grid(spmv_tiles(A), 8, resident);
}

// A reduction's grid never exceeds its virtual blocks (common.h).
template <typename K>
static int spmv_reduce_grid(const sspcg_matrix* A, K kernel, size_t dyn_lds)
{
    return std::min(spmv_persistent_grid(A, kernel, dyn_lds), virtual_blocks(spmv_tiles(A)));
}

// Dynamic LDS of the SpMV kernels: the staged windows of x.
template <typename T>
static size_t lds_bytes(const sspcg_matrix* A) { return sizeof(T) * (size_t)sell_view<T>(A).lds_n; }

int matrix_check_symmetric(const sspcg_matrix* A, const double* val, bool* sym, hipStream_t st)
{
    const int blocks = (int)((A->n + kRowBlock - 1) / kRowBlock);
    SSPCG_HIP(hipMemsetAsync(A->dflags, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_check_symmetric, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->row_ptr,
                       A->col, val, A->dflags);
    SSPCG_LAUNCHED("k_check_symmetric");
    int32_t h = 1;
    SSPCG_HIP(hipMemcpyAsync(&h, A->dflags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipStreamSynchronize(st));
    *sym = h == 0;
    return SSPCG_OK;
}

static size_t area_align(size_t v) { return (v + 255) / 256 * 256; }

size_t analysis_bytes(int64_t n)
{
    const int64_t nslices = (n + kSlice - 1) / kSlice;
    return 256 + 2 * area_align(sizeof(int32_t) * (size_t)nslices) +
           area_align(sizeof(int32_t) * (size_t)nslices * kMaxUnion);
}

void bind_analysis(sspcg_matrix* A, void* base)
{
    char* p = static_cast<char*>(base);
    const size_t per = area_align(sizeof(int32_t) * (size_t)A->nslices);
    A->dflags = reinterpret_cast<int32_t*>(p);
    A->a_width = reinterpret_cast<int32_t*>(p + 256);
    A->a_ulen = reinterpret_cast<int32_t*>(p + 256 + per);
    A->a_union = reinterpret_cast<int32_t*>(p + 256 + 2 * per);
}

int matrix_inspect(sspcg_matrix* A, const double* val, bool values_only, LayoutPlan* plan,
                   hipStream_t st, bool write_dinv, bool allow_sym)
{
    const int64_t nrows_padded = A->nslices * kSlice;
    const int blocks = (int)((nrows_padded + kRowBlock - 1) / kRowBlock);
    std::vector<int32_t> width(A->nslices), ulen(A->nslices);
    SSPCG_HIP(hipMemsetAsync(A->dflags, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_inspect, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nnz, A->nslices,
                       A->row_ptr, A->col, val, A->dflags, A->a_width,
                       write_dinv ? A->dinv : nullptr, write_dinv ? A->dinv32 : nullptr,
                       values_only);
    SSPCG_LAUNCHED("k_inspect");
    int32_t hflags = 0;
    SSPCG_HIP(hipMemcpyAsync(&hflags, A->dflags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipMemcpyAsync(width.data(), A->a_width, sizeof(int32_t) * A->nslices,
                             hipMemcpyDeviceToHost, st));
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
    hipLaunchKernelGGL(k_slice_union, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nslices,
                       A->row_ptr, A->col, A->a_union, A->a_ulen);
    SSPCG_LAUNCHED("k_slice_union");
    SSPCG_HIP(hipMemcpyAsync(ulen.data(), A->a_ulen, sizeof(int32_t) * A->nslices,
                             hipMemcpyDeviceToHost, st));
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
    // has at most 32 offsets and costs at most 2 % more stored entries than the
    // per-slice lists -- or A is symmetric and one triangle of the union
    // needs fewer entries than the per-slice lists
    plan->uoff.clear();
    plan->usym = false;
    if (plan->nshared == A->nslices) {
        std::vector<int32_t> hun((size_t)A->nslices * kMaxUnion);
        SSPCG_HIP(hipMemcpyAsync(hun.data(), A->a_union, sizeof(int32_t) * hun.size(),
                                 hipMemcpyDeviceToHost, st));
        SSPCG_HIP(hipStreamSynchronize(st));
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
        if (fits && !all.empty()) {
            std::sort(all.begin(), all.end());
            const int uw = (int)all.size();
            const double rows = (double)A->nslices * kSlice;
            // symmetric half storage: a list o_k = -o_{uw-1-k} and A = A^T
            bool mirrored = uw % 2 == 1;
            for (int k = 0; k < uw && mirrored; ++k) mirrored = all[k] == -all[uw - 1 - k];
            const int half = uw - uw / 2;   // stored entries per row
            if (allow_sym && mirrored && rows * half <= (double)plan->slots) {
                bool sym = false;
                const int rc = matrix_check_symmetric(A, val, &sym, st);
                if (rc != SSPCG_OK) return rc;
                plan->usym = sym;
            }
            if (plan->usym || rows * uw <= 1.02 * (double)plan->slots) plan->uoff = all;
        }
    }
    return SSPCG_OK;
}

int matrix_pack(sspcg_matrix* A, hipStream_t st)
{
    const int blocks = (int)((A->nslices * kSlice + kRowBlock - 1) / kRowBlock);
    hipLaunchKernelGGL(k_pack_union, dim3(blocks), dim3(kRowBlock), 0, st, A->nslices,
                       A->slice_ptr, A->slice_aux, A->a_union, A->soff);
    SSPCG_LAUNCHED("k_pack_union");
    return SSPCG_OK;
}

int matrix_fill(sspcg_matrix* A, const double* val, bool values_only, hipStream_t st)
{
    const int64_t nrows_padded = A->nslices * kSlice;
    const int blocks = (int)((nrows_padded + kRowBlock - 1) / kRowBlock);
    if (A->uniform) {
        const int stored = uniform_stored(A);
        hipLaunchKernelGGL(k_fill_uniform, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nslices,
                           A->row_ptr, A->col, val, A->uoff, A->uw, A->uw - stored,
                           sell_view<double>(A).uwv, A->usym ? 1 : 2, sell_view<float>(A).uwv,
                           A->usym ? 1 : 4, A->sval,
                           A->sval32);
        SSPCG_LAUNCHED("k_fill_uniform");
        SSPCG_HIP(hipStreamSynchronize(st));
        return SSPCG_OK;
    }
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kRowBlock), 0, st, A->n, A->nslices, A->row_ptr,
                       A->col, val, A->slice_ptr, A->slice_aux, A->soff, A->scol, A->sval,
                       A->sval32, values_only);
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
    const size_t lds = lds_bytes<T>(A);
    if (mode == 0)
        hipLaunchKernelGGL((k_spmv<T, 0>), dim3(G), dim3(kRowBlock), lds, st, S, x, y, zprev,
                           znext, c1, c2, c3, ctrl);
    else if (mode == 1)
        hipLaunchKernelGGL((k_spmv<T, 1>), dim3(G), dim3(kRowBlock), lds, st, S, x, y, zprev,
                           znext, c1, c2, c3, ctrl);
    else
        hipLaunchKernelGGL((k_spmv<T, 2>), dim3(G), dim3(kRowBlock), lds, st, S, x, y, zprev,
                           znext, c1, c2, c3, ctrl);
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
    const size_t lds = lds_bytes<double>(A);
    int G;
    if (S.lds_n > 0) {
        G = spmv_reduce_grid(A, k_residual<TR, true>, lds);
        hipLaunchKernelGGL((k_residual<TR, true>), dim3(G), dim3(kRowBlock), lds, st, S, x, b, r,
                           z1, dinvT, partials);
    } else {
        G = spmv_reduce_grid(A, k_residual<TR, false>, lds);
        hipLaunchKernelGGL((k_residual<TR, false>), dim3(G), dim3(kRowBlock), lds, st, S, x, b, r,
                           z1, dinvT, partials);
    }
    SSPCG_LAUNCHED("k_residual");
    *G_out = virtual_blocks(spmv_tiles(A));
    return SSPCG_OK;
}

template int launch_residual<double>(const sspcg_matrix*, const double*, const double*, double*,
                                     double*, double*, int*, hipStream_t);
template int launch_residual<float>(const sspcg_matrix*, const double*, const double*, float*,
                                    float*, double*, int*, hipStream_t);

int launch_pcg_spmv(const sspcg_matrix* A, const double* p, double* q, double* partials,
                    int* G_out, const Ctrl* ctrl, hipStream_t st)
{
    const Sell<double> S = sell_view<double>(A);
    const size_t lds = lds_bytes<double>(A);
    int G;
    if (S.lds_n > 0) {
        G = spmv_persistent_grid(A, k_pcg_spmv<true>, lds);
        hipLaunchKernelGGL((k_pcg_spmv<true>), dim3(G), dim3(kRowBlock), lds, st, S, p, q, partials,
                           ctrl);
    } else {
        G = spmv_persistent_grid(A, k_pcg_spmv<false>, lds);
        hipLaunchKernelGGL((k_pcg_spmv<false>), dim3(G), dim3(kRowBlock), lds, st, S, p, q,
                           partials, ctrl);
    }
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
