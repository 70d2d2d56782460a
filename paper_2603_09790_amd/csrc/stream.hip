// STREAM-style triad a = b + q c in FP64: the achievable HBM bandwidth that
// the byte rates of the solver's kernels are compared with (the published
// 8 TB/s peak is not reached by any access pattern).  Not part of the method.
//
// Each thread moves 16-byte vectors with non-temporal loads and stores (the
// arrays are far larger than the caches, as the solver's blocks are), one
// vector of each operand per loop trip, in a grid of two workgroups per CU
// that walk contiguous per-die ranges of 256-vector tiles.  That shape was
// the fastest of a sweep over 1, 2, 4 and 8 vectors per trip and 1, 2, 3, 4
// and 8 workgroups per CU (1 GiB arrays, two devices): 5.9-6.1 TB/s, against
// 5.1-5.2 TB/s with four vectors per trip and eight workgroups per CU --
// more bytes in flight per CU made the triad slower, not faster.

#include "launch.h"

namespace sspcg {

namespace {

constexpr int kTriadUnroll = 1;
constexpr int kTriadBlocksPerCu = 2;
typedef double d2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kRowBlock) void k_triad(int64_t nv, const d2* __restrict__ b,
                                                     const d2* __restrict__ c, double q,
                                                     d2* __restrict__ a)
{
    // tile = kTriadUnroll * kRowBlock vectors; thread t takes t, t + 256, ...
    constexpr int64_t kTile = (int64_t)kTriadUnroll * kRowBlock;
    const int64_t ntiles = (nv + kTile - 1) / kTile;
    const TileRange tr = xcd_tiles(ntiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t base = t * kTile + threadIdx.x;
        d2 bv[kTriadUnroll], cv[kTriadUnroll];
#pragma unroll
        for (int u = 0; u < kTriadUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kRowBlock;
            if (i < nv) {
                bv[u] = __builtin_nontemporal_load(b + i);
                cv[u] = __builtin_nontemporal_load(c + i);
            }
        }
#pragma unroll
        for (int u = 0; u < kTriadUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kRowBlock;
            if (i < nv) {
                d2 r;
                r.x = fma(q, cv[u].x, bv[u].x);
                r.y = fma(q, cv[u].y, bv[u].y);
                __builtin_nontemporal_store(r, a + i);
            }
        }
    }
}

// The odd last element when n is odd.
__global__ void k_triad_tail(int64_t i, const double* b, const double* c, double q, double* a)
{
    a[i] = fma(q, c[i], b[i]);
}

}  // namespace

int launch_triad(int64_t n, const double* b, const double* c, double q, double* a,
                 hipStream_t st)
{
    const int64_t nv = n / 2;
    if (nv > 0) {
        const int64_t ntiles = (nv + (int64_t)kTriadUnroll * kRowBlock - 1)
                               / ((int64_t)kTriadUnroll * kRowBlock);
        const int G = persistent_grid(ntiles, kTriadBlocksPerCu,
                                      resident_blocks((const void*)k_triad, kRowBlock));
        hipLaunchKernelGGL(k_triad, dim3(G), dim3(kRowBlock), 0, st, nv,
                           reinterpret_cast<const d2*>(b), reinterpret_cast<const d2*>(c), q,
                           reinterpret_cast<d2*>(a));
        SSPCG_HIP(hipGetLastError());
    }
    if (n % 2) {
        hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(1), 0, st, n - 1, b, c, q, a);
        SSPCG_HIP(hipGetLastError());
    }
    return SSPCG_OK;
}

}  // namespace sspcg
