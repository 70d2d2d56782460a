// Internal declarations shared by the HIP sources of libsspcg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "sspcg.h"

namespace sspcg {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kSlice = 64;         // rows per slice of the sliced layout (one per lane)
constexpr int kRowBlock = 256;     // threads of the row-parallel kernels
constexpr int kFinBlock = 1024;    // threads of the single-block finishing kernels
constexpr int kNumXcd = 8;         // accelerator complex dies of an MI355X
constexpr int kMaxGrid = 4096;     // upper bound on blocks of persistent kernels
constexpr int kMaxPartials = SSPCG_MAX_S * SSPCG_MAX_S + SSPCG_MAX_S;  // values per block
// Doubles per outer iteration in the device history of the s-step solve:
// relres, eta_alpha, eta_beta, conjugacy defect ||B2 - W beta||_F.
constexpr int kHistStride = 4;

// Device-side control block of a running solve.  Kernels of the outer loop
// read `done` on entry and return at once when it is set, so the host can
// enqueue iterations ahead of the convergence test.
struct Ctrl {
    int32_t done;       // 1 once the solve has ended
    int32_t status;     // sspcg_status when done
    int32_t iter;       // x updates taken
    int32_t max_iter;   // limit on x updates
    double nb;          // reference norm of the relative residual
    double tol;         // stop when ||r|| <= tol * nb
    double relres;      // last relative residual
    double rho[2];      // classical PCG: r^T z, double-buffered by iteration parity
    double sums[4];     // results of the setup reductions
    int32_t x_pending;  // 1 while x still lacks Q alpha of the last r update
    int32_t pad_i;
    double pad[4];
};
static_assert(sizeof(Ctrl) == 128, "Ctrl layout");

// Sliced layout of a CSR matrix: slice c holds rows 64c..64c+63, one per
// lane; entry k of lane l sits at slot slice_ptr[c] + 64k + l.  Two kinds of
// slice:
//  - shared offsets (slice_aux[c] < 0): the slice's rows draw their columns
//    from one sorted list of at most 32 offsets o_k = col - row, stored once
//    at soff[-slice_aux[c] - 1 + k]; entry k of a row is its value at column
//    row + o_k, or 0 where the row has no such entry (its gather then reads
//    any element of x: an exact zero term for finite x).  This is the case
//    for stencil matrices and removes the column indices from the stream.
//  - explicit columns (slice_aux[c] >= 0): entry k holds the row's k-th
//    stored entry, its column at col[slice_aux[c] + 64k + l]; rows are padded
//    to the slice's longest row with value 0 and the row as column.
// Either way the entries of a row keep the CSR order.
//
// Uniform layout (uniform != 0): when the offsets of all slices fit one
// global sorted list of at most 32 (structured-grid stencils), every row is
// stored against that list, no per-slice data is needed and a lane's
// entries are grouped in 16-byte vectors (2 FP64 or 4 FP32 values): stored
// entry t of lane l of slice c sits at c*64*uwv + (t/V)*64*V + l*V + t%V,
// V = 16 / sizeof(T), uwv = the stored entries per row rounded up to a
// multiple of V.
// Symmetric half storage (usym != 0): when A is symmetric, bit for bit, and
// its list is o_k = -o_{uw-1-k} (uw odd, o_{uw/2} = 0), only the entries
// k >= h = uw/2 are stored, as t = k - h.  Entry k < h of row i is then
// entry t = h - k of row i + o_k (zero when that row is below 0), which
// halves the value stream.  Both precisions store single values (V = 1),
// so uwv is the stored count itself.
template <typename T>
struct Sell {
    int32_t n;
    int32_t uniform;
    int32_t uw, uwv;            // uniform: offsets in the list, stored entries per row
    int32_t usym;               // uniform: symmetric half storage
    int32_t uo[32];             // uniform: the global offset list, in the kernel arguments
    // LDS staging of x (uniform layout): the gathers x[row + o_k] of a
    // 256-row tile starting at row a fall into windows of x, one per run of
    // consecutive offsets (o, o+1, ...), runs less than a tile apart sharing
    // one: window j is x[a + cl_lo[j] .. a + cl_lo[j] + cl_len[j]), cl_lo[j]
    // its first offset rounded down to a multiple of 4, cl_len[j] (a multiple
    // of 4) >= 256 + the span of its offsets, stored at sx[cl_base[j] ..).
    // Each workgroup copies its windows to LDS with contiguous loads, then
    // reads entry k of tile row t at sx[lds_k[k] + t].  lds_n = 0: gathers
    // from memory (more than kMaxWindows windows, a window longer than the
    // copy covers, or the layout is not uniform).
    int32_t lds_n;              // staged elements per tile (the sum of cl_len)
    int32_t ncl;                // windows
    int32_t lds_self;           // LDS index of x[row] for tile row 0 (the offset 0)
    int32_t cl_lo[12];          // window j: first offset,
    int32_t cl_len[12];         //   length,
    int32_t cl_base[12];        //   first LDS element (all multiples of 4)
    int32_t lds_k[32];          // LDS index of entry k for tile row 0 (stored pads: any window)
    int64_t nslices;
    const int64_t* slice_ptr;   // nslices + 1 slot offsets, multiples of 64
    const int64_t* slice_aux;   // kind and offset of each slice, see above
    const int32_t* col;         // explicit column indices
    const int32_t* soff;        // shared offset lists
    const T* val;
    const T* dinv;              // 1 / diag(A)
};

// Longest shared offset list a slice may use (the offsets travel in kernel
// arguments for the uniform layout).
constexpr int kMaxUnion = 32;
constexpr int kMaxWindows = 12;    // LDS windows of x per tile at most
constexpr int kStageRounds = 2;    // 16-byte vectors each thread copies per window at most
constexpr int kMaxStaged = 4096;   // staged elements per tile at most (32 KB in FP64)
static_assert(sizeof(Sell<double>::uo) == kMaxUnion * sizeof(int32_t), "offset list size");
static_assert(sizeof(Sell<double>::cl_lo) == kMaxWindows * sizeof(int32_t), "window list size");

// Grid of a persistent row kernel: at most `blocks_per_cu` workgroups per CU
// and never more than fit at once (`resident`, from the occupancy of the
// kernel), so no workgroup waits for another to finish its tile list; a
// multiple of kNumXcd blocks.
int persistent_grid(int64_t ntiles, int blocks_per_cu, int resident = 1 << 20);
int num_cus();
// Workgroups of `kernel` (256 threads, dyn_lds bytes of dynamic LDS) that
// fit on one CU at once.
int resident_blocks(const void* kernel, int threads, size_t dyn_lds = 0);

// Error plumbing for the C ABI.
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define SSPCG_HIP(call)                                        \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ::sspcg::hip_fail(e_, #call); \
    } while (0)
// SSPCG_DEBUG_SYNC=1 in the environment: synchronize and check after every
// launch, so an asynchronous failure is reported by the launch that caused it.
bool debug_sync();
#define SSPCG_LAUNCHED(what)                                   \
    do {                                                       \
        hipError_t e_ = hipGetLastError();                     \
        if (e_ == hipSuccess && ::sspcg::debug_sync())         \
            e_ = hipDeviceSynchronize();                       \
        if (e_ != hipSuccess) return ::sspcg::hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------------ device

// Workgroups are dispatched to the dies round-robin (block b runs on die
// b % 8), and each die has its own L2.  Give every die a contiguous range of
// tiles so that the neighbours a stencil row gathers stay in that die's L2.
struct TileRange {
    int64_t first, end, step;
};

__device__ inline TileRange xcd_tiles(int64_t ntiles)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (G >= kNumXcd && G % kNumXcd == 0) {
        const int x = b % kNumXcd, j = b / kNumXcd, per = G / kNumXcd;
        const int64_t lo = ntiles * x / kNumXcd, hi = ntiles * (x + 1) / kNumXcd;
        return {lo + j, hi, per};
    }
    return {b, ntiles, G};
}

// Reductions group their rows by "virtual blocks": VB(ntiles) groups of
// tiles, a number that depends on the problem size only.  The workgroups of
// a launch -- as many as fit, which depends on the kernel's register use --
// walk the virtual blocks (workgroup b takes b, b + G, ...), and every
// virtual block writes its own partial sums, so the sums and their rounding
// do not depend on the grid: a change of occupancy or of compiler leaves the
// results, and the iterations built on them, the same bit for bit.  Virtual
// block v takes the tiles xcd_tiles would give workgroup v of a grid of VB,
// so with G a multiple of 8 every workgroup stays on the die of its tiles.
// 512 at most: at 192^3 the s-step iteration took 2.024 ms with 512, 2.027
// with 1024 and 2.044 with 2048 (each virtual block ends in a block-wide
// reduction, and the single-workgroup finish sums VB values); contiguous
// chunks per virtual block instead of strided tiles made the block update
// 20-40 % slower.
constexpr int kVirtualBlocks = 512;

__host__ __device__ inline int virtual_blocks(int64_t ntiles)
{
    const int64_t v = ntiles < kVirtualBlocks ? ntiles : kVirtualBlocks;
    if (v >= kNumXcd) return (int)(v - v % kNumXcd);
    return (int)(v > 0 ? v : 1);
}

__device__ inline TileRange vblock_tiles(int64_t ntiles, int VB, int v)
{
    if (VB >= kNumXcd && VB % kNumXcd == 0) {
        const int x = v % kNumXcd, j = v / kNumXcd, per = VB / kNumXcd;
        const int64_t lo = ntiles * x / kNumXcd, hi = ntiles * (x + 1) / kNumXcd;
        return {lo + j, hi, per};
    }
    return {v, ntiles, VB};
}

// Tile of a non-persistent launch (one tile per workgroup, grid = ntiles):
// the first 8*floor(ntiles/8) tiles are split into 8 contiguous ranges, one
// per die, walked in dispatch order; the remaining tiles map to themselves.
__device__ inline int64_t xcd_block_tile()
{
    const int64_t b = blockIdx.x, G = gridDim.x;
    const int64_t full = G / kNumXcd * kNumXcd;
    if (b >= full) return b;
    return (b % kNumXcd) * (full / kNumXcd) + b / kNumXcd;
}

template <int K>
__device__ inline void zero_acc(double (&a)[K])
{
#pragma unroll
    for (int e = 0; e < K; ++e) a[e] = 0.0;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Reduces K per-thread accumulators over the block in a fixed order and
// writes the partial sums of virtual block v to partials[k * VB + v].  Every
// thread of the block must call it; it may be called again for the next
// virtual block (the trailing barrier frees the shared staging).
template <int K, int NT>
__device__ inline void block_partials(double (&acc)[K], double* __restrict__ partials, int v,
                                      int VB)
{
    __shared__ double sm[NT / kWave][K > 0 ? K : 1];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) sm[wave][k] = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += NT) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / kWave; ++w) s += sm[w][k];
        partials[(int64_t)k * VB + v] = s;
    }
    __syncthreads();
}

// Sum of partials[e * G + 0 .. G-1] by one wavefront in a fixed order.
// Unrolled so that a lane's loads are in flight together; each lane still
// adds its values in order, so the result does not depend on the unrolling.
__device__ inline double wave_finish(const double* __restrict__ partials, int e, int G)
{
    const int lane = threadIdx.x & (kWave - 1);
    double s = 0.0;
#pragma unroll 8
    for (int g = lane; g < G; g += kWave) s += partials[(int64_t)e * G + g];
    return wave_sum(s);
}

}  // namespace sspcg
