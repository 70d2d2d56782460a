// C ABI of libsspcg: argument checking, workspace layout and the drivers of
// the s-step PCG solve (Algorithm 1 with Algorithm 2 and FGS Gram solves),
// its mixed-precision refinement form and classical Jacobi PCG.
//
// Control flow.  The host enqueues whole outer iterations without waiting:
// the stop test runs on the device (k_norm_step), which sets Ctrl::done, and
// every later kernel of the loop returns at once when it sees the flag.  The
// host enqueues `check_every` iterations per batch, copies Ctrl to pinned
// memory behind each batch, and reads the copy of the previous batch while
// the current one runs, so the GPU never idles on a host round trip.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"

namespace sspcg {

// Device memory of sspcg_solve_static: one file-scope array that every GPU
// the library runs on holds until the process ends.  In host code this name
// is a host-side stand-in, not a device address: host code only ever uses the
// address hipGetSymbolAddress returns for it on each device (static_state).
__device__ __align__(256) unsigned char scratch[SSPCG_STATIC_SCRATCH_BYTES];

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

int hip_fail(hipError_t e, const char* what)
{
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return SSPCG_ERR_HIP;
}

bool debug_sync()
{
    static const bool on = [] {
        const char* v = std::getenv("SSPCG_DEBUG_SYNC");
        return v && v[0] == '1';
    }();
    return on;
}

}  // namespace sspcg

using namespace sspcg;

namespace {

#define API_TRY try {
#define API_CATCH                                  \
    }                                              \
    catch (const std::exception& ex)               \
    {                                              \
        set_error(std::string("exception: ") + ex.what()); \
        return SSPCG_ERR_HIP;                      \
    }                                              \
    catch (...)                                    \
    {                                              \
        set_error("unknown exception");            \
        return SSPCG_ERR_HIP;                      \
    }

#define RETURN_IF(x)                \
    do {                            \
        int rc_ = (x);              \
        if (rc_ != SSPCG_OK) return rc_; \
    } while (0)


inline hipStream_t as_stream(sspcg_stream s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline int64_t ld_for(int64_t n) { return (int64_t)align_up((size_t)n, kSlice); }

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int arg_error(const std::string& what)
{
    set_error(what);
    return SSPCG_ERR_ARG;
}

// HIP events a solve uses: two to poll the control block, two for its GPU
// time.  sspcg_solve creates them per call; the allocation-free entry point
// uses a set made once per device.
struct SolveEvents {
    hipEvent_t poll[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;
};

struct OwnedEvents {
    SolveEvents ev;
    int create()
    {
        SSPCG_HIP(hipEventCreateWithFlags(&ev.poll[0], hipEventDisableTiming));
        SSPCG_HIP(hipEventCreateWithFlags(&ev.poll[1], hipEventDisableTiming));
        SSPCG_HIP(hipEventCreate(&ev.t0));
        SSPCG_HIP(hipEventCreate(&ev.t1));
        return SSPCG_OK;
    }
    ~OwnedEvents()
    {
        for (hipEvent_t e : {ev.poll[0], ev.poll[1], ev.t0, ev.t1})
            if (e) (void)hipEventDestroy(e);
    }
};

// Workspace of a solve, carved from the caller's buffer.
struct Workspace {
    size_t ctrl = 0, small = 0, part = 0, part2 = 0, hist = 0, vec = 0, total = 0;
    int64_t ld = 0;
    size_t elem = 8;
    int ncols = 0;
};

size_t partial_bytes(int s)
{
    const int k = std::max({s * s, s * (s + 1) / 2 + s, 4});
    return align_up((size_t)k * kMaxGrid * sizeof(double), 256);
}

Workspace layout_sspcg(int64_t n, const sspcg_params* p)
{
    Workspace w;
    w.ld = ld_for(n);
    w.elem = p->precision == SSPCG_MIXED ? sizeof(float) : sizeof(double);
    const int s = p->s;
    size_t off = 0;
    w.ctrl = off;
    off += 256;
    w.small = off;
    off += align_up(sizeof(double) * (2 * s * s + s), 256);
    w.part = off;
    off += partial_bytes(s);
    w.hist = off;
    off += align_up(sizeof(double) * kHistStride * (size_t)std::max(p->max_outer, 1), 256);
    w.vec = off;
    // r, Z, AZ, Q, AQ (+ the correction d of the mixed form)
    w.ncols = 4 * s + 1 + (p->precision == SSPCG_MIXED ? 1 : 0);
    off += align_up(w.elem * (size_t)w.ld * w.ncols, 256);
    w.total = off;
    return w;
}

Workspace layout_pcg(int64_t n, const sspcg_params* p)
{
    Workspace w;
    w.ld = ld_for(n);
    size_t off = 0;
    w.ctrl = off;
    off += 256;
    w.part = off;
    off += partial_bytes(1);
    w.part2 = off;
    off += partial_bytes(1);
    w.hist = off;
    off += align_up(sizeof(double) * (size_t)std::max(p->max_outer, 1), 256);
    w.vec = off;
    w.ncols = 4;   // r, z, p, q
    off += align_up(sizeof(double) * (size_t)w.ld * 4, 256);
    w.total = off;
    return w;
}

int check_params(const sspcg_matrix* A, const sspcg_params* p, bool pcg)
{
    if (!p) return arg_error("params is NULL");
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return arg_error("tol must be positive");
    if (p->max_outer < 1) return arg_error("max_outer must be >= 1");
    if (p->check_every < 1) return arg_error("check_every must be >= 1");
    if (pcg) return SSPCG_OK;
    if (p->s < 1 || p->s > SSPCG_MAX_S) return arg_error("s must be in 1..16");
    if (p->sweeps < 1 || p->sweeps > 1000) return arg_error("sweeps must be in 1..1000");
    if (!(p->sweep_tol >= 0.0) || !(p->sweep_tol < 1.0)) return arg_error("sweep_tol must be in [0,1)");
    if (!(p->lambda_min >= 0.0) || !(p->lambda_max > p->lambda_min) || !std::isfinite(p->lambda_max))
        return arg_error("need 0 <= lambda_min < lambda_max");
    if (p->gram != SSPCG_GRAM_FGS && p->gram != SSPCG_GRAM_CHOLESKY)
        return arg_error("unknown gram solver");
    if (p->basis != SSPCG_BASIS_CHEBYSHEV && p->basis != SSPCG_BASIS_MONOMIAL)
        return arg_error("unknown basis");
    if (p->precision != SSPCG_FP64 && p->precision != SSPCG_MIXED)
        return arg_error("unknown precision");
    if (p->precision == SSPCG_MIXED) {
        if (!(p->inner_tol > 0.0 && p->inner_tol < 1.0)) return arg_error("inner_tol must be in (0,1)");
        if (p->max_refine < 0) return arg_error("max_refine must be >= 0");
        if (!A->sval32) {
            set_error("mixed precision needs a matrix created with SSPCG_MATRIX_FP32");
            return SSPCG_ERR_UNSUPPORTED;
        }
    }
    return SSPCG_OK;
}

// Enqueues `iters` iterations through `step(k)` in batches, polling the
// device control block between batches.  Returns when the device reports
// done or the iteration limit is enqueued and finished.
int run_polled(Ctrl* dctrl, Ctrl* hctrl, int64_t max_iter, int check_every, hipStream_t st,
               const SolveEvents& events, const std::function<int(int64_t)>& step,
               const std::function<void(int64_t, int64_t)>& on_batch_done = nullptr)
{
    int64_t bstart[2] = {0, 0}, bend[2] = {0, 0};
    hipEvent_t const* ev = events.poll;
    int rc = SSPCG_OK;
    int64_t k = 0;
    int batch = 0;
    bool done = false;
    while (!done && k < max_iter) {
        const int64_t kend = std::min<int64_t>(k + check_every, max_iter);
        bstart[batch & 1] = k;
        bend[batch & 1] = kend;
        for (; k < kend && rc == SSPCG_OK; ++k) rc = step(k);
        if (rc != SSPCG_OK) break;
        hipError_t e = hipMemcpyAsync(&hctrl[batch & 1], dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(ev[batch & 1], st);
        if (e != hipSuccess) {
            rc = hip_fail(e, "poll copy");
            break;
        }
        if (batch > 0) {
            e = hipEventSynchronize(ev[(batch - 1) & 1]);
            if (e != hipSuccess) {
                rc = hip_fail(e, "poll wait");
                break;
            }
            done = hctrl[(batch - 1) & 1].done != 0;
            if (on_batch_done) on_batch_done(bstart[(batch - 1) & 1], bend[(batch - 1) & 1]);
        }
        ++batch;
    }
    hipError_t e = hipStreamSynchronize(st);
    if (rc == SSPCG_OK && e == hipSuccess && batch > 0 && on_batch_done)
        on_batch_done(bstart[(batch - 1) & 1], bend[(batch - 1) & 1]);
    if (rc != SSPCG_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    SSPCG_HIP(hipMemcpy(&hctrl[0], dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    return SSPCG_OK;
}

// Optional per-phase timing of the outer loop: HIP events at the phase
// boundaries of every iteration; a ring of event slots covers the iterations
// in flight (two polling batches), read back when their batch has finished.
class PhaseTimer {
  public:
    static constexpr int kMarks = 8;   // xr | norm | mpk | rect | fgs | update | fgs
    int init(bool on, int check_every)
    {
        on_ = on;
        if (!on_) return SSPCG_OK;
        ring_ = 3 * check_every + 1;
        ev_.assign((size_t)ring_ * kMarks + 4, nullptr);
        for (auto& e : ev_) SSPCG_HIP(hipEventCreate(&e));
        return SSPCG_OK;
    }
    ~PhaseTimer()
    {
        for (auto& e : ev_)
            if (e) (void)hipEventDestroy(e);
    }
    // marks of the start phase (before the loop): mpk | update | fgs
    void start_mark(int i, hipStream_t st)
    {
        if (on_) (void)hipEventRecord(ev_[(size_t)ring_ * kMarks + i], st);
    }
    void mark(int64_t k, int i, hipStream_t st)
    {
        if (on_) (void)hipEventRecord(ev_[slot(k, i)], st);
    }
    void collect_start()
    {
        if (!on_) return;
        start_[0] = elapsed(ev_[(size_t)ring_ * kMarks + 0], ev_[(size_t)ring_ * kMarks + 1]);
        start_[1] = elapsed(ev_[(size_t)ring_ * kMarks + 1], ev_[(size_t)ring_ * kMarks + 2]);
        start_[2] = elapsed(ev_[(size_t)ring_ * kMarks + 2], ev_[(size_t)ring_ * kMarks + 3]);
    }
    void collect(int64_t k0, int64_t k1)
    {
        if (!on_) return;
        if ((int64_t)it_.size() < k1) it_.resize(k1);
        for (int64_t k = k0; k < k1; ++k)
            for (int i = 0; i + 1 < kMarks; ++i) it_[k][i] = elapsed(ev_[slot(k, i)], ev_[slot(k, i + 1)]);
    }
    // Sums the phases that did work: iteration k runs x/r and the norm for
    // k < iters and the rest for k < iters - 1 (the stop test ends it).
    void fill(sspcg_profile* pr, int s, int64_t iters) const
    {
        if (!on_) return;
        pr->launches[SSPCG_PHASE_SPMV] += s;
        pr->ms[SSPCG_PHASE_SPMV] += start_[0];
        pr->launches[SSPCG_PHASE_GRAM_UPDATE] += 1;
        pr->ms[SSPCG_PHASE_GRAM_UPDATE] += start_[1];
        pr->launches[SSPCG_PHASE_FGS] += 1;
        pr->ms[SSPCG_PHASE_FGS] += start_[2];
        for (int64_t k = 0; k < iters && k < (int64_t)it_.size(); ++k) {
            const auto& t = it_[k];
            pr->launches[SSPCG_PHASE_XR] += 1;
            pr->ms[SSPCG_PHASE_XR] += t[0];
            pr->launches[SSPCG_PHASE_NORM] += 1;
            pr->ms[SSPCG_PHASE_NORM] += t[1];
            if (k + 1 >= iters) continue;
            pr->launches[SSPCG_PHASE_SPMV] += s;
            pr->ms[SSPCG_PHASE_SPMV] += t[2];
            pr->launches[SSPCG_PHASE_GRAM_RECT] += 1;
            pr->ms[SSPCG_PHASE_GRAM_RECT] += t[3];
            pr->launches[SSPCG_PHASE_FGS] += 2;
            pr->ms[SSPCG_PHASE_FGS] += t[4] + t[6];
            pr->launches[SSPCG_PHASE_GRAM_UPDATE] += 1;
            pr->ms[SSPCG_PHASE_GRAM_UPDATE] += t[5];
        }
        pr->outer_iters += iters;
    }

  private:
    size_t slot(int64_t k, int i) const { return (size_t)(k % ring_) * kMarks + i; }
    static double elapsed(hipEvent_t a, hipEvent_t b)
    {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    bool on_ = false;
    int ring_ = 0;
    std::vector<hipEvent_t> ev_;
    std::vector<std::array<double, kMarks - 1>> it_;
    double start_[3] = {0, 0, 0};
};

// Algorithm 2 after z_1: s SpMV launches; each but the last forms the next
// basis vector in its epilogue.  Chebyshev: z_2 = alpha dinv.*p_2 - sigma z_1,
// z_{q+1} = 2 alpha dinv.*p_{q+1} - 2 sigma z_q - gamma z_{q-1}; monomial:
// z_{q+1} = dinv.*p_{q+1}.
// Captures `n` calls of step(k) on stream st into a graph.  The iterations
// take no per-iteration argument (the device control block carries the
// iteration count), so the graph replays any batch.
int capture_batch(hipStream_t st, int n, const std::function<int(int64_t)>& step,
                  hipGraph_t* graph, hipGraphExec_t* exec)
{
    SSPCG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    int rc = SSPCG_OK;
    for (int k = 0; k < n && rc == SSPCG_OK; ++k) rc = step(k);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != SSPCG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    const hipError_t e2 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e2, "hipGraphInstantiate");
    }
    *graph = g;
    return SSPCG_OK;
}

template <typename T>
int enqueue_mpk(const sspcg_matrix* A, int s, int basis, double al, double sg, T* Z, T* AZ,
                int64_t ld, const Ctrl* ctrl, hipStream_t st)
{
    for (int q = 1; q <= s; ++q) {
        T* zq = Z + (int64_t)(q - 1) * ld;
        T* y = AZ + (int64_t)(q - 1) * ld;
        int rc;
        if (q == s)
            rc = launch_spmv<T>(A, 0, zq, y, nullptr, nullptr, 0.0, 0.0, 0.0, ctrl, st);
        else if (basis == SSPCG_BASIS_MONOMIAL)
            rc = launch_spmv<T>(A, 1, zq, y, nullptr, Z + (int64_t)q * ld, 1.0, 0.0, 0.0, ctrl, st);
        else if (q == 1)
            rc = launch_spmv<T>(A, 1, zq, y, nullptr, Z + (int64_t)q * ld, al, sg, 0.0, ctrl, st);
        else
            rc = launch_spmv<T>(A, 2, zq, y, Z + (int64_t)(q - 2) * ld, Z + (int64_t)q * ld,
                                2.0 * al, 2.0 * sg, 1.0, ctrl, st);
        if (rc != SSPCG_OK) return rc;
    }
    return SSPCG_OK;
}

// The s-step iteration proper, on vectors of type T.  On entry r holds the
// residual, Z(:,1) = M^{-1} r and the device Ctrl is initialized.
template <typename T>
int run_sspcg(const sspcg_matrix* A, const sspcg_params* p, const Workspace& w, char* base, T* x,
              const T* dinv, int64_t max_iter, double* dhist, Ctrl* hctrl, sspcg_profile* prof,
              const SolveEvents& ev, hipStream_t st)
{
    const int s = p->s;
    const int64_t n = A->n, ld = w.ld;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + w.ctrl);
    double* Wbuf = reinterpret_cast<double*>(base + w.small);
    double* alpha = Wbuf + s * s;
    double* beta = alpha + s;
    double* part = reinterpret_cast<double*>(base + w.part);
    T* r = reinterpret_cast<T*>(base + w.vec);
    T* Z = r + ld;
    T* AZ = Z + (int64_t)s * ld;
    T* Q = AZ + (int64_t)s * ld;
    T* AQ = Q + (int64_t)s * ld;
    const double al = 2.0 / (p->lambda_max - p->lambda_min);
    const double sg = (p->lambda_max + p->lambda_min) / (p->lambda_max - p->lambda_min);
    PhaseTimer tm;
    int rc = tm.init(p->profile != 0, p->check_every);
    if (rc != SSPCG_OK) return rc;
    int G = 0;
    tm.start_mark(0, st);
    rc = enqueue_mpk<T>(A, s, p->basis, al, sg, Z, AZ, ld, ctrl, st);
    tm.start_mark(1, st);
    if (rc == SSPCG_OK)
        rc = launch_update_gram<T>(n, s, Z, Q, AZ, AQ, nullptr, r, nullptr, nullptr, ld, part, &G,
                                   ctrl, st);
    tm.start_mark(2, st);
    if (rc == SSPCG_OK)
        rc = launch_fgs_step(s, 0, part, G, Wbuf, alpha, p->sweeps, p->sweep_tol, p->gram, ctrl,
                             dhist, st);
    tm.start_mark(3, st);
    if (rc != SSPCG_OK) return rc;
    auto step = [&](int64_t k) -> int {
        int g = 0;
        tm.mark(k, 0, st);
        // r and z_1 now; x += Q alpha rides on the next block update, which
        // streams this Q anyway (or on the pending-x launch after the loop)
        int e = launch_xr<T>(n, s, Q, AQ, alpha, ld, nullptr, r, dinv, Z, part, &g, ctrl, st);
        tm.mark(k, 1, st);
        if (e == SSPCG_OK) e = launch_norm_step(part, g, ctrl, dhist, st);
        tm.mark(k, 2, st);
        if (e == SSPCG_OK) e = enqueue_mpk<T>(A, s, p->basis, al, sg, Z, AZ, ld, ctrl, st);
        tm.mark(k, 3, st);
        if (e == SSPCG_OK) e = launch_gram_rect<T>(n, s, Q, AZ, ld, part, &g, ctrl, st);
        tm.mark(k, 4, st);
        if (e == SSPCG_OK)
            e = launch_fgs_step(s, 1, part, g, Wbuf, beta, p->sweeps, p->sweep_tol, p->gram, ctrl,
                                dhist, st);
        tm.mark(k, 5, st);
        if (e == SSPCG_OK)
            e = launch_update_gram<T>(n, s, Z, Q, AZ, AQ, beta, r, x, alpha, ld, part, &g, ctrl, st);
        tm.mark(k, 6, st);
        if (e == SSPCG_OK)
            e = launch_fgs_step(s, 0, part, g, Wbuf, alpha, p->sweeps, p->sweep_tol, p->gram, ctrl,
                                dhist, st);
        tm.mark(k, 7, st);
        return e;
    };
    bool started = false;
    auto on_batch = [&](int64_t k0, int64_t k1) {
        if (!started) {
            tm.collect_start();
            started = true;
        }
        tm.collect(k0, k1);
    };
    if (p->use_graph && !p->profile && st != nullptr) {
        // one batch of iterations captured once, replayed until done
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        rc = capture_batch(st, p->check_every, step, &graph, &exec);
        if (rc != SSPCG_OK) return rc;
        auto replay = [&](int64_t k) -> int {
            if (k % p->check_every != 0) return SSPCG_OK;   // one launch per batch
            hipError_t e = hipGraphLaunch(exec, st);
            return e == hipSuccess ? SSPCG_OK : hip_fail(e, "hipGraphLaunch");
        };
        const int64_t batches = (max_iter + p->check_every - 1) / p->check_every;
        rc = run_polled(ctrl, hctrl, batches * p->check_every, p->check_every, st, ev, replay);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (rc == SSPCG_OK) rc = launch_x_pending<T>(n, s, Q, alpha, ld, x, ctrl, st);
        return rc;
    }
    rc = run_polled(ctrl, hctrl, max_iter, p->check_every, st, ev, step, on_batch);
    if (rc == SSPCG_OK && prof) tm.fill(prof, s, hctrl[0].iter);
    if (rc == SSPCG_OK) rc = launch_x_pending<T>(n, s, Q, alpha, ld, x, ctrl, st);
    return rc;
}

// Writes the initial control block through the pinned mirror.
int init_ctrl(Ctrl* hctrl, Ctrl* dctrl, double nb, double tol, int64_t max_iter, double rho0,
              hipStream_t st)
{
    Ctrl c;
    std::memset(&c, 0, sizeof(c));
    c.done = 0;
    c.status = SSPCG_NOT_CONVERGED;
    c.iter = 0;
    c.max_iter = (int32_t)max_iter;
    c.nb = nb;
    c.tol = tol;
    c.relres = 0.0;
    c.rho[0] = rho0;
    hctrl[0] = c;
    SSPCG_HIP(hipMemcpyAsync(dctrl, &hctrl[0], sizeof(Ctrl), hipMemcpyHostToDevice, st));
    return SSPCG_OK;
}

// Reads the setup sums {||b-Ax||^2, ||r_stored||^2, ||b||^2, r^T z} (blocking).
int setup_sums(Ctrl* hctrl, Ctrl* dctrl, const double* part, int G, double* out, hipStream_t st)
{
    int rc = launch_finish(part, 4, G, dctrl->sums, st);
    if (rc != SSPCG_OK) return rc;
    SSPCG_HIP(hipMemcpyAsync(&hctrl[1], dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    SSPCG_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < 4; ++i) out[i] = hctrl[1].sums[i];
    return SSPCG_OK;
}

// GPU time of a solve between two of the solve's events.
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    Timer(const SolveEvents& ev, hipStream_t s) : a(ev.t0), b(ev.t1), st(s)
    {
        (void)hipEventRecord(a, st);
    }
    double stop()
    {
        float ms = 0.0f;
        if (a && b && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess)
            (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
};

// ||b - A x|| / ||b|| in FP64 for the returned x (r and part are free
// workspace once the iteration has ended); not part of the timed solve.
int true_relres(const sspcg_matrix* A, const double* b, const double* x, double* r, double* part,
                Ctrl* dctrl, Ctrl* hctrl, hipStream_t st, double* out)
{
    int G = 0;
    double sums[4];
    int rc = launch_residual<double>(A, x, b, r, static_cast<double*>(nullptr), part, &G, st);
    if (rc == SSPCG_OK) rc = setup_sums(hctrl, dctrl, part, G, sums, st);
    if (rc != SSPCG_OK) return rc;
    *out = sums[2] > 0.0 ? std::sqrt(sums[0]) / std::sqrt(sums[2]) : 0.0;
    return SSPCG_OK;
}

int solve_fp64(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
               const Workspace& w, char* base, Ctrl* hctrl, const SolveEvents& ev,
               hipStream_t st, sspcg_result* res, double* history, sspcg_profile* prof)
{
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + w.ctrl);
    double* part = reinterpret_cast<double*>(base + w.part);
    double* dhist = reinterpret_cast<double*>(base + w.hist);
    double* r = reinterpret_cast<double*>(base + w.vec);
    double* Z = r + w.ld;
    Timer tm(ev, st);
    int G = 0;
    int rc = launch_residual<double>(A, x, b, r, Z, part, &G, st);
    double sums[4];
    if (rc == SSPCG_OK) rc = setup_sums(hctrl, ctrl, part, G, sums, st);
    if (rc != SSPCG_OK) return rc;
    const double nb = std::sqrt(sums[2]);
    res->outer_iters = 0;
    if (!std::isfinite(nb) || !std::isfinite(sums[0])) {
        res->device_ms = tm.stop();
        res->relres = res->relres_true = std::sqrt(sums[0]) / nb;
        set_error("non-finite right-hand side or starting residual");
        return res->status = SSPCG_ERR_NONFINITE;
    }
    if (nb == 0.0) {
        rc = launch_fill<double>(A->n, x, 0.0, st);
        res->device_ms = tm.stop();
        res->relres = res->relres_true = 0.0;
        return res->status = rc;
    }
    const double rel0 = std::sqrt(sums[0]) / nb;
    if (rel0 <= p->tol) {
        res->device_ms = tm.stop();
        res->relres = res->relres_true = rel0;
        return res->status = SSPCG_OK;
    }
    rc = init_ctrl(hctrl, ctrl, nb, p->tol, p->max_outer, 0.0, st);
    if (rc == SSPCG_OK)
        rc = run_sspcg<double>(A, p, w, base, x, A->dinv, p->max_outer, history ? dhist : nullptr,
                               hctrl, prof, ev, st);
    res->device_ms = tm.stop();
    if (rc != SSPCG_OK) return res->status = rc;
    const Ctrl c = hctrl[0];
    res->outer_iters = c.iter;
    res->inner_iters_total = c.iter;
    res->relres = c.relres;
    res->status = c.done ? c.status : SSPCG_NOT_CONVERGED;
    if (history && c.iter > 0)
        SSPCG_HIP(hipMemcpy(history, dhist, sizeof(double) * kHistStride * (size_t)c.iter,
                            hipMemcpyDeviceToHost));
    RETURN_IF(true_relres(A, b, x, r, part, ctrl, hctrl, st, &res->relres_true));
    return res->status;
}

int solve_mixed(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                const Workspace& w, char* base, Ctrl* hctrl, const SolveEvents& ev,
                hipStream_t st, sspcg_result* res, double* history, sspcg_profile* prof)
{
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + w.ctrl);
    double* part = reinterpret_cast<double*>(base + w.part);
    float* r = reinterpret_cast<float*>(base + w.vec);
    float* Z = r + w.ld;
    float* d = r + (int64_t)(4 * p->s + 1) * w.ld;
    Timer tm(ev, st);
    double nb = 0.0, relres = 0.0;
    int nref = 0, inner_total = 0, status = SSPCG_NOT_CONVERGED;
    for (;;) {
        int G = 0;
        double sums[4];
        int rc = launch_residual<float>(A, x, b, r, Z, part, &G, st);
        if (rc == SSPCG_OK) rc = setup_sums(hctrl, ctrl, part, G, sums, st);
        if (rc != SSPCG_OK) return rc;
        if (nref == 0) {
            nb = std::sqrt(sums[2]);
            if (!std::isfinite(nb)) {
                status = SSPCG_ERR_NONFINITE;
                relres = nb;
                set_error("non-finite right-hand side");
                break;
            }
            if (nb == 0.0) {
                rc = launch_fill<double>(A->n, x, 0.0, st);
                if (rc != SSPCG_OK) return rc;
                status = SSPCG_OK;
                relres = 0.0;
                break;
            }
        }
        relres = std::sqrt(sums[0]) / nb;
        if (history) history[nref] = relres;
        if (!std::isfinite(relres)) {
            status = SSPCG_ERR_NONFINITE;
            break;
        }
        if (relres <= p->tol) {
            status = SSPCG_OK;
            break;
        }
        if (nref >= p->max_refine || sums[1] == 0.0) {
            status = SSPCG_NOT_CONVERGED;
            break;
        }
        // reduce by inner_tol, or only to half the outer target when closer
        const double itol = std::min(std::max(p->inner_tol, 0.5 * p->tol / relres), 0.5);
        rc = init_ctrl(hctrl, ctrl, std::sqrt(sums[1]), itol, p->max_outer, 0.0, st);
        if (rc == SSPCG_OK) rc = launch_fill<float>(A->n, d, 0.0f, st);
        if (rc == SSPCG_OK)
            rc = run_sspcg<float>(A, p, w, base, d, A->dinv32, p->max_outer, nullptr, hctrl, prof,
                                  ev, st);
        if (rc != SSPCG_OK) return rc;
        const Ctrl c = hctrl[0];
        inner_total += c.iter;
        if (c.status != SSPCG_OK && c.status != SSPCG_NOT_CONVERGED) {
            status = c.status;
            break;
        }
        rc = launch_axpy_up<float>(A->n, x, d, nullptr, st);
        if (rc != SSPCG_OK) return rc;
        ++nref;
    }
    res->device_ms = tm.stop();
    res->outer_iters = inner_total;
    res->inner_iters_total = inner_total;
    res->refinements = nref;
    // the outer stop test is on the FP64 true residual of the returned x
    res->relres = res->relres_true = relres;
    return res->status = status;
}

int solve_pcg(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
              const Workspace& w, char* base, Ctrl* hctrl, const SolveEvents& ev, hipStream_t st,
              sspcg_result* res, double* history)
{
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + w.ctrl);
    double* part = reinterpret_cast<double*>(base + w.part);
    double* part2 = reinterpret_cast<double*>(base + w.part2);
    double* dhist = reinterpret_cast<double*>(base + w.hist);
    double* r = reinterpret_cast<double*>(base + w.vec);
    double* z = r + w.ld;
    double* pv = z + w.ld;
    double* q = pv + w.ld;
    const int64_t n = A->n;
    Timer tm(ev, st);
    int G = 0;
    double sums[4];
    int rc = launch_residual<double>(A, x, b, r, z, part2, &G, st);
    if (rc == SSPCG_OK) rc = setup_sums(hctrl, ctrl, part2, G, sums, st);
    if (rc != SSPCG_OK) return rc;
    const double nb = std::sqrt(sums[2]);
    res->outer_iters = 0;
    if (!std::isfinite(nb) || !std::isfinite(sums[0])) {
        res->device_ms = tm.stop();
        res->relres = res->relres_true = std::sqrt(sums[0]) / nb;
        set_error("non-finite right-hand side or starting residual");
        return res->status = SSPCG_ERR_NONFINITE;
    }
    if (nb == 0.0) {
        rc = launch_fill<double>(n, x, 0.0, st);
        res->device_ms = tm.stop();
        res->relres = res->relres_true = 0.0;
        return res->status = rc;
    }
    const double rel0 = std::sqrt(sums[0]) / nb;
    if (rel0 <= p->tol) {
        res->device_ms = tm.stop();
        res->relres = res->relres_true = rel0;
        return res->status = SSPCG_OK;
    }
    rc = init_ctrl(hctrl, ctrl, nb, p->tol, p->max_outer, sums[3], st);
    if (rc != SSPCG_OK) return rc;
    SSPCG_HIP(hipMemcpyAsync(pv, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    double* hist = history ? dhist : nullptr;
    auto step = [&](int64_t k) -> int {
        int g1 = 0, g2 = 0;
        int e = launch_pcg_spmv(A, pv, q, part, &g1, ctrl, st);
        if (e == SSPCG_OK) e = launch_pcg_update(A, k, x, r, z, pv, q, part, g1, part2, &g2, ctrl, st);
        if (e == SSPCG_OK) e = launch_pcg_pupdate(n, k, z, pv, part2, g2, ctrl, hist, st);
        return e;
    };
    rc = run_polled(ctrl, hctrl, p->max_outer, p->check_every, st, ev, step);
    res->device_ms = tm.stop();
    if (rc != SSPCG_OK) return res->status = rc;
    const Ctrl c = hctrl[0];
    res->outer_iters = c.iter;
    res->inner_iters_total = c.iter;
    res->relres = c.relres;
    res->status = c.done ? c.status : SSPCG_NOT_CONVERGED;
    if (history && c.iter > 0)
        SSPCG_HIP(hipMemcpy(history, dhist, sizeof(double) * (size_t)c.iter, hipMemcpyDeviceToHost));
    RETURN_IF(true_relres(A, b, x, z, part2, ctrl, hctrl, st, &res->relres_true));
    return res->status;
}

int check_matrix(const sspcg_matrix* A)
{
    if (!A || !A->sval) return arg_error("matrix handle is NULL or destroyed");
    return SSPCG_OK;
}

int check_vec(const void* p, int dtype, const char* name)
{
    if (!p) return arg_error(std::string(name) + " is NULL");
    if (!aligned(p, dtype == SSPCG_F32 ? 4 : 8)) return arg_error(std::string(name) + " is misaligned");
    return SSPCG_OK;
}

int check_dtype(const sspcg_matrix* A, int dtype)
{
    if (dtype != SSPCG_F64 && dtype != SSPCG_F32) return arg_error("unknown dtype");
    if (dtype == SSPCG_F32 && A && !A->sval32) {
        set_error("FP32 kernels need a matrix created with SSPCG_MATRIX_FP32");
        return SSPCG_ERR_UNSUPPORTED;
    }
    return SSPCG_OK;
}

int check_work(void* work, size_t bytes, int s)
{
    if (!work) return arg_error("work is NULL");
    if (!aligned(work, 256)) return arg_error("work must be 256-byte aligned");
    if (bytes < partial_bytes(s)) {
        set_error("kernel workspace too small");
        return SSPCG_ERR_WORKSPACE;
    }
    return SSPCG_OK;
}


int check_csr_args(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col,
                   const double* val, int32_t flags)
{
    if (n < 1 || nnz < n) return arg_error("need n >= 1 and nnz >= n (diagonal stored)");
    if (!row_ptr || !col || !val) return arg_error("CSR pointer is NULL");
    if (!aligned(row_ptr, 4) || !aligned(col, 4) || !aligned(val, 8)) return arg_error("CSR array misaligned");
    if (flags & ~(SSPCG_MATRIX_FP32 | SSPCG_MATRIX_FULL_STORAGE)) return arg_error("unknown flag");
    return SSPCG_OK;
}

// Places of the matrix's arrays in the caller's `aux` buffer (byte offsets,
// each 256-byte aligned).  The analysis area and the Jacobi scaling come
// first and depend on n alone; the layout's arrays follow the plan.
struct AuxLayout {
    size_t dinv = 0, dinv32 = 0, fixed = 0;
    size_t slice_ptr = 0, slice_aux = 0, col = 0, soff = 0;   // per-slice layout
    size_t uoff = 0;                                           // uniform layout
    size_t val = 0, val32 = 0;
    int64_t slots = 0;                                         // uniform: stored slots
    size_t total = 0;                                          // 0: too large
};

AuxLayout aux_layout(const sspcg_matrix* A, const LayoutPlan& plan)
{
    AuxLayout L;
    const bool f32 = (A->flags & SSPCG_MATRIX_FP32) != 0;
    const int64_t rows = A->nslices * kSlice;
    size_t off = analysis_bytes(A->n);
    L.dinv = off;
    off += align_up(sizeof(double) * (size_t)A->n, 256);
    L.dinv32 = off;
    if (f32) off += align_up(sizeof(float) * (size_t)A->n, 256);
    L.fixed = off;
    if (!plan.uoff.empty()) {
        const int64_t uw = (int64_t)plan.uoff.size();
        const int64_t stored = uw - (plan.usym ? uw / 2 : 0);
        // the full storage groups FP64 values in pairs and FP32 values in
        // quads; the half storage keeps single values
        const int64_t stored64 = plan.usym ? stored : (stored + 1) / 2 * 2;
        const int64_t stored32 = plan.usym ? stored : (stored + 3) / 4 * 4;
        L.slots = rows * stored;
        if (rows * stored64 >= ((int64_t)1 << 40)) return L;
        L.uoff = off;
        off += 256;
        L.val = off;
        off += align_up(sizeof(double) * (size_t)(rows * stored64), 256);
        L.val32 = off;
        if (f32) off += align_up(sizeof(float) * (size_t)(rows * stored32), 256);
    } else if (!plan.slice_ptr.empty()) {
        if (plan.slots >= ((int64_t)1 << 40)) return L;
        L.slice_ptr = off;
        off += align_up(sizeof(int64_t) * (size_t)(A->nslices + 1), 256);
        L.slice_aux = off;
        off += align_up(sizeof(int64_t) * (size_t)A->nslices, 256);
        L.col = off;
        off += align_up(sizeof(int32_t) * (size_t)plan.ncol, 256);
        L.soff = off;
        off += align_up(sizeof(int32_t) * (size_t)plan.nsoff, 256);
        L.val = off;
        off += align_up(sizeof(double) * (size_t)plan.slots, 256);
        L.val32 = off;
        if (f32) off += align_up(sizeof(float) * (size_t)plan.slots, 256);
    }
    L.total = off;
    return L;
}

// The poll buffer must be pinned host memory: the pipelined polling copies
// into it asynchronously.
int check_poll(void* poll)
{
    if (!poll) return arg_error("poll is NULL (pinned host memory of SSPCG_POLL_BYTES bytes)");
    if (!aligned(poll, 64)) return arg_error("poll must be 64-byte aligned");
    hipPointerAttribute_t at;
    const hipError_t e = hipPointerGetAttributes(&at, poll);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return arg_error("poll is not pinned host memory (hipHostMalloc or pin_memory)");
    }
    if (at.type != hipMemoryTypeHost) return arg_error("poll must be pinned host memory");
    return SSPCG_OK;
}

// Per-device state of sspcg_solve_static, made at the first call on a
// device with that device current: the device address of `scratch` there
// and the solve's HIP events.  Both are kept until the process ends.
struct StaticState {
    void* scratch = nullptr;
    SolveEvents ev;
};
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
StaticState g_static[kMaxDevices];
bool g_static_ready[kMaxDevices] = {};

int static_state(int dev, const StaticState** out)
{
    if (dev < 0 || dev >= kMaxDevices) return arg_error("device index out of range");
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticState& S = g_static[dev];
    if (!g_static_ready[dev]) {
        void* ptr = nullptr;
        SSPCG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("hipGetSymbolAddress returned no address for the static scratch");
            return SSPCG_ERR_HIP;
        }
        OwnedEvents ev;
        RETURN_IF(ev.create());
        S.scratch = ptr;
        S.ev = ev.ev;
        ev.ev = SolveEvents();   // kept: the state owns them now
        g_static_ready[dev] = true;
    }
    *out = &S;
    return SSPCG_OK;
}

}  // namespace

extern "C" {

int sspcg_abi_version(void) { return SSPCG_ABI_VERSION; }

const char* sspcg_status_string(int status)
{
    switch (status) {
    case SSPCG_OK: return "ok";
    case SSPCG_NOT_CONVERGED: return "not converged";
    case SSPCG_ERR_ARG: return "invalid argument";
    case SSPCG_ERR_HIP: return "HIP runtime error";
    case SSPCG_ERR_BREAKDOWN: return "breakdown (non-positive diagonal of a Gram matrix or of A)";
    case SSPCG_ERR_WORKSPACE: return "workspace too small";
    case SSPCG_ERR_NONFINITE: return "non-finite value";
    case SSPCG_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
    }
}

const char* sspcg_last_error(void) { return g_error.c_str(); }

void sspcg_default_params(sspcg_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->s = 4;
    p->sweeps = 2;
    p->lambda_min = 0.0;
    p->lambda_max = 2.0;
    p->tol = 1e-8;
    p->max_outer = 20000;
    p->precision = SSPCG_FP64;
    p->inner_tol = 1e-4;
    p->max_refine = 20;
    p->gram = SSPCG_GRAM_FGS;
    p->check_every = 8;
    p->profile = 0;
    p->sweep_tol = 0.0;
    p->basis = SSPCG_BASIS_CHEBYSHEV;
    p->use_graph = 0;
}

size_t sspcg_matrix_scratch_bytes(int32_t n)
{
    return analysis_bytes(std::max<int64_t>(n, 1));
}

int sspcg_matrix_aux_bytes(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col,
                           const double* val, int32_t flags, void* scratch, size_t scratch_bytes,
                           sspcg_stream stream, size_t* aux_bytes)
{
    API_TRY
    if (!aux_bytes) return arg_error("aux_bytes is NULL");
    *aux_bytes = 0;
    RETURN_IF(check_csr_args(n, nnz, row_ptr, col, val, flags));
    if (!scratch || !aligned(scratch, 256)) return arg_error("scratch is NULL or not 256-byte aligned");
    if (scratch_bytes < analysis_bytes(n)) {
        set_error("scratch smaller than sspcg_matrix_scratch_bytes(n)");
        return SSPCG_ERR_WORKSPACE;
    }
    sspcg_matrix A;
    A.n = n;
    A.nnz = nnz;
    A.flags = flags;
    A.row_ptr = row_ptr;
    A.col = col;
    A.nslices = (n + kSlice - 1) / kSlice;
    bind_analysis(&A, scratch);
    LayoutPlan plan;
    RETURN_IF(matrix_inspect(&A, val, false, &plan, as_stream(stream), false,
                             (flags & SSPCG_MATRIX_FULL_STORAGE) == 0));
    const AuxLayout L = aux_layout(&A, plan);
    if (L.total == 0) return arg_error("matrix too large");
    *aux_bytes = L.total;
    return SSPCG_OK;
    API_CATCH
}

int sspcg_matrix_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col,
                        const double* val, int32_t flags, void* aux, size_t aux_bytes,
                        sspcg_stream stream, sspcg_matrix** out)
{
    API_TRY
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    RETURN_IF(check_csr_args(n, nnz, row_ptr, col, val, flags));
    if (!aux || !aligned(aux, 256)) return arg_error("aux is NULL or not 256-byte aligned");
    hipStream_t st = as_stream(stream);
    std::unique_ptr<sspcg_matrix> A(new sspcg_matrix());
    A->n = n;
    A->nnz = nnz;
    A->flags = flags;
    A->row_ptr = row_ptr;
    A->col = col;
    (void)hipGetDevice(&A->device);
    A->nslices = (n + kSlice - 1) / kSlice;
    A->aux = aux;
    char* base = static_cast<char*>(aux);
    // the analysis area and the Jacobi scaling have fixed places: the first
    // pass over the matrix checks it and writes 1/diag(A)
    const AuxLayout L0 = aux_layout(A.get(), LayoutPlan());
    if (aux_bytes < L0.fixed) {
        set_error("aux smaller than sspcg_matrix_aux_bytes reported");
        return SSPCG_ERR_WORKSPACE;
    }
    bind_analysis(A.get(), base);
    A->dinv = reinterpret_cast<double*>(base + L0.dinv);
    A->dinv32 = (flags & SSPCG_MATRIX_FP32) ? reinterpret_cast<float*>(base + L0.dinv32) : nullptr;
    LayoutPlan plan;
    RETURN_IF(matrix_inspect(A.get(), val, false, &plan, st, true,
                             (flags & SSPCG_MATRIX_FULL_STORAGE) == 0));
    const AuxLayout L = aux_layout(A.get(), plan);
    if (L.total == 0) return arg_error("matrix too large");
    if (aux_bytes < L.total) {
        set_error("aux smaller than sspcg_matrix_aux_bytes reported");
        return SSPCG_ERR_WORKSPACE;
    }
    A->aux_used = L.total;
    A->slots = plan.slots;
    A->nshared = plan.nshared;
    if (!plan.uoff.empty()) {
        // uniform layout: offsets and values only
        A->uniform = 1;
        A->uw = (int32_t)plan.uoff.size();
        A->usym = plan.usym ? 1 : 0;
        A->slots = L.slots;
        A->uoff = reinterpret_cast<int32_t*>(base + L.uoff);
        A->sval = reinterpret_cast<double*>(base + L.val);
        A->sval32 = (flags & SSPCG_MATRIX_FP32) ? reinterpret_cast<float*>(base + L.val32) : nullptr;
        std::copy(plan.uoff.begin(), plan.uoff.end(), A->uoff_host);
        plan_lds(A.get());
        SSPCG_HIP(hipMemcpyAsync(A->uoff, plan.uoff.data(), sizeof(int32_t) * plan.uoff.size(),
                                 hipMemcpyHostToDevice, st));
    } else {
        A->slice_ptr = reinterpret_cast<int64_t*>(base + L.slice_ptr);
        A->slice_aux = reinterpret_cast<int64_t*>(base + L.slice_aux);
        A->scol = reinterpret_cast<int32_t*>(base + L.col);
        A->soff = reinterpret_cast<int32_t*>(base + L.soff);
        A->sval = reinterpret_cast<double*>(base + L.val);
        A->sval32 = (flags & SSPCG_MATRIX_FP32) ? reinterpret_cast<float*>(base + L.val32) : nullptr;
        SSPCG_HIP(hipMemcpyAsync(A->slice_ptr, plan.slice_ptr.data(),
                                 sizeof(int64_t) * plan.slice_ptr.size(), hipMemcpyHostToDevice, st));
        SSPCG_HIP(hipMemcpyAsync(A->slice_aux, plan.slice_aux.data(),
                                 sizeof(int64_t) * plan.slice_aux.size(), hipMemcpyHostToDevice, st));
        RETURN_IF(matrix_pack(A.get(), st));
    }
    RETURN_IF(matrix_fill(A.get(), val, false, st));
    *out = A.release();
    return SSPCG_OK;
    API_CATCH
}

int sspcg_matrix_update_values(sspcg_matrix* A, const double* val, sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (!val || !aligned(val, 8)) return arg_error("val is NULL or misaligned");
    hipStream_t st = as_stream(stream);
    // check everything before the matrix is touched
    RETURN_IF(matrix_inspect(A, val, true, nullptr, nullptr, st, false));
    if (A->usym) {
        bool sym = false;
        RETURN_IF(matrix_check_symmetric(A, val, &sym, st));
        if (!sym) {
            set_error("new values are not symmetric, but the matrix stores one triangle (it was "
                      "symmetric when created; SSPCG_MATRIX_FULL_STORAGE keeps both)");
            return SSPCG_ERR_UNSUPPORTED;
        }
    }
    RETURN_IF(matrix_inspect(A, val, true, nullptr, nullptr, st));
    return matrix_fill(A, val, true, st);
    API_CATCH
}

int sspcg_matrix_destroy(sspcg_matrix* A)
{
    API_TRY
    delete A;
    return SSPCG_OK;
    API_CATCH
}

int sspcg_matrix_info(const sspcg_matrix* A, int64_t* n, int64_t* nnz, int64_t* slots,
                      int64_t* slices, int64_t* shared_slices, int64_t* device_bytes,
                      int64_t* symmetric)
{
    RETURN_IF(check_matrix(A));
    if (symmetric) *symmetric = A->usym;
    if (n) *n = A->n;
    if (nnz) *nnz = A->nnz;
    if (slots) *slots = A->slots;
    if (slices) *slices = A->nslices;
    if (shared_slices) *shared_slices = A->nshared;
    if (device_bytes) *device_bytes = (int64_t)A->aux_used;
    return SSPCG_OK;
}

int sspcg_workspace_bytes(const sspcg_matrix* A, const sspcg_params* p, size_t* bytes)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (!bytes) return arg_error("bytes is NULL");
    RETURN_IF(check_params(A, p, false));
    // large enough for either solver with these parameters
    *bytes = std::max(layout_sspcg(A->n, p).total, layout_pcg(A->n, p).total);
    return SSPCG_OK;
    API_CATCH
}

int sspcg_solve(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                void* work, size_t work_bytes, void* poll, sspcg_stream stream,
                sspcg_result* res, double* history, sspcg_profile* profile)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (!res) return arg_error("res is NULL");
    std::memset(res, 0, sizeof(*res));
    RETURN_IF(check_vec(b, SSPCG_F64, "b"));
    RETURN_IF(check_vec(x, SSPCG_F64, "x"));
    RETURN_IF(check_params(A, p, false));
    if (!work || !aligned(work, 256)) return arg_error("work is NULL or not 256-byte aligned");
    RETURN_IF(check_poll(poll));
    const Workspace w = layout_sspcg(A->n, p);
    if (work_bytes < w.total) {
        set_error("workspace too small");
        return res->status = SSPCG_ERR_WORKSPACE;
    }
    hipStream_t st = as_stream(stream);
    char* base = static_cast<char*>(work);
    Ctrl* hctrl = static_cast<Ctrl*>(poll);
    sspcg_profile* prof = p->profile ? profile : nullptr;
    if (prof) std::memset(prof, 0, sizeof(*prof));
    OwnedEvents ev;
    RETURN_IF(ev.create());
    if (p->precision == SSPCG_MIXED)
        return solve_mixed(A, b, x, p, w, base, hctrl, ev.ev, st, res, history, prof);
    return solve_fp64(A, b, x, p, w, base, hctrl, ev.ev, st, res, history, prof);
    API_CATCH
}

int sspcg_solve_static(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                       void* poll, sspcg_stream stream, sspcg_result* res)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (!res) return arg_error("res is NULL");
    std::memset(res, 0, sizeof(*res));
    RETURN_IF(check_vec(b, SSPCG_F64, "b"));
    RETURN_IF(check_vec(x, SSPCG_F64, "x"));
    RETURN_IF(check_params(A, p, false));
    RETURN_IF(check_poll(poll));
    if (p->profile || p->use_graph) {
        set_error("sspcg_solve_static: profile and use_graph need HIP events or graphs it does "
                  "not create; use sspcg_solve");
        return res->status = SSPCG_ERR_UNSUPPORTED;
    }
    const Workspace w = layout_sspcg(A->n, p);
    if (w.total > (size_t)SSPCG_STATIC_SCRATCH_BYTES) {
        set_error("sspcg_solve_static: the solve needs " + std::to_string(w.total) +
                  " bytes of workspace, more than the static scratch of " +
                  std::to_string((size_t)SSPCG_STATIC_SCRATCH_BYTES) + " bytes; use sspcg_solve");
        return res->status = SSPCG_ERR_WORKSPACE;
    }
    int dev = -1;
    SSPCG_HIP(hipGetDevice(&dev));
    if (dev != A->device) return arg_error("the current device is not the matrix's device");
    const StaticState* sst = nullptr;
    RETURN_IF(static_state(dev, &sst));
    hipStream_t st = as_stream(stream);
    char* base = static_cast<char*>(sst->scratch);
    Ctrl* hctrl = static_cast<Ctrl*>(poll);
    if (p->precision == SSPCG_MIXED)
        return solve_mixed(A, b, x, p, w, base, hctrl, sst->ev, st, res, nullptr, nullptr);
    return solve_fp64(A, b, x, p, w, base, hctrl, sst->ev, st, res, nullptr, nullptr);
    API_CATCH
}

int sspcg_pcg_solve(const sspcg_matrix* A, const double* b, double* x, const sspcg_params* p,
                    void* work, size_t work_bytes, void* poll, sspcg_stream stream,
                    sspcg_result* res, double* history)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (!res) return arg_error("res is NULL");
    std::memset(res, 0, sizeof(*res));
    RETURN_IF(check_vec(b, SSPCG_F64, "b"));
    RETURN_IF(check_vec(x, SSPCG_F64, "x"));
    RETURN_IF(check_params(A, p, true));
    if (!work || !aligned(work, 256)) return arg_error("work is NULL or not 256-byte aligned");
    RETURN_IF(check_poll(poll));
    const Workspace w = layout_pcg(A->n, p);
    if (work_bytes < w.total) {
        set_error("workspace too small");
        return res->status = SSPCG_ERR_WORKSPACE;
    }
    OwnedEvents ev;
    RETURN_IF(ev.create());
    return solve_pcg(A, b, x, p, w, static_cast<char*>(work), static_cast<Ctrl*>(poll), ev.ev,
                     as_stream(stream), res, history);
    API_CATCH
}

int sspcg_interval_work_bytes(const sspcg_matrix* A, int32_t steps, size_t* bytes)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (!bytes) return arg_error("bytes is NULL");
    if (steps < 1 || steps > SSPCG_MAX_INTERVAL_STEPS)
        return arg_error("steps must be in 1..SSPCG_MAX_INTERVAL_STEPS");
    *bytes = interval_work_bytes(A->n, steps);
    return SSPCG_OK;
    API_CATCH
}

int sspcg_interval(const sspcg_matrix* A, int32_t method, int32_t steps, double rtol,
                   const double* v0, void* work, size_t work_bytes, sspcg_stream stream,
                   double* lambda_min, double* lambda_max, int32_t* steps_taken)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    if (method != SSPCG_INTERVAL_LANCZOS && method != SSPCG_INTERVAL_POWER)
        return arg_error("unknown interval method");
    if (steps < 1 || steps > SSPCG_MAX_INTERVAL_STEPS)
        return arg_error("steps must be in 1..SSPCG_MAX_INTERVAL_STEPS");
    if (!(rtol >= 0.0) || !std::isfinite(rtol)) return arg_error("rtol must be finite and >= 0");
    RETURN_IF(check_vec(v0, SSPCG_F64, "v0"));
    if (!lambda_min || !lambda_max) return arg_error("lambda_min / lambda_max is NULL");
    if (!work || !aligned(work, 256)) return arg_error("work is NULL or not 256-byte aligned");
    if (work_bytes < interval_work_bytes(A->n, steps)) {
        set_error("interval workspace too small");
        return SSPCG_ERR_WORKSPACE;
    }
    int taken = 0;
    const int rc = run_interval(A, method, steps, rtol, v0, work, as_stream(stream), lambda_min,
                                lambda_max, &taken);
    if (steps_taken) *steps_taken = taken;
    return rc;
    API_CATCH
}

size_t sspcg_kernel_work_bytes(int32_t s)
{
    return partial_bytes(std::max(1, std::min<int32_t>(s, SSPCG_MAX_S)));
}

int sspcg_spmv(const sspcg_matrix* A, int32_t dtype, const void* x, void* y, sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    RETURN_IF(check_dtype(A, dtype));
    RETURN_IF(check_vec(x, dtype, "x"));
    RETURN_IF(check_vec(y, dtype, "y"));
    hipStream_t st = as_stream(stream);
    if (dtype == SSPCG_F32)
        return launch_spmv<float>(A, 0, static_cast<const float*>(x), static_cast<float*>(y),
                                  nullptr, nullptr, 0, 0, 0, nullptr, st);
    return launch_spmv<double>(A, 0, static_cast<const double*>(x), static_cast<double*>(y),
                               nullptr, nullptr, 0, 0, 0, nullptr, st);
    API_CATCH
}

int sspcg_mpk(const sspcg_matrix* A, int32_t dtype, const void* r, int32_t s, double lmin,
              double lmax, int32_t basis, void* Z, void* P, int64_t ld, sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    RETURN_IF(check_dtype(A, dtype));
    RETURN_IF(check_vec(r, dtype, "r"));
    RETURN_IF(check_vec(Z, dtype, "Z"));
    RETURN_IF(check_vec(P, dtype, "P"));
    if (s < 1 || s > SSPCG_MAX_S) return arg_error("s must be in 1..16");
    if (ld < A->n) return arg_error("ld < n");
    if (!(lmin >= 0.0) || !(lmax > lmin)) return arg_error("need 0 <= lmin < lmax");
    if (basis != SSPCG_BASIS_CHEBYSHEV && basis != SSPCG_BASIS_MONOMIAL) return arg_error("unknown basis");
    const double al = 2.0 / (lmax - lmin), sg = (lmax + lmin) / (lmax - lmin);
    hipStream_t st = as_stream(stream);
    if (dtype == SSPCG_F32) {
        float* z = static_cast<float*>(Z);
        float* pp = static_cast<float*>(P);
        RETURN_IF(launch_mpk_start<float>(A->n, static_cast<const float*>(r), A->dinv32, z, pp, st));
        return enqueue_mpk<float>(A, s, basis, al, sg, z, pp + ld, ld, nullptr, st);
    }
    double* z = static_cast<double*>(Z);
    double* pp = static_cast<double*>(P);
    RETURN_IF(launch_mpk_start<double>(A->n, static_cast<const double*>(r), A->dinv, z, pp, st));
    return enqueue_mpk<double>(A, s, basis, al, sg, z, pp + ld, ld, nullptr, st);
    API_CATCH
}

int sspcg_block_update_gram(int64_t n, int32_t s, int32_t dtype, const void* Z, void* Q,
                            const void* AZ, void* AQ, const double* beta, const void* r,
                            int64_t ld, double* W, double* b1, void* work, size_t work_bytes,
                            sspcg_stream stream)
{
    API_TRY
    if (n < 1 || n >= ((int64_t)1 << 31)) return arg_error("n out of range");
    if (s < 1 || s > SSPCG_MAX_S) return arg_error("s must be in 1..16");
    if (ld < n) return arg_error("ld < n");
    RETURN_IF(check_dtype(nullptr, dtype));
    RETURN_IF(check_vec(Z, dtype, "Z"));
    RETURN_IF(check_vec(Q, dtype, "Q"));
    RETURN_IF(check_vec(AZ, dtype, "AZ"));
    RETURN_IF(check_vec(AQ, dtype, "AQ"));
    RETURN_IF(check_vec(r, dtype, "r"));
    if (beta && !aligned(beta, 8)) return arg_error("beta misaligned");
    if (!W || !b1) return arg_error("W or b1 is NULL");
    RETURN_IF(check_work(work, work_bytes, s));
    hipStream_t st = as_stream(stream);
    double* part = static_cast<double*>(work);
    int G = 0;
    if (dtype == SSPCG_F32)
        RETURN_IF(launch_update_gram<float>(n, s, static_cast<const float*>(Z), static_cast<float*>(Q),
                                            static_cast<const float*>(AZ), static_cast<float*>(AQ),
                                            beta, static_cast<const float*>(r), nullptr, nullptr,
                                            ld, part, &G, nullptr, st));
    else
        RETURN_IF(launch_update_gram<double>(n, s, static_cast<const double*>(Z),
                                             static_cast<double*>(Q), static_cast<const double*>(AZ),
                                             static_cast<double*>(AQ), beta,
                                             static_cast<const double*>(r), nullptr, nullptr, ld,
                                             part, &G, nullptr, st));
    return launch_gram_out(s, 0, part, G, W, b1, st);
    API_CATCH
}

int sspcg_gram_rect(int64_t n, int32_t s, int32_t dtype, const void* Q, const void* AZ, int64_t ld,
                    double* B2, void* work, size_t work_bytes, sspcg_stream stream)
{
    API_TRY
    if (n < 1 || n >= ((int64_t)1 << 31)) return arg_error("n out of range");
    if (s < 1 || s > SSPCG_MAX_S) return arg_error("s must be in 1..16");
    if (ld < n) return arg_error("ld < n");
    RETURN_IF(check_dtype(nullptr, dtype));
    RETURN_IF(check_vec(Q, dtype, "Q"));
    RETURN_IF(check_vec(AZ, dtype, "AZ"));
    if (!B2) return arg_error("B2 is NULL");
    RETURN_IF(check_work(work, work_bytes, s));
    hipStream_t st = as_stream(stream);
    double* part = static_cast<double*>(work);
    int G = 0;
    if (dtype == SSPCG_F32)
        RETURN_IF(launch_gram_rect<float>(n, s, static_cast<const float*>(Q),
                                          static_cast<const float*>(AZ), ld, part, &G, nullptr, st));
    else
        RETURN_IF(launch_gram_rect<double>(n, s, static_cast<const double*>(Q),
                                           static_cast<const double*>(AZ), ld, part, &G, nullptr, st));
    return launch_gram_out(s, 1, part, G, B2, nullptr, st);
    API_CATCH
}

int sspcg_fgs(int32_t s, int32_t nrhs, const double* W, const double* B, int32_t sweeps,
              double sweep_tol, int32_t gram_solver, double* X, int32_t* status,
              sspcg_stream stream)
{
    API_TRY
    if (!(sweep_tol >= 0.0) || !(sweep_tol < 1.0)) return arg_error("sweep_tol must be in [0,1)");
    if (s < 1 || s > SSPCG_MAX_S) return arg_error("s must be in 1..16");
    if (nrhs < 1 || nrhs > 4096) return arg_error("nrhs must be in 1..4096");
    if (sweeps < 1 || sweeps > 100000) return arg_error("sweeps out of range");
    if (gram_solver != SSPCG_GRAM_FGS && gram_solver != SSPCG_GRAM_CHOLESKY)
        return arg_error("unknown gram solver");
    if (!W || !B || !X || !status) return arg_error("NULL pointer");
    return launch_fgs_direct(s, nrhs, W, B, sweeps, sweep_tol, gram_solver, X, status,
                             as_stream(stream));
    API_CATCH
}

int sspcg_xr_update(const sspcg_matrix* A, int32_t s, int32_t dtype, const void* Q, const void* AQ,
                    const double* alpha, int64_t ld, void* x, void* r, void* z1, double* rr,
                    void* work, size_t work_bytes, sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    RETURN_IF(check_dtype(A, dtype));
    if (s < 1 || s > SSPCG_MAX_S) return arg_error("s must be in 1..16");
    if (ld < A->n) return arg_error("ld < n");
    RETURN_IF(check_vec(Q, dtype, "Q"));
    RETURN_IF(check_vec(AQ, dtype, "AQ"));
    RETURN_IF(check_vec(x, dtype, "x"));
    RETURN_IF(check_vec(r, dtype, "r"));
    if (z1) RETURN_IF(check_vec(z1, dtype, "z1"));
    if (!alpha || !rr) return arg_error("alpha or rr is NULL");
    RETURN_IF(check_work(work, work_bytes, s));
    hipStream_t st = as_stream(stream);
    double* part = static_cast<double*>(work);
    int G = 0;
    if (dtype == SSPCG_F32)
        RETURN_IF(launch_xr<float>(A->n, s, static_cast<const float*>(Q), static_cast<const float*>(AQ),
                                   alpha, ld, static_cast<float*>(x), static_cast<float*>(r),
                                   A->dinv32, static_cast<float*>(z1), part, &G, nullptr, st));
    else
        RETURN_IF(launch_xr<double>(A->n, s, static_cast<const double*>(Q),
                                    static_cast<const double*>(AQ), alpha, ld, static_cast<double*>(x),
                                    static_cast<double*>(r), A->dinv, static_cast<double*>(z1), part,
                                    &G, nullptr, st));
    return launch_finish(part, 1, G, rr, st);
    API_CATCH
}

int sspcg_csr_value_grad(const sspcg_matrix* A, const double* lambda, const double* x, double* gval,
                         sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    RETURN_IF(check_vec(lambda, SSPCG_F64, "lambda"));
    RETURN_IF(check_vec(x, SSPCG_F64, "x"));
    RETURN_IF(check_vec(gval, SSPCG_F64, "gval"));
    return launch_value_grad(A, lambda, x, gval, as_stream(stream));
    API_CATCH
}

int sspcg_diffusion7_assemble(const sspcg_matrix* A, const double* theta, double* val,
                              sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    RETURN_IF(check_vec(theta, SSPCG_F64, "theta"));
    RETURN_IF(check_vec(val, SSPCG_F64, "val"));
    return launch_diffusion7_assemble(A, theta, val, as_stream(stream));
    API_CATCH
}

int sspcg_diffusion7_theta_grad(const sspcg_matrix* A, const double* theta, const double* gval,
                                double* gtheta, sspcg_stream stream)
{
    API_TRY
    RETURN_IF(check_matrix(A));
    RETURN_IF(check_vec(theta, SSPCG_F64, "theta"));
    RETURN_IF(check_vec(gval, SSPCG_F64, "gval"));
    RETURN_IF(check_vec(gtheta, SSPCG_F64, "gtheta"));
    return launch_diffusion7_theta_grad(A, theta, gval, gtheta, as_stream(stream));
    API_CATCH
}

int sspcg_stream_triad(int64_t n, const double* b, const double* c, double q, double* a,
                       sspcg_stream stream)
{
    API_TRY
    if (n < 0) return arg_error("n < 0");
    if (n == 0) return SSPCG_OK;
    for (const void* v : {(const void*)b, (const void*)c, (const void*)a})
        if (!v || !aligned(v, 16)) return arg_error("a, b and c must be 16-byte aligned");
    return launch_triad(n, b, c, q, a, as_stream(stream));
    API_CATCH
}

}  // extern "C"
