// Host drivers of the CG solves and the C ABI of hns.h.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>

#include "kernels.h"

// the line factors of a Dirichlet set (defined with the entry points below)
extern "C" {
static hns_status line_factors(hns_operator *op, int bit, const double **out);
static hns_status line_factors32(hns_operator *op, int bit, const float **out);
}

namespace hns {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

// ---------------------------------------------------------------------------
// Workspace: one per concurrent solve, pooled on the operator
// ---------------------------------------------------------------------------
struct Workspace {
    int64_t n = 0;
    bool mixed = false;
    void *block = nullptr;
    double *r = nullptr, *p = nullptr, *q = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    double *partials = nullptr;   // kPartTotal doubles
    double *z = nullptr;          // M^-1 r of the line / IC(0) preconditioner (on first use)
    double *y = nullptr;          // scratch of the IC(0) triangular solves (on first use)
    double *mf = nullptr;         // element results of a matrix-free product (on first use)
    double *p2 = nullptr;         // second direction buffer of the fused iterations (on first use)
    bool fused = false;           // the last chunk ran fused iterations (two timed kernels)
    Scalars *sc = nullptr;        // [0] FP64 / outer loop, [1] inner FP32 loop
    Scalars *host = nullptr;      // pinned mirror of sc[0..1]
    std::vector<hipEvent_t> ev;   // timing events, a (start, end) pair per kernel of an iteration
    uint32_t token = 0;           // last iteration tag handed out (IterArgs::token)
    bool borrowed = false;        // buffers lent by the caller (nothing freed, no timing events)

    static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

    static size_t bytes_for(int64_t n, bool mixed)
    {
        size_t b = 3 * al(n * sizeof(double));
        if (mixed) b += 4 * al(n * sizeof(float));
        b += al(kPartTotal * sizeof(double)) + al(2 * sizeof(Scalars));
        return b;
    }

    // points the buffers into `base` (bytes_for(n, mixed) bytes, 256-byte
    // aligned, plus al(8 n) more for z when with_z)
    void carve(char *c, bool with_z)
    {
        r = (double *)c, c += al(n * sizeof(double));
        p = (double *)c, c += al(n * sizeof(double));
        q = (double *)c, c += al(n * sizeof(double));
        if (mixed) {
            r32 = (float *)c, c += al(n * sizeof(float));
            p32 = (float *)c, c += al(n * sizeof(float));
            q32 = (float *)c, c += al(n * sizeof(float));
            d32 = (float *)c, c += al(n * sizeof(float));
        }
        partials = (double *)c, c += al(kPartTotal * sizeof(double));
        sc = (Scalars *)c, c += al(2 * sizeof(Scalars));
        if (with_z) z = (double *)c;
    }

    hns_status allocate(int64_t n_, bool mixed_)
    {
        n = n_;
        mixed = mixed_;
        hipError_t e = hipMalloc(&block, bytes_for(n, mixed));
        if (e != hipSuccess) {
            block = nullptr;
            set_error("workspace allocation of %zu bytes failed: %s", bytes_for(n, mixed),
                      hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        carve((char *)block, false);
        HNS_TRY_HIP(hipMemset(sc, 0, 2 * sizeof(Scalars)));
        HNS_TRY_HIP(hipHostMalloc((void **)&host, 2 * sizeof(Scalars), hipHostMallocDefault));
        memset(host, 0, 2 * sizeof(Scalars));
        return HNS_OK;
    }

    // buffers lent by the caller: device memory `base` as carve() lays it
    // out, and a host mirror of the two scalar blocks
    void borrow(int64_t n_, bool mixed_, void *base, bool with_z, Scalars *host_mirror,
                uint32_t token0)
    {
        n = n_;
        mixed = mixed_;
        borrowed = true;
        carve((char *)base, with_z);
        host = host_mirror;
        memset(host, 0, 2 * sizeof(Scalars));
        token = token0;
    }

    hns_status ensure_events(size_t count)
    {
        while (ev.size() < count) {
            hipEvent_t e;
            HNS_TRY_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        return HNS_OK;
    }

    hns_status ensure_z()
    {
        if (z) return HNS_OK;
        hipError_t e = hipMalloc(&z, n * sizeof(double));
        if (e != hipSuccess) {
            z = nullptr;
            set_error("allocation of the preconditioned residual failed: %s",
                      hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        return HNS_OK;
    }

    hns_status ensure_y()
    {
        if (y) return HNS_OK;
        hipError_t e = hipMalloc(&y, n * sizeof(double));
        if (e != hipSuccess) {
            y = nullptr;
            set_error("allocation of the triangular-solve scratch failed: %s",
                      hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        return HNS_OK;
    }

    hns_status ensure_mf(size_t count)
    {
        if (mf || count == 0) return HNS_OK;
        hipError_t e = hipMalloc(&mf, count * sizeof(double));
        if (e != hipSuccess) {
            mf = nullptr;
            set_error("allocation of the matrix-free element results failed: %s",
                      hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        return HNS_OK;
    }

    hns_status ensure_p2()
    {
        if (p2) return HNS_OK;
        hipError_t e = hipMalloc(&p2, n * sizeof(double));
        if (e != hipSuccess) {
            p2 = nullptr;
            set_error("allocation of the second direction buffer failed: %s",
                      hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        return HNS_OK;
    }

    ~Workspace()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (borrowed) return;
        if (p2) (void)hipFree(p2);
        if (z) (void)hipFree(z);
        if (y) (void)hipFree(y);
        if (mf) (void)hipFree(mf);
        if (block) (void)hipFree(block);
        if (host) (void)hipHostFree(host);
    }
};

static hns_status acquire_ws(hns_operator *op, bool mixed, Workspace **out)
{
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> g(op->ws_mutex);
        for (size_t i = 0; i < op->ws_free.size(); ++i) {
            if (op->ws_free[i]->mixed || !mixed) {
                w = op->ws_free[i];
                op->ws_free.erase(op->ws_free.begin() + i);
                break;
            }
        }
    }
    if (!w) {
        w = new Workspace();
        hns_status st = w->allocate(op->n, mixed);
        if (st != HNS_OK) {
            delete w;
            return st;
        }
    }
    // a matrix-free operator's products need their element scratch
    hns_status st = w->ensure_mf(op->A.mf_scratch());
    if (st != HNS_OK) {
        std::lock_guard<std::mutex> g(op->ws_mutex);
        op->ws_free.push_back(w);
        return st;
    }
    *out = w;
    return HNS_OK;
}

static void release_ws(hns_operator *op, Workspace *w)
{
    std::lock_guard<std::mutex> g(op->ws_mutex);
    op->ws_free.push_back(w);
}

// copy the two scalar blocks host <-> device on the solve's stream
static hns_status push_scalars(Workspace *w, int which, hipStream_t s)
{
    HNS_TRY_HIP(hipMemcpyAsync(w->sc + which, w->host + which, sizeof(Scalars),
                               hipMemcpyHostToDevice, s));
    return HNS_OK;
}

static hns_status pull_scalars(Workspace *w, int which, hipStream_t s)
{
    HNS_TRY_HIP(hipMemcpyAsync(w->host + which, w->sc + which, sizeof(Scalars),
                               hipMemcpyDeviceToHost, s));
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

static void reset_scalars(Scalars &h, double tol)
{
    memset(&h, 0, sizeof(Scalars));
    h.tol2 = tol * tol;
}

// ---------------------------------------------------------------------------
// Solve drivers
// ---------------------------------------------------------------------------
struct SolveCtx {
    hns_operator *op;
    int bit;
    bool singular;
    const double *b;
    double *x;
    double tol;
    int max_iter;
    hipStream_t s;
    Workspace *w;
    const double *lfac = nullptr;   // line-preconditioner factors of this mask (FP64 solves)
    const IC0Dev *ic = nullptr;     // IC(0) factor of this mask (FP64 solves)
    const float *lfac32 = nullptr;  // FP32 line factors (inner iterations of mixed solves)
    bool scaled = false;            // point Jacobi as CG on the Jacobi-scaled operator
};

// Enqueue `count` CG iterations of one recurrence.  parity0 is the number of
// iterations executed since its last (re)start: it selects the rho slot of
// each iteration.  Iterations enqueued after the stop flag was raised are
// no-ops on the device, so the caller re-derives parity from the device's
// iteration counter after each chunk.
// Chunks of a recurrence that the single-workgroup kernel runs (latency-bound
// sizes: point Jacobi, FP64 or FP32, not while per-kernel timing is on).  It
// stops by itself at the tolerance, so its chunks may be long: one launch and
// one host read instead of one per check_every iterations.
constexpr int kSmallChunk = 1024;

static bool small_chunks(const hns_operator *op, const Workspace *w, Prec prec, const void *lfac,
                         const IC0Dev *ic, bool scaled)
{
    const int period = w->borrowed ? 0 : op->profile;
    return !lfac && !ic && !scaled && period <= 0 && op->n <= op->small_n &&
           op->A.fmt != HNS_MATRIX_FREE && (prec == Prec::F64 || prec == Prec::F32);
}

// Fused scaled iterations (two launches each, the direction update inside the
// next product): automatic ("fuse_dir" = -1) while one vector of the
// recurrence is at most 4 MiB.  Measured on the basin operators (15-point
// stencil, MI355X): 1.04-1.27x per iteration up to that size, where the
// launch and the vector pass saved outweigh the neighbours' r and p loads
// the product adds; even or slower beyond it (FP64 0.94x at 1.39M rows).
constexpr size_t kFuseBytes = size_t(4) << 20;

static bool fuse_wanted(const hns_operator *op, bool fp32)
{
    if (op->fuse_dir >= 0) return op->fuse_dir == 1;
    return (size_t)op->n * (fp32 ? sizeof(float) : sizeof(double)) <= kFuseBytes;
}

static hns_status enqueue_iterations(hns_operator *op, Workspace *w, Prec prec, int bit, void *x,
                                     void *r, void *p, void *q, const void *dinv, Scalars *sc,
                                     int count, int parity0, hipStream_t s,
                                     const void *lfac = nullptr, const IC0Dev *ic = nullptr,
                                     bool scaled = false)
{
    const int period = w->borrowed ? 0 : op->profile;
    if (period > 0) HNS_TRY(w->ensure_events(6 * (size_t)count));
    IterArgs a{&op->A, prec, op->n, x, r, p, q, dinv, op->bc, bit, sc, w->partials};
    a.mf = w->mf;
    if (scaled) {
        a.A = &op->S;
        a.dinv = nullptr;
        a.wjac = op->jac_w;
    }
    if (lfac) {
        a.lfac = lfac;
        a.z = w->z;
        a.line_len = op->line_len;
    }
    if (ic) {
        a.ic = ic;
        a.z = w->z;
        a.y = w->y;
    }
    // latency-bound sizes: the whole chunk in one workgroup
    if (small_chunks(op, w, prec, lfac, ic, scaled)) return launch_cg_small(a, parity0, count, s);
    // sampled: the iteration in the middle of each period window, so a chunk's
    // first iteration (launched after the host's read of the previous chunk,
    // on an idle GPU) is never timed unless every iteration is
    w->fused = scaled && fuse_wanted(op, prec == Prec::F32) && !w->borrowed && scaled_fusable(a);
    if (w->fused) {
        // two launches per iteration, p alternating between p and p2
        if (count <= 0) return HNS_OK;
        HNS_TRY(w->ensure_p2());
        void *bufs[2] = {p, w->p2};
        uint32_t prev_token = 0;
        int prev_parity = 0;
        for (int it = 0; it < count; ++it) {
            const bool timed = period > 0 && (it % period) == period / 2;
            if (++w->token == 0) w->token = 1;
            a.token = w->token;
            const int parity = (parity0 + it) & 1;
            HNS_TRY(launch_scaled_fused_step(a, it == 0 ? nullptr : bufs[(it - 1) & 1],
                                             bufs[it & 1], prev_token, prev_parity, parity, s,
                                             timed ? &w->ev[6 * it] : nullptr));
            prev_token = a.token;
            prev_parity = parity;
        }
        return launch_scaled_fused_close(a, bufs[(count - 1) & 1], prev_token, prev_parity, s);
    }
    for (int it = 0; it < count; ++it) {
        const bool timed = period > 0 && (it % period) == period / 2;
        if (++w->token == 0) w->token = 1;   // unique per workspace, never 0
        a.token = w->token;
        HNS_TRY(launch_iteration(a, (parity0 + it) & 1, s, timed ? &w->ev[6 * it] : nullptr));
    }
    return HNS_OK;
}

// After the chunk has completed: add the kernel durations of the sampled
// iterations among the first `done` (those that did work) to the operator's
// counters.
static hns_status account_iterations(hns_operator *op, Workspace *w, bool fp32, int done)
{
    const int period = w->borrowed ? 0 : op->profile;
    if (period <= 0 || done <= 0) return HNS_OK;
    const int base = fp32 ? 3 : 0;
    const int kernels = w->fused ? 2 : 3;   // fused: product (with the direction update), update
    for (int it = period / 2; it < done; it += period)
        for (int k = 0; k < kernels; ++k) {
            float ms = 0.0f;
            HNS_TRY_HIP(hipEventElapsedTime(&ms, w->ev[6 * it + 2 * k], w->ev[6 * it + 2 * k + 1]));
            op->prof_ms[base + k] += ms;
            op->prof_count[base + k] += 1;
        }
    return HNS_OK;
}

// Run chunks of one recurrence (scalar block `which`) until its stop flag is
// raised or the iteration budget is spent.  *since_start counts the
// iterations executed since the recurrence's last (re)start.
static hns_status run_chunks(const SolveCtx &c, int which, Prec prec, void *x, void *r, void *p,
                             void *q, const void *dinv, int *since_start)
{
    hns_operator *op = c.op;
    Workspace *w = c.w;
    Scalars &h = w->host[which];
    while (h.stop == 0) {
        const int left = c.max_iter - h.iter;
        if (left <= 0) break;
        const void *lf = prec == Prec::F64   ? (const void *)c.lfac
                         : prec == Prec::F32 ? (const void *)c.lfac32
                                             : nullptr;
        const int per = small_chunks(op, w, prec, lf, prec == Prec::F64 ? c.ic : nullptr, c.scaled)
                            ? std::max(op->check_every, kSmallChunk)
                            : op->check_every;
        const int chunk = left < per ? left : per;
        const int before = h.iter;
        HNS_TRY(enqueue_iterations(op, w, prec, c.bit, x, r, p, q, dinv, w->sc + which, chunk,
                                   *since_start, c.s, lf, prec == Prec::F64 ? c.ic : nullptr,
                                   c.scaled));
        HNS_TRY(pull_scalars(w, which, c.s));
        *since_start += h.iter - before;
        HNS_TRY(account_iterations(op, w, prec == Prec::F32, h.iter - before));
    }
    return HNS_OK;
}

// r = b - A x in FP64 (projected in the pure-Neumann case) into w->r; sum of
// squares into sc[0].rr, |b|^2 into sc[0].bb.
static hns_status true_residual_fp64(const SolveCtx &c)
{
    hns_operator *op = c.op;
    Workspace *w = c.w;
    HNS_TRY(launch_spmv_plain(op->A, false, c.x, w->q, op->bc, c.bit, c.s, w->mf));
    HNS_TRY(launch_residual(op->n, c.b, w->q, w->r, op->bc, c.bit, c.singular, w->sc,
                            w->partials, c.s));
    HNS_TRY(launch_project_norm(op->n, w->r, c.singular, w->sc, w->partials, c.s));
    return HNS_OK;
}

// Start of a solve: statistics of b, Dirichlet entries of x zeroed, then the
// FP64 true residual, and one read of the scalars for all of them.
static hns_status begin_solve(const SolveCtx &c, hns_solve_info *info)
{
    hns_operator *op = c.op;
    Workspace *w = c.w;
    reset_scalars(w->host[0], c.tol);
    HNS_TRY(push_scalars(w, 0, c.s));
    HNS_TRY(launch_bstats(op->n, c.b, op->bc, c.bit, w->sc, w->partials, c.s));
    HNS_TRY(launch_prepare_x(op->n, c.x, op->bc, c.bit, false, c.s));
    HNS_TRY(true_residual_fp64(c));
    HNS_TRY(pull_scalars(w, 0, c.s));
    if (w->host[0].nonfinite > 0) {
        set_error("right-hand side has %.0f non-finite entries", w->host[0].nonfinite);
        return HNS_ERR_INVALID;
    }
    info->removed_mean = c.singular ? w->host[0].sumb / (double)op->n : 0.0;
    return HNS_OK;
}

static hns_status finish_solve(const SolveCtx &c, hns_solve_info *info, hns_status status)
{
    hns_operator *op = c.op;
    Workspace *w = c.w;
    const Scalars &h = w->host[0];
    info->relres_true = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    if (status >= 0 && c.singular) {
        HNS_TRY(launch_normalise(op->n, c.x, op->lumped, op->lumped_sum, w->sc, w->partials,
                                 c.s));
    }
    HNS_TRY_HIP(hipStreamSynchronize(c.s));
    info->status = status;
    return status;
}

// A single-right-hand-side solve advanced one chunk of iterations at a time:
// hns_solve runs it to the end, a per-slot batch session interleaves several
// on one stream.  begin() computes the statistics of b and the first FP64
// true residual; enqueue() starts a recurrence segment when one is due and
// enqueues one chunk of CG iterations and the read of its scalars; after()
// runs once the stream has been waited for: when the recurrence stopped (or
// the iteration cap was reached) it recomputes the FP64 true residual and
// decides between the end of the solve, a restart and a residual
// replacement; end() normalises and reports.
//
// Recurrences:
//  - FP64 vectors (prec F64, or F32Store: FP32 matrix and diagonal): whenever
//    the recursive residual has fallen below the tolerance (F64) or by
//    `replace_drop` (F32Store), b - A x is recomputed with the FP64 matrix;
//    at the tolerance the solve ends if it agrees, else the recurrence
//    continues from it (a full restart in F64, a residual replacement that
//    keeps the direction in F32Store).
//  - mixed: one FP32 recurrence (matrix, vectors and diagonal in FP32) keeps
//    its search direction across refinement steps; whenever its recursive
//    residual has dropped by `replace_drop` since the last FP64 residual, the
//    FP32 iterate is added to the FP64 solution, the true residual is
//    recomputed in FP64, and the recurrence continues from it.
struct ChunkedSolve {
    SolveCtx c;
    hns_solve_info *info = nullptr;
    bool mixed = false;
    Prec prec = Prec::F64;       // FP64-vector recurrence: F64 or F32Store
    bool finished = false;
    bool zero_b = false;
    hns_status status = HNS_NOT_CONVERGED;
    bool fresh = true;
    int since = 0, replacements = 0, stalls = 0, floor_checks = 0, before = 0;
    double tol2 = 0, drop2 = 0, rr_true = 0, bb = 0, rr_prev = 0, rr_best = INFINITY;
    const void *dinv = nullptr;

    int which() const { return mixed ? 1 : 0; }

    hns_status begin()
    {
        hns_operator *op = c.op;
        Workspace *w = c.w;
        info->outer_iterations = 0;
        HNS_TRY(begin_solve(c, info));
        Scalars &h = w->host[0];
        if (!(h.bb > 0.0)) {  // b = 0
            HNS_TRY(launch_prepare_x(op->n, c.x, nullptr, -1, true, c.s));
            zero_b = true;
            status = HNS_OK;
            finished = true;
            return HNS_OK;
        }
        tol2 = c.tol * c.tol;
        if (mixed) {
            const double drop = replace_drop_of(
                op, small_chunks(op, w, Prec::F32, c.lfac32, nullptr, c.scaled));
            drop2 = drop * drop;
            rr_prev = h.rr;
            if (!(h.rr > tol2 * h.bb)) {
                status = HNS_OK;
                finished = true;
            }
        } else {
            const bool storage = (prec == Prec::F32Store);
            dinv = storage ? (const void *)op->dinv32 : (const void *)op->dinv;
            drop2 = storage ? replace_drop_of(op, false) * replace_drop_of(op, false) : 0.0;
            rr_true = h.rr;
            bb = h.bb;
            rr_prev = h.rr;
            if (!(rr_true > tol2 * bb)) {
                status = HNS_OK;
                finished = true;
            }
        }
        return HNS_OK;
    }

    // start of a recurrence segment from the FP64 true residual in w->r
    hns_status start_segment()
    {
        hns_operator *op = c.op;
        Workspace *w = c.w;
        Scalars &h = w->host[0];
        if (mixed) {
            Scalars &hi = w->host[1];
            const double thr2 = std::max(drop2, tol2 * h.bb / h.rr);
            if (!c.scaled) HNS_TRY(launch_cast(op->n, w->r, w->r32, w->d32, c.s));
            reset_scalars(hi, 0.0);
            hi.tol2 = thr2;
            hi.bb = h.rr;
            hi.iter = info->iterations;
            HNS_TRY(push_scalars(w, 1, c.s));
            if (c.scaled)   // r32 = (float)(D^-1/2 r_A), p = r32, correction d32 = 0
                HNS_TRY(launch_scale_in(op->n, Prec::F32, w->r, w->r32, w->p32, w->d32,
                                        op->jac_s, w->sc + 1, w->partials, c.s));
            else if (c.lfac32)
                HNS_TRY(launch_init_line(op->n, op->line_len, w->r32, w->p32, c.lfac32, false,
                                         false, w->sc + 1, w->partials, c.s));
            else
                HNS_TRY(launch_init_dir(op->n, Prec::F32, w->r32, w->p32, op->dinv32, false,
                                        false, w->sc + 1, w->partials, c.s));
        } else {
            if (prec == Prec::F32Store) {  // next stop: residual down by `drop` (or at tol)
                h.tol2 = std::max(tol2 * bb / rr_true, drop2);
                h.bb = rr_true;
            } else {
                h.tol2 = tol2;
                h.bb = bb;
            }
            h.stop = 0;
            HNS_TRY(push_scalars(w, 0, c.s));
            if (c.scaled)   // r = D^-1/2 r_A in place, p = r, correction dx = 0
                HNS_TRY(launch_scale_in(op->n, Prec::F64, w->r, w->r, w->p, w->z, op->jac_s,
                                        w->sc, w->partials, c.s));
            else if (c.ic && prec == Prec::F64)
                HNS_TRY(launch_init_ic0(op->n, *c.ic, w->r, w->p, w->z, w->y, w->sc,
                                        w->partials, c.s));
            else if (c.lfac && prec == Prec::F64)
                HNS_TRY(launch_init_line(op->n, op->line_len, w->r, w->p, c.lfac, false, false,
                                         w->sc, w->partials, c.s));
            else
                HNS_TRY(launch_init_dir(op->n, prec, w->r, w->p, dinv, false, false, w->sc,
                                        w->partials, c.s));
        }
        // no read here: if the start already stopped the recurrence
        // (converged, non-finite), the chunk's kernels exit at once and its
        // read reports it
        since = 0;
        fresh = false;
        return HNS_OK;
    }

    // At most `budget` (and `check_every`) iterations, then the read of the
    // recurrence's scalars into the pinned mirror; nothing is waited for.
    hns_status enqueue(int budget)
    {
        hns_operator *op = c.op;
        Workspace *w = c.w;
        if (fresh) HNS_TRY(start_segment());
        Scalars &hr = w->host[which()];
        before = hr.iter;
        const Prec p = mixed ? Prec::F32 : prec;
        const void *lf = p == Prec::F64   ? (const void *)c.lfac
                         : p == Prec::F32 ? (const void *)c.lfac32
                                          : nullptr;
        const int per = small_chunks(op, w, p, lf, p == Prec::F64 ? c.ic : nullptr, c.scaled)
                            ? std::max(op->check_every, kSmallChunk)
                            : op->check_every;
        const int chunk = std::min({c.max_iter - hr.iter, per, budget});
        if (chunk > 0 && hr.stop == 0) {
            void *x = mixed ? (void *)w->d32 : c.scaled ? (void *)w->z : (void *)c.x;
            void *r = mixed ? (void *)w->r32 : (void *)w->r;
            void *pp = mixed ? (void *)w->p32 : (void *)w->p;
            void *q = mixed ? (void *)w->q32 : (void *)w->q;
            const void *di = c.scaled ? nullptr : mixed ? (const void *)op->dinv32 : dinv;
            HNS_TRY(enqueue_iterations(op, w, p, c.bit, x, r, pp, q, di, w->sc + which(), chunk,
                                       since, c.s, lf, p == Prec::F64 ? c.ic : nullptr,
                                       c.scaled));
        }
        HNS_TRY_HIP(hipMemcpyAsync(&w->host[which()], w->sc + which(), sizeof(Scalars),
                                   hipMemcpyDeviceToHost, c.s));
        return HNS_OK;
    }

    hns_status after()
    {
        hns_operator *op = c.op;
        Workspace *w = c.w;
        Scalars &h = w->host[0];
        Scalars &hr = w->host[which()];
        since += hr.iter - before;
        HNS_TRY(account_iterations(op, w, mixed, hr.iter - before));
        if (hr.stop == 0 && hr.iter < c.max_iter) return HNS_OK;   // still running
        if (mixed) {
            Scalars &hi = w->host[1];
            info->iterations = hi.iter;
            const bool broke = (hi.stop == 2);
            // collect the FP32 correction and recompute the true residual in FP64
            if (c.scaled)
                HNS_TRY(launch_scale_out(op->n, Prec::F32, c.x, w->d32, op->jac_s, c.s));
            else
                HNS_TRY(launch_accumulate(op->n, c.x, w->d32, c.s));
            HNS_TRY(true_residual_fp64(c));
            HNS_TRY(pull_scalars(w, 0, c.s));
            ++replacements;
            if (h.rr <= tol2 * h.bb) return done(HNS_OK);
            if (hi.stop != 1 && !broke) return done(HNS_NOT_CONVERGED);  // budget spent
            stalls = (h.rr > 0.81 * rr_prev) ? stalls + 1 : 0;
            if (stalls >= 3) {
                set_error("mixed-precision refinement stagnated at relative residual %g",
                          std::sqrt(h.rr / h.bb));
                return done(HNS_NOT_CONVERGED);
            }
            rr_prev = h.rr;
            if (broke) {
                if (stalls > 0) {
                    set_error("FP32 CG broke down without progress after %d iterations",
                              hi.iter);
                    return done(HNS_ERR_BREAKDOWN);
                }
                fresh = true;  // new direction from the new true residual
                return HNS_OK;
            }
            HNS_TRY(launch_set_threshold(w->sc + 1, std::max(drop2, tol2 * h.bb / h.rr), h.rr,
                                         c.s));
            if (c.scaled)
                HNS_TRY(launch_replace_scaled(op->n, w->r, w->r32, w->p32, op->jac_s, w->sc + 1,
                                              w->partials, (since - 1) & 1, c.s));
            else if (c.lfac32)
                HNS_TRY(launch_replace_line(op->n, op->line_len, w->r, w->r32, (float *)w->z,
                                            w->p32, c.lfac32, w->sc + 1, w->partials,
                                            (since - 1) & 1, op->A.vec_packs(), c.s));
            else
                HNS_TRY(launch_replace_residual(op->n, Prec::F32, w->r, w->r32, w->p32,
                                                op->dinv32, w->sc + 1, w->partials,
                                                (since - 1) & 1, c.s));
            hi.stop = 0;
            return HNS_OK;
        }
        const bool storage = (prec == Prec::F32Store);
        if (c.scaled) HNS_TRY(launch_scale_out(op->n, Prec::F64, c.x, w->z, op->jac_s, c.s));
        info->iterations = h.iter;
        if (h.stop == 2) {
            set_error("CG breakdown after %d iterations (p^T A p = %g)", h.iter, h.gamma);
            return done(HNS_ERR_BREAKDOWN);
        }
        const bool hit = (h.stop == 1);
        // true residual, FP64 matrix
        const int iters = h.iter;
        HNS_TRY(true_residual_fp64(c));
        HNS_TRY(pull_scalars(w, 0, c.s));
        h.iter = iters;
        rr_true = h.rr;
        ++replacements;
        if (rr_true <= tol2 * bb) return done(HNS_OK);
        if (!hit || h.iter >= c.max_iter) return done(HNS_NOT_CONVERGED);  // budget spent
        if (!storage) {
            // the rounding floor: three failed checks in a row that do not
            // halve the smallest true residual seen at a check end the solve
            floor_checks = (rr_true > 0.25 * rr_best) ? floor_checks + 1 : 0;
            rr_best = std::min(rr_best, rr_true);
            if (floor_checks >= 3) {
                set_error("true residual stalled at %g, above the tolerance (rounding floor)",
                          std::sqrt(rr_true / bb));
                return done(HNS_NOT_CONVERGED);
            }
            fresh = true;  // restart from the true residual
            return HNS_OK;
        }
        stalls = (rr_true > 0.81 * rr_prev) ? stalls + 1 : 0;
        if (stalls >= 3) {
            set_error("FP32-storage refinement stagnated at relative residual %g",
                      std::sqrt(rr_true / bb));
            return done(HNS_NOT_CONVERGED);
        }
        rr_prev = rr_true;
        // residual replacement: keep the direction, continue from r_true
        h.tol2 = std::max(tol2 * bb / rr_true, drop2);
        HNS_TRY(launch_set_threshold(w->sc, h.tol2, rr_true, c.s));
        HNS_TRY(launch_replace_residual(op->n, prec, w->r, nullptr, w->p, dinv, w->sc,
                                        w->partials, (since - 1) & 1, c.s));
        h.stop = 0;
        return HNS_OK;
    }

    hns_status done(hns_status st)
    {
        status = st;
        finished = true;
        return HNS_OK;
    }

    hns_status end()
    {
        if (!zero_b) {
            if (mixed) {
                info->outer_iterations = replacements;
            } else {
                // report the FP64 residual against |b|^2
                Scalars &h = c.w->host[0];
                h.bb = bb;
                h.rr = rr_true;
                info->outer_iterations = (prec == Prec::F32Store) ? replacements : 1;
            }
        }
        return finish_solve(c, info, status);
    }
};

static hns_status run_to_end(ChunkedSolve &cs)
{
    HNS_TRY(cs.begin());
    while (!cs.finished) {
        HNS_TRY(cs.enqueue(INT_MAX));
        HNS_TRY_HIP(hipStreamSynchronize(cs.c.s));
        HNS_TRY(cs.after());
    }
    return cs.end();
}

// Classic mixed-precision refinement: each FP64 correction step solves
// A32 d = r / |r| by a fresh FP32 CG to `inner_tol`, then x += |r| d.
static hns_status solve_mixed_restart(const SolveCtx &c, hns_solve_info *info)
{
    hns_operator *op = c.op;
    Workspace *w = c.w;
    HNS_TRY(begin_solve(c, info));
    Scalars &h = w->host[0];
    Scalars &hi = w->host[1];
    info->outer_iterations = 0;
    if (!(h.bb > 0.0)) {
        HNS_TRY(launch_prepare_x(op->n, c.x, nullptr, -1, true, c.s));
        return finish_solve(c, info, HNS_OK);
    }
    const double tol2 = c.tol * c.tol;
    hns_status status = HNS_NOT_CONVERGED;
    int total_inner = 0, outer = 0;
    double rr_prev = h.rr;
    for (;;) {
        if (h.rr <= tol2 * h.bb) {
            status = HNS_OK;
            break;
        }
        if (outer >= op->max_outer || total_inner >= c.max_iter) break;
        if (outer > 0 && h.rr > 0.25 * rr_prev) {
            set_error("refinement stagnated at relative residual %g", std::sqrt(h.rr / h.bb));
            break;
        }
        rr_prev = h.rr;
        ++outer;
        HNS_TRY(launch_cast_scaled(op->n, w->r, w->r32, w->d32, w->sc, c.s));
        reset_scalars(hi, op->inner_tol);
        HNS_TRY(push_scalars(w, 1, c.s));
        HNS_TRY(launch_init_dir(op->n, Prec::F32, w->r32, w->p32, op->dinv32, false, true,
                                w->sc + 1, w->partials, c.s));
        int since = 0;
        SolveCtx ci = c;
        ci.max_iter = c.max_iter - total_inner;
        HNS_TRY(run_chunks(ci, 1, Prec::F32, w->d32, w->r32, w->p32, w->q32, op->dinv32, &since));
        total_inner += hi.iter;
        if (hi.stop == 2 && hi.iter == 0) {
            status = HNS_ERR_BREAKDOWN;
            set_error("FP32 inner CG broke down at its first iteration");
            break;
        }
        HNS_TRY(launch_correct(op->n, c.x, w->d32, w->sc, c.s));
        HNS_TRY(true_residual_fp64(c));
        HNS_TRY(pull_scalars(w, 0, c.s));
    }
    info->iterations = total_inner;
    info->outer_iterations = outer;
    return finish_solve(c, info, status);
}

static hns_status solve_fp64(const SolveCtx &c, hns_solve_info *info, Prec prec = Prec::F64)
{
    ChunkedSolve cs;
    cs.c = c;
    cs.info = info;
    cs.prec = prec;
    return run_to_end(cs);
}

static hns_status solve_mixed(const SolveCtx &c, hns_solve_info *info)
{
    switch (c.op->mixed_variant) {
    case 1: return solve_mixed_restart(c, info);
    case 2: return solve_fp64(c, info, Prec::F32Store);
    default: {
        ChunkedSolve cs;
        cs.c = c;
        cs.info = info;
        cs.mixed = true;
        return run_to_end(cs);
    }
    }
}

// The Jacobi-scaled operator D^-1/2 A D^-1/2 (unit diagonal, upper diagonals
// only; FP32 values too when A keeps them), s = D^-1/2 and w = diag(A) in
// FP32, computed on the device on first use.
static hns_status scaled_operator(hns_operator *op)
{
    std::lock_guard<std::mutex> g(op->line_mutex);
    if (op->S.dia) return HNS_OK;
    const DevMatrix &A = op->A;
    const int64_t n = op->n;
    DevMatrix S;
    S.n = n;
    S.nnz = A.nnz;
    S.fmt = HNS_FMT_SDIA;
    S.ndiag = A.ndiag;
    for (int k = 0; k < kMaxDiagWide; ++k) S.off[k] = A.off[k];
    S.unit = true;
    S.spmv_it64 = A.spmv_it64;
    S.spmv_it32 = A.spmv_it32;
    S.vec_it = A.vec_it;
    S.spmv_rows64 = A.spmv_rows64;
    double *sh = nullptr;
    float *w = nullptr;
    auto fail = [&](hipError_t e, const char *what) {
        S.release();
        if (sh) (void)hipFree(sh);
        if (w) (void)hipFree(w);
        set_error("Jacobi scaling: %s failed: %s", what, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
    };
    const size_t vals = (size_t)A.ndiag * n;
    hipError_t e = hipMalloc(&S.dia, vals * sizeof(double));
    if (e != hipSuccess) return fail(e, "allocation");
    if (A.dia32) {
        e = hipMalloc(&S.dia32, vals * sizeof(float));
        if (e != hipSuccess) return fail(e, "allocation");
    }
    e = hipMalloc(&sh, n * sizeof(double));
    if (e != hipSuccess) return fail(e, "allocation");
    e = hipMalloc(&w, n * sizeof(float));
    if (e != hipSuccess) return fail(e, "allocation");
    hns_status st = launch_jacobi_scale(n, A.ndiag, A.off, A.dia, sh, w, S.dia, S.dia32, nullptr);
    if (st == HNS_OK) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return fail(e, "scaling kernels");
    } else {
        S.release();
        (void)hipFree(sh);
        (void)hipFree(w);
        return st;
    }
    op->S = S;
    op->jac_s = sh;
    op->jac_w = w;
    return HNS_OK;
}

// ---------------------------------------------------------------------------
// Per-slot batch sessions: every slot runs its own single-right-hand-side
// recurrence (the chunked solve of hns_solve, point Jacobi, on the
// Jacobi-scaled operator where hns_solve would use it), and an advance
// enqueues one chunk of every running slot before it waits once.  For one or
// two slots the shared operator read of the multi-right-hand-side block saves
// nothing next to the vector traffic (two columns move as many bytes as two
// single recurrences), while a half-empty block still moves both columns.
// ---------------------------------------------------------------------------
struct SlotSession {
    hns_operator *op = nullptr;
    int K = 0;
    bool mixed = false;
    bool scaled = false;
    bool line = false;   // the vertical-line block preconditioner (set_param "precond" = 1)
    struct Slot {
        int state = 0;   // 0 free, 1 running, 2 finished
        double *b = nullptr, *x = nullptr;
        Workspace *w = nullptr;
        ChunkedSolve cs;
        hns_solve_info info{};
    };
    std::vector<Slot> slots;
};

bool slot_session_wanted(const hns_operator *op, int capacity)
{
    return op->session_mode == 2 || (op->session_mode == 0 && capacity <= 2);
}

static bool session_scaled(const hns_operator *op, bool mixed)
{
    return op->jacobi_scaling && op->A.fmt == HNS_FMT_SDIA && op->A.ndiag >= 1 &&
           op->A.ndiag <= kMaxDiag && op->n > op->small_n && (!mixed || op->A.dia32);
}

// line blocks in a per-slot session: "precond" = 1 (a per-slot HNS_MIXED
// solve is always mixed_variant 0, which runs them); IC(0) sessions keep point
// Jacobi
static bool session_line(const hns_operator *op)
{
    return op->precond == 1;
}

size_t slot_session_bytes(const hns_operator *op, int capacity, bool mixed)
{
    const size_t n = (size_t)op->n;
    size_t per = Workspace::bytes_for(op->n, mixed) + 2 * ((n + 31) & ~size_t(31)) * sizeof(double) +
                 op->A.mf_scratch() * sizeof(double);
    if (session_line(op))
        per += n * sizeof(double);                                          // z
    else if (session_scaled(op, mixed) && !mixed)
        per += n * sizeof(double);                                          // scaled correction
    if (!session_line(op) && session_scaled(op, mixed) && fuse_wanted(op, mixed))
        per += n * sizeof(double);                                          // second p buffer
    return per * (size_t)capacity + 256;
}

void slot_session_close(SlotSession *ss)
{
    if (!ss) return;
    (void)hipDeviceSynchronize();
    for (auto &sl : ss->slots) {
        if (sl.b) (void)hipFree(sl.b);
        delete sl.w;
    }
    delete ss;
}

hns_status slot_session_open(hns_operator *op, int capacity, bool mixed, SlotSession **out)
{
    *out = nullptr;
    SlotSession *ss = new SlotSession();
    ss->op = op;
    ss->K = capacity;
    ss->mixed = mixed;
    ss->line = session_line(op);
    ss->scaled = !ss->line && session_scaled(op, mixed);
    ss->slots.resize(capacity);
    auto fail = [&](hns_status st) {
        slot_session_close(ss);
        return st;
    };
    if (ss->scaled) {
        const hns_status st = scaled_operator(op);
        if (st != HNS_OK) return fail(st);
        if (mixed && !op->S.dia32) ss->scaled = false;
    }
    const size_t n = (size_t)op->n;
    const size_t n_al = (n + 31) & ~size_t(31);   // x 256-byte aligned, as a workspace vector
    for (auto &sl : ss->slots) {
        hipError_t e = hipMalloc((void **)&sl.b, 2 * n_al * sizeof(double));
        if (e != hipSuccess) {
            sl.b = nullptr;
            set_error("batch session allocation failed: %s", hipGetErrorString(e));
            return fail(e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP);
        }
        sl.x = sl.b + n_al;
        sl.w = new Workspace();
        hns_status st = sl.w->allocate(op->n, mixed);
        if (st == HNS_OK && (ss->line || (ss->scaled && !mixed))) st = sl.w->ensure_z();
        if (st == HNS_OK) st = sl.w->ensure_mf(op->A.mf_scratch());
        if (st != HNS_OK) return fail(st);
    }
    *out = ss;
    return HNS_OK;
}

hns_status slot_session_add(SlotSession *ss, int count, const int *slots, const int *mask_bits,
                            const double *const *b_devs, const double *tols,
                            const int *max_iters, hipStream_t s)
{
    hns_operator *op = ss->op;
    for (int q = 0; q < count; ++q) {
        const int j = slots[q];
        if (j < 0 || j >= ss->K || ss->slots[j].state != 0 || !b_devs[q] || !(tols[q] > 0) ||
            !std::isfinite(tols[q]) || max_iters[q] < 0 || mask_bits[q] < -1 ||
            mask_bits[q] > 7 || (mask_bits[q] >= 0 && !op->bc)) {
            set_error("hns_batch_add: slot %d is not free or its arguments are invalid", j);
            return HNS_ERR_INVALID;
        }
        for (int r = 0; r < q; ++r)
            if (slots[r] == j) {
                set_error("hns_batch_add: slot %d listed twice", j);
                return HNS_ERR_INVALID;
            }
    }
    for (int q = 0; q < count; ++q) {
        SlotSession::Slot &sl = ss->slots[slots[q]];
        HNS_TRY_HIP(hipMemcpyAsync(sl.b, b_devs[q], (size_t)op->n * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
        HNS_TRY(launch_prepare_x(op->n, sl.x, nullptr, -1, true, s));
        memset(&sl.info, 0, sizeof(sl.info));
        const double *lfac = nullptr;
        const float *lfac32 = nullptr;
        if (ss->line) {   // factors of this Dirichlet set (built on its first use)
            if (ss->mixed)
                HNS_TRY(line_factors32(op, mask_bits[q], &lfac32));
            else
                HNS_TRY(line_factors(op, mask_bits[q], &lfac));
        }
        sl.cs = ChunkedSolve();
        sl.cs.c = SolveCtx{op,       mask_bits[q], op->kind == HNS_POISSON && mask_bits[q] < 0,
                           sl.b,     sl.x,         tols[q],
                           max_iters[q], s,        sl.w,
                           lfac,     nullptr,      lfac32,
                           ss->scaled};
        sl.cs.info = &sl.info;
        sl.cs.mixed = ss->mixed;
        const hns_status st = sl.cs.begin();
        if (st == HNS_ERR_INVALID) {   // non-finite right-hand side: finished at once
            sl.info.status = HNS_ERR_INVALID;
            sl.state = 2;
            continue;
        }
        HNS_TRY(st);
        if (sl.cs.finished) {
            HNS_TRY(sl.cs.end());
            sl.state = 2;
        } else {
            sl.state = 1;
        }
    }
    return HNS_OK;
}

hns_status slot_session_advance(SlotSession *ss, int iterations, hipStream_t s, int *active_out)
{
    int done = 0;
    for (;;) {
        std::vector<SlotSession::Slot *> run;
        for (auto &sl : ss->slots)
            if (sl.state == 1) run.push_back(&sl);
        if (run.empty() || done >= iterations) break;
        const int budget = std::min(ss->op->check_every, iterations - done);
        for (auto *sl : run) {
            sl->cs.c.s = s;
            HNS_TRY(sl->cs.enqueue(budget));
        }
        HNS_TRY_HIP(hipStreamSynchronize(s));
        for (auto *sl : run) {
            HNS_TRY(sl->cs.after());
            if (sl->cs.finished) {
                HNS_TRY(sl->cs.end());
                sl->state = 2;
            }
        }
        done += budget;
    }
    int active = 0;
    for (auto &sl : ss->slots) active += (sl.state == 1);
    if (active_out) *active_out = active;
    return HNS_OK;
}

hns_status slot_session_poll(SlotSession *ss, int *states, hns_solve_info *infos)
{
    for (int j = 0; j < ss->K; ++j) {
        const SlotSession::Slot &sl = ss->slots[j];
        states[j] = sl.state;
        if (infos) {
            infos[j] = sl.info;
            if (sl.state == 1) {
                infos[j].iterations = sl.w->host[ss->mixed ? 1 : 0].iter;
                infos[j].status = HNS_NOT_CONVERGED;
            }
        }
    }
    return HNS_OK;
}

hns_status slot_session_take(SlotSession *ss, int slot, double *x_dev, hns_solve_info *info,
                             hipStream_t s)
{
    SlotSession::Slot &sl = ss->slots[slot];
    if (sl.state != 2) {
        set_error("hns_batch_take: slot %d has no finished solve", slot);
        return HNS_ERR_INVALID;
    }
    HNS_TRY_HIP(hipMemcpyAsync(x_dev, sl.x, (size_t)ss->op->n * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    HNS_TRY_HIP(hipStreamSynchronize(s));
    if (info) *info = sl.info;
    sl.state = 0;
    return HNS_OK;
}

}  // namespace hns

// ===========================================================================
// C ABI
// ===========================================================================
using namespace hns;

extern "C" {

const char *hns_last_error(void) { return g_last_error.c_str(); }

const char *hns_status_string(hns_status s)
{
    switch (s) {
    case HNS_OK: return "ok";
    case HNS_NOT_CONVERGED: return "not converged";
    case HNS_ERR_INVALID: return "invalid argument";
    case HNS_ERR_HIP: return "HIP runtime error";
    case HNS_ERR_OOM: return "out of memory";
    case HNS_ERR_MESH: return "invalid mesh";
    case HNS_ERR_BREAKDOWN: return "CG breakdown";
    }
    return "unknown status";
}

// Water columns of the node numbering: the first L nodes share (x, y), and
// so does every later run of L nodes, each at its own (x, y).  Returns L, or 0
// when the numbering is not made of such columns.
static int detect_columns(const hns_mesh *mesh)
{
    const int64_t n = mesh->n_nodes;
    const double *X = mesh->xyz;
    if (n < 2 || !X) return 0;
    auto same_xy = [X](int64_t a, int64_t b) {
        return X[3 * a] == X[3 * b] && X[3 * a + 1] == X[3 * b + 1];
    };
    int64_t L = 1;
    while (L < n && same_xy(0, L)) ++L;
    if (L < 2 || n % L != 0 || L > (1 << 20)) return 0;
    for (int64_t c = 0; c < n; c += L) {
        for (int64_t k = 1; k < L; ++k)
            if (!same_xy(c, c + k)) return 0;
        if (c + L < n && same_xy(c, c + L)) return 0;
    }
    return (int)L;
}

// Column blocks of the assembled matrix for the line preconditioner.
static void keep_column_blocks(hns_operator *op, const HostCSR &A, int L, const uint8_t *bc)
{
    op->line_len = L;
    op->line_d.assign(A.n, 0.0);
    op->line_e.assign(A.n, 0.0);
    for (int64_t i = 0; i < A.n; ++i) {
        const bool top = (i % L) == L - 1;
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            if (A.col[k] == i) op->line_d[i] = A.val[k];
            if (!top && A.col[k] == i + 1) op->line_e[i] = A.val[k];
        }
    }
    if (bc) op->bc_host.assign(bc, bc + A.n);
}

// Dirichlet bits and column blocks of an operator assembled on the device
// (the diagonal and the coupling to the next node of a column, read back
// from the diagonal storage).
static hns_status finish_device_operator(hns_operator *op, const hns_mesh *mesh)
{
    const int64_t n = op->n;
    if (mesh->bc) {
        hipError_t e = hipMalloc((void **)&op->bc, (size_t)n);
        if (e != hipSuccess) {
            op->bc = nullptr;
            set_error("hipMalloc of %lld bytes failed: %s", (long long)n, hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        HNS_TRY_HIP(hipMemcpy(op->bc, mesh->bc, (size_t)n, hipMemcpyHostToDevice));
    }
    const int L = detect_columns(mesh);
    if (L < 2) return HNS_OK;
    op->line_len = L;
    op->line_d.assign(n, 0.0);
    op->line_e.assign(n, 0.0);
    HNS_TRY_HIP(hipMemcpy(op->line_d.data(), op->A.dia, n * sizeof(double),
                          hipMemcpyDeviceToHost));
    for (int k = 0; k < op->A.ndiag; ++k)
        if (op->A.off[k] == 1) {
            HNS_TRY_HIP(hipMemcpy(op->line_e.data(), op->A.dia + (size_t)(k + 1) * n,
                                  n * sizeof(double), hipMemcpyDeviceToHost));
            for (int64_t i = L - 1; i < n; i += L) op->line_e[i] = 0.0;   // column tops
        }
    if (mesh->bc) op->bc_host.assign(mesh->bc, mesh->bc + n);
    return HNS_OK;
}

static hns_status finish_diagonal(hns_operator *op, const HostCSR &A,
                                  const std::vector<double> &lumped, const uint8_t *bc_host);

static hns_status finish_operator(hns_operator *op, const HostCSR &A, uint32_t fmt_flag,
                                  const std::vector<double> &lumped, const uint8_t *bc_host)
{
    const bool keep32 = (op->flags & HNS_KEEP_FP32) != 0;
    uint32_t fmt = fmt_flag ? fmt_flag : choose_format(A);
    HNS_TRY(upload_matrix(A, fmt, keep32, op->A));
    return finish_diagonal(op, A, lumped, bc_host);
}

// A brick operator without a stored matrix: the element data of the
// matrix-free product, and the diagonal and lumped mass of the assembled one
static hns_status finish_matrix_free(hns_operator *op, const hns_hex_mesh *mesh, const HostCSR &A,
                                     double c_mass, double c_stiff,
                                     const std::vector<double> &lumped)
{
    HNS_TRY(upload_matrix_free(mesh, c_mass, c_stiff, op->nu_h, op->nu_v, A.nnz(), op->A));
    return finish_diagonal(op, A, lumped, mesh->bc);
}

// D^-1 (and its FP32 copy with HNS_KEEP_FP32), the Dirichlet bits and the
// lumped mass of an assembled matrix, uploaded
static hns_status finish_diagonal(hns_operator *op, const HostCSR &A,
                                  const std::vector<double> &lumped, const uint8_t *bc_host)
{
    const bool keep32 = (op->flags & HNS_KEEP_FP32) != 0;
    // Jacobi: inverse diagonal
    std::vector<double> dinv(A.n, 0.0);
    for (int64_t i = 0; i < A.n; ++i) {
        double d = 0.0;
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
            if (A.col[k] == i) d = A.val[k];
        if (!(d > 0.0) || !std::isfinite(d)) {
            // not positive definite: kept, but every solve reports breakdown
            if (op->bad_diag < 0) op->bad_diag = i;
            dinv[i] = 0.0;
            continue;
        }
        dinv[i] = 1.0 / d;
    }
    auto up = [](const void *src, size_t bytes, void **dst) -> hns_status {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) {
            *dst = nullptr;
            set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        HNS_TRY_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return HNS_OK;
    };
    HNS_TRY(up(dinv.data(), A.n * sizeof(double), (void **)&op->dinv));
    if (keep32) {
        std::vector<float> d32(dinv.begin(), dinv.end());
        HNS_TRY(up(d32.data(), A.n * sizeof(float), (void **)&op->dinv32));
    }
    if (bc_host) HNS_TRY(up(bc_host, A.n, (void **)&op->bc));
    HNS_TRY(up(lumped.data(), A.n * sizeof(double), (void **)&op->lumped));
    op->lumped_sum = 0.0;
    for (double m : lumped) op->lumped_sum += m;
    return HNS_OK;
}

// Auxiliary forms of the step right-hand sides.  The consistent mass shares
// the pattern and symmetry of A and takes diagonal storage where A's stencil
// allows it (no column indices: about a third of the CSR bytes on the layered
// meshes); the divergence forms are not symmetric and the surface mass lives
// on the surface rows only, so those stay in CSR.
static hns_status assemble_step_aux(hns_operator *op, const hns_mesh *mesh, const HostCSR &A)
{
    if (op->kind != HNS_HELMHOLTZ) {
        set_error("HNS_STEP_AUX needs a HNS_HELMHOLTZ operator");
        return HNS_ERR_INVALID;
    }
    {
        HostCSR M;
        HNS_TRY(assemble_host(mesh, 1.0, 0.0, 0.0, 0.0, M, nullptr));
        const uint32_t fmt = choose_format(M) == HNS_FMT_SDIA ? HNS_FMT_SDIA : HNS_FMT_CSR;
        HNS_TRY(upload_matrix(M, fmt, false, op->M));
    }
    for (int c = 0; c < 3; ++c) {
        HostCSR B, Bt;
        HNS_TRY(assemble_divergence_host(mesh, A, c, B));
        transpose_values(B, Bt);
        HNS_TRY(upload_matrix(B, HNS_FMT_CSR, false, op->B[c]));
        HNS_TRY(upload_matrix(Bt, HNS_FMT_CSR, false, op->Bt[c]));
    }
    {
        HostCSR Ms;
        HNS_TRY(assemble_surface_mass_host(mesh, Ms));
        HNS_TRY(upload_matrix(Ms, HNS_FMT_CSR, false, op->Ms));
    }
    hipError_t e = hipMalloc((void **)&op->step_tmp, 3 * (size_t)op->n * sizeof(double));
    if (e != hipSuccess) {
        op->step_tmp = nullptr;
        set_error("step scratch allocation failed: %s", hipGetErrorString(e));
        return HNS_ERR_OOM;
    }
    {   // the mesh itself, for the advection term
        std::vector<int64_t> ptr;
        std::vector<int32_t> tet;
        std::vector<int8_t> loc;
        tet_incidence(mesh->n_nodes, mesh->n_tets, mesh->tets, ptr, tet, loc);
        auto up = [](const void *src, size_t bytes, void **dst) -> hns_status {
            hipError_t err = hipMalloc(dst, bytes);
            if (err != hipSuccess) {
                *dst = nullptr;
                set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(err));
                return err == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
            }
            HNS_TRY_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
            return HNS_OK;
        };
        op->ntet = mesh->n_tets;
        HNS_TRY(up(mesh->xyz, 3 * (size_t)op->n * sizeof(double), (void **)&op->mesh_xyz));
        HNS_TRY(up(mesh->tets, 4 * (size_t)op->ntet * sizeof(int32_t), (void **)&op->mesh_tets));
        HNS_TRY(up(ptr.data(), ptr.size() * sizeof(int64_t), (void **)&op->inc_ptr));
        HNS_TRY(up(tet.data(), tet.size() * sizeof(int32_t), (void **)&op->inc_tet));
        HNS_TRY(up(loc.data(), loc.size() * sizeof(int8_t), (void **)&op->inc_loc));
    }
    op->has_aux = true;
    return HNS_OK;
}

hns_status hns_assemble(const hns_mesh *mesh, double nu_h, double nu_v, double dt, uint32_t flags,
                        hns_operator **out)
{
    if (!out) {
        set_error("out is null");
        return HNS_ERR_INVALID;
    }
    *out = nullptr;
    const uint32_t kind = flags & (HNS_POISSON | HNS_HELMHOLTZ);
    if (kind != HNS_POISSON && kind != HNS_HELMHOLTZ) {
        set_error("flags must select exactly one of HNS_POISSON / HNS_HELMHOLTZ");
        return HNS_ERR_INVALID;
    }
    if (!std::isfinite(nu_h) || !std::isfinite(nu_v) || !std::isfinite(dt) || nu_h < 0 ||
        nu_v < 0) {
        set_error("viscosities must be finite and non-negative, dt finite");
        return HNS_ERR_INVALID;
    }
    uint32_t fmt = flags & (HNS_FMT_CSR | HNS_FMT_SELL | HNS_FMT_SDIA);
    if (fmt != 0 && fmt != HNS_FMT_CSR && fmt != HNS_FMT_SELL && fmt != HNS_FMT_SDIA) {
        set_error("choose one storage format");
        return HNS_ERR_INVALID;
    }
    if (flags & HNS_MATRIX_FREE) {
        set_error("HNS_MATRIX_FREE is offered for brick elements (hns_assemble_hex) only");
        return HNS_ERR_INVALID;
    }
    hns_operator *op = new hns_operator();
    (void)hipGetDevice(&op->device);
    op->flags = flags;
    op->kind = kind;
    op->nu_h = nu_h;
    op->nu_v = nu_v;
    op->dt = dt;
    HostCSR A;
    std::vector<double> lumped;
    const double c_mass = (kind == HNS_HELMHOLTZ) ? 1.0 : 0.0;
    const double c_stiff = (kind == HNS_HELMHOLTZ) ? dt : 1.0;
    if ((flags & HNS_GPU_ASSEMBLY) && !(flags & (HNS_KEEP_HOST | HNS_STEP_AUX)) &&
        (fmt == 0 || fmt == HNS_FMT_SDIA)) {
        // pattern, offsets and values on the device where the operator fits
        // the unrolled diagonal storage
        bool done = false;
        hns_status st = check_mesh_arrays(mesh);
        if (st == HNS_OK)
            st = assemble_operator_device(mesh, c_mass, c_stiff, nu_h, nu_v,
                                          (flags & HNS_KEEP_FP32) != 0, op, &done);
        if (st == HNS_OK && done) st = finish_device_operator(op, mesh);
        if (st != HNS_OK) {
            hns_operator_destroy(op);
            return st;
        }
        if (done) {
            op->assembly = 2;
            *out = op;
            return HNS_OK;
        }
    }
    hns_status st = assemble_host(mesh, c_mass, c_stiff, nu_h, nu_v, A, &lumped,
                                  (flags & HNS_GPU_ASSEMBLY) != 0);
    if (flags & HNS_GPU_ASSEMBLY) op->assembly = 1;
    if (st == HNS_OK) {
        op->n = A.n;
        st = finish_operator(op, A, fmt, lumped, mesh->bc);
    }
    if (st == HNS_OK) {
        const int L = detect_columns(mesh);
        if (L >= 2) keep_column_blocks(op, A, L, mesh->bc);
        if (flags & HNS_KEEP_HOST) {
            op->host_A = A;
            if (mesh->bc && op->bc_host.empty()) op->bc_host.assign(mesh->bc, mesh->bc + A.n);
        }
    }
    if (st == HNS_OK && (flags & HNS_STEP_AUX)) st = assemble_step_aux(op, mesh, A);
    if (st != HNS_OK) {
        hns_operator_destroy(op);
        return st;
    }
    *out = op;
    return HNS_OK;
}

hns_status hns_assemble_hex(const hns_hex_mesh *mesh, double nu_h, double nu_v, double dt,
                            uint32_t flags, hns_operator **out)
{
    if (!out) {
        set_error("out is null");
        return HNS_ERR_INVALID;
    }
    *out = nullptr;
    const uint32_t kind = flags & (HNS_POISSON | HNS_HELMHOLTZ);
    if (kind != HNS_POISSON && kind != HNS_HELMHOLTZ) {
        set_error("flags must select exactly one of HNS_POISSON / HNS_HELMHOLTZ");
        return HNS_ERR_INVALID;
    }
    if (flags & (HNS_GPU_ASSEMBLY | HNS_STEP_AUX)) {
        set_error("HNS_GPU_ASSEMBLY and HNS_STEP_AUX are not available for brick elements");
        return HNS_ERR_INVALID;
    }
    const bool mfree = (flags & HNS_MATRIX_FREE) != 0;
    if (mfree && (flags & (HNS_KEEP_FP32 | HNS_KEEP_HOST | HNS_FMT_CSR | HNS_FMT_SELL |
                           HNS_FMT_SDIA))) {
        set_error("HNS_MATRIX_FREE takes no storage format, HNS_KEEP_FP32 or HNS_KEEP_HOST");
        return HNS_ERR_INVALID;
    }
    if (!std::isfinite(nu_h) || !std::isfinite(nu_v) || !std::isfinite(dt) || nu_h < 0 ||
        nu_v < 0) {
        set_error("viscosities must be finite and non-negative, dt finite");
        return HNS_ERR_INVALID;
    }
    const uint32_t fmt = flags & (HNS_FMT_CSR | HNS_FMT_SELL | HNS_FMT_SDIA);
    if (fmt != 0 && fmt != HNS_FMT_CSR && fmt != HNS_FMT_SELL && fmt != HNS_FMT_SDIA) {
        set_error("choose one storage format");
        return HNS_ERR_INVALID;
    }
    hns_operator *op = new hns_operator();
    (void)hipGetDevice(&op->device);
    op->flags = flags;
    op->kind = kind;
    op->nu_h = nu_h;
    op->nu_v = nu_v;
    op->dt = dt;
    HostCSR A;
    std::vector<double> lumped;
    const double c_mass = (kind == HNS_HELMHOLTZ) ? 1.0 : 0.0;
    const double c_stiff = (kind == HNS_HELMHOLTZ) ? dt : 1.0;
    hns_status st = assemble_hex_host(mesh, c_mass, c_stiff, nu_h, nu_v, A, &lumped);
    if (st == HNS_OK) {
        op->n = A.n;
        st = mfree ? finish_matrix_free(op, mesh, A, c_mass, c_stiff, lumped)
                   : finish_operator(op, A, fmt, lumped, mesh->bc);
    }
    if (st == HNS_OK) {
        // Q1 column blocks are tridiagonal (vertical neighbours only); the Q2
        // ones reach two levels, so the tridiagonal line factor does not apply
        hns_mesh nodes = {};
        nodes.n_nodes = mesh->n_nodes;
        nodes.xyz = mesh->xyz;
        const int L = mesh->order == 1 ? detect_columns(&nodes) : 0;
        if (L >= 2) keep_column_blocks(op, A, L, mesh->bc);
        if (flags & HNS_KEEP_HOST) {
            op->host_A = A;
            if (mesh->bc && op->bc_host.empty()) op->bc_host.assign(mesh->bc, mesh->bc + A.n);
        }
    }
    if (st != HNS_OK) {
        hns_operator_destroy(op);
        return st;
    }
    *out = op;
    return HNS_OK;
}

void hns_operator_destroy(hns_operator *op)
{
    if (!op) return;
    (void)hipDeviceSynchronize();
    op->A.release();
    op->S.release();
    op->M.release();
    for (auto &b : op->B) b.release();
    for (auto &b : op->Bt) b.release();
    op->Ms.release();
    void *ptrs[] = {op->dinv,     op->dinv32,    op->bc,      op->lumped,  op->step_tmp,
                    op->mesh_xyz, op->mesh_tets, op->inc_ptr, op->inc_tet, op->inc_loc,
                    op->jac_s,    op->jac_w};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (double *f : op->line_fac)
        if (f) (void)hipFree(f);
    for (float *f : op->line_fac32)
        if (f) (void)hipFree(f);
    for (IC0Dev *f : op->ic0_fac)
        if (f) {
            f->release();
            delete f;
        }
    for (Workspace *w : op->ws_free) delete w;
    for (BWorkspace *w : op->bws_free) destroy_bworkspace(w);
    delete op;
}

hns_status hns_profile_enable(hns_operator *op, int on)
{
    if (!op) {
        set_error("null operator");
        return HNS_ERR_INVALID;
    }
    if (on < 0) {
        set_error("profile period must be >= 0");
        return HNS_ERR_INVALID;
    }
    op->profile = on;
    if (on)
        for (int k = 0; k < 6; ++k) {
            op->prof_ms[k] = 0.0;
            op->prof_count[k] = 0;
        }
    return HNS_OK;
}

hns_status hns_profile_read(const hns_operator *op, int kernel, double *total_ms,
                            int64_t *launches)
{
    if (!op || kernel < 0 || kernel > 5 || !total_ms || !launches) {
        set_error("hns_profile_read: bad arguments");
        return HNS_ERR_INVALID;
    }
    *total_ms = op->prof_ms[kernel];
    *launches = op->prof_count[kernel];
    return HNS_OK;
}

int64_t hns_operator_n(const hns_operator *op) { return op ? op->n : -1; }
int64_t hns_operator_nnz(const hns_operator *op) { return op ? op->A.nnz : -1; }
uint32_t hns_operator_format(const hns_operator *op) { return op ? op->A.fmt : 0; }
int hns_operator_line_len(const hns_operator *op) { return op ? op->line_len : -1; }

int hns_operator_assembly(const hns_operator *op) { return op ? op->assembly : -1; }

int hns_operator_ndiag(const hns_operator *op)
{
    if (!op) return -1;
    return op->A.fmt == HNS_FMT_SDIA ? op->A.ndiag : 0;
}

hns_status hns_set_param(hns_operator *op, const char *name, double value)
{
    if (!op || !name) {
        set_error("null operator or name");
        return HNS_ERR_INVALID;
    }
    std::string k(name);
    if (k == "check_every" && value >= 1 && value <= 1e6) {
        op->check_every = (int)value;
    } else if (k == "inner_tol" && value > 0 && value < 1) {
        op->inner_tol = value;
    } else if (k == "max_outer" && value >= 1 && value <= 1000) {
        op->max_outer = (int)value;
    } else if (k == "mixed_variant" && (value == 0 || value == 1 || value == 2)) {
        op->mixed_variant = (int)value;
    } else if (k == "replace_drop" && value > 0 && value < 1) {
        op->replace_drop = value;
    } else if (k == "bspmm_vec" && (value == 0 || value == 1 || value == 2 || value == 4)) {
        op->bspmm_vec = (int)value;
        op->tuned.clear();
    } else if (k == "bspmm_tile" && value >= -1 && value <= kTileShapesAbi &&
               value == (int)value) {
        op->bspmm_tile = (int)value;
        op->tuned.clear();
    } else if (k == "use_graph" && (value == 0 || value == 1)) {
        op->use_graph = (int)value;
    } else if (k == "spmv_it64" && value >= 1 && value <= 64 && value == (int)value) {
        op->A.spmv_it64 = op->S.spmv_it64 = (int)value;
    } else if (k == "spmv_it32" && value >= 0 && value <= 64 && value == (int)value) {
        op->A.spmv_it32 = op->S.spmv_it32 = (int)value;
    } else if (k == "spmv_rows64" && (value == 0 || value == 1 || value == 2)) {
        op->A.spmv_rows64 = op->S.spmv_rows64 = (int)value;
    } else if (k == "vec_it" && value >= 0 && value <= 64 && value == (int)value) {
        op->A.vec_it = op->S.vec_it = (int)value;
    } else if (k == "jacobi_scaling" && (value == 0 || value == 1)) {
        op->jacobi_scaling = (int)value;
    } else if (k == "fuse_dir" && (value == -1 || value == 0 || value == 1)) {
        op->fuse_dir = (int)value;
    } else if (k == "session_mode" && (value == 0 || value == 1 || value == 2)) {
        op->session_mode = (int)value;
    } else if (k == "small_n" && value >= 0 && value <= (double)kSmallMaxN &&
               value == (int64_t)value) {
        op->small_n = (int64_t)value;
    } else if (k == "precond" && (value == 0 || value == 1 || value == 2)) {
        if (value == 2 && op->host_A.col.empty()) {
            set_error("precond = 2 (IC(0)) needs an operator assembled with HNS_KEEP_HOST");
            return HNS_ERR_INVALID;
        }
        if (value == 1) {
            if (op->line_len < 2) {
                set_error("precond = 1 needs a node numbering made of water columns");
                return HNS_ERR_INVALID;
            }
            const int G = line_grid(op->n, op->line_len);
            if (G < 1 || G > kMaxPart) {
                set_error("line preconditioner: %lld nodes in columns of %d do not fit the "
                          "launch shape", (long long)op->n, op->line_len);
                return HNS_ERR_INVALID;
            }
        }
        op->precond = (int)value;
    } else {
        set_error("unknown parameter or bad value: %s = %g", name, value);
        return HNS_ERR_INVALID;
    }
    return HNS_OK;
}

size_t hns_footprint_bytes(const hns_operator *op, int k, uint32_t mode, int include_operator)
{
    if (!op || k < 1) return 0;
    const bool mixed = (mode == HNS_MIXED);
    size_t b = k == 1 ? Workspace::bytes_for(op->n, mixed) : bworkspace_bytes(op->n, k, mixed);
    if (k == 1 && op->precond == 1) b += (size_t)op->n * sizeof(double);       // z
    if (k == 1 && op->precond == 2) b += 2 * (size_t)op->n * sizeof(double);   // z, y
    if (k == 1) b += op->A.mf_scratch() * sizeof(double);   // matrix-free element results
    // the second direction buffer of the fused scaled iterations
    if (k == 1 && op->jacobi_scaling && op->precond == 0 && op->A.fmt == HNS_FMT_SDIA &&
        op->A.ndiag >= 1 && op->A.ndiag <= kMaxDiag && op->n > op->small_n &&
        fuse_wanted(op, mixed))
        b += (size_t)op->n * sizeof(double);
    if (include_operator) {
        for (const double *f : op->line_fac)
            if (f) b += 2 * (size_t)op->n * sizeof(double);
        for (const IC0Dev *f : op->ic0_fac)
            if (f) b += f->bytes;
        b += op->A.bytes() + (size_t)op->n * (8 + 1 + 8);
        // the Jacobi-scaled operator, resident once a point-Jacobi solve has used it
        const bool scaled = op->S.dia || (op->jacobi_scaling && op->precond == 0 &&
                                          op->A.fmt == HNS_FMT_SDIA && op->A.ndiag >= 1 &&
                                          op->A.ndiag <= kMaxDiag && op->n > op->small_n);
        if (scaled)
            b += (size_t)op->A.ndiag * op->n * (op->A.dia32 ? 12 : 8) + (size_t)op->n * (8 + 4);
        if (op->dinv32) b += (size_t)op->n * 4;
        if (op->has_aux)
            b += op->M.bytes() + op->B[0].bytes() * 6 + op->Ms.bytes() + 24 * (size_t)op->n +
                 (3 * 8 + 8) * (size_t)op->n + (4 * 4 + 4 * (4 + 1)) * (size_t)op->ntet;
    }
    return b;
}

static hns_status check_solve_args(hns_operator *op, int mask_bit, const void *b, const void *x,
                                   double tol, int max_iter, uint32_t mode)
{
    if (!op || !b || !x) {
        set_error("null operator or vector");
        return HNS_ERR_INVALID;
    }
    if (mask_bit < -1 || mask_bit > 7) {
        set_error("mask_bit must be -1 or 0..7");
        return HNS_ERR_INVALID;
    }
    if (mask_bit >= 0 && !op->bc) {
        set_error("mask_bit given but the mesh had no Dirichlet bits");
        return HNS_ERR_INVALID;
    }
    if (!(tol > 0) || !std::isfinite(tol) || max_iter < 0) {
        set_error("tol must be positive and finite, max_iter >= 0");
        return HNS_ERR_INVALID;
    }
    if (mode != HNS_FP64 && mode != HNS_MIXED) {
        set_error("unknown mode %u", mode);
        return HNS_ERR_INVALID;
    }
    if (mode == HNS_MIXED && op->A.fmt == HNS_MATRIX_FREE) {
        set_error("matrix-free operators run HNS_FP64 solves only");
        return HNS_ERR_INVALID;
    }
    if (mode == HNS_MIXED && !op->dinv32) {
        set_error("HNS_MIXED needs an operator assembled with HNS_KEEP_FP32");
        return HNS_ERR_INVALID;
    }
    return HNS_OK;
}

// Device factors of the line preconditioner for Dirichlet set `bit` (-1 =
// none): the column blocks with Dirichlet rows and columns replaced by the
// identity, factorised top-down (u_0 = d_0, u_k = d_k - e_{k-1}^2 / u_{k-1});
// stored as the masked couplings e followed by the inverse pivots 1 / u.
// Column factors of Dirichlet set `bit` on the host: masked couplings e (n)
// then inverse pivots w (n) of the top-down Thomas factorisation.
static hns_status line_factors_host(const hns_operator *op, int bit, std::vector<double> &host)
{
    const int64_t n = op->n;
    const int L = op->line_len;
    const bool masked = bit >= 0 && !op->bc_host.empty();
    auto dir = [&](int64_t i) { return masked && ((op->bc_host[i] >> bit) & 1u); };
    host.assign(2 * (size_t)n, 0.0);
    double *e = host.data(), *w = host.data() + n;
    for (int64_t c0 = 0; c0 < n; c0 += L) {
        for (int64_t i = c0; i < c0 + L; ++i) {
            const bool top = (i == c0 + L - 1);
            e[i] = (top || dir(i) || dir(i + 1)) ? 0.0 : op->line_e[i];
            const double d = dir(i) ? 1.0 : op->line_d[i];
            const double u = (i == c0) ? d : d - e[i - 1] * (e[i - 1] * w[i - 1]);
            if (!(u > 0.0) || !std::isfinite(u)) {
                set_error("column block of node %lld is not positive definite", (long long)i);
                return HNS_ERR_BREAKDOWN;
            }
            w[i] = 1.0 / u;
        }
    }
    return HNS_OK;
}

static hns_status upload_factors(const void *host, size_t bytes, void **dev)
{
    hipError_t err = hipMalloc(dev, bytes);
    if (err != hipSuccess) {
        *dev = nullptr;
        set_error("allocation of line factors failed: %s", hipGetErrorString(err));
        return err == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
    }
    err = hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        set_error("upload of line factors failed: %s", hipGetErrorString(err));
        return HNS_ERR_HIP;
    }
    return HNS_OK;
}

// Device factors of Dirichlet set `bit` (FP64), computed on first use.
static hns_status line_factors(hns_operator *op, int bit, const double **out)
{
    std::lock_guard<std::mutex> g(op->line_mutex);
    double *&slot = op->line_fac[bit + 1];
    if (!slot) {
        std::vector<double> host;
        HNS_TRY(line_factors_host(op, bit, host));
        void *dev = nullptr;
        HNS_TRY(upload_factors(host.data(), host.size() * sizeof(double), &dev));
        slot = (double *)dev;
    }
    *out = slot;
    return HNS_OK;
}

// The same factors rounded to FP32, for the inner iterations of HNS_MIXED.
static hns_status line_factors32(hns_operator *op, int bit, const float **out)
{
    std::lock_guard<std::mutex> g(op->line_mutex);
    float *&slot = op->line_fac32[bit + 1];
    if (!slot) {
        std::vector<double> host;
        HNS_TRY(line_factors_host(op, bit, host));
        std::vector<float> h32(host.begin(), host.end());
        void *dev = nullptr;
        HNS_TRY(upload_factors(h32.data(), h32.size() * sizeof(float), &dev));
        slot = (float *)dev;
    }
    *out = slot;
    return HNS_OK;
}

void IC0Dev::release()
{
    void *ptrs[] = {perm, lptr, uptr, lcol, ucol, lval, uval, diag};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    perm = nullptr;
    lptr = uptr = nullptr;
    lcol = ucol = nullptr;
    lval = uval = diag = nullptr;
}

// Device IC(0) factor for Dirichlet set `bit`, factorised on first use.
static hns_status ic0_factors(hns_operator *op, int bit, const IC0Dev **out)
{
    std::lock_guard<std::mutex> g(op->line_mutex);
    IC0Dev *&slot = op->ic0_fac[bit + 1];
    if (!slot) {
        IC0Host H;
        HNS_TRY(ic0_factor_host(op->host_A, op->bc_host.empty() ? nullptr : op->bc_host.data(),
                                bit, H));
        IC0Dev *D = new IC0Dev();
        D->n = H.n;
        D->ncolors = H.ncolors;
        D->cstart = H.cstart;
        // the factor rows of each colour in column-major padded blocks
        std::vector<int32_t> lcol, ucol;
        std::vector<double> lval, uval;
        auto by_colour = [&](const std::vector<int64_t> &ptr, const std::vector<int32_t> &col,
                             const std::vector<double> &val, std::vector<int64_t> &base,
                             std::vector<int32_t> &width, std::vector<int32_t> &ecol,
                             std::vector<double> &eval) {
            base.assign(H.ncolors, 0);
            width.assign(H.ncolors, 0);
            int64_t total = 0;
            for (int c = 0; c < H.ncolors; ++c) {
                int64_t w = 0;
                for (int64_t r = H.cstart[c]; r < H.cstart[c + 1]; ++r)
                    w = std::max(w, ptr[r + 1] - ptr[r]);
                base[c] = total;
                width[c] = (int32_t)w;
                total += w * (H.cstart[c + 1] - H.cstart[c]);
            }
            ecol.assign(total, 0);
            eval.assign(total, 0.0);
            // the colours' blocks are disjoint: one thread per colour
            std::vector<std::thread> th;
            for (int c = 0; c < H.ncolors; ++c)
                th.emplace_back([&, c] {
                    const int64_t r0 = H.cstart[c], nc = H.cstart[c + 1] - r0;
                    for (int64_t j = 0; j < nc; ++j)
                        for (int64_t t = ptr[r0 + j]; t < ptr[r0 + j + 1]; ++t) {
                            const int64_t e = base[c] + (t - ptr[r0 + j]) * nc + j;
                            ecol[e] = col[t];
                            eval[e] = val[t];
                        }
                });
            for (auto &t : th) t.join();
        };
        by_colour(H.lptr, H.lcol, H.lval, D->lbase, D->lwidth, lcol, lval);
        by_colour(H.uptr, H.ucol, H.uval, D->ubase, D->uwidth, ucol, uval);
        auto up = [&](const void *src, size_t bytes, void **dst) -> hns_status {
            hipError_t e = hipMalloc(dst, bytes > 0 ? bytes : 8);
            if (e != hipSuccess) {
                *dst = nullptr;
                set_error("allocation of the IC(0) factor failed: %s", hipGetErrorString(e));
                return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
            }
            D->bytes += bytes;
            if (bytes) HNS_TRY_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
            return HNS_OK;
        };
        hns_status st = HNS_OK;
        auto run = [&]() -> hns_status {
            HNS_TRY(up(H.perm.data(), H.perm.size() * 4, (void **)&D->perm));
            HNS_TRY(up(H.lptr.data(), H.lptr.size() * 8, (void **)&D->lptr));
            HNS_TRY(up(H.uptr.data(), H.uptr.size() * 8, (void **)&D->uptr));
            HNS_TRY(up(lcol.data(), lcol.size() * 4, (void **)&D->lcol));
            HNS_TRY(up(ucol.data(), ucol.size() * 4, (void **)&D->ucol));
            HNS_TRY(up(lval.data(), lval.size() * 8, (void **)&D->lval));
            HNS_TRY(up(uval.data(), uval.size() * 8, (void **)&D->uval));
            HNS_TRY(up(H.diag.data(), H.diag.size() * 8, (void **)&D->diag));
            return HNS_OK;
        };
        st = run();
        if (st != HNS_OK) {
            D->release();
            delete D;
            return st;
        }
        slot = D;
    }
    *out = slot;
    return HNS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free solves (hns_solve_noalloc): the workspace of a solve lives
// in `scratch`, a file-scope device array of which every GPU the library
// runs on holds its own copy until the process ends.  Host code never uses
// the array's name as an address: the device address of each GPU's copy is
// looked up once per device (with that device current) and kept here.  The
// host mirror of the CG scalars is a file-scope host array per device.  Calls
// on one GPU share all of it, so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
namespace hns {

constexpr size_t kScratchBytes = size_t(96) << 20;   // 96 MiB per GPU
constexpr int kScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mutex;
static void *g_scratch_dev[kScratchDevices];          // scratch's address on each GPU
static Scalars g_scratch_host[kScratchDevices][2];    // host mirror of the scalars
static uint32_t g_scratch_token[kScratchDevices];     // iteration tags handed out so far

// Device address of `scratch` on the current device (looked up on the
// device's first call) and the device's index.
static hns_status scratch_address(void **out, int *dev_out)
{
    int dev = -1;
    HNS_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("hns_solve_noalloc: device %d is beyond the %d devices it supports", dev,
                  kScratchDevices);
        return HNS_ERR_INVALID;
    }
    std::lock_guard<std::mutex> g(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hns_solve_noalloc: address of the static scratch on device %d: %s", dev,
                      e != hipSuccess ? hipGetErrorString(e) : "null address");
            return HNS_ERR_HIP;
        }
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    *dev_out = dev;
    return HNS_OK;
}

}  // namespace hns

extern "C" {

size_t hns_noalloc_scratch_bytes(void) { return kScratchBytes; }

size_t hns_noalloc_bytes(const hns_operator *op, uint32_t mode)
{
    if (!op) return 0;
    const bool mixed = (mode == HNS_MIXED);
    // the correction vector of the Jacobi-scaled FP64 recurrence is counted
    // whether or not that recurrence runs
    return Workspace::bytes_for(op->n, mixed) + (mixed ? 0 : Workspace::al(op->n * sizeof(double)));
}

hns_status hns_solve_noalloc(hns_operator *op, int mask_bit, const double *b_dev, double *x_dev,
                             double tol, int max_iter, uint32_t mode, void *stream,
                             hns_solve_info *info)
{
    hns_solve_info local;
    if (!info) info = &local;
    memset(info, 0, sizeof(*info));
    hns_status st = check_solve_args(op, mask_bit, b_dev, x_dev, tol, max_iter, mode);
    if (st == HNS_OK && op->precond != 0) {
        set_error("hns_solve_noalloc runs point Jacobi only (set_param \"precond\" = 0): the "
                  "other preconditioners build factors on first use");
        st = HNS_ERR_INVALID;
    }
    if (st == HNS_OK && op->A.fmt == HNS_MATRIX_FREE) {
        set_error("hns_solve_noalloc: matrix-free operators need their element scratch");
        st = HNS_ERR_INVALID;
    }
    if (st == HNS_OK && op->bad_diag >= 0) {
        set_error("diagonal entry %lld is not positive: Jacobi-PCG needs an SPD operator",
                  (long long)op->bad_diag);
        st = HNS_ERR_BREAKDOWN;
    }
    const bool mixed = (mode == HNS_MIXED);
    const size_t need = (st == HNS_OK) ? hns_noalloc_bytes(op, mode) : 0;
    if (st == HNS_OK && need > kScratchBytes) {
        set_error("hns_solve_noalloc: %lld rows need %zu bytes of scratch, more than the %zu "
                  "bytes of the static scratch",
                  (long long)op->n, need, kScratchBytes);
        st = HNS_ERR_INVALID;
    }
    void *base = nullptr;
    int dev = 0;
    if (st == HNS_OK) st = scratch_address(&base, &dev);
    if (st != HNS_OK) {
        info->status = st;
        return st;
    }
    // hns_solve's recurrence where the operator already holds what it needs:
    // the Jacobi-scaled copy is built (and allocated) by hns_solve on its
    // first use, so without it the unscaled point-Jacobi recurrence runs (the
    // same iterates in exact arithmetic)
    bool scaled = op->jacobi_scaling && op->A.fmt == HNS_FMT_SDIA && op->A.ndiag >= 1 &&
                  op->A.ndiag <= kMaxDiag && op->n > op->small_n &&
                  (!mixed || op->mixed_variant == 0);
    if (scaled) {
        std::lock_guard<std::mutex> g(op->line_mutex);
        scaled = op->S.dia && (!mixed || op->S.dia32);
    }
    Workspace w;
    w.borrow(op->n, mixed, base, !mixed, g_scratch_host[dev], g_scratch_token[dev]);
    SolveCtx c{op,       mask_bit, op->kind == HNS_POISSON && mask_bit < 0, b_dev, x_dev, tol,
               max_iter, (hipStream_t)stream, &w, nullptr, nullptr, nullptr, scaled};
    st = mixed ? solve_mixed(c, info) : solve_fp64(c, info);
    g_scratch_token[dev] = w.token;
    info->status = st;
    return st;
}

hns_status hns_solve(hns_operator *op, int mask_bit, const double *b_dev, double *x_dev,
                     double tol, int max_iter, uint32_t mode, void *stream, hns_solve_info *info)
{
    hns_solve_info local;
    if (!info) info = &local;
    memset(info, 0, sizeof(*info));
    hns_status st = check_solve_args(op, mask_bit, b_dev, x_dev, tol, max_iter, mode);
    if (st != HNS_OK) {
        info->status = st;
        return st;
    }
    if (op->bad_diag >= 0) {
        set_error("diagonal entry %lld is not positive: Jacobi-PCG needs an SPD operator",
                  (long long)op->bad_diag);
        info->status = HNS_ERR_BREAKDOWN;
        return HNS_ERR_BREAKDOWN;
    }
    const double *lfac = nullptr;
    const float *lfac32 = nullptr;
    const IC0Dev *ic = nullptr;
    if (op->precond == 2) {
        if (mode != HNS_FP64 || (op->kind == HNS_POISSON && mask_bit < 0)) {
            set_error("the IC(0) preconditioner runs HNS_FP64 solves with a Dirichlet set only");
            info->status = HNS_ERR_INVALID;
            return HNS_ERR_INVALID;
        }
        st = ic0_factors(op, mask_bit, &ic);
        if (st != HNS_OK) {
            info->status = st;
            return st;
        }
    }
    if (op->precond == 1) {
        if (mode == HNS_MIXED && op->mixed_variant != 0) {
            set_error("the line preconditioner runs HNS_MIXED solves with mixed_variant 0 "
                      "(FP32 CG with FP64 residual replacement) only");
            info->status = HNS_ERR_INVALID;
            return HNS_ERR_INVALID;
        }
        st = mode == HNS_MIXED ? line_factors32(op, mask_bit, &lfac32)
                               : line_factors(op, mask_bit, &lfac);
        if (st != HNS_OK) {
            info->status = st;
            return st;
        }
    }
    // point Jacobi on the unrolled diagonal format (above the single-workgroup
    // size): plain CG on the Jacobi-scaled operator
    bool scaled = op->jacobi_scaling && op->precond == 0 && op->A.fmt == HNS_FMT_SDIA &&
                  op->A.ndiag >= 1 && op->A.ndiag <= kMaxDiag && op->n > op->small_n &&
                  (mode == HNS_FP64 || (mode == HNS_MIXED && op->mixed_variant == 0));
    if (scaled) {
        st = scaled_operator(op);
        if (st != HNS_OK) {
            info->status = st;
            return st;
        }
        if (mode == HNS_MIXED && !op->S.dia32) scaled = false;   // no FP32 values kept
    }
    Workspace *w = nullptr;
    st = acquire_ws(op, mode == HNS_MIXED, &w);
    if (st == HNS_OK && (lfac || lfac32 || ic || (scaled && mode == HNS_FP64))) {
        st = w->ensure_z();
        if (st == HNS_OK && ic) st = w->ensure_y();
        if (st != HNS_OK) release_ws(op, w);
    }
    if (st != HNS_OK) {
        info->status = st;
        return st;
    }
    SolveCtx c{op,   mask_bit, op->kind == HNS_POISSON && mask_bit < 0, b_dev, x_dev, tol,
               max_iter, (hipStream_t)stream, w, lfac, ic, lfac32, scaled};
    st = (mode == HNS_MIXED) ? solve_mixed(c, info) : solve_fp64(c, info);
    info->status = st;
    release_ws(op, w);
    return st;
}

hns_status hns_apply(hns_operator *op, int mask_bit, const double *x_dev, double *y_dev,
                     void *stream)
{
    if (!op || !x_dev || !y_dev || mask_bit < -1 || mask_bit > 7 || (mask_bit >= 0 && !op->bc)) {
        set_error("hns_apply: bad arguments");
        return HNS_ERR_INVALID;
    }
    if (op->A.fmt == HNS_MATRIX_FREE) {   // element scratch from the workspace pool
        Workspace *w = nullptr;
        HNS_TRY(acquire_ws(op, false, &w));
        hns_status st = launch_spmv_plain(op->A, false, x_dev, y_dev, op->bc, mask_bit,
                                          (hipStream_t)stream, w->mf);
        if (st == HNS_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
            set_error("hns_apply: the product failed on the device");
            st = HNS_ERR_HIP;
        }
        release_ws(op, w);
        return st;
    }
    HNS_TRY(launch_spmv_plain(op->A, false, x_dev, y_dev, op->bc, mask_bit, (hipStream_t)stream));
    HNS_TRY_HIP(hipStreamSynchronize((hipStream_t)stream));
    return HNS_OK;
}

static hns_status acquire_bws(hns_operator *op, int K, bool mixed, BWorkspace **out)
{
    {
        std::lock_guard<std::mutex> g(op->ws_mutex);
        for (size_t i = 0; i < op->bws_free.size(); ++i) {
            BWorkspace *w = op->bws_free[i];
            if (bworkspace_k(w) == K && (bworkspace_mixed(w) || !mixed)) {
                op->bws_free.erase(op->bws_free.begin() + i);
                *out = w;
                return HNS_OK;
            }
        }
    }
    return create_bworkspace(op->n, K, mixed, out);
}

static void release_bws(hns_operator *op, BWorkspace *w)
{
    std::lock_guard<std::mutex> g(op->ws_mutex);
    op->bws_free.push_back(w);
}

static hns_status check_batched_args(hns_operator *op, int k, const int *bits, const void *B,
                                     const void *X, double tol, int max_iter, uint32_t mode)
{
    if (k < 1 || k > 1024 || !bits) {
        set_error("k must be in [1, 1024] with k mask bits");
        return HNS_ERR_INVALID;
    }
    for (int j = 0; j < k; ++j)
        if (bits[j] < -1 || bits[j] > 7 || (bits[j] >= 0 && !op->bc)) {
            set_error("bad mask bit %d for column %d", bits[j], j);
            return HNS_ERR_INVALID;
        }
    return check_solve_args(op, -1, B, X, tol, max_iter, mode);
}

hns_status hns_solve_batched(hns_operator *op, int k, const int *mask_bits, const double *B_dev,
                             double *X_dev, double tol, int max_iter, uint32_t mode, void *stream,
                             hns_solve_info *infos)
{
    if (!infos) {
        set_error("infos must hold k entries");
        return HNS_ERR_INVALID;
    }
    for (int j = 0; j < k && j < 1024; ++j) memset(&infos[j], 0, sizeof(hns_solve_info));
    HNS_TRY(check_batched_args(op, k, mask_bits, B_dev, X_dev, tol, max_iter, mode));
    if (op->precond != 0) {
        set_error("multi-right-hand-side solves use the point Jacobi preconditioner only");
        return HNS_ERR_INVALID;
    }
    if (op->A.fmt == HNS_MATRIX_FREE) {
        set_error("multi-right-hand-side solves need a stored matrix (not HNS_MATRIX_FREE)");
        return HNS_ERR_INVALID;
    }
    if (op->bad_diag >= 0) {
        set_error("diagonal entry %lld is not positive: Jacobi-PCG needs an SPD operator",
                  (long long)op->bad_diag);
        for (int j = 0; j < k; ++j) infos[j].status = HNS_ERR_BREAKDOWN;
        return HNS_ERR_BREAKDOWN;
    }
    const bool mixed = (mode == HNS_MIXED);
    hipStream_t s = (hipStream_t)stream;
    BWorkspace *w = nullptr;
    HNS_TRY(acquire_bws(op, k, mixed, &w));
    int V = 1;
    hns_status st = batched_plan(op, w, k, mixed, s, &V);
    if (st == HNS_OK)
        st = solve_batched_impl(op, w, k, mask_bits, B_dev, X_dev, tol, max_iter, mixed, V, s,
                                infos);
    release_bws(op, w);
    return st;
}

hns_status hns_tune_batched(hns_operator *op, int k, uint32_t mode, void *stream,
                            double *times_us, int *best_plan)
{
    if (!op || !times_us || !best_plan || k < 1 || k > 1024 ||
        (mode != HNS_FP64 && mode != HNS_MIXED) || (mode == HNS_MIXED && !op->dinv32)) {
        set_error("hns_tune_batched: bad arguments");
        return HNS_ERR_INVALID;
    }
    if (op->A.fmt == HNS_MATRIX_FREE) {
        set_error("hns_tune_batched: matrix-free operators have no batched product");
        return HNS_ERR_INVALID;
    }
    const bool mixed = (mode == HNS_MIXED);
    BWorkspace *w = nullptr;
    HNS_TRY(acquire_bws(op, k, mixed, &w));
    hns_status st = tune_batched(op, w, k, mixed, (hipStream_t)stream, times_us, best_plan);
    release_bws(op, w);
    if (st == HNS_OK) {
        if (op->bspmm_tile < 0) plan_cache_put(plan_key(op, k, mixed), *best_plan);
        std::lock_guard<std::mutex> g(op->ws_mutex);
        bool found = false;
        for (auto &t : op->tuned)
            if (t[0] == k && t[1] == (int)mixed) {
                t[2] = *best_plan;
                found = true;
            }
        if (!found) op->tuned.push_back({k, (int)mixed, *best_plan});
    }
    return st;
}

}  // extern "C"
