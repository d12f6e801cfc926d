// amg_solve: Algorithm 1 (the basic AMG iteration) and the outer Krylov
// drivers. Every vector operation runs on the GPU; Krylov scalars stay in a
// device array, and the host reads one residual norm per iteration for the
// stopping test.
#include <chrono>
#include <cmath>

#include "context.h"

namespace amgp2 {

// ---------------------------------------------------------------- profiling
ProfScope::ProfScope(amg_ctx *hh, const std::string &cls, double bytes) : h(hh), idx(0) {
    if (!h->prof) return;
    if (h->prof_finest_only && cls.size() > 3 && cls.compare(cls.size() - 3, 3, ".L0") != 0) return;
    amg_ctx::Pending pe;
    pe.cls = cls;
    pe.bytes = bytes;
    // timing-only events: no system-scope fence (its L2 writeback and
    // invalidate would lengthen the interval and slow the next kernel);
    // profile_collect synchronises the stream before reading them
    for (hipEvent_t *e : {&pe.a, &pe.b}) {
        if (!h->event_pool.empty()) {
            *e = h->event_pool.back();
            h->event_pool.pop_back();
        } else {
            AMG_HIP(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
        }
    }
    AMG_HIP(hipEventRecord(pe.a, h->stream));
    h->pending.push_back(pe);
    idx = h->pending.size();
}

ProfScope::~ProfScope() {
    if (!h->prof || idx == 0) return;
    (void)hipEventRecord(h->pending[idx - 1].b, h->stream);
}

void profile_collect(amg_ctx *h) {
    if (h->pending.empty()) return;
    AMG_HIP(hipStreamSynchronize(h->stream));
    for (auto &pe : h->pending) {
        float ms = 0.f;
        AMG_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
        ProfStat &st = h->stats[pe.cls];
        st.launches += 1;
        st.ms += ms;
        st.bytes += pe.bytes;
        h->event_pool.push_back(pe.a);
        h->event_pool.push_back(pe.b);
    }
    h->pending.clear();
}

// algorithmic bytes of one pass over rows [.., ..) of a block operator
static double row_bytes(const DMat &m, int64_t nnz, int nrows) {
    return static_cast<double>(nnz) * (m.np * 8.0 + 4.0) + nrows * 4.0;
}

static RowArgs row_args(const DMat &m) {
    RowArgs a;
    a.nrows = m.nrows;
    a.rowptr = m.rowptr.p;
    a.col = m.col.p;
    a.val = m.val.p;
    a.nnz = m.nnz;
    return a;
}

static std::string tag(const char *cls, int l) { return std::string(cls) + ".L" + std::to_string(l); }

// ---------------------------------------------------------------- level ops
void apply_level(amg_ctx *h, int l, const double *x, double *y) {
    Level &L = h->lv[l];
    RowArgs a = row_args(L.A);
    a.x = x;
    a.y = y;
    ProfScope ps(h, tag("spmv", l), row_bytes(L.A, L.A.nnz, L.n) + 3.0 * L.n * 16.0);
    a.trip = L.trip;
    launch_row(L.mode, OP_SPMV, L.G, a, h->stream);
}

// r = b - A x on the level's first `rows` rows (all of them: -1)
static void residual(amg_ctx *h, int l, const double *b, const double *x, double *r, int rows = -1) {
    Level &L = h->lv[l];
    RowArgs a = row_args(L.A);
    if (rows >= 0) a.nrows = rows;
    a.x = x;
    a.b = b;
    a.y = r;
    ProfScope ps(h, tag("resid", l), row_bytes(L.A, L.A.nnz, L.n) + 3.0 * L.n * 24.0);
    a.trip = L.trip;
    launch_row(L.mode, OP_RESID, L.G, a, h->stream);
}

static double level_omega(amg_ctx *h, int l) {
    if (!h->level_omega.empty())
        return h->level_omega[std::min<size_t>(l, h->level_omega.size() - 1)];
    return h->prm.omega;
}

// (on the level's leading nA rows: the systems of a batch that continue
// below the level; every row outside batches)
static void jacobi_step(amg_ctx *h, int l, const double *b, double *x, bool zero_init) {
    Level &L = h->lv[l];
    const double om = level_omega(h, l);
    const int nb = L.mode == 3 ? 9 : 1;
    if (zero_init) {
        ProfScope ps(h, tag("jacobi0", l), 3.0 * L.n * 16.0 + nb * 8.0 * L.n);
        launch_jacobi_zero(L.mode, L.nA, L.dinv.p, L.n, b, om, x, h->stream);
        return;
    }
    RowArgs a = row_args(L.A);
    a.nrows = L.nA;
    a.x = x;
    a.b = b;
    a.y = L.t.p;
    a.dinv = L.dinv.p;
    a.dinv_n = L.n;
    a.omega = om;
    {
        ProfScope ps(h, tag("jacobi", l), row_bytes(L.A, L.A.nnz, L.n) + 3.0 * L.n * 24.0 + nb * 8.0 * L.n);
        a.trip = L.trip;
        launch_row(L.mode, OP_JACOBI, L.G, a, h->stream);
    }
    launch_copy(x, L.t.p, 3 * static_cast<int64_t>(L.nA), h->stream);
}

// One block Gauss-Seidel sweep by colours. x_zero: x is zero on entry (and
// its buffer holds the zeros), so the first colour's rows see only zero
// neighbours: x_i = D_i^{-1} b_i without reading their matrix rows.
static void gs_sweep(amg_ctx *h, int l, const double *b, double *x, bool forward, bool x_zero) {
    Level &L = h->lv[l];
    const int ncol = static_cast<int>(L.cptr.size()) - 1;
    const int nb = L.mode == 3 ? 9 : 1;
    for (int q = 0; q < ncol; ++q) {
        const int c = forward ? q : ncol - 1 - q;
        const int r0 = L.cptr[c], r1 = L.cptr[c + 1];
        if (r1 == r0) continue;
        if (q == 0 && x_zero) {
            ProfScope ps(h, tag("gs", l), (r1 - r0) * (4.0 + 48.0 + nb * 8.0));
            launch_diag_solve(L.mode, r1 - r0, L.g_rowid.p + r0, L.dinv.p, L.n, b, x, h->stream);
            continue;
        }
        RowArgs a;
        a.nrows = r1 - r0;
        a.rowptr = L.Ag.rowptr.p + r0;
        a.col = L.Ag.col.p;
        a.val = L.Ag.val.p;
        a.nnz = L.Ag.nnz;
        a.rowid = L.g_rowid.p + r0;
        a.x = x;
        a.b = b;
        a.y = x;
        a.dinv = L.dinv.p;
        a.dinv_n = L.n;
        a.xcd_chunks = L.gs_xcd;
        // matrix rows of this colour + row pointer, row id, b_i, x_i read and
        // write, inverted diagonal block
        const double bytes = static_cast<double>(L.colour_nnz[c]) * (L.Ag.np * 8.0 + 4.0) +
                             a.nrows * (8.0 + 24.0 + 48.0 + nb * 8.0);
        ProfScope ps(h, tag("gs", l), bytes);
        a.trip = L.tripg;
        launch_row(L.mode, OP_GS, L.Gg, a, h->stream);
    }
}

// zero_init: x is zero on entry; filled: its buffer already holds the zeros
void smooth(amg_ctx *h, int l, const double *b, double *x, bool pre, bool zero_init, bool filled) {
    const amg_params &p = h->prm;
    const int steps = pre ? p.pre : p.post;
    Level &L = h->lv[l];
    const bool need_fill = zero_init && !filled && (steps == 0 || p.smoother != AMG_SMOOTH_JA);
    if (need_fill) launch_fill(x, 0.0, 3 * static_cast<int64_t>(L.nA), h->stream);
    for (int k = 0; k < steps; ++k) {
        if (p.smoother == AMG_SMOOTH_JA)
            jacobi_step(h, l, b, x, zero_init && k == 0);
        else
            gs_sweep(h, l, b, x, pre || h->post_forward, pre && zero_init && k == 0);
    }
}

static void coarse_solve(amg_ctx *h, const double *b, double *x) {
    ProfScope ps(h, "coarse", static_cast<double>(h->coarse_m) * h->coarse_m * 8.0);
    launch_dense_gemv(h->coarse_inv.p, h->coarse_m, h->coarse_nc, b, x, h->stream);
}

// a batch of SPD systems: the systems ending on level l (its rows past nA)
// by their explicit inverses
static void ending_systems(amg_ctx *h, int l, const double *b, double *x) {
    Level &L = h->lv[l];
    if (L.dseg.count == 0) return;
    ProfScope ps(h, "coarse", L.dseg.bytes);
    launch_dense_segs<double>(L.dseg.view(), b, b, x, x, h->stream);
}

static void run_dense_tail(amg_ctx *h, const double *b, double *x) {
    ProfScope ps(h, "dense_tail", static_cast<double>(h->tail_m) * h->tail_m * 8.0);
    launch_dense_gemv(h->tail_dense.p, h->tail_m, h->tail_nc, b, x, h->stream);
}

static void run_tail(amg_ctx *h, const double *b, double *x, bool x_zero) {
    TailArgs a = h->tail_args;
    a.b_in = b;
    a.x_out = x;
    a.x_in_zero = x_zero ? 1 : 0;
    ProfScope ps(h, "tail", h->tail_bytes);
    launch_tail(h->lv[0].mode, a, h->tail_lds, 1, h->stream);
}

// Algorithm 1: AMG(K_l, x_l, b_l). x_zero: x_l is zero on entry (the first
// Jacobi step then needs no operator pass); filled: its buffer holds the zeros.
static void cycle(amg_ctx *h, int l, const double *b, double *x, bool x_zero, bool filled) {
    Level &L = h->lv[l];
    if (h->nsys > 0) ending_systems(h, l, b, x);
    if (L.coarsest) {
        if (h->nsys == 0) coarse_solve(h, b, x);
        return;
    }
    if (l == h->tail_start) {
        run_tail(h, b, x, x_zero);
        return;
    }
    if (l == h->dense_start && x_zero) {
        run_dense_tail(h, b, x);
        return;
    }
    smooth(h, l, b, x, true, x_zero, filled);
    residual(h, l, b, x, L.r.p, L.nA);
    Level &C = h->lv[l + 1];
    {
        // b_{l+1} = P^T r; the same pass zeroes x_{l+1} for the recursion
        RowArgs a = row_args(L.R);
        a.x = L.r.p;
        a.y = C.b.p;
        a.zero_out = C.x.p;
        ProfScope ps(h, tag("restrict", l), row_bytes(L.R, L.R.nnz, L.R.nrows) + 3.0 * (L.n + 2 * C.n) * 8.0);
        launch_row(1, OP_SPMV, L.Gr, a, h->stream);
    }
    if (C.coarsest) {
        if (h->nsys > 0) ending_systems(h, l + 1, C.b.p, C.x.p);
        else coarse_solve(h, C.b.p, C.x.p);
    } else {
        // x_{l+1} = 0, then nu recursive calls (nu = 1: V-cycle, 2: W-cycle)
        const int nu = std::max(1, h->prm.nu);
        for (int k = 0; k < nu; ++k) cycle(h, l + 1, C.b.p, C.x.p, k == 0, k == 0);
    }
    {
        RowArgs a = row_args(L.P);
        a.x = C.x.p;
        a.y = x;
        ProfScope ps(h, tag("prolong", l), row_bytes(L.P, L.P.nnz, L.P.nrows) + 3.0 * (2.0 * L.n + C.n) * 8.0);
        launch_row(1, OP_SPMV_ADD, L.Gp, a, h->stream);
    }
    smooth(h, l, b, x, false, false, false);
}

void vcycle(amg_ctx *h, int l, const double *b, double *x) { cycle(h, l, b, x, true, false); }

// z = M^{-1} r: `cycles` successive applications of Algorithm 1 on the
// finest level, the first from z = 0, each further one from the current z.
// z_filled: z already holds zeros.
static void precondition_eager(amg_ctx *h, const double *r, double *z, bool z_filled) {
    if (h->saddle) {
        saddle_precondition(h, r, z);
        return;
    }
    if (h->mixed) {
        precondition_mp(h, r, z);
        return;
    }
    const int cyc = std::max(1, h->prm.cycles);
    for (int k = 0; k < cyc; ++k) cycle(h, 0, r, z, k == 0, k == 0 && z_filled);
}

// The preconditioner's launches recorded once into a HIP graph per (r, z)
// pair and replayed: one launch call instead of hundreds. The recording
// runs on a stream of the library's own (a capture cannot run on the legacy
// default stream) and contains kernels only: no host synchronisation, no
// memset nodes, no event records (profiling runs eagerly).
static hipGraphExec_t graph_for(amg_ctx *h, const double *r, double *z, bool z_filled) {
    for (const auto &g : h->graphs)
        if (g.r == r && g.z == z && g.filled == z_filled) return g.exec;
    if (h->graphs.size() >= 8) return nullptr;
    hipStream_t cs = nullptr;
    AMG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    // the capture stream must see everything ordered before it on the caller's stream
    hipEvent_t ev;
    AMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    AMG_HIP(hipEventRecord(ev, h->stream));
    AMG_HIP(hipStreamWaitEvent(cs, ev, 0));
    const hipStream_t saved = h->stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    h->stream = cs;
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    try {
        precondition_eager(h, r, z, z_filled);
    } catch (...) {
        (void)hipStreamEndCapture(cs, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        h->stream = saved;
        (void)hipStreamDestroy(cs);
        (void)hipEventDestroy(ev);
        throw;
    }
    h->stream = saved;
    AMG_HIP(hipStreamEndCapture(cs, &graph));
    AMG_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    AMG_HIP(hipGraphDestroy(graph));
    AMG_HIP(hipStreamSynchronize(cs));
    AMG_HIP(hipStreamDestroy(cs));
    AMG_HIP(hipEventDestroy(ev));
    h->graphs.push_back({r, z, z_filled, exec});
    return exec;
}

// z = M^{-1} r for pointers that stay the same from call to call
static void precondition_impl(amg_ctx *h, const double *r, double *z, bool z_filled) {
    if (h->prm.graph && !h->prof) {
        if (hipGraphExec_t g = graph_for(h, r, z, z_filled)) {
            AMG_HIP(hipGraphLaunch(g, h->stream));
            return;
        }
    }
    precondition_eager(h, r, z, z_filled);
}

// z = M^{-1} r for pointers that change from call to call (the flexible
// GMRES basis): through staging vectors so that one recording serves all
void precondition_staged(amg_ctx *h, const double *r, double *z) {
    if (!h->prm.graph || h->prof) {
        precondition_eager(h, r, z, false);
        return;
    }
    if (h->g_in.n != static_cast<size_t>(h->n_dof)) {
        h->g_in.alloc(h->n_dof);
        h->g_out.alloc(h->n_dof);
    }
    launch_copy(h->g_in.p, r, h->n_dof, h->stream);
    precondition_impl(h, h->g_in.p, h->g_out.p, false);
    launch_copy(z, h->g_out.p, h->n_dof, h->stream);
}

void precondition(amg_ctx *h, const double *r, double *z) { precondition_impl(h, r, z, false); }

}  // namespace amgp2

// ---------------------------------------------------------------- Krylov
namespace amgp2 {

static double read_scalar(amg_ctx *h, int idx) {
    AMG_HIP(hipMemcpyAsync(h->h_sc, h->sc.p, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    AMG_HIP(hipStreamSynchronize(h->stream));
    return h->h_sc[idx];
}

// The scalars' copy to the host, waited on separately (scalars_wait), so
// that work enqueued in between overlaps the host's round trip.
static void scalars_begin(amg_ctx *h) {
    if (!h->sc_ready) AMG_HIP(hipEventCreateWithFlags(&h->sc_ready, hipEventDisableTiming));
    AMG_HIP(hipMemcpyAsync(h->h_sc, h->sc.p, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    AMG_HIP(hipEventRecord(h->sc_ready, h->stream));
}
static void scalars_wait(amg_ctx *h) { AMG_HIP(hipEventSynchronize(h->sc_ready)); }

// CG's stopping test waits for the scalars of iteration k on the host; while
// the last test's relative residual is still above KRYLOV_AHEAD * tol, the
// next preconditioner application, which only reads r and writes z, is
// enqueued before that wait, so the round trip overlaps the GPU's cycle. If
// the test then stops the solve, that application has changed nothing else.

static void dot_into(amg_ctx *h, const double *a, const double *b, int dst, int post = RED_NONE) {
    ProfScope ps(h, "blas", 2.0 * h->n_dof * 8.0);
    const int nb = launch_dot_partial(a, b, h->n_dof, h->partial.p, h->stream);
    launch_reduce(h->partial.p, nb, h->sc.p, dst, h->stream, post);
}

// q = A p on the finest level and <p, q> into sc[SC_PQ]
static void spmv_dot(amg_ctx *h, const double *p, double *q, int post) {
    Level &L = h->lv[0];
    RowArgs a = row_args(L.A);
    a.x = p;
    a.y = q;
    a.partial = h->partial.p;
    {
        ProfScope ps(h, "spmv.L0", row_bytes(L.A, L.A.nnz, L.n) + 3.0 * L.n * 16.0);
        a.trip = L.trip;
        launch_row(L.mode, OP_SPMV_DOT, L.G, a, h->stream);
    }
    launch_reduce(h->partial.p, row_blocks(L.n, L.G), h->sc.p, SC_PQ, h->stream, post);
}

// x += alpha p, r -= alpha q, <r, r> into sc[SC_RR]; zeroes z for the next
// preconditioner application
static void cg_update(amg_ctx *h, double *x, double *r, const double *p, const double *q, double *z) {
    ProfScope ps(h, "blas", 7.0 * h->n_dof * 8.0);
    const int nb = launch_cg_update(x, r, p, q, h->sc.p, h->n_dof, h->partial.p, z, h->stream);
    launch_reduce(h->partial.p, nb, h->sc.p, SC_RR, h->stream);
}

double true_relres(amg_ctx *h, const double *b, const double *x, double r0norm) {
    residual(h, 0, b, x, h->kw.p);
    dot_into(h, h->kw.p, h->kw.p, SC_TMP);
    const double rr = read_scalar(h, SC_TMP);
    return r0norm > 0.0 ? std::sqrt(rr) / r0norm : 0.0;
}

static int finish(amg_ctx *h, const double *b, const double *x, double r0, int it, int status,
                  std::chrono::steady_clock::time_point t0, amg_result *res) {
    const double rel = true_relres(h, b, x, r0);
    if (status == AMG_OK && !(rel == rel)) status = AMG_DIVERGED;
    if (res) {
        res->iters = it;
        res->status = status;
        res->relres = rel;
        res->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    profile_collect(h);
    return status;
}

// classify the recursive residual: converged, diverged, or continue (-1)
static int check(double rr, double rr0, double tol) {
    if (!(rr == rr) || std::isinf(rr)) return AMG_DIVERGED;
    const double rel = std::sqrt(rr / rr0);
    if (rel > 1e3) return AMG_DIVERGED;
    if (rel <= tol) return AMG_OK;
    return -1;
}

int solve_pcg(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = h->n_dof;
    double *r = h->kr.p, *z = h->kz.p, *p = h->kp.p, *q = h->kq.p;
    residual(h, 0, b, x, r);
    dot_into(h, r, r, SC_RR);
    const double rr0 = read_scalar(h, SC_RR);
    const double r0 = std::sqrt(rr0);
    if (rr0 == 0.0) return finish(h, b, x, r0, 0, AMG_OK, t0, res);
    if (!(rr0 == rr0)) return finish(h, b, x, r0, 0, AMG_DIVERGED, t0, res);
    precondition(h, r, z);
    dot_into(h, r, z, SC_RZ);
    launch_copy(p, z, n, h->stream);
    int it = 0, status = AMG_NOT_CONVERGED;
    double rel = 1.0;
    while (it < maxit) {
        spmv_dot(h, p, q, RED_CG_ALPHA);
        cg_update(h, x, r, p, q, z);
        ++it;
        scalars_begin(h);
        const bool ahead = it < maxit && rel > KRYLOV_AHEAD * tol;
        if (ahead) precondition_impl(h, r, z, true);
        scalars_wait(h);
        const double rr = h->h_sc[SC_RR];
        if (!(h->h_sc[SC_PQ] > 0.0)) { status = AMG_BREAKDOWN; break; }
        const int c = check(rr, rr0, tol);
        if (c >= 0) { status = c; break; }
        rel = std::sqrt(rr / rr0);
        if (!ahead) precondition_impl(h, r, z, true);
        dot_into(h, r, z, SC_TMP, RED_CG_BETA);
        launch_cg_direction(p, z, h->sc.p, n, h->stream);
    }
    return finish(h, b, x, r0, it, status, t0, res);
}

int solve_fcg(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = h->n_dof;
    double *r = h->kr.p, *z = h->kz.p, *p = h->kp.p, *q = h->kq.p;
    residual(h, 0, b, x, r);
    dot_into(h, r, r, SC_RR);
    const double rr0 = read_scalar(h, SC_RR);
    const double r0 = std::sqrt(rr0);
    if (rr0 == 0.0) return finish(h, b, x, r0, 0, AMG_OK, t0, res);
    if (!(rr0 == rr0)) return finish(h, b, x, r0, 0, AMG_DIVERGED, t0, res);
    int it = 0, status = AMG_NOT_CONVERGED;
    double rel = 1.0;
    bool ahead = false;  // this iteration's preconditioner already enqueued
    while (it < maxit) {
        if (!ahead) precondition_impl(h, r, z, it > 0);
        if (it == 0) {
            launch_copy(p, z, n, h->stream);
        } else {
            // p = z - (<z, q_prev> / <p_prev, q_prev>) p_prev
            dot_into(h, z, q, SC_TMP, RED_FCG_BETA);
            launch_cg_direction(p, z, h->sc.p, n, h->stream);
        }
        spmv_dot(h, p, q, RED_NONE);
        dot_into(h, p, r, SC_PR, RED_FCG_ALPHA);
        cg_update(h, x, r, p, q, z);
        ++it;
        scalars_begin(h);
        ahead = it < maxit && rel > KRYLOV_AHEAD * tol;
        if (ahead) precondition_impl(h, r, z, true);
        scalars_wait(h);
        const double rr = h->h_sc[SC_RR];
        if (!(h->h_sc[SC_PQ] > 0.0)) { status = AMG_BREAKDOWN; break; }
        const int c = check(rr, rr0, tol);
        if (c >= 0) { status = c; break; }
        rel = std::sqrt(rr / rr0);
    }
    return finish(h, b, x, r0, it, status, t0, res);
}

// Stand-alone AMG: repeated Algorithm 1 from the current iterate.
int solve_stationary(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    double *r = h->kr.p;
    residual(h, 0, b, x, r);
    dot_into(h, r, r, SC_RR);
    const double rr0 = read_scalar(h, SC_RR);
    const double r0 = std::sqrt(rr0);
    if (rr0 == 0.0) return finish(h, b, x, r0, 0, AMG_OK, t0, res);
    int it = 0, status = AMG_NOT_CONVERGED;
    const int cyc = std::max(1, h->prm.cycles);
    while (it < maxit) {
        for (int k = 0; k < cyc; ++k) cycle(h, 0, b, x, false, false);
        residual(h, 0, b, x, r);
        dot_into(h, r, r, SC_RR);
        ++it;
        const int c = check(read_scalar(h, SC_RR), rr0, tol);
        if (c >= 0) { status = c; break; }
    }
    return finish(h, b, x, r0, it, status, t0, res);
}

}  // namespace amgp2
