// The mixed-precision preconditioner: Algorithm 1 on FP32 vectors, with the
// finest operator in FP32 and the coarser ones in BF16 with per-row FP32
// scales (AMG_PREC_MIXED), or FP32 everywhere (AMG_PREC_FP32). The outer
// Krylov loop, its residual and dot products stay in FP64 (flexible CG or
// flexible GMRES absorb the variation of the reduced-precision cycle), and
// the coarsest solve stays the FP64 explicit inverse. The coarse end that is
// assembled as one operator (from level dense_start down) is applied from an
// FP32 copy of that FP64-assembled operator.
#include <algorithm>
#include <cmath>

#include "context.h"

namespace amgp2 {

// The reduced-precision kernels read half (FP32) or a quarter (BF16) of the
// bytes per entry, so their best lanes per row can differ from the FP64
// kernels': time them on their own, starting from the FP64 choice and
// switching only for a 3% gain.
static void autotune_mp(amg_ctx *h, Level &L) {
    hipStream_t s = h->stream;
    LevelMP &M = L.mp;
    const int cand[] = {8, 16, 32, 64};
    const int64_t nv = 3 * static_cast<int64_t>(L.n);
    launch_fill_f32(M.x.p, 0.f, nv, s);
    launch_fill_f32(M.b.p, 1.f, nv, s);
    launch_fill_f32(M.t.p, 0.f, nv, s);
    hipEvent_t e0, e1;
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
    auto time_it = [&](auto &&launch) {
        launch();
        launch();
        float best_ms = 1e30f;
        for (int r = 0; r < 7; ++r) {
            evict_caches(h);
            AMG_HIP(hipEventRecord(e0, s));
            launch();
            AMG_HIP(hipEventRecord(e1, s));
            AMG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
            best_ms = std::min(best_ms, ms);
        }
        return best_ms;
    };
    // (lanes G, entries per lane and trip T); the heuristic lane count with
    // T = 1 is kept unless another choice is at least 5% faster. T > 1 is
    // tried only where a trip of the row group (G T entries) is at most twice
    // the mean row.
    const double avg_row = static_cast<double>(L.A.nnz) / std::max(1, L.n);
    auto pick = [&](int G0, int &trip_out, auto &&time_of) {
        int bestG = G0, bestT = 1;
        float best = time_of(G0, 1);
        for (int T : {1, 2, 4})
            for (int G : cand) {
                if ((G == G0 && T == 1) || (T > 1 && G * T > 2.0 * avg_row)) continue;
                const float ms = time_of(G, T);
                if (ms < 0.95f * best) {
                    best = ms;
                    bestG = G;
                    bestT = T;
                }
            }
        trip_out = bestT;
        return bestG;
    };
    M.G = pick(M.G, M.trip, [&](int G, int P) {
        RowArgsMP a;
        a.nrows = L.n;
        a.rowptr = L.A.rowptr.p;
        a.col = L.A.col.p;
        a.val = M.aval();
        a.rscale = M.scale.p;
        a.nnz = L.A.nnz;
        a.x = M.x.p;
        a.b = M.b.p;
        a.y = M.r.p;
        a.trip = P;
        return time_it([&] { launch_row_mp(L.mode, OP_RESID, G, M.kind, a, s); });
    });
    if (!L.cptr.empty()) {
        // a whole forward sweep, colour by colour, as the smoother runs it;
        // then per-XCD contiguous rows for the chosen kernel
        auto sweep_time = [&](int G, int P, int xcd) {
            return time_it([&] {
                for (size_t c = 0; c + 1 < L.cptr.size(); ++c) {
                    if (L.cptr[c + 1] == L.cptr[c]) continue;
                    RowArgsMP a;
                    a.nrows = L.cptr[c + 1] - L.cptr[c];
                    a.rowptr = L.Ag.rowptr.p + L.cptr[c];
                    a.col = L.Ag.col.p;
                    a.val = M.agval();
                    a.rscale = M.scale.p;
                    a.nnz = L.Ag.nnz;
                    a.rowid = L.g_rowid.p + L.cptr[c];
                    a.x = M.t.p;
                    a.b = M.b.p;
                    a.y = M.t.p;
                    a.dinv = M.dinv.p;
                    a.dinv_n = L.n;
                    a.xcd_chunks = xcd;
                    a.trip = P;
                    launch_row_mp(L.mode, OP_GS, G, M.kind, a, s);
                }
            });
        };
        M.Gg = pick(M.Gg, M.tripg, [&](int G, int P) { return sweep_time(G, P, 0); });
        M.xcd = sweep_time(M.Gg, M.tripg, 1) < 0.95f * sweep_time(M.Gg, M.tripg, 0) ? 1 : 0;
    }
    AMG_HIP(hipEventDestroy(e0));
    AMG_HIP(hipEventDestroy(e1));
}

void build_mixed(amg_ctx *h) {
    hipStream_t s = h->stream;
    const int prec = h->prm.precision;
    h->mixed = prec != AMG_PREC_FP64;
    if (!h->mixed) return;
    for (size_t l = 0; l < h->lv.size(); ++l) {
        Level &L = h->lv[l];
        LevelMP &M = L.mp;
        const size_t nv = static_cast<size_t>(L.vlen());
        M.x.alloc(nv);
        M.b.alloc(nv);
        M.r.alloc(nv);
        M.t.alloc(nv);
        if (L.coarsest) continue;
        M.kind = (l == 0 || prec == AMG_PREC_FP32) ? VAL_F32 : VAL_BF16;
        const int64_t np = L.A.np;
        if (M.kind == VAL_F32) {
            M.a32.alloc(np * L.A.nnz);
            launch_planes_f32(L.A.val.p, M.a32.p, np * L.A.nnz, s);
            if (!L.cptr.empty()) {
                M.ag32.alloc(np * L.Ag.nnz);
                launch_planes_f32(L.Ag.val.p, M.ag32.p, np * L.Ag.nnz, s);
            }
        } else {
            M.scale.alloc(static_cast<size_t>(L.mode) * L.n);
            launch_row_scales(L.mode, L.n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.A.nnz, M.scale.p, s);
            M.a16.alloc(np * L.A.nnz);
            launch_planes_bf16(L.mode, L.n, L.A.rowptr.p, nullptr, L.A.val.p, L.A.nnz, M.scale.p, M.a16.p, s);
            if (!L.cptr.empty()) {
                M.ag16.alloc(np * L.Ag.nnz);
                launch_planes_bf16(L.mode, L.Ag.nrows, L.Ag.rowptr.p, L.g_rowid.p, L.Ag.val.p, L.Ag.nnz, M.scale.p,
                                   M.ag16.p, s);
            }
        }
        M.dinv.alloc(L.dinv.n);
        launch_to_f32(L.dinv.p, M.dinv.p, static_cast<int64_t>(L.dinv.n), s);
        M.pval.alloc(L.P.nnz);
        launch_to_f32(L.P.val.p, M.pval.p, L.P.nnz, s);
        M.rval.alloc(L.R.nnz);
        launch_to_f32(L.R.val.p, M.rval.p, L.R.nnz, s);
        // the tuner starts from the heuristic lane count, not from the FP64
        // kernels' tuned choice, so that its result does not inherit their
        // timing noise
        M.G = M.Gg = lanes_for(L.A.nnz, L.n);
        // (not the levels inside the assembled coarse end: those kernels do
        // not run in the cycle)
        if (h->prm.autotune && (h->dense_start < 0 || static_cast<int>(l) < h->dense_start)) autotune_mp(h, L);
    }
    refresh_tail_f32(h);
}

// FP32 copies of the saddle blocks, transfers and smoother scalings, and of
// the Braess-Sarazin Schur hierarchies (after build_mixed)
void build_saddle_mp(amg_ctx *h) {
    hipStream_t s = h->stream;
    auto conv = [&](DevBuf<float> &dst, const DevBuf<double> &src) {
        dst.alloc(std::max<size_t>(1, src.n));
        if (src.n) launch_to_f32(src.p, dst.p, static_cast<int64_t>(src.n), s);
    };
    for (Level &L : h->lv) {
        LevelMP &M = L.mp;
        conv(M.sB, L.B.val);
        conv(M.sBt, L.Bt.val);
        if (L.C.nnz > 0) conv(M.sC, L.C.val);
        if (L.H.nnz > 0) {
            conv(M.sH, L.H.val);
            conv(M.sHt, L.Ht.val);
        }
        if (L.sgs_scale.n) conv(M.sgs, L.sgs_scale);
        if (L.bs_ahat.n) conv(M.ahat, L.bs_ahat);
        if (L.nA > 0 && M.dinv.n == 0) conv(M.dinv, L.dinv);
        // assembled Schur coarse ends: FP32 copies for the FP32 cycle
        if (L.schur.dense_from >= 0 && L.schur.tdense.inv32.n == 0) L.schur.tdense.make_f32(s);
        for (SchurLevel &q : L.schur.lv) {
            conv(q.s32, q.S.val);
            if (q.Sg.nnz > 0) conv(q.sg32, q.Sg.val);
            if (q.dinv.n) conv(q.dinv32, q.dinv);
            const size_t m = std::max<size_t>(1, q.S.nrows);
            q.x32.alloc(m);
            q.b32.alloc(m);
            q.r32.alloc(m);
        }
    }
    AMG_HIP(hipStreamSynchronize(s));
}

void refresh_tail_f32(amg_ctx *h) {
    h->tail_dense32.release();
    h->tail_dense16.release();
    if (h->mixed && h->tail_m > 0) {
        // the coarse end below the finest level, in the coarse levels' value
        // type: BF16 in the FP32/BF16 cycle, FP32 in the FP32 cycle; rows
        // padded to a multiple of 8 values for the GEMV's 16-byte loads
        const int m = h->tail_m;
        h->tail_ld = (m + 7) / 8 * 8;
        const int64_t mm = static_cast<int64_t>(m) * h->tail_ld;
        if (h->prm.precision == AMG_PREC_MIXED) {
            h->tail_dense16.alloc(mm);
            launch_dense_copy(h->tail_dense.p, m, h->tail_ld, VAL_BF16, h->tail_dense16.p, h->stream);
        } else {
            h->tail_dense32.alloc(mm);
            launch_dense_copy(h->tail_dense.p, m, h->tail_ld, VAL_F32, h->tail_dense32.p, h->stream);
        }
    }
    AMG_HIP(hipStreamSynchronize(h->stream));
}

static std::string tag(const char *cls, int l) { return std::string(cls) + ".L" + std::to_string(l); }

static RowArgsMP args_natural(Level &L) {
    RowArgsMP a;
    a.nrows = L.n;
    a.rowptr = L.A.rowptr.p;
    a.col = L.A.col.p;
    a.val = L.mp.aval();
    a.rscale = L.mp.scale.p;
    a.nnz = L.A.nnz;
    a.trip = L.mp.trip;
    return a;
}

static double mat_bytes(const Level &L, int64_t nnz, int rows) {
    return static_cast<double>(nnz) * (L.A.np * L.mp.vbytes() + 4.0) + rows * 4.0 +
           (L.mp.kind == VAL_BF16 ? rows * 4.0 * L.mode : 0.0);
}

// (on the leading nA rows: in a batch, the systems still coarsening)
static void residual_mp(amg_ctx *h, int l, const float *b, const float *x, float *r) {
    Level &L = h->lv[l];
    RowArgsMP a = args_natural(L);
    a.nrows = L.nA;
    a.x = x;
    a.b = b;
    a.y = r;
    ProfScope ps(h, tag("resid", l), mat_bytes(L, L.A.nnz, L.nA) + 3.0 * L.nA * 12.0);
    launch_row_mp(L.mode, OP_RESID, L.mp.G, L.mp.kind, a, h->stream);
}

// One damped Jacobi step. The step reads x and writes its result out of
// place: into the other buffer of the level's pair (mp.x, mp.t), which the
// cycle then carries on with (returned), or, on a batch level whose rows past
// nA hold ending systems that live in x only, into mp.t and back to x.
static float *jacobi_mp(amg_ctx *h, int l, const float *b, float *x, bool zero) {
    Level &L = h->lv[l];
    const float om = static_cast<float>(
        h->level_omega.empty() ? h->prm.omega : h->level_omega[std::min<size_t>(l, h->level_omega.size() - 1)]);
    const int nb = L.mode == 3 ? 9 : 1;
    if (zero) {
        ProfScope ps(h, tag("jacobi0", l), 3.0 * L.nA * 8.0 + nb * 4.0 * L.nA);
        launch_jacobi_zero_mp(L.mode, L.nA, L.n, L.mp.dinv.p, b, om, x, h->stream);
        return x;
    }
    const bool swap = L.nA == L.n;
    float *out = swap && x == L.mp.t.p ? L.mp.x.p : L.mp.t.p;
    AMG_REQUIRE(out != x, AMG_EINVAL, "jacobi_mp: output aliases the input");
    RowArgsMP a = args_natural(L);
    a.nrows = L.nA;
    a.x = x;
    a.b = b;
    a.y = out;
    a.dinv = L.mp.dinv.p;
    a.dinv_n = L.n;
    a.omega = om;
    {
        ProfScope ps(h, tag("jacobi", l), mat_bytes(L, L.A.nnz, L.nA) + 3.0 * L.nA * 12.0 + nb * 4.0 * L.nA);
        launch_row_mp(L.mode, OP_JACOBI, L.mp.G, L.mp.kind, a, h->stream);
    }
    if (swap) return out;
    launch_copy_f32(x, out, 3 * static_cast<int64_t>(L.nA), h->stream);
    return x;
}

static void gs_mp(amg_ctx *h, int l, const float *b, float *x, bool forward, bool x_zero) {
    Level &L = h->lv[l];
    const int ncol = static_cast<int>(L.cptr.size()) - 1;
    const int nb = L.mode == 3 ? 9 : 1;
    for (int q = 0; q < ncol; ++q) {
        const int c = forward ? q : ncol - 1 - q;
        const int r0 = L.cptr[c], r1 = L.cptr[c + 1];
        if (r1 == r0) continue;
        if (q == 0 && x_zero) {
            ProfScope ps(h, tag("gs", l), (r1 - r0) * (4.0 + 24.0 + nb * 4.0));
            launch_diag_solve_mp(L.mode, r1 - r0, L.g_rowid.p + r0, L.mp.dinv.p, L.n, b, x, h->stream);
            continue;
        }
        RowArgsMP a;
        a.nrows = r1 - r0;
        a.rowptr = L.Ag.rowptr.p + r0;
        a.col = L.Ag.col.p;
        a.val = L.mp.agval();
        a.rscale = L.mp.scale.p;
        a.nnz = L.Ag.nnz;
        a.rowid = L.g_rowid.p + r0;
        a.x = x;
        a.b = b;
        a.y = x;
        a.dinv = L.mp.dinv.p;
        a.dinv_n = L.n;
        a.xcd_chunks = L.mp.xcd;
        a.trip = L.mp.tripg;
        ProfScope ps(h, tag("gs", l), mat_bytes(L, L.colour_nnz[c], a.nrows) + a.nrows * (4.0 + 12.0 + 24.0 + nb * 4.0));
        launch_row_mp(L.mode, OP_GS, L.mp.Gg, L.mp.kind, a, h->stream);
    }
}

// returns the buffer holding x_l afterwards (Jacobi steps alternate buffers)
static float *smooth_mp(amg_ctx *h, int l, const float *b, float *x, bool pre, bool zero_init, bool filled) {
    const amg_params &p = h->prm;
    const int steps = pre ? p.pre : p.post;
    Level &L = h->lv[l];
    if (zero_init && !filled && (steps == 0 || p.smoother != AMG_SMOOTH_JA))
        launch_fill_f32(x, 0.f, 3 * static_cast<int64_t>(L.nA), h->stream);
    for (int k = 0; k < steps; ++k) {
        if (p.smoother == AMG_SMOOTH_JA)
            x = jacobi_mp(h, l, b, x, zero_init && k == 0);
        else
            gs_mp(h, l, b, x, pre || h->post_forward, pre && zero_init && k == 0);
    }
    return x;
}

// coarsest level: the FP64 explicit inverse
static void coarse_mp(amg_ctx *h, int l, const float *b, float *x) {
    Level &L = h->lv[l];
    const int64_t nv = 3 * static_cast<int64_t>(L.n);
    launch_to_f64(b, L.b.p, nv, h->stream);
    {
        ProfScope ps(h, "coarse", static_cast<double>(h->coarse_m) * h->coarse_m * 8.0);
        launch_dense_gemv(h->coarse_inv.p, h->coarse_m, h->coarse_nc, L.b.p, L.x.p, h->stream);
    }
    launch_to_f32(L.x.p, x, nv, h->stream);
}

// a batch of SPD systems: the systems ending on level l (its rows past nA)
// by their FP64 explicit inverses, as the single-system coarsest level
static void ending_systems_mp(amg_ctx *h, int l, const float *b, float *x) {
    Level &L = h->lv[l];
    if (L.dseg.count == 0) return;
    const int64_t a0 = 3 * static_cast<int64_t>(L.nA), m = 3 * static_cast<int64_t>(L.n) - a0;
    launch_to_f64(b + a0, L.b.p + a0, m, h->stream);
    {
        ProfScope ps(h, "coarse", L.dseg.bytes);
        launch_dense_segs<double>(L.dseg.view(), L.b.p, L.b.p, L.x.p, L.x.p, h->stream);
    }
    launch_to_f32(L.x.p + a0, x + a0, m, h->stream);
}

// Algorithm 1 on level l from x (zero on entry if x_zero; filled: its
// buffer holds the zeros). Returns the buffer that holds x_l on return: x,
// or the other buffer of the level's pair after an odd number of Jacobi
// steps.
static float *cycle_mp(amg_ctx *h, int l, const float *b, float *x, bool x_zero, bool filled) {
    Level &L = h->lv[l];
    if (h->nsys > 0) ending_systems_mp(h, l, b, x);
    if (L.coarsest) {
        if (h->nsys == 0) coarse_mp(h, l, b, x);
        return x;
    }
    if (l == h->dense_start && x_zero) {
        const bool bf = h->tail_dense16.n > 0;
        ProfScope ps(h, "dense_tail", static_cast<double>(h->tail_m) * h->tail_m * (bf ? 2.0 : 4.0));
        if (bf)
            launch_dense_gemv_bf16(h->tail_dense16.p, h->tail_m, h->tail_ld, h->tail_nc, b, x, h->stream);
        else
            launch_dense_gemv_f32(h->tail_dense32.p, h->tail_m, h->tail_ld, h->tail_nc, b, x, h->stream);
        return x;
    }
    x = smooth_mp(h, l, b, x, true, x_zero, filled);
    residual_mp(h, l, b, x, L.mp.r.p);
    Level &C = h->lv[l + 1];
    {
        RowArgsMP a;
        a.nrows = L.R.nrows;
        a.rowptr = L.R.rowptr.p;
        a.col = L.R.col.p;
        a.val = L.mp.rval.p;
        a.nnz = L.R.nnz;
        a.x = L.mp.r.p;
        a.y = C.mp.b.p;
        a.zero_out = C.mp.x.p;
        ProfScope ps(h, tag("restrict", l), L.R.nnz * 8.0 + 3.0 * (L.n + 2 * C.n) * 4.0);
        launch_row_mp(1, OP_SPMV, L.Gr, VAL_F32, a, h->stream);
    }
    float *e = C.mp.x.p;
    if (C.coarsest) {
        if (h->nsys > 0) ending_systems_mp(h, l + 1, C.mp.b.p, e);
        else coarse_mp(h, l + 1, C.mp.b.p, e);
    } else {
        const int nu = std::max(1, h->prm.nu);
        for (int k = 0; k < nu; ++k) e = cycle_mp(h, l + 1, C.mp.b.p, e, k == 0, k == 0);
    }
    {
        RowArgsMP a;
        a.nrows = L.P.nrows;
        a.rowptr = L.P.rowptr.p;
        a.col = L.P.col.p;
        a.val = L.mp.pval.p;
        a.nnz = L.P.nnz;
        a.x = e;
        a.y = x;
        ProfScope ps(h, tag("prolong", l), L.P.nnz * 8.0 + 3.0 * (2.0 * L.n + C.n) * 4.0);
        launch_row_mp(1, OP_SPMV_ADD, L.Gp, VAL_F32, a, h->stream);
    }
    return smooth_mp(h, l, b, x, false, false, false);
}

void precondition_mp(amg_ctx *h, const double *r, double *z) {
    Level &L = h->lv[0];
    const int64_t nv = 3 * static_cast<int64_t>(L.n);
    launch_to_f32(r, L.mp.b.p, nv, h->stream);
    const int cyc = std::max(1, h->prm.cycles);
    float *x = L.mp.x.p;
    for (int k = 0; k < cyc; ++k) x = cycle_mp(h, 0, L.mp.b.p, x, k == 0, false);
    launch_to_f64(x, z, nv, h->stream);
}

}  // namespace amgp2
