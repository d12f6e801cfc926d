// amg_solve_multi: K right-hand sides on one SPD hierarchy. The V-cycle of
// Algorithm 1 and the outer PCG / flexible CG run on interleaved blocks of K
// vectors (multi.h), so every matrix pass serves all K; each right-hand side
// keeps its own Krylov scalars, stopping test and iteration count, and one
// that has converged (or broken down) keeps its iterate while the others go
// on. Arithmetic per right-hand side is that of amg_solve up to the order of
// the floating-point sums.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>

#include "context.h"
#include "multi.h"

namespace amgp2 {

static double mlevel_omega(amg_ctx *h, int l) {
    if (!h->level_omega.empty()) return h->level_omega[std::min<size_t>(l, h->level_omega.size() - 1)];
    return h->prm.omega;
}

// The cycle on block vectors. T = double (FP64 hierarchy) or float (the
// reduced-precision copies: FP32 finest, FP32 or BF16 below).
template <typename T>
struct MCycle {
    amg_ctx *h;
    MultiWork &W;
    int K;
    static constexpr bool RP = std::is_same<T, float>::value;

    int kind(const Level &L) const { return RP ? (L.mp.kind == VAL_BF16 ? MK_BF16 : MK_F32) : MK_F64; }
    const void *aval(const Level &L) const { return RP ? L.mp.aval() : static_cast<const void *>(L.A.val.p); }
    const void *agval(const Level &L) const { return RP ? L.mp.agval() : static_cast<const void *>(L.Ag.val.p); }
    const void *dinv(const Level &L) const {
        return RP ? static_cast<const void *>(L.mp.dinv.p) : static_cast<const void *>(L.dinv.p);
    }
    T *vx(int l) { return RP ? reinterpret_cast<T *>(W.lv[l].x32.p) : reinterpret_cast<T *>(W.lv[l].x.p); }
    T *vb(int l) { return RP ? reinterpret_cast<T *>(W.lv[l].b32.p) : reinterpret_cast<T *>(W.lv[l].b.p); }
    T *vr(int l) { return RP ? reinterpret_cast<T *>(W.lv[l].r32.p) : reinterpret_cast<T *>(W.lv[l].r.p); }
    T *vt(int l) { return RP ? reinterpret_cast<T *>(W.lv[l].t32.p) : reinterpret_cast<T *>(W.lv[l].t.p); }
    int64_t len(int l) const { return 3 * static_cast<int64_t>(h->lv[l].n) * K; }

    MRowArgs natural(const Level &L) const {
        MRowArgs a;
        a.nrows = L.n;
        a.rowptr = L.A.rowptr.p;
        a.col = L.A.col.p;
        a.val = aval(L);
        a.rscale = L.mp.scale.n ? L.mp.scale.p : nullptr;
        a.nnz = L.A.nnz;
        return a;
    }

    void fill0(T *x, int64_t n) {
        if (RP)
            launch_fill_f32(reinterpret_cast<float *>(x), 0.f, n, h->stream);
        else
            launch_fill(reinterpret_cast<double *>(x), 0.0, n, h->stream);
    }
    void copy(T *dst, const T *src, int64_t n) {
        if (RP)
            launch_copy_f32(reinterpret_cast<float *>(dst), reinterpret_cast<const float *>(src), n, h->stream);
        else
            launch_copy(reinterpret_cast<double *>(dst), reinterpret_cast<const double *>(src), n, h->stream);
    }

    // one damped Jacobi step, out of place into the other buffer of the
    // level's pair (vt, or vx when x is vt); returns the buffer with the result
    T *jacobi(int l, const T *b, T *x, bool zero) {
        Level &L = h->lv[l];
        const double om = mlevel_omega(h, l);
        if (zero) {
            launch_mjacobi_zero(L.mode, RP ? MK_F32 : MK_F64, K, L.n, dinv(L), b, om, x, h->stream);
            return x;
        }
        T *out = x == vt(l) ? vx(l) : vt(l);
        MRowArgs a = natural(L);
        a.x = x;
        a.b = b;
        a.y = out;
        a.dinv = dinv(L);
        a.dinv_n = L.n;
        a.omega = om;
        launch_mrow(L.mode, M_JACOBI, kind(L), K, a, h->stream);
        return out;
    }

    void gs(int l, const T *b, T *x, bool forward, bool x_zero) {
        Level &L = h->lv[l];
        const int ncol = static_cast<int>(L.cptr.size()) - 1;
        for (int q = 0; q < ncol; ++q) {
            const int c = forward ? q : ncol - 1 - q;
            const int r0 = L.cptr[c], r1 = L.cptr[c + 1];
            if (r1 == r0) continue;
            if (q == 0 && x_zero) {
                launch_mdiag_solve(L.mode, RP ? MK_F32 : MK_F64, K, r1 - r0, L.g_rowid.p + r0, dinv(L), L.n, b, x,
                                   h->stream);
                continue;
            }
            MRowArgs a;
            a.nrows = r1 - r0;
            a.rowptr = L.Ag.rowptr.p + r0;
            a.col = L.Ag.col.p;
            a.val = agval(L);
            a.rscale = L.mp.scale.n ? L.mp.scale.p : nullptr;
            a.nnz = L.Ag.nnz;
            a.rowid = L.g_rowid.p + r0;
            a.x = x;
            a.b = b;
            a.y = x;
            a.dinv = dinv(L);
            a.dinv_n = L.n;
            launch_mrow(L.mode, M_GS, kind(L), K, a, h->stream);
        }
    }

    T *smooth(int l, const T *b, T *x, bool pre, bool zero_init) {
        const amg_params &p = h->prm;
        const int steps = pre ? p.pre : p.post;
        if (zero_init && (steps == 0 || p.smoother != AMG_SMOOTH_JA)) fill0(x, len(l));
        for (int k = 0; k < steps; ++k) {
            if (p.smoother == AMG_SMOOTH_JA)
                x = jacobi(l, b, x, zero_init && k == 0);
            else
                gs(l, b, x, pre, pre && zero_init && k == 0);
        }
        return x;
    }

    // the coarsest level: the FP64 explicit inverse on all K columns
    void coarse(int l, const T *b, T *x) {
        const int64_t n = len(l);
        if (RP) {
            launch_to_f64(reinterpret_cast<const float *>(b), W.lv[l].b.p, n, h->stream);
            launch_mdense(MK_F64, h->coarse_inv.p, h->coarse_m, h->coarse_m, h->coarse_nc * K, W.lv[l].b.p,
                          W.lv[l].x.p, h->stream);
            launch_to_f32(W.lv[l].x.p, reinterpret_cast<float *>(x), n, h->stream);
        } else {
            launch_mdense(MK_F64, h->coarse_inv.p, h->coarse_m, h->coarse_m, h->coarse_nc * K, b, x, h->stream);
        }
    }

    // returns the buffer that holds x_l on return (Jacobi steps alternate)
    T *cycle(int l, const T *b, T *x, bool x_zero) {
        Level &L = h->lv[l];
        if (L.coarsest) {
            coarse(l, b, x);
            return x;
        }
        if (l == h->dense_start && x_zero) {
            const int nc = h->tail_nc * K;
            if (!RP)
                launch_mdense(MK_F64, h->tail_dense.p, h->tail_m, h->tail_m, nc, b, x, h->stream);
            else if (h->tail_dense16.n)
                launch_mdense(MK_BF16, h->tail_dense16.p, h->tail_m, h->tail_ld, nc, b, x, h->stream);
            else
                launch_mdense(MK_F32, h->tail_dense32.p, h->tail_m, h->tail_ld, nc, b, x, h->stream);
            return x;
        }
        x = smooth(l, b, x, true, x_zero);
        {
            MRowArgs a = natural(L);
            a.x = x;
            a.b = b;
            a.y = vr(l);
            launch_mrow(L.mode, M_RESID, kind(L), K, a, h->stream);
        }
        Level &C = h->lv[l + 1];
        {
            MRowArgs a;
            a.nrows = L.R.nrows;
            a.rowptr = L.R.rowptr.p;
            a.col = L.R.col.p;
            a.val = RP ? static_cast<const void *>(L.mp.rval.p) : static_cast<const void *>(L.R.val.p);
            a.nnz = L.R.nnz;
            a.x = vr(l);
            a.y = vb(l + 1);
            a.zero_out = vx(l + 1);
            launch_mrow(1, M_SPMV, RP ? MK_F32 : MK_F64, K, a, h->stream);
        }
        T *e = vx(l + 1);
        if (C.coarsest) {
            coarse(l + 1, vb(l + 1), e);
        } else {
            const int nu = std::max(1, h->prm.nu);
            for (int k = 0; k < nu; ++k) e = cycle(l + 1, vb(l + 1), e, k == 0);
        }
        {
            MRowArgs a;
            a.nrows = L.P.nrows;
            a.rowptr = L.P.rowptr.p;
            a.col = L.P.col.p;
            a.val = RP ? static_cast<const void *>(L.mp.pval.p) : static_cast<const void *>(L.P.val.p);
            a.nnz = L.P.nnz;
            a.x = e;
            a.y = x;
            launch_mrow(1, M_SPMV_ADD, RP ? MK_F32 : MK_F64, K, a, h->stream);
        }
        return smooth(l, b, x, false, false);
    }

    // z = M^{-1} r on FP64 blocks of the finest level
    void precondition(const double *r, double *z) {
        const int64_t n = len(0);
        const int cyc = std::max(1, h->prm.cycles);
        if (RP) {
            launch_to_f32(r, W.lv[0].b32.p, n, h->stream);
            T *x = reinterpret_cast<T *>(W.lv[0].x32.p);
            for (int k = 0; k < cyc; ++k) x = cycle(0, reinterpret_cast<const T *>(W.lv[0].b32.p), x, k == 0);
            launch_to_f64(reinterpret_cast<const float *>(x), z, n, h->stream);
        } else {
            // (z pairs with the level's t buffer; the result ends in z)
            T *x = reinterpret_cast<T *>(z);
            for (int k = 0; k < cyc; ++k) x = cycle(0, reinterpret_cast<const T *>(r), x, k == 0);
            if (x != reinterpret_cast<T *>(z)) copy(reinterpret_cast<T *>(z), x, n);
        }
    }
};

static void multi_alloc(amg_ctx *h, MultiWork &W, int K) {
    if (W.K == K && W.lv.size() == h->lv.size()) return;  // kept from the last call with this K
    W.K = K;
    W.lv.resize(h->lv.size());
    for (size_t l = 0; l < h->lv.size(); ++l) {
        const size_t n = 3 * static_cast<size_t>(h->lv[l].n) * K;
        MultiLevelWork &w = W.lv[l];
        if (h->mixed) {
            w.x32.alloc(n);
            w.b32.alloc(n);
            w.r32.alloc(n);
            w.t32.alloc(n);
            if (h->lv[l].coarsest) {
                w.x.alloc(n);
                w.b.alloc(n);
            }
        } else {
            w.x.alloc(n);
            w.b.alloc(n);
            w.r.alloc(n);
            w.t.alloc(n);
        }
    }
    const size_t nd = static_cast<size_t>(h->n_dof) * K;
    for (DevBuf<double> *v : {&W.B, &W.X, &W.R, &W.Z, &W.P, &W.Q}) v->alloc(nd);
    W.partial.alloc(static_cast<size_t>(mdot_blocks(h->n_dof)) * 3 * K);
    W.dots.alloc(3 * K);
    W.coef.alloc(static_cast<size_t>(MultiWork::SLOTS) * 2 * MULTI_MAX_K);
    if (!W.h_coef)
        AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&W.h_coef),
                              MultiWork::SLOTS * 2 * MULTI_MAX_K * sizeof(double)));
    if (!W.h_dots) AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&W.h_dots), 3 * MULTI_MAX_K * sizeof(double)));
}

// y = A x on the finest level (FP64), K columns
static void mapply(amg_ctx *h, int K, const double *x, double *y) {
    Level &L = h->lv[0];
    MRowArgs a;
    a.nrows = L.n;
    a.rowptr = L.A.rowptr.p;
    a.col = L.A.col.p;
    a.val = L.A.val.p;
    a.nnz = L.A.nnz;
    a.x = x;
    a.y = y;
    launch_mrow(L.mode, M_SPMV, MK_F64, K, a, h->stream);
}

// dots of up to 3 pairs over the K columns, read back to the host (the
// synchronisation also completes every coefficient copy issued before)
static std::vector<double> mdots(amg_ctx *h, MultiWork &W, int np, const double *a0, const double *b0,
                                 const double *a1 = nullptr, const double *b1 = nullptr,
                                 const double *a2 = nullptr, const double *b2 = nullptr) {
    const double *A[3] = {a0, a1, a2}, *B[3] = {b0, b1, b2};
    launch_mdot(np, W.K, h->n_dof, A, B, W.partial.p, W.dots.p, h->stream);
    AMG_HIP(hipMemcpyAsync(W.h_dots, W.dots.p, static_cast<size_t>(np) * W.K * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    AMG_HIP(hipStreamSynchronize(h->stream));
    W.used = 0;
    return std::vector<double>(W.h_dots, W.h_dots + np * W.K);
}

// y = cy y + cx x with per-column coefficients, staged through a pinned slot
// (slots are reused only after a synchronisation in mdots)
static void mcomb(amg_ctx *h, MultiWork &W, double *y, const std::vector<double> &cy, const double *x,
                  const std::vector<double> &cx) {
    if (W.used == MultiWork::SLOTS) {
        AMG_HIP(hipStreamSynchronize(h->stream));
        W.used = 0;
    }
    const int slot = W.used++;
    double *c = W.h_coef + static_cast<size_t>(slot) * 2 * MULTI_MAX_K;
    double *d = W.coef.p + static_cast<size_t>(slot) * 2 * MULTI_MAX_K;
    for (int r = 0; r < W.K; ++r) {
        c[r] = cy[r];
        c[W.K + r] = cx[r];
    }
    AMG_HIP(hipMemcpyAsync(d, c, 2 * W.K * sizeof(double), hipMemcpyHostToDevice, h->stream));
    launch_mlincomb(W.K, h->n_dof, y, d, x, d + W.K, h->stream);
}

int solve_multi(amg_ctx *h, int nrhs, const double *B, double *X, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    AMG_REQUIRE(!h->saddle && h->nsys == 0, AMG_EINVAL, "amg_solve_multi: SPD systems only");
    AMG_REQUIRE(h->prm.krylov == AMG_KRYLOV_PCG || h->prm.krylov == AMG_KRYLOV_FCG, AMG_EINVAL,
                "amg_solve_multi: needs PCG or FCG");
    AMG_REQUIRE(!h->post_forward, AMG_EINVAL, "amg_solve_multi: needs the symmetric cycle");
    AMG_REQUIRE(nrhs >= 1 && nrhs <= MULTI_MAX_K, AMG_EINVAL, "amg_solve_multi: 1 to 8 right-hand sides");
    const int K = nrhs <= 2 ? 2 : (nrhs <= 4 ? 4 : 8);
    MultiWork &W = h->multi;
    multi_alloc(h, W, K);
    W.used = 0;
    hipStream_t s = h->stream;
    const int64_t nd = h->n_dof;
    launch_interleave(K, nrhs, nd, B, W.B.p, true, s);
    launch_interleave(K, nrhs, nd, X, W.X.p, true, s);
    MCycle<double> c64{h, W, K};
    MCycle<float> c32{h, W, K};
    auto prec = [&](const double *r, double *z) {
        if (h->mixed)
            c32.precondition(r, z);
        else
            c64.precondition(r, z);
    };
    const std::vector<double> one(K, 1.0), zero(K, 0.0), mone(K, -1.0);
    // R = B - A X
    mapply(h, K, W.X.p, W.R.p);
    mcomb(h, W, W.R.p, mone, W.B.p, one);
    std::vector<double> rr0 = mdots(h, W, 1, W.R.p, W.R.p);
    std::vector<int> status(K, AMG_NOT_CONVERGED), iters(K, 0), active(K, 0);
    for (int r = 0; r < K; ++r) {
        if (r >= nrhs || rr0[r] == 0.0) {
            status[r] = AMG_OK;
        } else if (!(rr0[r] == rr0[r]) || std::isinf(rr0[r])) {
            status[r] = AMG_DIVERGED;
        } else {
            active[r] = 1;
        }
    }
    auto any_active = [&]() { return std::any_of(active.begin(), active.end(), [](int a) { return a != 0; }); };
    const bool fcg = h->prm.krylov == AMG_KRYLOV_FCG;
    std::vector<double> rz(K, 0.0), pq_prev(K, 0.0), alpha(K, 0.0), beta(K, 0.0), malpha(K, 0.0);
    int it = 0;
    if (!fcg && any_active()) {
        prec(W.R.p, W.Z.p);
        const std::vector<double> d = mdots(h, W, 1, W.R.p, W.Z.p);
        for (int r = 0; r < K; ++r) rz[r] = d[r];
        launch_copy(W.P.p, W.Z.p, nd * K, s);
    }
    // While every running column's last relative residual is above
    // KRYLOV_AHEAD * tol, the next preconditioner application goes ahead of
    // the stopping test's read, and its dot (<r, z> for CG, <z, q> for FCG)
    // comes back in the same read: one host round trip less per iteration,
    // the same arithmetic.
    double relmin = 1.0;
    bool ahead = false;             // z of this iteration already computed
    std::vector<double> zdot(K);    // its dot, read with the last stopping test
    while (it < maxit && any_active()) {
        if (fcg) {
            if (!ahead) prec(W.R.p, W.Z.p);
            if (it == 0) {
                launch_copy(W.P.p, W.Z.p, nd * K, s);
            } else {
                // beta = -<z, q_prev> / <p_prev, q_prev>: p = z + beta p_prev
                const std::vector<double> d = ahead ? zdot : mdots(h, W, 1, W.Z.p, W.Q.p);
                for (int r = 0; r < K; ++r) beta[r] = active[r] && pq_prev[r] != 0.0 ? -d[r] / pq_prev[r] : 0.0;
                mcomb(h, W, W.P.p, beta, W.Z.p, one);
            }
        }
        mapply(h, K, W.P.p, W.Q.p);
        const std::vector<double> d = fcg ? mdots(h, W, 2, W.P.p, W.Q.p, W.P.p, W.R.p) : mdots(h, W, 1, W.P.p, W.Q.p);
        for (int r = 0; r < K; ++r) {
            alpha[r] = 0.0;
            if (!active[r]) continue;
            const double pq = d[r];
            if (!(pq > 0.0) || !std::isfinite(pq)) {
                status[r] = (pq == pq) ? AMG_BREAKDOWN : AMG_DIVERGED;
                active[r] = 0;
                continue;
            }
            alpha[r] = (fcg ? d[K + r] : rz[r]) / pq;
            pq_prev[r] = pq;
        }
        for (int r = 0; r < K; ++r) malpha[r] = -alpha[r];
        mcomb(h, W, W.X.p, one, W.P.p, alpha);
        mcomb(h, W, W.R.p, one, W.Q.p, malpha);
        ++it;
        ahead = it < maxit && relmin > KRYLOV_AHEAD * tol;
        std::vector<double> rrv;
        if (ahead) {
            prec(W.R.p, W.Z.p);
            rrv = fcg ? mdots(h, W, 2, W.R.p, W.R.p, W.Z.p, W.Q.p) : mdots(h, W, 2, W.R.p, W.R.p, W.R.p, W.Z.p);
            std::copy(rrv.begin() + K, rrv.end(), zdot.begin());
        } else {
            rrv = mdots(h, W, 1, W.R.p, W.R.p);
        }
        relmin = 1e300;
        for (int r = 0; r < K; ++r) {
            if (!active[r]) continue;
            iters[r] = it;
            const double rr = rrv[r];
            if (!(rr == rr) || std::isinf(rr) || std::sqrt(rr / rr0[r]) > 1e3) {
                status[r] = AMG_DIVERGED;
                active[r] = 0;
            } else if (std::sqrt(rr / rr0[r]) <= tol) {
                status[r] = AMG_OK;
                active[r] = 0;
            } else {
                relmin = std::min(relmin, std::sqrt(rr / rr0[r]));
            }
        }
        if (!fcg && it < maxit && any_active()) {
            if (!ahead) prec(W.R.p, W.Z.p);
            const std::vector<double> dz = ahead ? zdot : mdots(h, W, 1, W.R.p, W.Z.p);
            for (int r = 0; r < K; ++r) {
                beta[r] = active[r] && rz[r] != 0.0 ? dz[r] / rz[r] : 0.0;
                if (active[r]) rz[r] = dz[r];
            }
            mcomb(h, W, W.P.p, beta, W.Z.p, one);
        }
    }
    // true residuals
    mapply(h, K, W.X.p, W.R.p);
    mcomb(h, W, W.R.p, mone, W.B.p, one);
    std::vector<double> rr = mdots(h, W, 1, W.R.p, W.R.p);
    launch_interleave(K, nrhs, nd, W.X.p, X, false, s);
    AMG_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = AMG_OK;
    for (int r = 0; r < nrhs; ++r) {
        const double rel = rr0[r] > 0.0 ? std::sqrt(rr[r] / rr0[r]) : 0.0;
        int st = status[r];
        if (st == AMG_OK && !(rel == rel)) st = AMG_DIVERGED;
        if (res) {
            res[r].iters = iters[r];
            res[r].status = st;
            res[r].relres = rel;
            res[r].solve_ms = ms;
        }
        worst = std::max(worst, st);
    }
    return worst;
}

}  // namespace amgp2
