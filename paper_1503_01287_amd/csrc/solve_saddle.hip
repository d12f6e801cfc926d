// Saddle point systems K [u; p] = [f; g], K = [[A, B^T], [B, -C]]
// (Section 2.4): Algorithm 1 with the segregated Gauss-Seidel (Uzawa) or the
// Braess-Sarazin smoother of Section 3.3, the saddle Galerkin hierarchy K_{l+1} = P^T K_l P
// with P = diag(I, J, H), and right-preconditioned flexible GMRES (the
// paper's outer method for these systems, Section 4.4).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "context.h"
#include "multi.h"

namespace amgp2 {

static int lanes(int64_t nnz, int nrows) {
    const double avg = nrows > 0 ? static_cast<double>(nnz) / nrows : 1.0;
    int G = 4;
    while (G < 64 && G < avg) G *= 2;
    return G;
}

static BlkArgs blk(const DMat &m) {
    BlkArgs a;
    a.nrows = m.nrows;
    a.rowptr = m.rowptr.p;
    a.col = m.col.p;
    a.val = m.val.p;
    a.nnz = m.nnz;
    return a;
}

static std::string tag(const char *cls, int l) { return std::string(cls) + ".L" + std::to_string(l); }

void saddle_setup_level(amg_ctx *h, Level &L) {
    hipStream_t s = h->stream;
    L.Gb = lanes(L.B.nnz, L.B.nrows);
    L.Gbt = lanes(L.Bt.nnz, L.Bt.nrows);
    L.sgs_scale.alloc(std::max(1, L.n_pres));
    launch_sgs_scale(L.n_pres, L.B.rowptr.p, L.B.col.p, L.B.val.p, L.B.nnz, L.dinv.p, L.n, h->prm.sgs_damping,
                     L.C.nnz > 0 ? L.C.rowptr.p : nullptr, L.C.col.p, L.C.val.p, L.C.nnz, L.sgs_scale.p, s);
    if (h->prm.smoother == AMG_SMOOTH_BS) {
        L.bs_ahat.alloc(3 * static_cast<size_t>(std::max(1, L.n)));
        launch_bs_diag(L.n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.A.nnz, L.bs_ahat.p, s);
    }
    AMG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- precision views
// The cycle below runs on FP64 data (T = double) or on the FP32 copies of the
// reduced-precision cycle (T = float); SV<T> gives the level's arrays of each.
template <typename T>
struct SV;
template <>
struct SV<double> {
    static double *x(Level &L) { return L.x.p; }
    static double *b(Level &L) { return L.b.p; }
    static double *r(Level &L) { return L.r.p; }
    static double *t(Level &L) { return L.t.p; }
    static const double *B(const Level &L) { return L.B.val.p; }
    static const double *Bt(const Level &L) { return L.Bt.val.p; }
    static const double *C(const Level &L) { return L.C.val.p; }
    static const double *H(const Level &L) { return L.H.val.p; }
    static const double *Ht(const Level &L) { return L.Ht.val.p; }
    static const double *dinv(const Level &L) { return L.dinv.p; }
    static const double *sgs(const Level &L) { return L.sgs_scale.p; }
    static const double *ahat(const Level &L) { return L.bs_ahat.p; }
    static const double *S(const SchurLevel &q) { return q.S.val.p; }
    static const double *Sg(const SchurLevel &q) { return q.Sg.val.p; }
    static const double *sdinv(const SchurLevel &q) { return q.dinv.p; }
    static double *sx(SchurLevel &q) { return q.x.p; }
    static double *sb(SchurLevel &q) { return q.b.p; }
    static double *sr(SchurLevel &q) { return q.r.p; }
};
template <>
struct SV<float> {
    static float *x(Level &L) { return L.mp.x.p; }
    static float *b(Level &L) { return L.mp.b.p; }
    static float *r(Level &L) { return L.mp.r.p; }
    static float *t(Level &L) { return L.mp.t.p; }
    static const float *B(const Level &L) { return L.mp.sB.p; }
    static const float *Bt(const Level &L) { return L.mp.sBt.p; }
    static const float *C(const Level &L) { return L.mp.sC.p; }
    static const float *H(const Level &L) { return L.mp.sH.p; }
    static const float *Ht(const Level &L) { return L.mp.sHt.p; }
    static const float *dinv(const Level &L) { return L.mp.dinv.p; }
    static const float *sgs(const Level &L) { return L.mp.sgs.p; }
    static const float *ahat(const Level &L) { return L.mp.ahat.p; }
    static const float *S(const SchurLevel &q) { return q.s32.p; }
    static const float *Sg(const SchurLevel &q) { return q.sg32.p; }
    static const float *sdinv(const SchurLevel &q) { return q.dinv32.p; }
    static float *sx(SchurLevel &q) { return q.x32.p; }
    static float *sb(SchurLevel &q) { return q.b32.p; }
    static float *sr(SchurLevel &q) { return q.r32.p; }
};

template <typename T>
static BlkArgsT<T> blkT(const DMat &m, const T *val) {
    BlkArgsT<T> a;
    a.nrows = m.nrows;
    a.rowptr = m.rowptr.p;
    a.col = m.col.p;
    a.val = val;
    a.nnz = m.nnz;
    return a;
}

static void fillv(double *x, int64_t n, hipStream_t s) { launch_fill(x, 0.0, n, s); }
static void fillv(float *x, int64_t n, hipStream_t s) { launch_fill_f32(x, 0.f, n, s); }
static void axpbyv(double *y, const double *x, double a, double b, int64_t n, hipStream_t s) {
    launch_axpby(y, x, a, b, n, s);
}
static void axpbyv(float *y, const float *x, float a, float b, int64_t n, hipStream_t s) {
    launch_axpby_f(y, x, a, b, n, s);
}

// r_u = f - A u on the first nrows velocity nodes (3x3 blocks)
static void a_resid(amg_ctx *h, int l, const double *b, const double *x, double *r, int nrows) {
    Level &L = h->lv[l];
    RowArgs a;
    a.nrows = nrows;
    a.rowptr = L.A.rowptr.p;
    a.col = L.A.col.p;
    a.val = L.A.val.p;
    a.nnz = L.A.nnz;
    a.x = x;
    a.b = b;
    a.y = r;
    ProfScope ps(h, tag("resid", l), static_cast<double>(L.A.nnz) * 76.0 + L.n * 76.0);
    a.trip = L.trip;
    launch_row(3, OP_RESID, L.G, a, h->stream);
}
static void a_resid(amg_ctx *h, int l, const float *b, const float *x, float *r, int nrows) {
    Level &L = h->lv[l];
    RowArgsMP a;
    a.nrows = nrows;
    a.rowptr = L.A.rowptr.p;
    a.col = L.A.col.p;
    a.val = L.mp.aval();
    a.rscale = L.mp.scale.p;
    a.nnz = L.A.nnz;
    a.x = x;
    a.b = b;
    a.y = r;
    a.trip = L.mp.trip;
    ProfScope ps(h, tag("resid", l), static_cast<double>(L.A.nnz) * (9.0 * L.mp.vbytes() + 4.0) + L.n * 40.0);
    launch_row_mp(3, OP_RESID, L.mp.G, L.mp.kind, a, h->stream);
}
// velocity restriction (R = P^T, scalar per component) into the next level
static void restrict_u(amg_ctx *h, int l, const double *r, double *bc) {
    Level &L = h->lv[l];
    RowArgs a;
    a.nrows = L.R.nrows;
    a.rowptr = L.R.rowptr.p;
    a.col = L.R.col.p;
    a.val = L.R.val.p;
    a.nnz = L.R.nnz;
    a.x = r;
    a.y = bc;
    launch_row(1, OP_SPMV, L.Gr, a, h->stream);
}
static void restrict_u(amg_ctx *h, int l, const float *r, float *bc) {
    Level &L = h->lv[l];
    RowArgsMP a;
    a.nrows = L.R.nrows;
    a.rowptr = L.R.rowptr.p;
    a.col = L.R.col.p;
    a.val = L.mp.rval.p;
    a.nnz = L.R.nnz;
    a.x = r;
    a.y = bc;
    launch_row_mp(1, OP_SPMV, L.Gr, VAL_F32, a, h->stream);
}
static void prolong_u(amg_ctx *h, int l, const double *xc, double *x) {
    Level &L = h->lv[l];
    RowArgs a;
    a.nrows = L.P.nrows;
    a.rowptr = L.P.rowptr.p;
    a.col = L.P.col.p;
    a.val = L.P.val.p;
    a.nnz = L.P.nnz;
    a.x = xc;
    a.y = x;
    launch_row(1, OP_SPMV_ADD, L.Gp, a, h->stream);
}
static void prolong_u(amg_ctx *h, int l, const float *xc, float *x) {
    Level &L = h->lv[l];
    RowArgsMP a;
    a.nrows = L.P.nrows;
    a.rowptr = L.P.rowptr.p;
    a.col = L.P.col.p;
    a.val = L.mp.pval.p;
    a.nnz = L.P.nnz;
    a.x = xc;
    a.y = x;
    launch_row_mp(1, OP_SPMV_ADD, L.Gp, VAL_F32, a, h->stream);
}

// r = [f - A u - B^T p ; g - B u + C p] on level l for the first nrows_u
// velocity nodes and nrows_p pressure nodes (r and b are full level vectors)
template <typename T>
static void saddle_residual_rows(amg_ctx *h, int l, const T *b, const T *x, T *r, int nrows_u, int nrows_p) {
    Level &L = h->lv[l];
    const int64_t nu = 3 * static_cast<int64_t>(L.n);
    a_resid(h, l, b, x, r, nrows_u);
    BlkArgsT<T> bt = blkT<T>(L.Bt, SV<T>::Bt(L));
    bt.nrows = nrows_u;
    bt.x = x + nu;
    bt.y = r;
    launch_blk<T>(3, 1, BLK_SUB, L.Gbt, bt, h->stream);
    // g - B u + C p in one pass over the pressure rows
    BlkArgsT<T> bb = blkT<T>(L.B, SV<T>::B(L));
    bb.nrows = nrows_p;
    bb.x = x;
    bb.b = b + nu;
    bb.y = r + nu;
    if (L.C.nnz > 0) {
        bb.c_rowptr = L.C.rowptr.p;
        bb.c_col = L.C.col.p;
        bb.c_val = SV<T>::C(L);
        bb.c_x = x + nu;
        bb.c_sign = T(1);
    }
    launch_blk<T>(1, 3, BLK_RESID, L.Gb, bb, h->stream);
}

static void saddle_residual(amg_ctx *h, int l, const double *b, const double *x, double *r) {
    saddle_residual_rows<double>(h, l, b, x, r, h->lv[l].n, h->lv[l].n_pres);
}

// y = K_l x
void saddle_apply(amg_ctx *h, int l, const double *x, double *y) {
    Level &L = h->lv[l];
    const int64_t nu = 3 * static_cast<int64_t>(L.n);
    {
        RowArgs a;
        a.nrows = L.n;
        a.rowptr = L.A.rowptr.p;
        a.col = L.A.col.p;
        a.val = L.A.val.p;
        a.nnz = L.A.nnz;
        a.x = x;
        a.y = y;
        ProfScope ps(h, tag("spmv", l), static_cast<double>(L.A.nnz) * 76.0 + L.n * 52.0);
        a.trip = L.trip;
        launch_row(3, OP_SPMV, L.G, a, h->stream);
    }
    BlkArgs bt = blk(L.Bt);
    bt.x = x + nu;
    bt.y = y;
    launch_blk(3, 1, BLK_ADD, L.Gbt, bt, h->stream);
    // B u - C p in one pass over the pressure rows
    BlkArgs bb = blk(L.B);
    bb.x = x;
    bb.y = y + nu;
    if (L.C.nnz > 0) {
        bb.c_rowptr = L.C.rowptr.p;
        bb.c_col = L.C.col.p;
        bb.c_val = L.C.val.p;
        bb.c_x = x + nu;
        bb.c_sign = -1.0;
    }
    launch_blk(1, 3, BLK_SPMV, L.Gb, bb, h->stream);
}

// One segregated Gauss-Seidel step (reading of Section 3.3: K_hat =
// [[M_A, 0], [B, -omega^{-1} S_d]], M_A = damped block Jacobi, S_d =
// diag(B M_A^{-1} B^T + C)): du = M_A^{-1} r_u, dp = omega S_d^{-1}(B du - r_p),
// on the smoothed rows of the level. x_zero: the iterate is zero, so the
// residual is the right-hand side.
template <typename T>
static void sgs_step(amg_ctx *h, int l, const T *b, T *x, bool x_zero) {
    Level &L = h->lv[l];
    const int64_t nu = 3 * static_cast<int64_t>(L.n);
    const T *r = b;
    if (!x_zero) {
        saddle_residual_rows<T>(h, l, b, x, SV<T>::r(L), L.nA, L.npA);
        r = SV<T>::r(L);
    }
    // from a zero guess the step writes x outright (no fill before it)
    launch_sgs_u<T>(L.nA, L.n, SV<T>::dinv(L), r, static_cast<T>(h->prm.sgs_damping), SV<T>::t(L), x, x_zero,
                    h->stream);
    BlkArgsT<T> bb = blkT<T>(L.B, SV<T>::B(L));
    bb.nrows = L.npA;
    bb.x = SV<T>::t(L);
    bb.b = r + nu;
    bb.y = x + nu;
    bb.y_zero = x_zero ? 1 : 0;
    bb.dscale = SV<T>::sgs(L);
    bb.omega = static_cast<T>(h->prm.sgs_omega);
    launch_blk<T>(1, 3, BLK_SGS_P, L.Gb, bb, h->stream);
}

// Scalar V(1,1) cycle on level k of the Schur hierarchy of saddle level l,
// from a zero guess: Gauss-Seidel colour by colour on the smoothed rows
// (forward before the coarse correction, backward after it), restriction
// with H^T and prolongation with H of saddle level l + k; rows that end on
// this level are solved by their explicit inverses.
template <typename T>
static void schur_vcycle(amg_ctx *h, int l, int k, const T *b, T *x) {
    SchurHier &sh = h->lv[l].schur;
    SchurLevel &q = sh.lv[k];
    hipStream_t s = h->stream;
    if (k == sh.dense_from) {
        launch_dense_segs<T>(sh.tdense.view(), static_cast<const T *>(nullptr), b, static_cast<T *>(nullptr), x, s);
        return;
    }
    if (q.dseg.count > 0)
        launch_dense_segs<T>(q.dseg.view(), static_cast<const T *>(nullptr), b, static_cast<T *>(nullptr), x, s);
    if (q.nA == 0) return;
    const int nc = static_cast<int>(q.cptr.size()) - 1;
    fillv(x, q.nA, s);
    for (int c = 0; c < nc; ++c)
        launch_scalar_gs<T>(q.cptr[c + 1] - q.cptr[c], q.Sg.rowptr.p + q.cptr[c], q.Sg.col.p, SV<T>::Sg(q),
                            q.rowid.p + q.cptr[c], SV<T>::sdinv(q), b, x, q.G, s);
    BlkArgsT<T> ra = blkT<T>(q.S, SV<T>::S(q));
    ra.nrows = q.nA;
    ra.x = x;
    ra.b = b;
    ra.y = SV<T>::sr(q);
    launch_blk<T>(1, 1, BLK_RESID, q.G, ra, s);
    const Level &V = h->lv[l + k];
    SchurLevel &n = sh.lv[k + 1];
    BlkArgsT<T> ht = blkT<T>(V.Ht, SV<T>::Ht(V));
    ht.x = SV<T>::sr(q);
    ht.y = SV<T>::sb(n);
    launch_blk<T>(1, 1, BLK_SPMV, V.Ght, ht, s);
    schur_vcycle<T>(h, l, k + 1, SV<T>::sb(n), SV<T>::sx(n));
    BlkArgsT<T> hh = blkT<T>(V.H, SV<T>::H(V));
    hh.x = SV<T>::sx(n);
    hh.y = x;
    launch_blk<T>(1, 1, BLK_ADD, V.Gh, hh, s);
    for (int c = nc - 1; c >= 0; --c)
        launch_scalar_gs<T>(q.cptr[c + 1] - q.cptr[c], q.Sg.rowptr.p + q.cptr[c], q.Sg.col.p, SV<T>::Sg(q),
                            q.rowid.p + q.cptr[c], SV<T>::sdinv(q), b, x, q.G, s);
}

// The Schur cycle of saddle level l from Schur level k down is a fixed linear
// map of its right-hand side (zero initial guess), block diagonal over the
// systems of a batch. From the first level k >= 1 (k >= 0 below the finest
// saddle level) whose systems all have at most SCHUR_DENSE_MAX rows, it is
// assembled once, column by column from unit right-hand sides (one per
// system at a time), and applied as one segmented GEMV: the same map as the
// colour sweeps it replaces, up to rounding order.
constexpr int SCHUR_DENSE_MAX = 1500;

// The Schur cycle of setup_schur_dense on SCHUR_COLS columns at once, for
// its assembly: the scalar Schur levels run as the multi-right-hand-side
// row kernels (multi.h) over 3 x SCHUR_K interleaved columns (S applied to
// each column), so that the operators are read once for all of them. Same
// steps as schur_vcycle (forward sweep by colours from zero, residual,
// H^T, recursion, H, backward sweep; systems ending on a level by their
// explicit inverses); the sweeps take the correction form x_i += (b_i -
// sum_j S_ij x_j) / S_ii, equal to the direct form up to rounding.
constexpr int SCHUR_K = 16;
constexpr int SCHUR_COLS = 3 * SCHUR_K;

struct SchurBlockWork {
    std::vector<DevBuf<double>> x, b, r;
};

static void schur_block_cycle(amg_ctx *h, int l, int k, SchurBlockWork &W, const double *b, double *x) {
    SchurHier &sh = h->lv[l].schur;
    SchurLevel &q = sh.lv[k];
    hipStream_t s = h->stream;
    if (q.dseg.count > 0) launch_dense_segs_block(q.dseg.view(), SCHUR_COLS, b, x, s);
    if (q.nA == 0) return;
    launch_fill(x, 0.0, static_cast<int64_t>(q.nA) * SCHUR_COLS, s);
    const int nc = static_cast<int>(q.cptr.size()) - 1;
    auto sweep = [&](int c) {
        const int rows = q.cptr[c + 1] - q.cptr[c];
        if (rows == 0) return;
        MRowArgs a;
        a.nrows = rows;
        a.rowptr = q.Sg.rowptr.p + q.cptr[c];
        a.col = q.Sg.col.p;
        a.val = q.Sg.val.p;
        a.nnz = q.Sg.nnz;
        a.rowid = q.rowid.p + q.cptr[c];
        a.x = x;
        a.b = b;
        a.y = x;
        a.dinv = q.dinv.p;
        a.dinv_n = q.S.nrows;
        launch_mrow(1, M_GS, MK_F64, SCHUR_K, a, s);
    };
    for (int c = 0; c < nc; ++c) sweep(c);
    {
        MRowArgs a;
        a.nrows = q.nA;
        a.rowptr = q.S.rowptr.p;
        a.col = q.S.col.p;
        a.val = q.S.val.p;
        a.nnz = q.S.nnz;
        a.x = x;
        a.b = b;
        a.y = W.r[k].p;
        launch_mrow(1, M_RESID, MK_F64, SCHUR_K, a, s);
    }
    const Level &V = h->lv[l + k];
    {
        MRowArgs a;
        a.nrows = V.Ht.nrows;
        a.rowptr = V.Ht.rowptr.p;
        a.col = V.Ht.col.p;
        a.val = V.Ht.val.p;
        a.nnz = V.Ht.nnz;
        a.x = W.r[k].p;
        a.y = W.b[k + 1].p;
        launch_mrow(1, M_SPMV, MK_F64, SCHUR_K, a, s);
    }
    schur_block_cycle(h, l, k + 1, W, W.b[k + 1].p, W.x[k + 1].p);
    {
        MRowArgs a;
        a.nrows = V.H.nrows;
        a.rowptr = V.H.rowptr.p;
        a.col = V.H.col.p;
        a.val = V.H.val.p;
        a.nnz = V.H.nnz;
        a.x = W.x[k + 1].p;
        a.y = x;
        launch_mrow(1, M_SPMV_ADD, MK_F64, SCHUR_K, a, s);
    }
    for (int c = nc - 1; c >= 0; --c) sweep(c);
}

void setup_schur_dense(amg_ctx *h, int l) {
    SchurHier &sh = h->lv[l].schur;
    if (!h->prm.fuse_coarse) return;  // launch by launch (amg_params::fuse_coarse = 0)
    const int K = static_cast<int>(sh.lv.size()) - 1;  // the last level is already explicit
    int k0 = -1;
    for (int k = (l == 0 ? 1 : 0); k < K; ++k) {
        const auto &rows = sh.lv[k].blk_rows;
        if (!rows.empty() && *std::max_element(rows.begin(), rows.end()) <= SCHUR_DENSE_MAX) {
            k0 = k;
            break;
        }
    }
    if (k0 < 0) return;
    SchurLevel &q = sh.lv[k0];
    hipStream_t s = h->stream;
    sh.dense_from = -1;
    sh.tdense = DenseSegs();
    int mmax = 0;
    for (size_t b = 0; b < q.blk_rows.size(); ++b) {
        if (q.blk_rows[b] == 0) continue;
        sh.tdense.add(q.blk_rows[b], 0, 0, q.blk_off[b]);
        mmax = std::max(mmax, q.blk_rows[b]);
    }
    sh.tdense.finalize(s);
    const DenseSegView v = sh.tdense.view();
    // SCHUR_COLS unit columns of every system per blocked cycle
    SchurBlockWork W;
    const int nlev = static_cast<int>(sh.lv.size());
    W.x.resize(nlev);
    W.b.resize(nlev);
    W.r.resize(nlev);
    for (int k = k0; k < nlev; ++k) {
        const size_t len = static_cast<size_t>(std::max(1, sh.lv[k].S.nrows)) * SCHUR_COLS;
        W.x[k].alloc(len);
        W.b[k].alloc(len);
        W.r[k].alloc(len);
    }
    const int64_t n0 = static_cast<int64_t>(std::max(1, q.S.nrows)) * SCHUR_COLS;
    for (int j0 = 0; j0 < mmax; j0 += SCHUR_COLS) {
        launch_fill(W.b[k0].p, 0.0, n0, s);
        launch_segment_units_block(v, j0, SCHUR_COLS, W.b[k0].p, s);
        schur_block_cycle(h, l, k0, W, W.b[k0].p, W.x[k0].p);
        launch_segment_store_block(v, j0, SCHUR_COLS, W.x[k0].p, sh.tdense.inv.p, s);
    }
    AMG_HIP(hipStreamSynchronize(s));
    sh.dense_from = k0;
}

// One Braess-Sarazin step (Section 3.3): K_hat = [[A_hat, B^T], [B, B A_hat^{-1} B^T - S_hat]]
// with A_hat = 2 diag(A) and S_hat^{-1} one scalar V-cycle for
// S = C + B A_hat^{-1} B^T. Solving K_hat [du; dp] = [r_u; r_p]:
// S_hat dp = B A_hat^{-1} r_u - r_p, du = A_hat^{-1}(r_u - B^T dp).
// The cycle is linear and odd, so it is run on -(B A_hat^{-1} r_u - r_p)
// and returns -dp exactly (negation commutes with every rounding).
template <typename T>
static void bs_step(amg_ctx *h, int l, const T *b, T *x, bool x_zero) {
    Level &L = h->lv[l];
    hipStream_t s = h->stream;
    const int64_t nu = 3 * static_cast<int64_t>(L.n);
    // from a zero guess the residual is b and the step writes x outright
    const T *r = b;
    if (!x_zero) {
        saddle_residual_rows<T>(h, l, b, x, SV<T>::r(L), L.nA, L.npA);
        r = SV<T>::r(L);
    }
    launch_scale<T>(3 * static_cast<int64_t>(L.nA), SV<T>::ahat(L), r, SV<T>::t(L), s);
    SchurLevel &q0 = L.schur.lv[0];
    BlkArgsT<T> bb = blkT<T>(L.B, SV<T>::B(L));
    bb.nrows = L.npA;
    bb.x = SV<T>::t(L);
    bb.b = r + nu;
    bb.y = SV<T>::sb(q0);
    launch_blk<T>(1, 3, BLK_RESID, L.Gb, bb, s);
    schur_vcycle<T>(h, l, 0, SV<T>::sb(q0), SV<T>::sx(q0));
    if (x_zero)
        launch_neg<T>(L.npA, SV<T>::sx(q0), x + nu, s);
    else
        axpbyv(x + nu, SV<T>::sx(q0), T(-1), T(1), L.npA, s);
    // u += ahat (r_u + B^T s_x), one pass
    BlkArgsT<T> bt = blkT<T>(L.Bt, SV<T>::Bt(L));
    bt.nrows = L.nA;
    bt.x = SV<T>::sx(q0);
    bt.b = r;
    bt.y = x;
    bt.dscale = SV<T>::ahat(L);
    bt.y_zero = x_zero ? 1 : 0;
    launch_blk<T>(3, 1, BLK_ADD_SCALED, L.Gbt, bt, s);
}

// One multiplicative Vanka sweep (Section 3.3): the patches colour by
// colour, each x_P += omega K_P^{-1} (b - K x)_P with the residual of the
// current iterate (FP64 only).
static void vanka_step(amg_ctx *h, int l, const double *b, double *x) {
    Level &L = h->lv[l];
    const VankaView v = vanka_view(L);
    const int nc = static_cast<int>(L.vanka.cptr.size()) - 1;
    ProfScope ps(h, tag("vanka", l), L.vanka.inv_bytes);  // algorithmic: the patch inverses
    VankaData &V = L.vanka;
    for (int c = 0; c < nc; ++c) {
        const int cnt = V.cptr[c + 1] - V.cptr[c];
        if (V.path == 2)
            launch_vanka_colour_tiled(v, V.order.p + V.cptr[c], V.tpre.p + V.cptr[c], V.upre.p + V.cptr[c],
                                      V.rpre[VankaData::rg_index(V.rg)].p + V.cptr[c], cnt, V.ntiles[c], V.nunits[c],
                                      V.nrunits[VankaData::rg_index(V.rg)][c], V.cc, V.rg,
                                      V.roff.p, V.rbuf.p, V.poff.p, V.pbuf.p, b, x, h->prm.vanka_omega, h->stream);
        else if (V.path == 3)
            launch_vanka_colour_rows(v, V.order.p + V.cptr[c], V.tpre.p + V.cptr[c],
                                     V.rpre[VankaData::rg_index(V.rg)].p + V.cptr[c], cnt, V.ntiles[c],
                                     V.nrunits[VankaData::rg_index(V.rg)][c], V.rg, V.aw, V.roff.p, V.rbuf.p, b, x,
                                     h->prm.vanka_omega, h->stream);
        else if (V.path == 1)
            launch_vanka_colour_split(v, V.order.p + V.cptr[c], V.tpre.p + V.cptr[c], cnt, V.ntiles[c], V.max_nodes,
                                      V.roff.p, V.rbuf.p, b, x, h->prm.vanka_omega, h->stream);
        else
            launch_vanka_colour(v, V.order.p + V.cptr[c], cnt, V.max_nodes, b, x, h->prm.vanka_omega, h->stream);
    }
}
static void vanka_step(amg_ctx *, int, const float *, float *) {
    throw Error(AMG_EUNSUPPORTED, "the Vanka smoother runs in FP64");
}

template <typename T>
static void saddle_step(amg_ctx *h, int l, const T *b, T *x, bool x_zero) {
    if (h->prm.smoother == AMG_SMOOTH_BS)
        bs_step<T>(h, l, b, x, x_zero);
    else if (h->prm.smoother == AMG_SMOOTH_VANKA)
        vanka_step(h, l, b, x);
    else
        sgs_step<T>(h, l, b, x, x_zero);
}

// Algorithm 1 on saddle level l: systems that end on this level take their
// explicit inverse; the others are smoothed, restricted with P^T = diag(I, J, H)^T,
// corrected from level l + 1 and smoothed again.
template <typename T>
static void saddle_cycle(amg_ctx *h, int l, const T *b, T *x, bool x_zero) {
    Level &L = h->lv[l];
    const int64_t nu = 3 * static_cast<int64_t>(L.n);
    if (l == h->saddle_tail_from && x_zero) {
        ProfScope ps(h, "saddle_tail", h->saddle_tail.bytes);
        launch_dense_segs<T>(h->saddle_tail.view(), b, b + nu, x, x + nu, h->stream);
        return;
    }
    if (L.dseg.count > 0) {
        ProfScope ps(h, "coarse", L.dseg.bytes);
        launch_dense_segs<T>(L.dseg.view(), b, b + nu, x, x + nu, h->stream);
    }
    if (L.nA == 0) return;
    const amg_params &p = h->prm;
    // a zero guess is filled in unless the first smoothing step writes every
    // row of x without reading it (sGS, Braess-Sarazin)
    if (x_zero && !((p.smoother == AMG_SMOOTH_SGS || p.smoother == AMG_SMOOTH_BS) && p.pre >= 1)) {
        fillv(x, 3 * static_cast<int64_t>(L.nA), h->stream);
        fillv(x + nu, L.npA, h->stream);
    }
    for (int k = 0; k < p.pre; ++k) saddle_step<T>(h, l, b, x, x_zero && k == 0);
    saddle_residual_rows<T>(h, l, b, x, SV<T>::r(L), L.nA, L.npA);
    Level &C = h->lv[l + 1];
    const int64_t ncu = 3 * static_cast<int64_t>(C.n);
    restrict_u(h, l, SV<T>::r(L), SV<T>::b(C));
    {
        BlkArgsT<T> ht = blkT<T>(L.Ht, SV<T>::Ht(L));
        ht.x = SV<T>::r(L) + nu;
        ht.y = SV<T>::b(C) + ncu;
        launch_blk<T>(1, 1, BLK_SPMV, L.Ght, ht, h->stream);
    }
    const int nu_rec = C.nA > 0 ? std::max(1, p.nu) : 1;
    for (int k = 0; k < nu_rec; ++k) saddle_cycle<T>(h, l + 1, SV<T>::b(C), SV<T>::x(C), k == 0);
    prolong_u(h, l, SV<T>::x(C), x);
    {
        BlkArgsT<T> hh = blkT<T>(L.H, SV<T>::H(L));
        hh.x = SV<T>::x(C) + ncu;
        hh.y = x + nu;
        launch_blk<T>(1, 1, BLK_ADD, L.Gh, hh, h->stream);
    }
    for (int k = 0; k < p.post; ++k) saddle_step<T>(h, l, b, x, false);
}

// z = M^{-1} r (FP64 vectors). The reduced-precision cycle converts r to
// FP32 on the finest level and z back to FP64; the outer FGMRES stays FP64.
void saddle_precondition(amg_ctx *h, const double *r, double *z) {
    const int cyc = std::max(1, h->prm.cycles);
    if (h->mixed) {
        Level &L0 = h->lv[0];
        const int64_t n = L0.vlen();
        launch_to_f32(r, L0.mp.b.p, n, h->stream);
        for (int k = 0; k < cyc; ++k) saddle_cycle<float>(h, 0, L0.mp.b.p, L0.mp.x.p, k == 0);
        launch_to_f64(L0.mp.x.p, z, n, h->stream);
        return;
    }
    for (int k = 0; k < cyc; ++k) saddle_cycle<double>(h, 0, r, z, k == 0);
}

void saddle_smooth(amg_ctx *h, int l, const double *b, double *x) { saddle_step<double>(h, l, b, x, false); }

// Below the finest level a saddle cycle is entered from a zero guess, so the
// cycle from level d down is a fixed linear map of its right-hand side, block
// diagonal over the systems of a batch (the smoothers, transfers and coarse
// solves are linear; Vanka's and Braess-Sarazin's inner solves included).
// From the first level d >= 1 on which every system has at most
// SADDLE_TAIL_MAX rows, the GEMV would beat the cycle and the assembly fits
// the setup budget, it is assembled once, column by column from unit
// right-hand sides (one per system at a time) through the FP64 cycle (which
// applies the map of level d + 1, assembled first, instead of recursing),
// and applied as one segmented GEMV: the same map as the launches it replaces,
// up to rounding order, kept where it measures faster than those launches. Visits
// of level d from a nonzero guess (the second recursion of a W-cycle) still
// run the cycle itself. Called after the reduced-precision copies exist.
constexpr int SADDLE_TAIL_MAX = 5000;
constexpr double SADDLE_TAIL_BYTES_MAX = 2.0e9;
constexpr double SADDLE_TAIL_SETUP_MS = 2000.0;

void setup_saddle_tail(amg_ctx *h) {
    h->saddle_tail_from = -1;
    h->saddle_tail = DenseSegs();
    // the choice below is timed: without the tuner, setups stay timing-free
    if (!h->saddle || !h->prm.fuse_coarse || !h->prm.autotune) return;
    const int last = static_cast<int>(h->lv.size()) - 1;
    hipStream_t s = h->stream;
    hipEvent_t e0, e1;
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
    // one cycle from level d from a zero guess, FP64 or in the precision the
    // solves use
    auto time_cycle = [&](int d, bool fp64) {
        Level &L = h->lv[d];
        const int64_t nv = std::max<int64_t>(1, L.vlen());
        const bool mp = h->mixed && !fp64;
        if (mp) launch_fill_f32(L.mp.b.p, 1.f, nv, s);
        else launch_fill(L.b.p, 1.0, nv, s);
        float best = 1e30f;
        for (int r = 0; r < 4; ++r) {
            evict_caches(h);
            AMG_HIP(hipEventRecord(e0, s));
            if (mp) saddle_cycle<float>(h, d, L.mp.b.p, L.mp.x.p, true);
            else saddle_cycle<double>(h, d, L.b.p, L.x.p, true);
            AMG_HIP(hipEventRecord(e1, s));
            AMG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) best = std::min(best, ms);
        }
        return best;
    };
    for (int d = 1; d < last; ++d) {
        Level &L = h->lv[d];
        if (L.sys_n.empty()) {
            L.sys_noff.assign(1, 0);
            L.sys_n.assign(1, L.n);
            L.sys_poff.assign(1, 0);
            L.sys_np.assign(1, L.n_pres);
        }
        if (L.nA == 0) break;  // every system ends here: already one explicit solve
        int mmax = 0;
        double bytes = 0.0;
        for (size_t j = 0; j < L.sys_n.size(); ++j) {
            const int m = 3 * L.sys_n[j] + L.sys_np[j];
            mmax = std::max(mmax, m);
            bytes += 8.0 * m * static_cast<double>(m);
        }
        if (mmax > SADDLE_TAIL_MAX || bytes > SADDLE_TAIL_BYTES_MAX) continue;
        // the GEMV streams the maps at no more than about 5 TB/s: assemble
        // them only where that already beats the launches they would
        // replace, and where the assembly (one FP64 cycle per column) stays
        // within SADDLE_TAIL_SETUP_MS; otherwise try a coarser level
        const float sparse_ms = time_cycle(d, false);
        const double gemv_bytes = h->mixed ? 0.5 * bytes : bytes;  // FP32 copy in FP32 cycles
        if (gemv_bytes / 5.0e9 >= 0.9 * sparse_ms) continue;
        const float asm_ms = h->mixed ? time_cycle(d, true) : sparse_ms;
        if (static_cast<double>(mmax) * asm_ms > SADDLE_TAIL_SETUP_MS) continue;
        // the maps' layout on level lev (one square block per system);
        // returns the largest block
        auto layout = [&](int lev, DenseSegs &T) {
            Level &V = h->lv[lev];
            if (V.sys_n.empty()) {
                V.sys_noff.assign(1, 0);
                V.sys_n.assign(1, V.n);
                V.sys_poff.assign(1, 0);
                V.sys_np.assign(1, V.n_pres);
            }
            int mm = 0;
            for (size_t j = 0; j < V.sys_n.size(); ++j) {
                const int m = 3 * V.sys_n[j] + V.sys_np[j];
                mm = std::max(mm, m);
                if (m > 0) T.add(m, 3 * V.sys_noff[j], 3 * V.sys_n[j], V.sys_poff[j]);
            }
            T.finalize(s);
            return mm;
        };
        // the GEMV's own time, on a zero map of the same layout, before the
        // assembly (one FP64 cycle per column) is paid for
        {
            DenseSegs trial;
            layout(d, trial);
            if (trial.inv.n) launch_fill(trial.inv.p, 0.0, static_cast<int64_t>(trial.inv.n), s);
            if (h->mixed) trial.make_f32(s);
            h->saddle_tail = std::move(trial);
            h->saddle_tail_from = d;
            const float est_ms = time_cycle(d, false);
            h->saddle_tail_from = -1;
            h->saddle_tail = DenseSegs();
            if (!(est_ms < 0.95f * sparse_ms)) continue;
        }
        // the map of level lev, column by column from unit right-hand sides
        // through the FP64 cycle (as it stands: with the map of a coarser
        // level in place, the cycle applies that map instead of recursing)
        auto assemble = [&](int lev, DenseSegs &T) {
            Level &V = h->lv[lev];
            const int mm = layout(lev, T);
            const DenseSegView v = T.view();
            const int64_t nv = std::max<int64_t>(1, V.vlen()), nu = 3 * static_cast<int64_t>(V.n);
            DevBuf<double> unit(nv), col(nv);
            for (int j = 0; j < mm; ++j) {
                launch_fill(unit.p, 0.0, nv, s);
                launch_segment_units(v, j, unit.p, unit.p + nu, s);
                saddle_cycle<double>(h, lev, unit.p, col.p, true);
                launch_segment_store_column(v, j, col.p, col.p + nu, T.inv.p, s);
            }
            AMG_HIP(hipStreamSynchronize(s));
        };
        // A V-cycle from level d visits level d + 1 from a zero guess: if
        // that level still coarsens, its own (smaller) map is assembled first
        // and level d's column cycles apply it instead of recursing.
        if (h->prm.nu == 1 && d + 1 < last && h->lv[d + 1].nA > 0) {
            DenseSegs inner;
            assemble(d + 1, inner);
            h->saddle_tail = std::move(inner);
            h->saddle_tail_from = d + 1;
        }
        DenseSegs T;
        assemble(d, T);
        if (h->mixed) T.make_f32(s);  // the FP32 cycle reads an FP32 copy
        AMG_HIP(hipStreamSynchronize(s));
        h->saddle_tail = std::move(T);
        h->saddle_tail_from = d;
        const float dense_ms = time_cycle(d, false);
        if (!(dense_ms < 0.95f * sparse_ms)) {
            h->saddle_tail_from = -1;
            h->saddle_tail = DenseSegs();
        }
        break;
    }
    AMG_HIP(hipEventDestroy(e0));
    AMG_HIP(hipEventDestroy(e1));
}


static double norm2(amg_ctx *h, const double *v);

// stand-alone AMG: repeated Algorithm 1 from the current iterate
int solve_stationary_saddle(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    system_residual(h, b, x, h->kw.p);
    const double r0 = norm2(h, h->kw.p);
    int it = 0, status = AMG_NOT_CONVERGED;
    double rel = 0.0;
    if (r0 == 0.0) status = AMG_OK;
    while (status == AMG_NOT_CONVERGED && it < maxit) {
        const int cyc = std::max(1, h->prm.cycles);
        for (int k = 0; k < cyc; ++k) saddle_cycle(h, 0, b, x, false);
        ++it;
        system_residual(h, b, x, h->kw.p);
        rel = norm2(h, h->kw.p) / r0;
        if (!(rel == rel) || rel > 1e3) status = AMG_DIVERGED;
        else if (rel <= tol) status = AMG_OK;
    }
    if (res) {
        res->iters = it;
        res->status = status;
        res->relres = rel;
        res->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    profile_collect(h);
    return status;
}

void system_matvec(amg_ctx *h, const double *x, double *y) {
    if (h->saddle)
        saddle_apply(h, 0, x, y);
    else
        apply_level(h, 0, x, y);
}

void system_residual(amg_ctx *h, const double *b, const double *x, double *r) {
    if (h->saddle) {
        saddle_residual(h, 0, b, x, r);
    } else {
        system_matvec(h, x, r);
        launch_axpby(r, b, 1.0, -1.0, h->n_dof, h->stream);
    }
}

void precondition_any(amg_ctx *h, const double *r, double *z) { precondition_staged(h, r, z); }

// ---------------------------------------------------------------- FGMRES
static double norm2(amg_ctx *h, const double *v) {
    const int nb = launch_dot_partial(v, v, h->n_dof, h->partial.p, h->stream);
    launch_reduce(h->partial.p, nb, h->sc.p, SC_TMP, h->stream);
    AMG_HIP(hipMemcpyAsync(h->h_sc, h->sc.p, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    AMG_HIP(hipStreamSynchronize(h->stream));
    return std::sqrt(h->h_sc[SC_TMP]);
}

// Right-preconditioned flexible GMRES(m); the Hessenberg matrix and its
// Givens rotations live on the host (m <= a few hundred). Classical
// Gram-Schmidt with delayed reorthogonalisation (DCGS2: Swirydowicz,
// Langou, Ananthan, Yang and Thomas, Numer. Linear Algebra Appl. 2021):
// step j preconditions the pending vector u_j (orthogonalised once), and one
// pass over the basis takes the dots of V_0..V_{j+1} with u_j and with the
// new w = A z_j, after which one update finishes v_j (the second pass) and
// orthogonalises w once. Two passes over the basis per step instead of the
// four of CGS2, one host synchronisation. Column j - 1 of the Hessenberg
// matrix is complete at step j (u_j = V s + gamma v_j adds eta_j s to it and
// makes its subdiagonal eta_j gamma); the residual estimate of column j is
// taken provisionally with its pending subdiagonal eta_{j+1}, and when that
// meets the tolerance (or the cycle ends) one more pass over the basis
// completes the column before the exact test. FGMRES allows any z_j: the
// relation A Z = V H holds column by column with z_j = M^{-1} u_j.
int solve_fgmres(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = h->n_dof;
    const int m = std::max(1, h->prm.restart);
    if (h->gm_m != m) {
        h->gm_V.alloc(static_cast<size_t>(m + 1) * n);
        h->gm_Z.alloc(static_cast<size_t>(m) * n);
        h->gm_h.alloc(static_cast<size_t>(2 * (m + 2) + 4));
        h->gm_y.alloc(static_cast<size_t>(m + 1));
        h->gm_part.alloc(static_cast<size_t>(2 * (m + 2)) * multidot_blocks(n));
        h->gm_m = m;
    }
    double *V = h->gm_V.p, *Z = h->gm_Z.p;
    // H: rotated (upper triangular) columns, row-major i * m + j; Hr: the
    // raw Hessenberg columns (column j at j * (m + 1))
    std::vector<double> H(static_cast<size_t>(m + 1) * m), Hr(static_cast<size_t>(m + 1) * m), cs(m), sn(m),
        g(m + 1), hcol(m + 2), eta(m + 1, 1.0);
    const size_t nh = static_cast<size_t>(2 * (m + 2) + 4);
    if (h->gm_hpin_n < nh) {
        if (h->gm_hpin) AMG_HIP(hipHostFree(h->gm_hpin));
        h->gm_hpin = nullptr;
        AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->gm_hpin), nh * sizeof(double)));
        h->gm_hpin_n = nh;
    }
    double *hbuf = h->gm_hpin;
    std::vector<char> done_col(m, 0);
    system_residual(h, b, x, V);
    const double r0 = norm2(h, V);
    auto finish = [&](int it, int status) {
        system_residual(h, b, x, h->kw.p);
        const double rel = r0 > 0.0 ? norm2(h, h->kw.p) / r0 : 0.0;
        if (status == AMG_OK && !(rel == rel)) status = AMG_DIVERGED;
        if (res) {
            res->iters = it;
            res->status = status;
            res->relres = rel;
            res->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        profile_collect(h);
        return status;
    };
    if (r0 == 0.0) return finish(0, AMG_OK);
    if (!(r0 == r0)) return finish(0, AMG_DIVERGED);
    int it = 0;
    double beta = r0;
    double est_last = 1.0;  // the last residual estimate (relative)
    int status = AMG_NOT_CONVERGED;
    // rotations 0..c-1 applied to raw column c, rotation c formed, g updated;
    // returns the residual estimate after c + 1 columns
    auto rotate = [&](int c) {
        const double *raw = Hr.data() + static_cast<size_t>(c) * (m + 1);
        for (int i = 0; i <= c + 1; ++i) hcol[i] = raw[i];
        for (int i = 0; i < c; ++i) {
            const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
            hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
            hcol[i] = t;
        }
        const double den = std::hypot(hcol[c], hcol[c + 1]);
        cs[c] = den > 0.0 ? hcol[c] / den : 1.0;
        sn[c] = den > 0.0 ? hcol[c + 1] / den : 0.0;
        hcol[c] = den;
        g[c + 1] = -sn[c] * g[c];
        g[c] = cs[c] * g[c];
        for (int i = 0; i <= c; ++i) H[static_cast<size_t>(i) * m + c] = hcol[i];
        return std::fabs(g[c + 1]) / r0;
    };
    // the same estimate without changing the rotations (provisional column)
    auto estimate = [&](int c) {
        const double *raw = Hr.data() + static_cast<size_t>(c) * (m + 1);
        for (int i = 0; i <= c + 1; ++i) hcol[i] = raw[i];
        for (int i = 0; i < c; ++i) {
            const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
            hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
            hcol[i] = t;
        }
        const double den = std::hypot(hcol[c], hcol[c + 1]);
        return den > 0.0 ? std::fabs(hcol[c + 1] / den * g[c]) / r0 : 0.0;
    };
    while (it < maxit) {
        // V_0 = r / beta (r is in V_0 already)
        h->h_sc[SC_TMP] = beta;
        AMG_HIP(hipMemcpyAsync(h->sc.p + SC_TMP, &h->h_sc[SC_TMP], sizeof(double), hipMemcpyHostToDevice, h->stream));
        launch_scale_by_inverse(V, V, n, h->sc.p, SC_TMP, h->stream);
        std::fill(g.begin(), g.end(), 0.0);
        std::fill(done_col.begin(), done_col.end(), 0);
        g[0] = beta;
        int nc = 0;  // complete, rotated columns
        bool stop = false;
        bool ahead = false;  // this step's preconditioner already enqueued
        double *hd = h->gm_h.p;
        if (!h->sc_ready) AMG_HIP(hipEventCreateWithFlags(&h->sc_ready, hipEventDisableTiming));
        for (int j = 0; j < m && it + j < maxit && !stop; ++j) {
            double *vj = V + static_cast<int64_t>(j) * n, *w = V + static_cast<int64_t>(j + 1) * n;
            double *zj = Z + static_cast<int64_t>(j) * n;
            if (!ahead) precondition_any(h, vj, zj);
            ahead = false;
            system_matvec(h, zj, w);
            const int k = j + 2;
            int nb = launch_multidot2(V, n, k, vj, w, n, h->gm_part.p, h->stream);
            launch_multidot_reduce(h->gm_part.p, nb, 2 * k, hd, h->stream);
            launch_dcgs2_update(V, n, j, hd, n, j > 0, h->stream);
            AMG_HIP(hipMemcpyAsync(hbuf, hd, (2 * k + 3) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            AMG_HIP(hipEventRecord(h->sc_ready, h->stream));
            // the pending vector u_{j+1} is final for step j + 1: its
            // preconditioner goes ahead of the host's wait while the last
            // estimate is far from the tolerance
            if (j + 1 < m && it + j + 1 < maxit && est_last > KRYLOV_AHEAD * tol) {
                precondition_any(h, w, Z + static_cast<int64_t>(j + 1) * n);
                ahead = true;
            }
            AMG_HIP(hipEventSynchronize(h->sc_ready));
            const double *dA = hbuf, *dB = hbuf + k;
            const double gam = hbuf[2 * k], d = hbuf[2 * k + 1], et = hbuf[2 * k + 2];
            double est = 0.0;
            if (j > 0 && !done_col[j - 1]) {
                // u_j = V s + gamma v_j completes column j - 1
                double *c1 = Hr.data() + static_cast<size_t>(j - 1) * (m + 1);
                for (int i = 0; i < j; ++i) c1[i] += eta[j] * dA[i];
                c1[j] = eta[j] * gam;
                done_col[j - 1] = 1;
                est = rotate(j - 1);
                est_last = est;
                nc = j;
                if (!(est == est) || est > 1e3) {
                    status = AMG_DIVERGED;
                    break;
                }
                if (est <= tol || gam == 0.0) break;  // column j is not used
            }
            // column j with its pending subdiagonal
            double *cj = Hr.data() + static_cast<size_t>(j) * (m + 1);
            for (int i = 0; i < j; ++i) cj[i] = dB[i];
            cj[j] = d;
            cj[j + 1] = et;
            eta[j + 1] = et;
            const bool last = j + 1 == m || it + j + 1 >= maxit;
            if (last || et == 0.0 || estimate(j) <= tol) {
                // complete column j now: s = V_{0..j} . u_{j+1}, |u_{j+1}|^2
                nb = launch_multidot(V, n, k, w, n, h->gm_part.p, h->stream);
                launch_multidot_reduce(h->gm_part.p, nb, k, hd, h->stream);
                AMG_HIP(hipMemcpyAsync(hbuf, hd, k * sizeof(double), hipMemcpyDeviceToHost, h->stream));
                AMG_HIP(hipStreamSynchronize(h->stream));
                double ss = 0.0;
                for (int i = 0; i <= j; ++i) {
                    ss += hbuf[i] * hbuf[i];
                    cj[i] += et * hbuf[i];
                }
                const double g2 = hbuf[j + 1] - ss;
                cj[j + 1] = et * (g2 > 0.0 ? std::sqrt(g2) : 0.0);
                done_col[j] = 1;
                est = rotate(j);
                est_last = est;
                nc = j + 1;
                if (!(est == est) || est > 1e3) {
                    status = AMG_DIVERGED;
                    break;
                }
                stop = est <= tol || cj[j + 1] == 0.0;
            }
        }
        it += nc;
        const int j = nc;
        // y = R^{-1} g, x += Z y
        std::vector<double> y(j, 0.0);
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[static_cast<size_t>(i) * m + k] * y[k];
            y[i] = H[static_cast<size_t>(i) * m + i] != 0.0 ? s / H[static_cast<size_t>(i) * m + i] : 0.0;
        }
        if (j > 0) {
            AMG_HIP(hipMemcpyAsync(h->gm_y.p, y.data(), j * sizeof(double), hipMemcpyHostToDevice, h->stream));
            launch_multi_add(Z, n, j, h->gm_y.p, x, n, h->stream);
        }
        if (status == AMG_DIVERGED) break;
        system_residual(h, b, x, V);
        beta = norm2(h, V);
        if (beta / r0 <= tol) {
            status = AMG_OK;
            break;
        }
        if (nc == 0) break;  // no progress possible (breakdown on the first column)
    }
    return finish(it, status);
}

}  // namespace amgp2
