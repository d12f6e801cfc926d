// amg_setup: the level hierarchy of Section 3.2.
//   host : separated graphs (K_ll and K_qq patterns), greedy independent sets,
//          averaging interpolation, colouring, the coarsest dense inverse;
//   GPU  : Galerkin products P^T A P (k_spgemm.hip), diagonal-block inverses,
//          colour-grouped copies of the operators.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <tuple>

#include <memory>

#include "context.h"
#include "saddle.h"

namespace amgp2 {

void DenseSegs::finalize(hipStream_t s) {
    count = static_cast<int>(h_m.size());
    std::vector<int> rs(count + 1, 0);
    bytes = 0.0;
    for (int k = 0; k < count; ++k) {
        rs[k + 1] = rs[k] + h_m[k];
        bytes += 8.0 * h_m[k] * h_m[k];
    }
    rows = rs[count];
    moff.upload(h_moff, s);
    rstart.upload(rs, s);
    uoff.upload(h_uoff, s);
    nu.upload(h_nu, s);
    poff.upload(h_poff, s);
    inv.alloc(count ? static_cast<size_t>(h_moff.back() + static_cast<int64_t>(h_m.back()) * h_m.back()) : 0);
}

void DenseSegs::make_f32(hipStream_t s) {
    inv32.alloc(inv.n);
    if (inv.n) launch_to_f32(inv.p, inv32.p, static_cast<int64_t>(inv.n), s);
    bytes *= 0.5;
}

static void upload_pattern(DMat &m, const HostCSR &h, hipStream_t s) {
    m.nrows = h.nrows;
    m.ncols = h.ncols;
    m.nnz = h.nnz();
    m.rowptr.upload(h.rowptr, s);
    m.col.upload(h.col, s);
}

// Scalar host matrix -> device (1 plane).
static void upload_scalar(DMat &m, const HostCSR &h, hipStream_t s) {
    upload_pattern(m, h, s);
    m.np = 1;
    m.val.upload(h.val, s);
}

// Row-major blocks (np values per entry) -> planes.
static void upload_blocks(DMat &m, int nrows, int ncols, const int32_t *rowptr, const int32_t *col,
                          const double *val, int np, hipStream_t s) {
    m.nrows = nrows;
    m.ncols = ncols;
    m.nnz = rowptr[nrows];
    m.np = np;
    m.rowptr.upload(rowptr, nrows + 1, s);
    m.col.upload(col, static_cast<size_t>(m.nnz), s);
    // the caller's blocks as they are, then into planes on the device
    DevBuf<double> aos;
    aos.upload(val, static_cast<size_t>(np) * m.nnz, s);
    m.val.alloc(std::max<size_t>(1, static_cast<size_t>(np) * m.nnz));
    launch_aos_to_planes(aos.p, np, m.nnz, m.val.p, s);
    AMG_HIP(hipStreamSynchronize(s));
}

// B^T of a host 1x3-block matrix (nrows x ncols) as 3x1 blocks (3 planes).
static void upload_transpose_1x3(DMat &m, int nrows, int ncols, const int32_t *rowptr, const int32_t *col,
                                 const double *val, hipStream_t s) {
    const int64_t nnz = rowptr[nrows];
    std::vector<int> rp(ncols + 1, 0), cl(nnz);
    for (int64_t k = 0; k < nnz; ++k) ++rp[col[k] + 1];
    std::partial_sum(rp.begin(), rp.end(), rp.begin());
    std::vector<int> next(rp.begin(), rp.end() - 1);
    std::vector<double> planes(3 * static_cast<size_t>(nnz));
    for (int i = 0; i < nrows; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int q = next[col[k]]++;
            cl[q] = i;
            for (int c = 0; c < 3; ++c) planes[static_cast<size_t>(c) * nnz + q] = val[3 * k + c];
        }
    m.nrows = ncols;
    m.ncols = nrows;
    m.nnz = nnz;
    m.np = 3;
    m.rowptr.upload(rp, s);
    m.col.upload(cl, s);
    m.val.upload(planes, s);
    AMG_HIP(hipStreamSynchronize(s));
}

static HostCSR download_pattern(const DMat &m, hipStream_t s) {
    HostCSR h;
    h.nrows = m.nrows;
    h.ncols = m.ncols;
    h.rowptr = m.rowptr.download(s);
    h.col = m.col.download(s);
    return h;
}

// C = X Y, one of X / Y scalar (np = 1), the other with np planes.
// search_y: Y's rows are long (binary search in them); otherwise Y is a
// prolongation with a few entries per row (linear scan).
static DMat spgemm(amg_ctx *h, const DMat &X, const DMat &Y, bool search_y) {
    hipStream_t s = h->stream;
    AMG_REQUIRE(X.ncols == Y.nrows, AMG_EINVAL, "spgemm: shape mismatch");
    AMG_REQUIRE(X.np == 1 || Y.np == 1, AMG_EINVAL, "spgemm: one factor must be scalar");
    DMat C;
    C.nrows = X.nrows;
    C.ncols = Y.ncols;
    C.np = std::max(X.np, Y.np);
    DevBuf<int> cnt(std::max(1, C.nrows)), flag(1);
    flag.zero(s);
    launch_spgemm_count(C.nrows, X.rowptr.p, X.col.p, Y.rowptr.p, Y.col.p, cnt.p, flag.p, s);
    std::vector<int> hc = cnt.download(s);
    std::vector<int> hf = flag.download(s);
    AMG_REQUIRE(hf[0] == 0, AMG_EUNSUPPORTED,
                "Galerkin product: a coarse row has more distinct columns than the LDS hash holds");
    std::vector<int> rp(C.nrows + 1, 0);
    for (int i = 0; i < C.nrows; ++i) rp[i + 1] = rp[i] + hc[i];
    C.nnz = rp[C.nrows];
    C.rowptr.upload(rp, s);
    C.col.alloc(std::max<int64_t>(1, C.nnz));
    launch_spgemm_fill(C.nrows, X.rowptr.p, X.col.p, Y.rowptr.p, Y.col.p, C.rowptr.p, C.col.p, s);
    C.val.alloc(std::max<int64_t>(1, C.nnz * C.np));
    AMG_REQUIRE(search_y ? X.np == 1 : Y.np == 1, AMG_EINVAL, "spgemm: factor layout");
    hipEvent_t e0, e1;
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
    flag.zero(s);
    AMG_HIP(hipEventRecord(e0, s));
    launch_spgemm_numeric_lds(search_y, C.np, C.nrows, X.rowptr.p, X.col.p, X.val.p, X.nnz, Y.rowptr.p, Y.col.p,
                              Y.val.p, Y.nnz, C.rowptr.p, C.col.p, C.val.p, C.nnz, flag.p, s);
    AMG_HIP(hipEventRecord(e1, s));
    AMG_HIP(hipEventSynchronize(e1));
    if (flag.download(s)[0] != 0) {
        // a factor row beyond the LDS staging: the unstaged kernels (same sums)
        if (!search_y)
            launch_spgemm_numeric_bx(X.np, C.nrows, X.rowptr.p, X.col.p, X.val.p, X.nnz, Y.rowptr.p, Y.col.p,
                                     Y.val.p, C.rowptr.p, C.col.p, C.val.p, C.nnz, s);
        else
            launch_spgemm_numeric_by(Y.np, C.nrows, X.rowptr.p, X.col.p, X.val.p, Y.rowptr.p, Y.col.p,
                                     Y.val.p, Y.nnz, C.rowptr.p, C.col.p, C.val.p, C.nnz, s);
        AMG_HIP(hipEventRecord(e1, s));
        AMG_HIP(hipEventSynchronize(e1));
    }
    float ms = 0.f;
    AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // algorithmic bytes: both factors and the product's pattern read once,
    // the product's values written once
    ProfStat &st = h->setup_stats["setup.spgemm_numeric"];
    st.launches += 1;
    st.ms += ms;
    st.bytes += static_cast<double>(X.nnz) * (X.np * 8.0 + 4.0) + static_cast<double>(Y.nnz) * (Y.np * 8.0 + 4.0) +
                static_cast<double>(C.nnz) * (C.np * 8.0 + 4.0) + 4.0 * (X.nrows + Y.nrows + C.nrows);
    return C;
}

// Lanes per row for a row kernel: the smallest power of two (4..64) not
// below the mean entries per row.
// The operator without its numerically zero entries (all planes zero, the
// diagonal of a square operator always kept): on these meshes the Dirichlet
// couplings removed by the symmetric elimination and couplings that vanish
// on the Kuhn split. False, with out untouched, when there are none.
static bool drop_zero_entries(const DMat &m, bool square, DMat &out, hipStream_t s) {
    if (m.nnz == 0 || m.nrows == 0) return false;
    DevBuf<int> cnt(static_cast<size_t>(m.nrows));
    launch_count_kept(m.np, m.nrows, square, m.rowptr.p, m.col.p, m.val.p, m.nnz, cnt.p, s);
    const std::vector<int> c = cnt.download(s);
    std::vector<int> rp(static_cast<size_t>(m.nrows) + 1, 0);
    for (int i = 0; i < m.nrows; ++i) rp[i + 1] = rp[i] + c[i];
    if (rp.back() == m.nnz) return false;
    out = DMat();
    out.nrows = m.nrows;
    out.ncols = m.ncols;
    out.np = m.np;
    out.nnz = rp.back();
    out.rowptr.upload(rp, s);
    out.col.alloc(static_cast<size_t>(std::max<int64_t>(1, out.nnz)));
    out.val.alloc(static_cast<size_t>(std::max<int64_t>(1, out.nnz * out.np)));
    launch_compact_rows(m.np, m.nrows, square, m.rowptr.p, m.col.p, m.val.p, m.nnz, out.rowptr.p, out.col.p,
                        out.val.p, out.nnz, s);
    AMG_HIP(hipStreamSynchronize(s));
    return true;
}

int lanes_for(int64_t nnz, int nrows) {
    const double avg = nrows > 0 ? static_cast<double>(nnz) / nrows : 1.0;
    int G = 4;
    while (G < 64 && G < avg) G *= 2;
    return G;
}

static void check_system(const amg_system *sys) {
    AMG_REQUIRE(sys != nullptr, AMG_EINVAL, "amg_setup: null system");
    AMG_REQUIRE(sys->n_lin >= 0 && sys->n_quad >= 0 && sys->n_lin + sys->n_quad > 0, AMG_EINVAL,
                "amg_setup: node counts must be positive");
    AMG_REQUIRE(sys->bs == 1 || sys->bs == 3, AMG_EINVAL, "amg_setup: bs must be 1 or 3");
    AMG_REQUIRE(sys->A_rowptr && sys->A_col && sys->A_val, AMG_EINVAL, "amg_setup: A is missing");
    const int n = sys->n_lin + sys->n_quad;
    if (sys->n_pres > 0) {
        AMG_REQUIRE(sys->bs == 3, AMG_EINVAL, "amg_setup: saddle systems need 3x3 velocity blocks");
        AMG_REQUIRE(sys->n_pres == sys->n_lin, AMG_EINVAL,
                    "amg_setup: pressure nodes must be the linear velocity nodes (n_pres == n_lin)");
        AMG_REQUIRE(sys->B_rowptr && sys->B_col && sys->B_val, AMG_EINVAL, "amg_setup: B is missing");
        for (int k = 0; k < sys->B_rowptr[sys->n_pres]; ++k)
            AMG_REQUIRE(sys->B_col[k] >= 0 && sys->B_col[k] < n, AMG_EINVAL, "amg_setup: B column out of range");
        if (sys->C_rowptr)
            for (int q = 0; q < sys->n_pres; ++q)
                for (int k = sys->C_rowptr[q]; k < sys->C_rowptr[q + 1]; ++k) {
                    AMG_REQUIRE(sys->C_col[k] >= 0 && sys->C_col[k] < sys->n_pres, AMG_EINVAL,
                                "amg_setup: C column out of range");
                    AMG_REQUIRE(k == sys->C_rowptr[q] || sys->C_col[k - 1] < sys->C_col[k], AMG_EINVAL,
                                "amg_setup: C columns not sorted/unique");
                }
    }
    AMG_REQUIRE(sys->A_rowptr[0] == 0, AMG_EINVAL, "amg_setup: A_rowptr[0] != 0");
    for (int i = 0; i < n; ++i) {
        const int b = sys->A_rowptr[i], e = sys->A_rowptr[i + 1];
        AMG_REQUIRE(e >= b, AMG_EINVAL, "amg_setup: A_rowptr not monotone");
        bool diag = false;
        for (int k = b; k < e; ++k) {
            const int j = sys->A_col[k];
            AMG_REQUIRE(j >= 0 && j < n, AMG_EINVAL, "amg_setup: column index out of range");
            AMG_REQUIRE(k == b || sys->A_col[k - 1] < j, AMG_EINVAL, "amg_setup: columns not sorted/unique");
            diag |= j == i;
        }
        AMG_REQUIRE(diag, AMG_EINVAL, "amg_setup: missing diagonal entry in row " + std::to_string(i));
    }
}

static void setup_smoother(amg_ctx *h, Level &L) {
    hipStream_t s = h->stream;
    const int nb = L.mode == 3 ? 9 : 1;
    L.dinv.alloc(static_cast<size_t>(nb) * L.n);
    DevBuf<int> flag(1);
    flag.zero(s);
    launch_diag_inverse(L.mode, L.n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.A.nnz, L.dinv.p, flag.p, s);
    std::vector<int> hf = flag.download(s);
    AMG_REQUIRE(hf[0] == 0, AMG_EINVAL, "amg_setup: singular or missing diagonal block");
    L.G = lanes_for(L.A.nnz, L.n);
    if (h->prm.smoother != AMG_SMOOTH_GS) return;
    // colour-grouped copy of A for the Gauss-Seidel sweeps
    const int ncol = greedy_colouring(L.hpat, L.colour);
    std::vector<int> order(L.n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L.colour[a] < L.colour[b]; });
    L.cptr.assign(ncol + 1, 0);
    for (int i = 0; i < L.n; ++i) ++L.cptr[L.colour[i] + 1];
    std::partial_sum(L.cptr.begin(), L.cptr.end(), L.cptr.begin());
    std::vector<int> grp(L.n + 1, 0);
    L.colour_nnz.assign(ncol, 0);
    const std::vector<int> arp = L.A.rowptr.download(s);  // stored rows (zero blocks dropped)
    for (int g = 0; g < L.n; ++g) {
        const int len = arp[order[g] + 1] - arp[order[g]];
        grp[g + 1] = grp[g] + len;
        L.colour_nnz[L.colour[order[g]]] += len;
    }
    L.Ag.nrows = L.n;
    L.Ag.ncols = L.n;
    L.Ag.nnz = L.A.nnz;
    L.Ag.np = L.A.np;
    L.Ag.rowptr.upload(grp, s);
    L.Ag.col.alloc(static_cast<size_t>(L.A.nnz));
    L.Ag.val.alloc(static_cast<size_t>(L.A.nnz) * L.A.np);
    L.g_rowid.upload(order, s);
    L.d_cptr.upload(L.cptr, s);
    launch_gather_rows(L.A.np, L.n, L.g_rowid.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.A.nnz, L.Ag.rowptr.p,
                       L.Ag.col.p, L.Ag.val.p, L.Ag.nnz, s);
    AMG_HIP(hipStreamSynchronize(s));
    L.Gg = L.G;
}

// Autotuner: lanes per row for the level's row kernels, measured with HIP
// events on the level's own operators (residual on the natural rows, one
// Gauss-Seidel launch on the largest colour). Runs on scratch vectors.
void evict_caches(amg_ctx *h) {
    constexpr size_t n = (512u << 20) / sizeof(double);
    if (h->tune_flush.n != n) h->tune_flush.alloc(n);
    launch_fill(h->tune_flush.p, 0.0, static_cast<int64_t>(n), h->stream);
}

// Copy of a Schur level's smoothed rows grouped by colour (rows in the order
// rowid), so that a colour sweep reads its rows' pointers by position,
// together with the row ids, instead of after them.
void group_schur_rows(SchurLevel &q, hipStream_t s) {
    const int m = q.cptr.empty() ? 0 : q.cptr.back();
    q.Sg = DMat();
    q.Sg.np = 1;
    q.Sg.nrows = m;
    q.Sg.ncols = q.S.ncols;
    if (m == 0) return;
    const std::vector<int> rp = q.S.rowptr.download(s), order = q.rowid.download(s);
    std::vector<int> grp(m + 1, 0);
    for (int g = 0; g < m; ++g) grp[g + 1] = grp[g] + rp[order[g] + 1] - rp[order[g]];
    q.Sg.nnz = grp[m];
    q.Sg.rowptr.upload(grp, s);
    q.Sg.col.alloc(std::max<int64_t>(1, q.Sg.nnz));
    q.Sg.val.alloc(std::max<int64_t>(1, q.Sg.nnz));
    launch_gather_rows(1, m, q.rowid.p, q.S.rowptr.p, q.S.col.p, q.S.val.p, q.S.nnz, q.Sg.rowptr.p, q.Sg.col.p,
                       q.Sg.val.p, q.Sg.nnz, s);
    AMG_HIP(hipStreamSynchronize(s));
}

void autotune_level(amg_ctx *h, Level &L, bool natural_only) {
    hipStream_t s = h->stream;
    const int cand[] = {8, 16, 32, 64};
    hipEvent_t e0, e1;
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
    launch_fill(L.x.p, 0.0, 3 * static_cast<int64_t>(L.n), s);
    launch_fill(L.b.p, 1.0, 3 * static_cast<int64_t>(L.n), s);
    launch_fill(L.t.p, 0.0, 3 * static_cast<int64_t>(L.n), s);
    // best of 7 timed repetitions after 2 warm-up runs (short kernels are noisy)
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
    // Candidates (lanes G, entries per lane and trip T) are timed against
    // the heuristic's choice (T = 1), which another candidate replaces only
    // when it is at least 5% faster: timing noise then does not flip the
    // choice from one setup to the next. T > 1 is tried only where a trip of
    // the row group (G T entries) is at most twice the mean row.
    const double avg_row = static_cast<double>(L.A.nnz) / std::max(1, L.n);
    auto pick = [&](int G0, auto &&time_of) {
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
        return std::make_tuple(bestG, bestT, best);
    };
    std::tie(L.G, L.trip, std::ignore) = pick(L.G, [&](int G, int P) {
        RowArgs a;
        a.nrows = L.n;
        a.rowptr = L.A.rowptr.p;
        a.col = L.A.col.p;
        a.val = L.A.val.p;
        a.nnz = L.A.nnz;
        a.x = L.x.p;
        a.b = L.b.p;
        a.y = L.r.p;
        a.trip = P;
        return time_it([&] { launch_row(L.mode, OP_RESID, G, a, s); });
    });
    if (!L.cptr.empty() && !natural_only) {
        // a whole forward sweep, colour by colour, as the smoother runs it,
        // with round-robin or per-XCD contiguous workgroup placement
        auto sweep_time = [&](int G, int P, int xcd) {
            return time_it([&] {
                for (size_t c = 0; c + 1 < L.cptr.size(); ++c) {
                    if (L.cptr[c + 1] == L.cptr[c]) continue;
                    RowArgs a;
                    a.nrows = L.cptr[c + 1] - L.cptr[c];
                    a.rowptr = L.Ag.rowptr.p + L.cptr[c];
                    a.col = L.Ag.col.p;
                    a.val = L.Ag.val.p;
                    a.nnz = L.Ag.nnz;
                    a.rowid = L.g_rowid.p + L.cptr[c];
                    a.x = L.t.p;
                    a.b = L.b.p;
                    a.y = L.t.p;
                    a.dinv = L.dinv.p;
                    a.dinv_n = L.n;
                    a.xcd_chunks = xcd;
                    a.trip = P;
                    launch_row(L.mode, OP_GS, G, a, s);
                }
            });
        };
        float rr_ms = 0.f;
        std::tie(L.Gg, L.tripg, rr_ms) = pick(L.Gg, [&](int G, int P) { return sweep_time(G, P, 0); });
        L.gs_xcd = sweep_time(L.Gg, L.tripg, 1) < 0.95f * rr_ms ? 1 : 0;
    }
    if (L.n_pres > 0 && L.B.nnz > 0) {
        // saddle levels: lanes of the B (1x3, pressure rows) and B^T (3x1,
        // velocity rows) kernels, same rule (heuristic kept unless >= 5% slower)
        const int64_t nu = 3 * static_cast<int64_t>(L.n);
        launch_fill(L.x.p, 0.0, L.vlen(), s);
        launch_fill(L.b.p, 1.0, L.vlen(), s);
        const int gcand[] = {4, 8, 16, 32, 64};
        auto pick_g = [&](int G0, auto &&time_of) {
            int bestG = G0;
            float best = time_of(G0);
            for (int G : gcand) {
                if (G == G0) continue;
                const float ms = time_of(G);
                if (ms < 0.95f * best) {
                    best = ms;
                    bestG = G;
                }
            }
            return bestG;
        };
        BlkArgs bb;
        bb.nrows = L.B.nrows;
        bb.rowptr = L.B.rowptr.p;
        bb.col = L.B.col.p;
        bb.val = L.B.val.p;
        bb.nnz = L.B.nnz;
        bb.x = L.x.p;
        bb.b = L.b.p + nu;
        bb.y = L.r.p + nu;
        L.Gb = pick_g(L.Gb, [&](int G) { return time_it([&] { launch_blk<double>(1, 3, BLK_RESID, G, bb, s); }); });
        BlkArgs bt;
        bt.nrows = L.Bt.nrows;
        bt.rowptr = L.Bt.rowptr.p;
        bt.col = L.Bt.col.p;
        bt.val = L.Bt.val.p;
        bt.nnz = L.Bt.nnz;
        bt.x = L.x.p + nu;
        bt.y = L.r.p;
        L.Gbt = pick_g(L.Gbt, [&](int G) { return time_it([&] { launch_blk<double>(3, 1, BLK_ADD, G, bt, s); }); });
    }
    AMG_HIP(hipEventDestroy(e0));
    AMG_HIP(hipEventDestroy(e1));
}

static void setup_coarsest(amg_ctx *h, Level &L) {
    hipStream_t s = h->stream;
    const int np = L.A.np;
    std::vector<int> rp = L.A.rowptr.download(s), cl = L.A.col.download(s);
    std::vector<double> v = L.A.val.download(s);
    if (L.mode == 3) {
        // [[A, B^T], [B, -C]] on the saddle coarsest level, A otherwise
        const int nu = 3 * L.n;
        const int m = nu + L.n_pres;
        std::vector<double> M(static_cast<size_t>(m) * m, 0.0);
        for (int i = 0; i < L.n; ++i)
            for (int k = rp[i]; k < rp[i + 1]; ++k)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        M[static_cast<size_t>(3 * i + r) * m + 3 * cl[k] + c] = v[static_cast<size_t>(r * 3 + c) * L.A.nnz + k];
        if (L.n_pres > 0) {
            std::vector<int> brp = L.B.rowptr.download(s), bcl = L.B.col.download(s);
            std::vector<double> bv = L.B.val.download(s);
            for (int q = 0; q < L.n_pres; ++q)
                for (int k = brp[q]; k < brp[q + 1]; ++k)
                    for (int c = 0; c < 3; ++c) {
                        const double b = bv[static_cast<size_t>(c) * L.B.nnz + k];
                        M[static_cast<size_t>(nu + q) * m + 3 * bcl[k] + c] = b;
                        M[static_cast<size_t>(3 * bcl[k] + c) * m + nu + q] = b;
                    }
            if (L.C.nnz > 0) {
                std::vector<int> crp = L.C.rowptr.download(s), ccl = L.C.col.download(s);
                std::vector<double> cv = L.C.val.download(s);
                for (int q = 0; q < L.n_pres; ++q)
                    for (int k = crp[q]; k < crp[q + 1]; ++k)
                        M[static_cast<size_t>(nu + q) * m + nu + ccl[k]] = -cv[k];
            }
            if (h->pinned >= 0) {
                // constants in the pressure kernel: fix the last pressure unknown
                h->pinned = m - 1;
                for (int j = 0; j < m; ++j) {
                    M[static_cast<size_t>(m - 1) * m + j] = 0.0;
                    M[static_cast<size_t>(j) * m + m - 1] = 0.0;
                }
                M[static_cast<size_t>(m - 1) * m + m - 1] = 1.0;
            }
        }
        AMG_REQUIRE(dense_inverse(M, m), AMG_EINVAL, "amg_setup: singular coarsest matrix");
        if (h->pinned >= 0) {
            // the pinned unknown's output is zero whatever its input holds
            for (int j = 0; j < m; ++j) M[static_cast<size_t>(m - 1) * m + j] = 0.0;
        }
        h->coarse_m = m;
        h->coarse_nc = 1;
        h->coarse_inv.upload(M, s);
        if (L.n_pres > 0) {
            L.dseg = DenseSegs();
            L.dseg.add(m, 0, nu, 0);
            L.dseg.finalize(s);
            AMG_HIP(hipMemcpyAsync(L.dseg.inv.p, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, s));
            AMG_HIP(hipStreamSynchronize(s));  // M is a local
        }
    } else {
        const int m = L.n;
        std::vector<double> M(static_cast<size_t>(m) * m, 0.0);
        for (int i = 0; i < L.n; ++i)
            for (int k = rp[i]; k < rp[i + 1]; ++k) M[static_cast<size_t>(i) * m + cl[k]] = v[k];
        AMG_REQUIRE(dense_inverse(M, m), AMG_EINVAL, "amg_setup: singular coarsest matrix");
        h->coarse_m = m;
        h->coarse_nc = 3;
        h->coarse_inv.upload(M, s);
    }
    (void)np;
    AMG_HIP(hipStreamSynchronize(s));
}

// Descriptors of levels t..L for the tail kernel; returns the doubles of
// level vectors one workgroup needs (x, b, r: 9 per node).
static int tail_descriptors(amg_ctx *h, int t, DevBuf<TailLevel> &buf, TailArgs &a, double &algo) {
    const amg_params &p = h->prm;
    const int L = static_cast<int>(h->lv.size()) - 1;
    std::vector<TailLevel> d(L - t + 1);
    int off = 0;
    algo = 0.0;
    for (int k = t; k <= L; ++k) {
        Level &V = h->lv[k];
        TailLevel &q = d[k - t];
        q.n = V.n;
        q.lds_off = off;
        off += 9 * V.n;
        if (k == L) break;
        q.nc = h->lv[k + 1].n;
        if (p.smoother == AMG_SMOOTH_GS) {
            q.ncolors = static_cast<int>(V.cptr.size()) - 1;
            q.cptr = V.d_cptr.p;
            q.g_rowptr = V.Ag.rowptr.p;
            q.g_col = V.Ag.col.p;
            q.g_val = V.Ag.val.p;
            q.g_nnz = V.Ag.nnz;
            q.g_rowid = V.g_rowid.p;
        }
        q.a_rowptr = V.A.rowptr.p;
        q.a_col = V.A.col.p;
        q.a_val = V.A.val.p;
        q.a_nnz = V.A.nnz;
        q.dinv = V.dinv.p;
        q.r_rowptr = V.R.rowptr.p;
        q.r_col = V.R.col.p;
        q.r_val = V.R.val.p;
        q.p_rowptr = V.P.rowptr.p;
        q.p_col = V.P.col.p;
        q.p_val = V.P.val.p;
        q.omega = h->level_omega.empty() ? p.omega
                                         : h->level_omega[std::min<size_t>(k, h->level_omega.size() - 1)];
        const double mat = static_cast<double>(V.A.nnz) * (V.A.np * 8.0 + 4.0);
        algo += (p.pre + p.post + 1) * mat + 2.0 * V.P.nnz * 12.0;
    }
    algo += static_cast<double>(h->coarse_m) * h->coarse_m * 8.0;
    buf.upload(d, h->stream);
    AMG_HIP(hipStreamSynchronize(h->stream));
    a = TailArgs();
    a.nlev = L - t + 1;
    a.smoother = p.smoother;
    a.pre = p.pre;
    a.post = p.post;
    a.lv = buf.p;
    a.cinv = h->coarse_inv.p;
    a.cm = h->coarse_m;
    a.cnc = h->coarse_nc;
    return off;
}

// The coarse end of the V-cycle is handled in one of two ways:
//  * dense tail: below the finest level a cycle always starts from x = 0, so
//    the V-cycle from level d down is a fixed linear map T of b_d
//    (pre-smoothing, restriction, coarser levels, prolongation,
//    post-smoothing). T is assembled once, one unit right-hand side per
//    workgroup of the tail kernel, and applied as a single GEMV.
//  * LDS tail: if even the finest level is small, the whole V-cycle runs in
//    one workgroup with the vectors in LDS.
// The first level of an SPD hierarchy that the assembled coarse end
// (setup_tail) will cover, or -1: the first level d >= 1 whose operator has
// at most TAIL_DENSE_MAX rows, for the symmetric V-cycle with JA or GS
int dense_tail_level(const amg_ctx *h) {
    const amg_params &p = h->prm;
    // (both forms implement the symmetric cycle: forward pre-, backward post-smoothing)
    if (h->saddle || h->nsys > 0 || !p.fuse_coarse || p.nu != 1 || h->post_forward) return -1;
    if (p.smoother != AMG_SMOOTH_JA && p.smoother != AMG_SMOOTH_GS) return -1;
    const int L = static_cast<int>(h->lv.size()) - 1;
    for (int k = 1; k < L; ++k) {
        const int m = h->lv[k].mode == 3 ? 3 * h->lv[k].n : h->lv[k].n;
        if (m <= TAIL_DENSE_MAX) return k;
    }
    return -1;
}

void setup_tail(amg_ctx *h) {
    h->tail_start = -1;
    h->dense_start = -1;
    h->tail_m = 0;
    h->tail_dense.release();
    const amg_params &p = h->prm;
    if (!p.fuse_coarse || p.nu != 1 || h->post_forward) return;
    if (p.smoother != AMG_SMOOTH_JA && p.smoother != AMG_SMOOTH_GS) return;
    const int L = static_cast<int>(h->lv.size()) - 1;
    if (L == 0) return;
    const int d = dense_tail_level(h);
    if (d > 0) {
        TailArgs u;
        double algo = 0.0;
        DevBuf<TailLevel> desc;
        const int stride = tail_descriptors(h, d, desc, u, algo);
        const int mode = h->lv[d].mode;
        const int m = mode == 3 ? 3 * h->lv[d].n : h->lv[d].n;
        h->tail_dense.alloc(static_cast<size_t>(m) * m);
        const int chunk = 2048;
        DevBuf<double> scratch(static_cast<size_t>(std::min(chunk, m)) * stride);
        u.unit_rhs = 1;
        u.m = m;
        u.x_out = h->tail_dense.p;
        u.gscratch = scratch.p;
        u.gstride = stride;
        for (int j0 = 0; j0 < m; j0 += chunk) {
            u.unit_base = j0;
            launch_tail(mode, u, 0, std::min(chunk, m - j0), h->stream);
        }
        AMG_HIP(hipStreamSynchronize(h->stream));
        h->tail_m = m;
        h->tail_nc = mode == 3 ? 1 : 3;
        h->dense_start = d;
    }
    // LDS tail from the finest level, if everything fits
    int64_t bytes = 0;
    for (int k = 0; k <= L; ++k) bytes += 72 * static_cast<int64_t>(h->lv[k].n);
    if (bytes <= TAIL_LDS_MAX && h->lv[0].A.nnz <= TAIL_NNZ_MAX) {
        double algo = 0.0;
        const int off = tail_descriptors(h, 0, h->tail_levels, h->tail_args, algo);
        h->tail_lds = off * static_cast<int>(sizeof(double));
        h->tail_bytes = algo;
        h->tail_start = 0;
    }
}

// Braess-Sarazin on saddle level l (Section 3.3): the Schur complement
// S_l = C_l + B_l A_hat^{-1} B_l^T on the structural pattern of B B^T (+ C),
// its scalar Galerkin hierarchy with the pressure interpolations H_k of the
// saddle levels below, a colouring per level for Gauss-Seidel and a dense
// inverse on the saddle coarsest level (last pressure unknown pinned when
// constants are in the pressure kernel).
void setup_schur(amg_ctx *h, int l) {
    hipStream_t s = h->stream;
    Level &L = h->lv[l];
    SchurHier &sh = L.schur;
    sh.lv.clear();
    {
        HostCSR bp = download_pattern(L.B, s), btp = download_pattern(L.Bt, s), cp;
        if (L.C.nnz > 0) cp = download_pattern(L.C, s);
        HostCSR pat = pattern_product(bp, btp, L.C.nnz > 0 ? &cp : nullptr);
        SchurLevel first;
        upload_pattern(first.S, pat, s);
        first.S.np = 1;
        first.S.val.alloc(std::max<int64_t>(1, first.S.nnz));
        const bool hc = L.C.nnz > 0;
        launch_schur_numeric(L.n_pres, L.B.rowptr.p, L.B.col.p, L.B.val.p, L.B.nnz, L.Bt.rowptr.p, L.Bt.col.p,
                             L.Bt.val.p, L.Bt.nnz, L.bs_ahat.p, hc ? L.C.rowptr.p : nullptr,
                             hc ? L.C.col.p : nullptr, hc ? L.C.val.p : nullptr, first.S.rowptr.p, first.S.col.p,
                             first.S.val.p, s);
        sh.lv.push_back(std::move(first));
    }
    const int last = static_cast<int>(h->lv.size()) - 1;
    for (int k = l; k < last; ++k) {
        const Level &V = h->lv[k];
        DMat SH = spgemm(h, sh.lv.back().S, V.H, false);
        SchurLevel nx;
        nx.S = spgemm(h, V.Ht, SH, true);
        sh.lv.push_back(std::move(nx));
    }
    for (size_t k = 0; k < sh.lv.size(); ++k) {
        SchurLevel &q = sh.lv[k];
        const int n = q.S.nrows;
        q.x.alloc(std::max(1, n));
        q.b.alloc(std::max(1, n));
        q.r.alloc(std::max(1, n));
        if (k + 1 == sh.lv.size()) break;
        HostCSR pat = download_pattern(q.S, s);
        std::vector<int> colour;
        const int nc = greedy_colouring(pat, colour);
        q.cptr.assign(nc + 1, 0);
        for (int i = 0; i < n; ++i) ++q.cptr[colour[i] + 1];
        std::partial_sum(q.cptr.begin(), q.cptr.end(), q.cptr.begin());
        std::vector<int> order(std::max(1, n)), next(q.cptr.begin(), q.cptr.end() - 1);
        for (int i = 0; i < n; ++i) order[next[colour[i]]++] = i;
        q.rowid.upload(order, s);
        group_schur_rows(q, s);
        q.dinv.alloc(std::max(1, n));
        DevBuf<int> flag(1);
        flag.zero(s);
        launch_diag_inverse(1, n, q.S.rowptr.p, q.S.col.p, q.S.val.p, q.S.nnz, q.dinv.p, flag.p, s);
        AMG_REQUIRE(flag.download(s)[0] == 0, AMG_EINVAL,
                    "amg_setup: Braess-Sarazin Schur complement has a zero or missing diagonal entry");
        q.G = lanes_for(q.S.nnz, n);
    }
    SchurLevel &c = sh.lv.back();
    const int m = c.S.nrows;
    std::vector<int> rp = c.S.rowptr.download(s), cl = c.S.col.download(s);
    std::vector<double> v = c.S.val.download(s);
    std::vector<double> M(static_cast<size_t>(m) * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) M[static_cast<size_t>(i) * m + cl[k]] = v[k];
    if (h->pinned >= 0 && m > 0) {
        for (int j = 0; j < m; ++j) {
            M[static_cast<size_t>(m - 1) * m + j] = 0.0;
            M[static_cast<size_t>(j) * m + m - 1] = 0.0;
        }
        M[static_cast<size_t>(m - 1) * m + m - 1] = 1.0;
    }
    AMG_REQUIRE(dense_inverse(M, m), AMG_EINVAL, "amg_setup: singular coarsest Schur complement");
    if (h->pinned >= 0 && m > 0)
        for (int j = 0; j < m; ++j) M[static_cast<size_t>(m - 1) * m + j] = 0.0;
    sh.m = m;
    sh.inv.upload(M, s);
    for (size_t k = 0; k + 1 < sh.lv.size(); ++k) sh.lv[k].nA = sh.lv[k].S.nrows;
    for (SchurLevel &q : sh.lv) {
        q.blk_off.assign(1, 0);
        q.blk_rows.assign(1, q.S.nrows);
    }
    c.nA = 0;
    c.dseg = DenseSegs();
    c.dseg.add(m, 0, 0, 0);
    c.dseg.finalize(s);
    AMG_HIP(hipMemcpyAsync(c.dseg.inv.p, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
}

VankaView vanka_view(Level &L) {
    VankaView v;
    v.npatch = L.vanka.npatch;
    v.pptr = L.vanka.pptr.p;
    v.pnode = L.vanka.pnode.p;
    v.moff = L.vanka.moff.p;
    v.inv = L.vanka.inv.p;
    v.n = L.n;
    v.arow = L.A.rowptr.p;
    v.acol = L.A.col.p;
    v.aval = L.A.val.p;
    v.annz = L.A.nnz;
    v.brow = L.B.rowptr.p;
    v.bcol = L.B.col.p;
    v.bval = L.B.val.p;
    v.bnnz = L.B.nnz;
    v.btrow = L.Bt.rowptr.p;
    v.btcol = L.Bt.col.p;
    v.btval = L.Bt.val.p;
    v.btnnz = L.Bt.nnz;
    if (L.C.nnz > 0) {
        v.crow = L.C.rowptr.p;
        v.ccol = L.C.col.p;
        v.cval = L.C.val.p;
    }
    return v;
}

// Multiplicative Vanka on saddle level l (Section 3.3): patch i = pressure
// DOF i and the velocity nodes of B's row i (structural pattern, sorted).
// Patches i and j conflict when A couples a node of one to a node of the
// other (A's pattern holds the diagonal, so shared nodes count) or when C
// couples their pressures; greedy first-fit colouring in index order of the
// conflict graph gives the processing order (colour, then index). The local
// matrices are assembled and inverted on the GPU.
void setup_vanka(amg_ctx *h, int l) {
    hipStream_t s = h->stream;
    Level &L = h->lv[l];
    VankaData &V = L.vanka;
    HostCSR bp = download_pattern(L.B, s);
    const int np = L.n_pres;
    V.npatch = np;
    V.max_nodes = 0;
    for (int i = 0; i < np; ++i) {
        std::sort(bp.col.begin() + bp.rowptr[i], bp.col.begin() + bp.rowptr[i + 1]);
        V.max_nodes = std::max(V.max_nodes, bp.rowptr[i + 1] - bp.rowptr[i]);
    }
    const HostCSR node_patch = transpose(bp);  // patches containing each node
    HostCSR cp;
    if (L.C.nnz > 0) cp = download_pattern(L.C, s);
    HostCSR conf;
    conf.nrows = conf.ncols = np;
    conf.rowptr.assign(np + 1, 0);
    std::vector<int> mark_node(L.n, -1), mark_patch(np, -1);
    for (int i = 0; i < np; ++i) {
        for (int k = bp.rowptr[i]; k < bp.rowptr[i + 1]; ++k) {
            const int u = bp.col[k];
            for (int q = L.hpat.rowptr[u]; q < L.hpat.rowptr[u + 1]; ++q) {
                const int w = L.hpat.col[q];
                if (mark_node[w] == i) continue;
                mark_node[w] = i;
                for (int t = node_patch.rowptr[w]; t < node_patch.rowptr[w + 1]; ++t) {
                    const int j = node_patch.col[t];
                    if (mark_patch[j] != i) {
                        mark_patch[j] = i;
                        conf.col.push_back(j);
                    }
                }
            }
        }
        if (L.C.nnz > 0)
            for (int k = cp.rowptr[i]; k < cp.rowptr[i + 1]; ++k) {
                const int j = cp.col[k];
                if (mark_patch[j] != i) {
                    mark_patch[j] = i;
                    conf.col.push_back(j);
                }
            }
        conf.rowptr[i + 1] = static_cast<int>(conf.col.size());
    }
    std::vector<int> colour;
    const int nc = greedy_colouring(conf, colour);
    V.cptr.assign(nc + 1, 0);
    for (int i = 0; i < np; ++i) ++V.cptr[colour[i] + 1];
    std::partial_sum(V.cptr.begin(), V.cptr.end(), V.cptr.begin());
    std::vector<int> order(std::max(1, np)), next(V.cptr.begin(), V.cptr.end() - 1);
    for (int i = 0; i < np; ++i) order[next[colour[i]]++] = i;
    std::vector<int64_t> moff(std::max(1, np), 0);
    int64_t total = 0;
    for (int i = 0; i < np; ++i) {
        moff[i] = total;
        const int64_t m = 3 * static_cast<int64_t>(bp.rowptr[i + 1] - bp.rowptr[i]) + 1;
        total += m * m;
    }
    AMG_REQUIRE(total * 8 <= (int64_t(96) << 30), AMG_ENOMEM,
                "amg_setup: the Vanka patch inverses would exceed 96 GiB");
    // the patch kernels keep 2 m + 4,096 doubles and n_P ints of a patch in LDS (96 KiB budget)
    AMG_REQUIRE((2 * (3 * V.max_nodes + 1) + 4096) * 8 + V.max_nodes * 4 <= 98304, AMG_EUNSUPPORTED,
                "amg_setup: a Vanka patch is too large for the patch kernels");
    V.pptr.upload(bp.rowptr, s);
    V.pnode.upload(bp.col, s);
    V.order.upload(order, s);
    V.moff.upload(moff, s);
    V.inv.alloc(static_cast<size_t>(std::max<int64_t>(1, total)));
    V.inv_bytes = 8.0 * static_cast<double>(total);
    const VankaView view = vanka_view(L);
    launch_vanka_assemble(view, V.max_nodes, s);
    DevBuf<int> flag(1);
    flag.zero(s);
    launch_vanka_invert(view, 3 * V.max_nodes + 1, flag.p, s);
    AMG_REQUIRE(flag.download(s)[0] == 0, AMG_EINVAL, "amg_setup: singular Vanka patch matrix");
    // two-kernel path: residual offsets and the apply's tiles, colour by colour
    std::vector<int64_t> roff(std::max(1, np), 0);
    int64_t rtot = 0;
    for (int i = 0; i < np; ++i) {
        roff[i] = rtot;
        rtot += 3 * static_cast<int64_t>(bp.rowptr[i + 1] - bp.rowptr[i]) + 1;
    }
    std::vector<int> tpre(std::max(1, np), 0);
    V.ntiles.assign(nc, 0);
    for (int c = 0; c < nc; ++c) {
        int t = 0;
        for (int k = V.cptr[c]; k < V.cptr[c + 1]; ++k) {
            tpre[k] = t;
            const int i = order[k];
            t += (3 * (bp.rowptr[i + 1] - bp.rowptr[i]) + 1 + 63) / 64;
        }
        V.ntiles[c] = t;
    }
    V.roff.upload(roff, s);
    V.tpre.upload(tpre, s);
    V.rbuf.alloc(static_cast<size_t>(std::max<int64_t>(1, rtot)));
    // the tiled path's residual: rg lanes per row, 256 / rg node rows (and
    // the pressure row) per unit, tables for every rg
    for (const int rg : {16, 32, 64}) {
        const int rows = 256 / rg, ri = VankaData::rg_index(rg);
        std::vector<int> rpre(std::max(1, np), 0);
        V.nrunits[ri].assign(nc, 0);
        for (int c = 0; c < nc; ++c) {
            int t = 0;
            for (int k = V.cptr[c]; k < V.cptr[c + 1]; ++k) {
                rpre[k] = t;
                const int i = order[k];
                t += (bp.rowptr[i + 1] - bp.rowptr[i] + 1 + rows - 1) / rows;
            }
            V.nrunits[ri][c] = t;
        }
        V.rpre[ri].upload(rpre, s);
    }
    V.rg = 16;
    // three-kernel path: 64-row x cc-column tiles of the inverses and their
    // partial sums, colour by colour, for a chunk width cc
    auto tile_tables = [&](int cc) {
        std::vector<int> upre(std::max(1, np), 0);
        std::vector<int64_t> poff(std::max(1, np), 0);
        V.nunits.assign(nc, 0);
        int64_t ptot = 0;
        for (int i = 0; i < np; ++i) {
            const int64_t m = 3 * static_cast<int64_t>(bp.rowptr[i + 1] - bp.rowptr[i]) + 1;
            poff[i] = ptot;
            ptot += ((m + cc - 1) / cc) * m;
        }
        for (int c = 0; c < nc; ++c) {
            int t = 0;
            for (int k = V.cptr[c]; k < V.cptr[c + 1]; ++k) {
                upre[k] = t;
                const int i = order[k];
                const int m = 3 * (bp.rowptr[i + 1] - bp.rowptr[i]) + 1;
                t += ((m + 63) / 64) * ((m + cc - 1) / cc);
            }
            V.nunits[c] = t;
        }
        V.cc = cc;
        V.upre.upload(upre, s);
        V.poff.upload(poff, s);
        if (static_cast<int64_t>(V.pbuf.n) < ptot) V.pbuf.alloc(static_cast<size_t>(std::max<int64_t>(1, ptot)));
    };
    // the sweep form for this level's patch sizes: one kernel per colour for
    // patches up to 256 unknowns, the tiled form above, unless (with the
    // tuners on) another form or chunk width is 3% faster on a scratch
    // vector pair
    const bool large = 3 * V.max_nodes + 1 > 256;
    V.path = large ? 2 : 0;
    tile_tables(256);
    if (h->prm.autotune) {
        const int64_t nv = L.vlen();
        DevBuf<double> xs(nv), bs(nv);
        launch_fill(xs.p, 0.0, nv, s);
        launch_fill(bs.p, 1.0, nv, s);
        hipEvent_t e0, e1;
        AMG_HIP(hipEventCreate(&e0));
        AMG_HIP(hipEventCreate(&e1));
        auto sweep = [&](int path) {
            for (int c = 0; c < nc; ++c) {
                const int cnt = V.cptr[c + 1] - V.cptr[c];
                if (path == 2)
                    launch_vanka_colour_tiled(view, V.order.p + V.cptr[c], V.tpre.p + V.cptr[c],
                                              V.upre.p + V.cptr[c], V.rpre[VankaData::rg_index(V.rg)].p + V.cptr[c],
                                              cnt, V.ntiles[c], V.nunits[c],
                                              V.nrunits[VankaData::rg_index(V.rg)][c], V.cc, V.rg, V.roff.p, V.rbuf.p, V.poff.p,
                                              V.pbuf.p, bs.p, xs.p, 0.5, s);
                else if (path == 3)
                    launch_vanka_colour_rows(view, V.order.p + V.cptr[c], V.tpre.p + V.cptr[c],
                                             V.rpre[VankaData::rg_index(V.rg)].p + V.cptr[c], cnt, V.ntiles[c],
                                             V.nrunits[VankaData::rg_index(V.rg)][c], V.rg, V.aw, V.roff.p, V.rbuf.p, bs.p,
                                             xs.p, 0.5, s);
                else if (path == 1)
                    launch_vanka_colour_split(view, V.order.p + V.cptr[c], V.tpre.p + V.cptr[c], cnt, V.ntiles[c],
                                              V.max_nodes, V.roff.p, V.rbuf.p, bs.p, xs.p, 0.5, s);
                else
                    launch_vanka_colour(view, V.order.p + V.cptr[c], cnt, V.max_nodes, bs.p, xs.p, 0.5, s);
            }
        };
        auto time_of = [&](int path) {
            sweep(path);
            float best = 1e30f;
            for (int r = 0; r < 3; ++r) {
                AMG_HIP(hipEventRecord(e0, s));
                sweep(path);
                AMG_HIP(hipEventRecord(e1, s));
                AMG_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
                best = std::min(best, ms);
            }
            return best;
        };
        float best = time_of(V.path);
        int best_path = V.path, best_cc = 256;
        for (const int path : {0, 1}) {
            if (path == V.path) continue;
            const float t = time_of(path);
            if (t < 0.97f * best) {
                best = t;
                best_path = path;
            }
        }
        for (const int cc : {128, 256, 512}) {
            if (cc == 256 && V.path == 2) continue;
            tile_tables(cc);
            const float t = time_of(2);
            if (t < 0.97f * best) {
                best = t;
                best_path = 2;
                best_cc = cc;
            }
        }
        tile_tables(best_cc);
        // the spread residual's width (wider lane groups for long rows), in
        // the tiled form and in the two-kernel form with that residual
        int best_rg = 16;
        for (const int rg : {16, 32, 64}) {
            V.rg = rg;
            for (const int path : {2, 3}) {
                if (path == 2 && rg == 16) continue;  // timed above
                const float t = time_of(path);
                if (t < 0.97f * best) {
                    best = t;
                    best_path = path;
                    best_rg = rg;
                }
            }
        }
        V.rg = best_rg;
        V.path = best_path;
        if (best_path == 3) {
            // wavefronts per correction tile: shorter column chains per lane
            int best_aw = 4;
            for (const int aw : {8, 16}) {
                V.aw = aw;
                const float t = time_of(3);
                if (t < 0.97f * best) {
                    best = t;
                    best_aw = aw;
                }
            }
            V.aw = best_aw;
        }
        AMG_HIP(hipEventDestroy(e0));
        AMG_HIP(hipEventDestroy(e1));
    }
    AMG_HIP(hipStreamSynchronize(s));
}

double jacobi_omega(const amg_ctx *h, int l) {
    if (h->level_omega.empty()) return h->prm.omega;
    return h->level_omega[std::min<size_t>(l, h->level_omega.size() - 1)];
}

// Learned damping: the row features of every non-coarsest level go through
// the network in one batch; predictions outside (0.2, 1.2) or not finite
// fall back to the fixed weight of that level.
void predict_level_omega(amg_ctx *h) {
    amg_mlp *m = h->prm.omega_model;
    const int L = static_cast<int>(h->lv.size()) - 1;
    if (!m || L <= 0) return;
    hipStream_t s = h->stream;
    std::vector<float> X(static_cast<size_t>(L) * MLP_NF);
    for (int l = 0; l < L; ++l) {
        const Level &V = h->lv[l];
        double f[MLP_NF];
        row_features(V.mode, V.n, V.A.rowptr.p, V.A.col.p, V.A.val.p, V.A.nnz, l, f, s);
        for (int k = 0; k < MLP_NF; ++k) X[static_cast<size_t>(l) * MLP_NF + k] = static_cast<float>(f[k]);
    }
    m->w.reserve(L);
    AMG_HIP(hipMemcpyAsync(m->w.X.p, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, s));
    mlp_forward(m->theta.p, m->w.X.p, L, m->w, s);
    std::vector<float> om(L);
    AMG_HIP(hipMemcpyAsync(om.data(), m->w.om.p, L * sizeof(float), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    std::vector<double> w(L + 1);
    bool used = false;
    for (int l = 0; l < L; ++l) {
        const double o = om[l];
        const bool ok = std::isfinite(o) && o > MLP_OMEGA_MIN && o < MLP_OMEGA_MIN + MLP_OMEGA_SPAN;
        w[l] = ok ? o : jacobi_omega(h, l);
        used = used || ok;
    }
    w[L] = w[L - 1];
    h->fixed_omega = h->level_omega;
    h->level_omega = std::move(w);
    h->learned = used;
}

// Power iteration on D^{-1} A_l from a fixed pseudo-random start: the
// Rayleigh quotient (A v, D^{-1} A v) / (v, A v) of the generalised problem
// A v = lambda D v (a lower bound of lambda_max that converges to it).
double lambda_max_dinv_a(amg_ctx *h, Level &L) {
    hipStream_t s = h->stream;
    const int64_t nv = 3 * static_cast<int64_t>(L.n);
    DevBuf<double> v(nv), y(nv), w(nv), partial(static_cast<size_t>(dot_blocks(nv))), sc(4);
    launch_fill_hash(v.p, nv, 0x5eed, s);
    auto dot = [&](const double *a, const double *b) {
        const int nb = launch_dot_partial(a, b, nv, partial.p, s);
        launch_reduce(partial.p, nb, sc.p, 0, s);
        double r = 0.0;
        AMG_HIP(hipMemcpyAsync(&r, sc.p, sizeof(double), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        return r;
    };
    RowArgs a;
    a.nrows = L.n;
    a.rowptr = L.A.rowptr.p;
    a.col = L.A.col.p;
    a.val = L.A.val.p;
    a.nnz = L.A.nnz;
    double lam = 0.0;
    for (int it = 0; it < 100; ++it) {
        a.x = v.p;
        a.y = y.p;
        launch_row(L.mode, OP_SPMV, L.G, a, s);                 // y = A v
        launch_jacobi_zero(L.mode, L.n, L.dinv.p, L.n, y.p, 1.0, w.p, s);  // w = D^{-1} A v
        const double vav = dot(v.p, y.p), ydy = dot(y.p, w.p), ww = dot(w.p, w.p);
        if (!(vav > 0.0) || !(ww > 0.0)) break;
        lam = ydy / vav;
        launch_axpby(v.p, w.p, 1.0 / std::sqrt(ww), 0.0, nv, s);   // v = w / |w|
    }
    return lam;
}

void cap_learned_omega(amg_ctx *h) {
    const int L = static_cast<int>(h->lv.size()) - 1;
    h->omega_cap.assign(L + 1, 0.0);
    for (int l = 0; l < L; ++l) {
        const double lam = lambda_max_dinv_a(h, h->lv[l]);
        h->omega_cap[l] = lam > 0.0 ? OMEGA_CAP_FACTOR * 2.0 / lam : 0.0;
    }
    if (!h->learned) return;
    for (int l = 0; l < L; ++l)
        if (h->omega_cap[l] > 0.0 && h->level_omega[l] > h->omega_cap[l]) h->level_omega[l] = h->omega_cap[l];
    h->level_omega[L] = h->level_omega[L - 1];
}

void build_hierarchy(amg_ctx *h, const amg_system *sys) {
    check_system(sys);
    h->saddle = sys->n_pres > 0;
    h->pinned = (h->saddle && sys->pressure_kernel) ? 0 : -1;
    hipStream_t s = h->stream;
    const amg_params &p = h->prm;
    h->lv.clear();
    h->lv.emplace_back();
    {
        SetupPhase ph(h, "upload");
        Level &L0 = h->lv.back();
        L0.n_lin = sys->n_lin;
        L0.n_quad = sys->n_quad;
        L0.n = sys->n_lin + sys->n_quad;
        L0.mode = sys->bs;
        upload_blocks(L0.A, L0.n, L0.n, sys->A_rowptr, sys->A_col, sys->A_val, sys->bs * sys->bs, s);
        L0.hpat.nrows = L0.hpat.ncols = L0.n;
        L0.hpat.rowptr.assign(sys->A_rowptr, sys->A_rowptr + L0.n + 1);
        L0.hpat.col.assign(sys->A_col, sys->A_col + L0.A.nnz);
        if (h->saddle) {
            // B: pressure rows (the vertices, = linear velocity nodes) x velocity nodes, 1x3 blocks
            L0.n_pres = sys->n_pres;
            upload_blocks(L0.B, sys->n_pres, L0.n, sys->B_rowptr, sys->B_col, sys->B_val, 3, s);
            upload_transpose_1x3(L0.Bt, sys->n_pres, L0.n, sys->B_rowptr, sys->B_col, sys->B_val, s);
            if (sys->C_rowptr && sys->C_col && sys->C_val)
                upload_blocks(L0.C, sys->n_pres, sys->n_pres, sys->C_rowptr, sys->C_col, sys->C_val, 1, s);
        }
    }
    const int max_levels = std::max(1, p.max_levels);
    while (true) {
        Level &L = h->lv.back();
        if (L.vlen() <= p.coarse_max || static_cast<int>(h->lv.size()) >= max_levels) break;
        HostCSR P, Hp;
        int ncl = 0, ncq = 0;
        auto ph_c = std::make_unique<SetupPhase>(h, "coarsen");
        if (p.separate) {
            HostCSR gl = subgraph(L.hpat, 0, L.n_lin), gq = subgraph(L.hpat, L.n_lin, L.n);
            HostCSR pl = averaging_interpolation(gl, greedy_independent_set(gl));
            HostCSR pq = averaging_interpolation(gq, greedy_independent_set(gq));
            ncl = pl.ncols;
            ncq = pq.ncols;
            P = block_diagonal(pl, pq);
            // pressure: the linear-node graph and its interpolation (H = I-block of P)
            if (h->saddle) Hp = std::move(pl);
        } else {
            HostCSR g = subgraph(L.hpat, 0, L.n);
            P = averaging_interpolation(g, greedy_independent_set(g));
            ncl = P.ncols;
        }
        if (P.ncols > 0.9 * L.n || P.ncols == 0) break;
        upload_scalar(L.P, P, s);
        HostCSR R = transpose(P);
        upload_scalar(L.R, R, s);
        L.hP = std::move(P);
        L.Gp = lanes_for(L.P.nnz, L.P.nrows);
        L.Gr = lanes_for(L.R.nnz, L.R.nrows);
        ph_c.reset();
        SetupPhase ph_g(h, "galerkin");
        DMat AP = spgemm(h, L.A, L.P, false);
        DMat Ac = spgemm(h, L.R, AP, true);
        Level next;
        next.n_lin = ncl;
        next.n_quad = ncq;
        next.n = ncl + ncq;
        next.mode = L.mode;
        next.A = std::move(Ac);
        next.hpat = download_pattern(next.A, s);
        if (h->saddle) {
            // K_{l+1} = P^T K_l P with P = diag(I, J, H): B_c = H^T B P,
            // B_c^T = P^T B^T H, C_c = H^T C H
            upload_scalar(L.H, Hp, s);
            upload_scalar(L.Ht, transpose(Hp), s);
            L.Gh = lanes_for(L.H.nnz, L.H.nrows);
            L.Ght = lanes_for(L.Ht.nnz, L.Ht.nrows);
            DMat BP = spgemm(h, L.B, L.P, false);
            next.B = spgemm(h, L.Ht, BP, true);
            DMat BtH = spgemm(h, L.Bt, L.H, false);
            next.Bt = spgemm(h, L.R, BtH, true);
            if (L.C.nnz > 0) {
                DMat CH = spgemm(h, L.C, L.H, false);
                next.C = spgemm(h, L.Ht, CH, true);
            }
            next.n_pres = ncl;
        }
        h->lv.push_back(std::move(next));
    }
    h->lv.back().coarsest = true;
    for (Level &L : h->lv) {
        L.nA = L.coarsest ? 0 : L.n;
        L.npA = L.coarsest ? 0 : L.n_pres;
    }
    if (p.omega_model && p.smoother == AMG_SMOOTH_JA && !h->saddle) {
        SetupPhase ph(h, "omega_network");
        predict_level_omega(h);
    }
    // Coarsening, the Galerkin products and the row features above used the
    // structural patterns. From here on every level keeps A without its
    // numerically zero blocks: the smoother setup, the tuners, the
    // reduced-precision copies and the solve-phase kernels stream that
    // (the same operator, fewer bytes); the structural A stays for export.
    {
        SetupPhase ph(h, "drop_zeros");
        for (Level &L : h->lv) {
            DMat c;
            if (drop_zero_entries(L.A, true, c, s)) {
                L.A_pat = std::move(L.A);
                L.A = std::move(c);
            }
        }
    }
    // The FP64 kernels' tuner runs where those kernels run in solves: with a
    // reduced-precision cycle only the finest level's natural-order kernels
    // (the outer Krylov operator); in the FP64 cycle every level above the
    // assembled coarse end.
    const bool reduced = p.precision != AMG_PREC_FP64;
    const int tail_from = dense_tail_level(h);
    for (size_t l = 0; l < h->lv.size(); ++l) {
        Level &L = h->lv[l];
        const size_t nv = static_cast<size_t>(L.vlen());
        L.x.alloc(nv);
        L.b.alloc(nv);
        L.r.alloc(nv);
        L.t.alloc(nv);
        if (!L.coarsest) {
            {
                SetupPhase ph(h, "smoother");
                setup_smoother(h, L);
                if (h->saddle) saddle_setup_level(h, L);
            }
            const bool used = reduced ? l == 0 : (tail_from < 0 || static_cast<int>(l) < tail_from);
            if (p.autotune && used) {
                SetupPhase ph(h, "autotune");
                autotune_level(h, L, reduced);
            }
        }
    }
    {
        SetupPhase ph(h, "coarsest");
        setup_coarsest(h, h->lv.back());
    }
    if (!h->saddle && p.smoother == AMG_SMOOTH_JA) {
        SetupPhase ph(h, "omega_bound");
        cap_learned_omega(h);
    }
    if (h->saddle && p.smoother == AMG_SMOOTH_BS)
        for (int l = 0; l + 1 < static_cast<int>(h->lv.size()); ++l) {
            {
                SetupPhase ph(h, "schur");
                setup_schur(h, l);
            }
            if (!h->batch_member) {
                SetupPhase ph(h, "schur_map");
                setup_schur_dense(h, l);
            }
        }
    if (h->saddle && p.smoother == AMG_SMOOTH_VANKA)
        for (int l = 0; l + 1 < static_cast<int>(h->lv.size()); ++l) {
            SetupPhase ph(h, "vanka");
            setup_vanka(h, l);
        }
    // B and B^T likewise, once the Schur complements and the Vanka patches
    // (defined on B's structural pattern) are built
    if (h->saddle)
        for (Level &L : h->lv) {
            DMat c;
            if (drop_zero_entries(L.B, false, c, s)) {
                L.B_pat = std::move(L.B);
                L.B = std::move(c);
            }
            if (drop_zero_entries(L.Bt, false, c, s)) L.Bt = std::move(c);
        }
    if (!h->saddle) {
        {
            SetupPhase ph(h, "coarse_map");
            setup_tail(h);
        }
        SetupPhase ph(h, "reduced_copies");
        build_mixed(h);
    } else if (p.precision != AMG_PREC_FP64) {
        SetupPhase ph(h, "reduced_copies");
        build_mixed(h);
        build_saddle_mp(h);
    }
    if (h->saddle && !h->batch_member) {
        SetupPhase ph(h, "saddle_map");
        setup_saddle_tail(h);
    }
    h->n_dof = static_cast<int>(h->lv[0].vlen());
    const size_t nd = static_cast<size_t>(h->n_dof);
    h->kr.alloc(nd);
    h->kz.alloc(nd);
    h->kp.alloc(nd);
    h->kq.alloc(nd);
    h->kw.alloc(nd);
    h->partial.alloc(static_cast<size_t>(std::max(1024 * 128, row_blocks(h->lv[0].n, 64))));
    h->tune_flush.release();
    h->sc.alloc(SC_COUNT);
    if (!h->h_sc) AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->h_sc), SC_COUNT * sizeof(double)));
    AMG_HIP(hipStreamSynchronize(s));
}

}  // namespace amgp2
