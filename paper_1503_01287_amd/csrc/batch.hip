// Batches of independent saddle point systems (many solves of uneven mesh
// size in one set of launches).
//
// Every system gets its own hierarchy, built exactly as a single amg_setup
// would build it (Section 3.2). The hierarchies are then merged level by
// level into one block-diagonal hierarchy: level l holds the systems whose
// hierarchy reaches level l, ordered by decreasing depth, so the systems
// that continue below l form a leading block (smoothed, restricted,
// corrected) and those ending on l a trailing block (solved by their
// explicit inverses, one segmented kernel). A V-cycle of the merged
// hierarchy is then the V-cycles of all systems at once: each kernel launch
// serves the whole batch. The outer flexible GMRES keeps per-system inner
// products, Hessenberg matrices, convergence tests and iteration counts.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <exception>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "context.h"

namespace amgp2 {

static int lanes_of(int64_t nnz, int nrows) {
    const double avg = nrows > 0 ? static_cast<double>(nnz) / nrows : 1.0;
    int G = 4;
    while (G < 64 && G < avg) G *= 2;
    return G;
}

// Block-diagonal concatenation: part j contributes rows[j] rows (its matrix
// may be null or empty) with its columns shifted by coff[j].
static void merge_mats(DMat &out, const std::vector<const DMat *> &parts, const std::vector<int> &rows,
                       const std::vector<int> &coff, int ncols, int np, hipStream_t s) {
    // block-diagonal concatenation on the device: each part's row pointers
    // shifted by the entries before it, its columns by its column offset,
    // its value planes copied into the merged planes
    out = DMat();
    out.np = np;
    out.ncols = ncols;
    int64_t nrows = 0, nnz = 0;
    for (size_t j = 0; j < parts.size(); ++j) {
        const DMat *m = parts[j];
        nrows += rows[j];
        if (m && m->nnz > 0) {
            AMG_REQUIRE(m->nrows == rows[j] && m->np == np, AMG_EINVAL, "batch: inconsistent level operators");
            nnz += m->nnz;
        }
    }
    AMG_REQUIRE(nnz <= INT32_MAX && nrows < INT32_MAX, AMG_EINVAL, "batch: merged level exceeds 32-bit indices");
    out.nrows = static_cast<int>(nrows);
    out.nnz = nnz;
    out.rowptr.alloc(static_cast<size_t>(nrows) + 1);
    out.col.alloc(static_cast<size_t>(std::max<int64_t>(1, nnz)));
    out.val.alloc(static_cast<size_t>(std::max<int64_t>(1, nnz * np)));
    launch_copy_shift_i32(nullptr, 1, 0, out.rowptr.p, s);  // rowptr[0] = 0
    int64_t r0 = 0, k0 = 0;
    for (size_t j = 0; j < parts.size(); ++j) {
        const DMat *m = parts[j];
        if (m && m->nnz > 0) {
            launch_copy_shift_i32(m->rowptr.p + 1, m->nrows, static_cast<int>(k0), out.rowptr.p + r0 + 1, s);
            launch_copy_shift_i32(m->col.p, m->nnz, coff[j], out.col.p + k0, s);
            for (int p = 0; p < np; ++p)
                AMG_HIP(hipMemcpyAsync(out.val.p + p * nnz + k0, m->val.p + p * m->nnz, m->nnz * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
            k0 += m->nnz;
        } else {
            launch_copy_shift_i32(nullptr, rows[j], static_cast<int>(k0), out.rowptr.p + r0 + 1, s);
        }
        r0 += rows[j];
    }
}

// out[p * T + off_j + k] = src_j[p * len_j + k] (T = sum len_j); null parts -> 0
static void merge_planes(DevBuf<double> &out, const std::vector<const double *> &src,
                         const std::vector<int64_t> &len, int np, hipStream_t s) {
    int64_t T = 0;
    for (int64_t v : len) T += v;
    out.alloc(static_cast<size_t>(std::max<int64_t>(1, T * np)));
    int64_t off = 0;
    for (size_t j = 0; j < src.size(); ++j) {
        for (int p = 0; p < np; ++p) {
            double *d = out.p + p * T + off;
            if (src[j])
                AMG_HIP(hipMemcpyAsync(d, src[j] + p * len[j], len[j] * sizeof(double), hipMemcpyDeviceToDevice, s));
            else
                launch_fill(d, 0.0, len[j], s);
        }
        off += len[j];
    }
}

static void copy_segment(DenseSegs &d, int k, const DenseSegs &from, hipStream_t s) {
    AMG_REQUIRE(from.count == 1 && from.h_m[0] == d.h_m[k], AMG_EINVAL, "batch: coarsest inverse size mismatch");
    const size_t mm = static_cast<size_t>(d.h_m[k]) * d.h_m[k];
    AMG_HIP(hipMemcpyAsync(d.inv.p + d.h_moff[k], from.inv.p, mm * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// chunks of [base, base + len) for system q
static void add_chunks(int64_t base, int64_t len, int q, std::vector<int64_t> &st, std::vector<int> &ln,
                       std::vector<int> &sg, std::vector<int64_t> *dst, int64_t dbase) {
    for (int64_t o = 0; o < len; o += BATCH_CHUNK) {
        st.push_back(base + o);
        ln.push_back(static_cast<int>(std::min<int64_t>(BATCH_CHUNK, len - o)));
        sg.push_back(q);
        if (dst) dst->push_back(dbase + o);
    }
}

// Every system's own hierarchy (amg_setup's, with the batch's overrides in
// `inst`), built by a pool of host threads, each with a stream of its own:
// the systems' host passes (independent sets, colourings, dense inverses)
// run on several cores and their kernels overlap on the GPU. Each build is
// the same as alone (no timed choices: the systems' tuners are off), so the
// result does not depend on the schedule. The first failing system (lowest
// index) reports its error. The phase "systems" is the wall time of the
// step; the systems' own phases are summed into h as "systems.<phase>"
// (time summed over the threads), their Galerkin kernels' statistics as
// the batch's own.
static void build_instances(amg_ctx *h, int nsys, const amg_system *sys,
                            std::vector<std::unique_ptr<amg_ctx>> &inst) {
    SetupPhase ph(h, "systems");
    const int hw = static_cast<int>(std::thread::hardware_concurrency());
    const int nthreads = std::max(1, std::min({nsys, hw > 0 ? hw : 1, 16}));
    int dev = 0;
    AMG_HIP(hipGetDevice(&dev));
    std::atomic<int> next{0};
    std::vector<std::exception_ptr> err(nsys);
    std::mutex held_mu;
    std::vector<void *> held;  // buffers the builds released, freed after them
    auto work = [&]() {
        std::vector<void *> mine;
        deferred_frees = &mine;
        struct Hand {
            std::vector<void *> &mine, &held;
            std::mutex &mu;
            ~Hand() {
                deferred_frees = nullptr;
                std::lock_guard<std::mutex> lock(mu);
                held.insert(held.end(), mine.begin(), mine.end());
            }
        } hand{mine, held, held_mu};
        hipStream_t st = nullptr;
        try {
            AMG_HIP(hipSetDevice(dev));
            AMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        } catch (...) {
            const int i = next.fetch_add(1);
            if (i < nsys) err[i] = std::current_exception();
            next = nsys;
            return;
        }
        for (int i; (i = next.fetch_add(1)) < nsys;) {
            try {
                inst[i]->stream = st;
                build_hierarchy(inst[i].get(), &sys[i]);
                AMG_HIP(hipStreamSynchronize(st));
            } catch (...) {
                err[i] = std::current_exception();
                (void)hipStreamSynchronize(st);
                next = nsys;  // the others stop taking systems
            }
            inst[i]->stream = h->stream;
        }
        (void)hipStreamDestroy(st);
    };
    if (nthreads == 1) {
        work();
    } else {
        std::vector<std::thread> pool;
        try {
            for (int t = 0; t < nthreads; ++t) pool.emplace_back(work);
        } catch (...) {
            // no more threads: the started ones finish the systems (joined
            // below); only if none started does the error surface
            if (pool.empty()) throw;
        }
        for (auto &t : pool) t.join();
    }
    for (void *q : held) (void)hipFree(q);
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
    const std::string pre = "setup.";
    for (const auto &in : inst)
        for (const auto &kv : in->setup_stats) {
            const bool phase = kv.first.compare(0, pre.size(), pre) == 0 && kv.first != "setup.spgemm_numeric";
            ProfStat &st = h->setup_stats[phase ? "setup.systems." + kv.first.substr(pre.size()) : kv.first];
            st.launches += kv.second.launches;
            st.ms += kv.second.ms;
            st.bytes += kv.second.bytes;
        }
}

void build_batch(amg_ctx *h, int nsys, const amg_system *sys) {
    hipStream_t s = h->stream;
    const amg_params &p = h->prm;
    std::vector<std::unique_ptr<amg_ctx>> inst(nsys);
    std::vector<int> depth(nsys);
    for (int i = 0; i < nsys; ++i) {
        AMG_REQUIRE(sys[i].n_pres > 0, AMG_EINVAL, "amg_setup_batched: every system must be a saddle point system");
        inst[i].reset(new amg_ctx());
        inst[i]->prm = p;
        inst[i]->prm.autotune = 0;
        inst[i]->prm.omega_model = nullptr;
        inst[i]->prm.precision = AMG_PREC_FP64;  // the merged hierarchy is converted once
        inst[i]->batch_member = true;            // explicit Schur tails are assembled once, merged
        inst[i]->stream = s;
    }
    build_instances(h, nsys, sys, inst);
    for (int i = 0; i < nsys; ++i) depth[i] = static_cast<int>(inst[i]->lv.size()) - 1;
    auto ph_merge = std::make_unique<SetupPhase>(h, "merge");
    std::vector<int> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return depth[a] > depth[b]; });
    const int maxd = depth[order[0]];
    const bool bs = p.smoother == AMG_SMOOTH_BS;

    std::vector<Level> merged(maxd + 1);
    for (int l = 0; l <= maxd; ++l) {
        std::vector<int> P;  // systems reaching level l, in merged order
        for (int i : order)
            if (depth[i] >= l) P.push_back(i);
        Level &M = merged[l];
        M.mode = 3;
        const size_t np_ = P.size();
        std::vector<int> noff(np_), poff(np_), nrow(np_), prow(np_);
        for (size_t j = 0; j < np_; ++j) {
            const Level &V = inst[P[j]]->lv[l];
            noff[j] = M.n;
            poff[j] = M.n_pres;
            nrow[j] = V.n;
            prow[j] = V.n_pres;
            M.n += V.n;
            M.n_pres += V.n_pres;
            M.nnz_pat_A += V.pattern_nnz_A();
            M.nnz_pat_B += V.pattern_nnz_B();
            M.n_lin += V.n_lin;
            M.n_quad += V.n_quad;
            if (depth[P[j]] > l) {
                M.nA += V.n;
                M.npA += V.n_pres;
            }
        }
        M.coarsest = M.nA == 0;
        M.sys_noff = noff;
        M.sys_n = nrow;
        M.sys_poff = poff;
        M.sys_np = prow;
        std::vector<const DMat *> pa, pb, pbt, pc;
        bool anyc = false;
        for (int i : P) {
            const Level &V = inst[i]->lv[l];
            pa.push_back(&V.A);
            pb.push_back(&V.B);
            pbt.push_back(&V.Bt);
            pc.push_back(&V.C);
            anyc |= V.C.nnz > 0;
        }
        merge_mats(M.A, pa, nrow, noff, M.n, 9, s);
        merge_mats(M.B, pb, prow, noff, M.n, 3, s);
        merge_mats(M.Bt, pbt, nrow, poff, M.n_pres, 3, s);
        if (anyc) merge_mats(M.C, pc, prow, poff, M.n_pres, 1, s);
        {
            std::vector<const double *> dv, sg, ah;
            std::vector<int64_t> ln, lp, l3;
            for (size_t j = 0; j < np_; ++j) {
                const Level &V = inst[P[j]]->lv[l];
                const bool sm = depth[P[j]] > l;
                dv.push_back(sm ? V.dinv.p : nullptr);
                sg.push_back(sm ? V.sgs_scale.p : nullptr);
                ah.push_back(sm && bs ? V.bs_ahat.p : nullptr);
                ln.push_back(V.n);
                lp.push_back(V.n_pres);
                l3.push_back(3 * static_cast<int64_t>(V.n));
            }
            merge_planes(M.dinv, dv, ln, 9, s);
            merge_planes(M.sgs_scale, sg, lp, 1, s);
            if (bs) merge_planes(M.bs_ahat, ah, l3, 1, s);
        }
        // transfers to the next level: the leading (still coarsening) systems
        if (M.nA > 0) {
            std::vector<const DMat *> pp, pr, ph, pht;
            std::vector<int> rows_p, rows_r, rows_h, rows_ht, cp, cr, ch, cht;
            int n1 = 0, np1 = 0;
            for (size_t j = 0; j < np_; ++j) {
                if (depth[P[j]] <= l) continue;
                const Level &V = inst[P[j]]->lv[l];
                const Level &W = inst[P[j]]->lv[l + 1];
                pp.push_back(&V.P);
                rows_p.push_back(V.n);
                cp.push_back(n1);
                pr.push_back(&V.R);
                rows_r.push_back(W.n);
                cr.push_back(noff[j]);
                ph.push_back(&V.H);
                rows_h.push_back(V.n_pres);
                ch.push_back(np1);
                pht.push_back(&V.Ht);
                rows_ht.push_back(W.n_pres);
                cht.push_back(poff[j]);
                n1 += W.n;
                np1 += W.n_pres;
            }
            merge_mats(M.P, pp, rows_p, cp, n1, 1, s);
            merge_mats(M.R, pr, rows_r, cr, M.n, 1, s);
            merge_mats(M.H, ph, rows_h, ch, np1, 1, s);
            merge_mats(M.Ht, pht, rows_ht, cht, M.n_pres, 1, s);
        }
        // systems ending on this level: their explicit inverses
        for (size_t j = 0; j < np_; ++j)
            if (depth[P[j]] == l) {
                const Level &V = inst[P[j]]->lv[l];
                M.dseg.add(3 * V.n + V.n_pres, 3 * noff[j], 3 * V.n, poff[j]);
            }
        if (!M.dseg.h_m.empty()) {
            M.dseg.finalize(s);
            int k = 0;
            for (size_t j = 0; j < np_; ++j)
                if (depth[P[j]] == l) copy_segment(M.dseg, k++, inst[P[j]]->lv[l].dseg, s);
        }
        // Braess-Sarazin: the Schur hierarchies of the leading systems, merged
        // with the same rule (level k holds the systems reaching level l + k)
        if (bs && M.nA > 0) {
            int K = 0;
            for (int i : P)
                if (depth[i] > l) K = std::max(K, depth[i] - l);
            M.schur.lv.resize(K + 1);
            for (int k = 0; k <= K; ++k) {
                SchurLevel &Q = M.schur.lv[k];
                std::vector<int> R;
                for (int i : P)
                    if (depth[i] > l && depth[i] >= l + k) R.push_back(i);
                std::vector<const DMat *> ps;
                std::vector<int> rows, off;
                std::vector<const double *> dv;
                std::vector<int64_t> ln;
                int tot = 0;
                for (int i : R) {
                    const SchurLevel &q = inst[i]->lv[l].schur.lv[k];
                    ps.push_back(&q.S);
                    rows.push_back(q.S.nrows);
                    off.push_back(tot);
                    const bool sm = depth[i] > l + k;
                    dv.push_back(sm ? q.dinv.p : nullptr);
                    ln.push_back(q.S.nrows);
                    if (sm) Q.nA += q.S.nrows;
                    tot += q.S.nrows;
                }
                merge_mats(Q.S, ps, rows, off, tot, 1, s);
                merge_planes(Q.dinv, dv, ln, 1, s);
                // colour lists of the smoothed systems, colour by colour
                int nc = 0;
                std::vector<std::vector<int>> rid(R.size());
                for (size_t j = 0; j < R.size(); ++j)
                    if (depth[R[j]] > l + k) {
                        const SchurLevel &q = inst[R[j]]->lv[l].schur.lv[k];
                        nc = std::max(nc, static_cast<int>(q.cptr.size()) - 1);
                        rid[j] = q.rowid.download(s);
                    }
                Q.cptr.assign(1, 0);
                std::vector<int> order_rows;
                for (int c = 0; c < nc; ++c) {
                    for (size_t j = 0; j < R.size(); ++j) {
                        if (depth[R[j]] <= l + k) continue;
                        const SchurLevel &q = inst[R[j]]->lv[l].schur.lv[k];
                        if (c + 1 >= static_cast<int>(q.cptr.size())) continue;
                        for (int g = q.cptr[c]; g < q.cptr[c + 1]; ++g) order_rows.push_back(rid[j][g] + off[j]);
                    }
                    Q.cptr.push_back(static_cast<int>(order_rows.size()));
                }
                if (order_rows.empty()) order_rows.push_back(0);
                Q.rowid.upload(order_rows, s);
                group_schur_rows(Q, s);
                for (size_t j = 0; j < R.size(); ++j)
                    if (depth[R[j]] == l + k) Q.dseg.add(rows[j], 0, 0, off[j]);
                if (!Q.dseg.h_m.empty()) {
                    Q.dseg.finalize(s);
                    int kk = 0;
                    for (size_t j = 0; j < R.size(); ++j)
                        if (depth[R[j]] == l + k) copy_segment(Q.dseg, kk++, inst[R[j]]->lv[l].schur.lv[k].dseg, s);
                }
                Q.blk_off = off;
                Q.blk_rows = rows;
                Q.G = lanes_of(Q.S.nnz, Q.S.nrows);
                Q.x.alloc(std::max(1, tot));
                Q.b.alloc(std::max(1, tot));
                Q.r.alloc(std::max(1, tot));
            }
        }
        M.G = lanes_of(M.A.nnz, M.n);
        M.Gg = M.G;
        M.Gb = lanes_of(M.B.nnz, M.B.nrows);
        M.Gbt = lanes_of(M.Bt.nnz, M.Bt.nrows);
        M.Gp = lanes_of(M.P.nnz, M.P.nrows);
        M.Gr = lanes_of(M.R.nnz, M.R.nrows);
        M.Gh = lanes_of(M.H.nnz, M.H.nrows);
        M.Ght = lanes_of(M.Ht.nnz, M.Ht.nrows);
        const size_t nv = static_cast<size_t>(M.vlen());
        M.x.alloc(nv);
        M.b.alloc(nv);
        M.r.alloc(nv);
        M.t.alloc(nv);
    }
    AMG_HIP(hipStreamSynchronize(s));
    ph_merge.reset();
    // the merged levels' kernels see other shapes than the systems' own; a
    // reduced-precision cycle runs only the finest level's natural-order
    // FP64 kernels (the outer Krylov operator)
    if (p.autotune) {
        SetupPhase ph(h, "autotune");
        const bool reduced = p.precision != AMG_PREC_FP64;
        for (size_t l = 0; l < merged.size(); ++l)
            if (merged[l].nA > 0 && (!reduced || l == 0)) autotune_level(h, merged[l], reduced);
    }

    // level-0 layout of every system, chunk tables
    h->nsys = nsys;
    h->b_order = order;
    const Level &L0 = merged[0];
    const int64_t nu0 = 3 * static_cast<int64_t>(L0.n);
    std::vector<int64_t> user(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i)
        user[i + 1] = user[i] + 3 * static_cast<int64_t>(sys[i].n_lin + sys[i].n_quad) + sys[i].n_pres;
    h->b_uoff.assign(nsys, 0);
    h->b_poff.assign(nsys, 0);
    h->b_nu.assign(nsys, 0);
    h->b_np.assign(nsys, 0);
    {
        int64_t u = 0, q = 0;
        for (int j = 0; j < nsys; ++j) {
            const amg_system &S = sys[order[j]];
            h->b_uoff[j] = u;
            h->b_poff[j] = q;
            h->b_nu[j] = 3 * static_cast<int64_t>(S.n_lin + S.n_quad);
            h->b_np[j] = S.n_pres;
            u += h->b_nu[j];
            q += h->b_np[j];
        }
    }
    std::vector<int64_t> st, ds, st_in, ds_in, st_out, ds_out;
    std::vector<int> ln, sg, ln_in, sg_in, ln_out, sg_out;
    std::vector<int> c0(nsys), c1(nsys), c2(nsys), c3(nsys);
    for (int j = 0; j < nsys; ++j) {
        c0[j] = static_cast<int>(st.size());
        add_chunks(h->b_uoff[j], h->b_nu[j], j, st, ln, sg, nullptr, 0);
        c1[j] = static_cast<int>(st.size());
    }
    for (int j = 0; j < nsys; ++j) {
        c2[j] = static_cast<int>(st.size());
        add_chunks(nu0 + h->b_poff[j], h->b_np[j], j, st, ln, sg, nullptr, 0);
        c3[j] = static_cast<int>(st.size());
    }
    for (int j = 0; j < nsys; ++j) {
        const int64_t ub = user[order[j]];
        add_chunks(ub, h->b_nu[j], j, st_in, ln_in, sg_in, &ds_in, h->b_uoff[j]);
        add_chunks(ub + h->b_nu[j], h->b_np[j], j, st_in, ln_in, sg_in, &ds_in, nu0 + h->b_poff[j]);
        add_chunks(h->b_uoff[j], h->b_nu[j], j, st_out, ln_out, sg_out, &ds_out, ub);
        add_chunks(nu0 + h->b_poff[j], h->b_np[j], j, st_out, ln_out, sg_out, &ds_out, ub + h->b_nu[j]);
    }
    h->b_chunks.build(st, ln, sg, {}, s);
    h->b_c0.upload(c0, s);
    h->b_c1.upload(c1, s);
    h->b_c2.upload(c2, s);
    h->b_c3.upload(c3, s);
    h->b_in.build(st_in, ln_in, sg_in, ds_in, s);
    h->b_out.build(st_out, ln_out, sg_out, ds_out, s);

    inst.clear();
    h->lv = std::move(merged);
    h->saddle = true;
    h->pinned = -1;
    if (bs) {
        SetupPhase ph(h, "schur_map");
        for (int l = 0; l + 1 < static_cast<int>(h->lv.size()); ++l)
            if (!h->lv[l].schur.lv.empty()) setup_schur_dense(h, l);
    }
    if (p.precision != AMG_PREC_FP64) {
        SetupPhase ph(h, "reduced_copies");
        build_mixed(h);
        build_saddle_mp(h);
    }
    {
        SetupPhase ph(h, "saddle_map");
        setup_saddle_tail(h);
    }
    h->n_dof = static_cast<int>(h->lv[0].vlen());
    const size_t nd = static_cast<size_t>(h->n_dof);
    h->b_b.alloc(nd);
    h->b_x.alloc(nd);
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

// ---------------------------------------------------------------- SPD batches
// Batches of independent SPD systems: every system gets the hierarchy
// amg_setup builds for it alone (FP64, no assembled coarse end); level l of
// the merged hierarchy concatenates the level-l operators of the systems
// that reach l, ordered by decreasing depth, so that the systems still
// coarsening lead it (nA rows: smoothed, restricted, corrected) and those
// ending on l follow (their explicit coarsest inverses, one segmented
// product). Greedy first-fit colouring in index order colours a
// block-diagonal graph as each block alone, so the merged colour lists
// (the leading systems' rows of each colour, in system order) sweep every
// system exactly as its own hierarchy would.
void build_batch_spd(amg_ctx *h, int nsys, const amg_system *sys) {
    hipStream_t s = h->stream;
    const amg_params &p = h->prm;
    std::vector<std::unique_ptr<amg_ctx>> inst(nsys);
    std::vector<int> depth(nsys);
    const int mode = sys[0].bs;
    for (int i = 0; i < nsys; ++i) {
        AMG_REQUIRE(sys[i].n_pres == 0, AMG_EINVAL, "amg_setup_batched: SPD and saddle point systems in one batch");
        AMG_REQUIRE(sys[i].bs == mode, AMG_EINVAL, "amg_setup_batched: SPD systems of one batch share bs");
        inst[i].reset(new amg_ctx());
        inst[i]->prm = p;
        inst[i]->prm.autotune = 0;
        inst[i]->prm.omega_model = nullptr;
        inst[i]->prm.precision = AMG_PREC_FP64;
        inst[i]->prm.fuse_coarse = 0;  // each system's coarse levels are merged, not assembled
        inst[i]->batch_member = true;
        inst[i]->stream = s;
    }
    build_instances(h, nsys, sys, inst);
    for (int i = 0; i < nsys; ++i) depth[i] = static_cast<int>(inst[i]->lv.size()) - 1;
    auto ph_merge = std::make_unique<SetupPhase>(h, "merge");
    std::vector<int> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return depth[a] > depth[b]; });
    const int maxd = depth[order[0]];
    const int nb = mode == 3 ? 9 : 1;
    std::vector<Level> merged(maxd + 1);
    for (int l = 0; l <= maxd; ++l) {
        std::vector<int> P;
        for (int i : order)
            if (depth[i] >= l) P.push_back(i);
        Level &M = merged[l];
        M.mode = mode;
        const size_t np_ = P.size();
        std::vector<int> noff(np_), nrow(np_);
        for (size_t j = 0; j < np_; ++j) {
            const Level &V = inst[P[j]]->lv[l];
            noff[j] = M.n;
            nrow[j] = V.n;
            M.n += V.n;
            M.n_lin += V.n_lin;
            M.n_quad += V.n_quad;
            M.nnz_pat_A += V.pattern_nnz_A();
            if (depth[P[j]] > l) M.nA += V.n;
        }
        M.coarsest = M.nA == 0;
        M.sys_noff = noff;
        M.sys_n = nrow;
        std::vector<const DMat *> pa;
        for (int i : P) pa.push_back(&inst[i]->lv[l].A);
        merge_mats(M.A, pa, nrow, noff, M.n, nb, s);
        {
            std::vector<const double *> dv;
            std::vector<int64_t> ln;
            for (size_t j = 0; j < np_; ++j) {
                const Level &V = inst[P[j]]->lv[l];
                dv.push_back(depth[P[j]] > l ? V.dinv.p : nullptr);
                ln.push_back(V.n);
            }
            merge_planes(M.dinv, dv, ln, nb, s);
        }
        if (M.nA > 0) {
            std::vector<const DMat *> pp, pr;
            std::vector<int> rows_p, rows_r, cp, cr;
            int n1 = 0;
            for (size_t j = 0; j < np_; ++j) {
                if (depth[P[j]] <= l) continue;
                const Level &V = inst[P[j]]->lv[l];
                const Level &W = inst[P[j]]->lv[l + 1];
                pp.push_back(&V.P);
                rows_p.push_back(V.n);
                cp.push_back(n1);
                pr.push_back(&V.R);
                rows_r.push_back(W.n);
                cr.push_back(noff[j]);
                n1 += W.n;
            }
            merge_mats(M.P, pp, rows_p, cp, n1, 1, s);
            merge_mats(M.R, pr, rows_r, cr, M.n, 1, s);
            // Gauss-Seidel: the leading systems' rows of each colour, in system order
            if (p.smoother == AMG_SMOOTH_GS) {
                int ncol = 0;
                for (size_t j = 0; j < np_; ++j)
                    if (depth[P[j]] > l) ncol = std::max(ncol, static_cast<int>(inst[P[j]]->lv[l].cptr.size()) - 1);
                const std::vector<int> arp = M.A.rowptr.download(s);
                std::vector<int> rows;
                M.cptr.assign(1, 0);
                M.colour_nnz.assign(ncol, 0);
                M.colour.assign(M.n, -1);
                // each system's rows bucketed by colour (in index order)
                std::vector<std::vector<int>> byc(np_), cst(np_);
                for (size_t j = 0; j < np_; ++j) {
                    if (depth[P[j]] <= l) continue;
                    const Level &V = inst[P[j]]->lv[l];
                    std::vector<int> &st = cst[j];
                    st.assign(ncol + 1, 0);
                    for (int i = 0; i < V.n; ++i) ++st[V.colour[i] + 1];
                    std::partial_sum(st.begin(), st.end(), st.begin());
                    std::vector<int> at(st.begin(), st.end() - 1);
                    byc[j].resize(V.n);
                    for (int i = 0; i < V.n; ++i) byc[j][at[V.colour[i]]++] = i;
                }
                for (int c = 0; c < ncol; ++c) {
                    for (size_t j = 0; j < np_; ++j) {
                        if (depth[P[j]] <= l) continue;
                        for (int t = cst[j][c]; t < cst[j][c + 1]; ++t) {
                            const int g = noff[j] + byc[j][t];
                            rows.push_back(g);
                            M.colour[g] = c;
                            M.colour_nnz[c] += arp[g + 1] - arp[g];
                        }
                    }
                    M.cptr.push_back(static_cast<int>(rows.size()));
                }
                std::vector<int> grp(rows.size() + 1, 0);
                for (size_t g = 0; g < rows.size(); ++g) grp[g + 1] = grp[g] + arp[rows[g] + 1] - arp[rows[g]];
                M.Ag = DMat();
                M.Ag.nrows = static_cast<int>(rows.size());
                M.Ag.ncols = M.n;
                M.Ag.np = M.A.np;
                M.Ag.nnz = grp.back();
                M.Ag.rowptr.upload(grp, s);
                M.Ag.col.alloc(static_cast<size_t>(std::max<int64_t>(1, M.Ag.nnz)));
                M.Ag.val.alloc(static_cast<size_t>(std::max<int64_t>(1, M.Ag.nnz * M.A.np)));
                if (rows.empty()) rows.push_back(0);
                M.g_rowid.upload(rows, s);
                M.d_cptr.upload(M.cptr, s);
                if (M.Ag.nrows > 0)
                    launch_gather_rows(M.A.np, M.Ag.nrows, M.g_rowid.p, M.A.rowptr.p, M.A.col.p, M.A.val.p,
                                       M.A.nnz, M.Ag.rowptr.p, M.Ag.col.p, M.Ag.val.p, M.Ag.nnz, s);
            }
        }
        // systems ending on this level: their coarsest inverses, as 3 n x 3 n
        // operators on their rows (A = A_s (x) I_3: the scalar inverse (x) I_3)
        for (size_t j = 0; j < np_; ++j)
            if (depth[P[j]] == l) {
                const Level &V = inst[P[j]]->lv[l];
                M.dseg.add(3 * V.n, 3 * noff[j], 3 * V.n, 0);
            }
        if (!M.dseg.h_m.empty()) {
            M.dseg.finalize(s);
            int k = 0;
            for (size_t j = 0; j < np_; ++j) {
                if (depth[P[j]] != l) continue;
                const amg_ctx &I = *inst[P[j]];
                const int m3 = M.dseg.h_m[k];
                AMG_REQUIRE(I.coarse_nc * I.coarse_m == m3, AMG_EINVAL, "batch: coarsest inverse size mismatch");
                std::vector<double> inv = I.coarse_inv.download(s), full;
                if (I.coarse_nc == 1) {
                    full.swap(inv);
                } else {
                    const int m = I.coarse_m;
                    full.assign(static_cast<size_t>(m3) * m3, 0.0);
                    for (int a = 0; a < m; ++a)
                        for (int b2 = 0; b2 < m; ++b2)
                            for (int c = 0; c < 3; ++c)
                                full[static_cast<size_t>(3 * a + c) * m3 + 3 * b2 + c] =
                                    inv[static_cast<size_t>(a) * m + b2];
                }
                AMG_HIP(hipMemcpyAsync(M.dseg.inv.p + M.dseg.h_moff[k], full.data(), full.size() * sizeof(double),
                                       hipMemcpyHostToDevice, s));
                AMG_HIP(hipStreamSynchronize(s));  // full is a local
                ++k;
            }
        }
        M.G = lanes_of(M.A.nnz, M.n);
        M.Gg = M.G;
        M.Gp = lanes_of(M.P.nnz, M.P.nrows);
        M.Gr = lanes_of(M.R.nnz, M.R.nrows);
        const size_t nv = 3 * static_cast<size_t>(std::max(1, M.n));
        M.x.alloc(nv);
        M.b.alloc(nv);
        M.r.alloc(nv);
        M.t.alloc(nv);
    }
    AMG_HIP(hipStreamSynchronize(s));
    ph_merge.reset();
    // (a reduced-precision cycle runs only the finest level's natural-order
    // FP64 kernels: the outer Krylov operator)
    if (p.autotune) {
        SetupPhase ph(h, "autotune");
        const bool reduced = p.precision != AMG_PREC_FP64;
        for (size_t l = 0; l < merged.size(); ++l)
            if (merged[l].nA > 0 && (!reduced || l == 0)) autotune_level(h, merged[l], reduced);
    }
    // level-0 layout of every system (velocity ranges only), chunk tables
    h->nsys = nsys;
    h->b_order = order;
    std::vector<int64_t> user(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i) user[i + 1] = user[i] + 3 * static_cast<int64_t>(sys[i].n_lin + sys[i].n_quad);
    h->b_uoff.assign(nsys, 0);
    h->b_poff.assign(nsys, 0);
    h->b_nu.assign(nsys, 0);
    h->b_np.assign(nsys, 0);
    {
        int64_t u = 0;
        for (int j = 0; j < nsys; ++j) {
            const amg_system &S = sys[order[j]];
            h->b_uoff[j] = u;
            h->b_nu[j] = 3 * static_cast<int64_t>(S.n_lin + S.n_quad);
            u += h->b_nu[j];
        }
    }
    std::vector<int64_t> st, ds_unused, st_in, ds_in, st_out, ds_out;
    std::vector<int> ln, sg, ln_in, sg_in, ln_out, sg_out;
    std::vector<int> c0(nsys), c1(nsys), c2(nsys), c3(nsys);
    for (int j = 0; j < nsys; ++j) {
        c0[j] = static_cast<int>(st.size());
        add_chunks(h->b_uoff[j], h->b_nu[j], j, st, ln, sg, nullptr, 0);
        c1[j] = static_cast<int>(st.size());
    }
    for (int j = 0; j < nsys; ++j) c2[j] = c3[j] = static_cast<int>(st.size());
    for (int j = 0; j < nsys; ++j) {
        const int64_t ub = user[order[j]];
        add_chunks(ub, h->b_nu[j], j, st_in, ln_in, sg_in, &ds_in, h->b_uoff[j]);
        add_chunks(h->b_uoff[j], h->b_nu[j], j, st_out, ln_out, sg_out, &ds_out, ub);
    }
    h->b_chunks.build(st, ln, sg, {}, s);
    h->b_c0.upload(c0, s);
    h->b_c1.upload(c1, s);
    h->b_c2.upload(c2, s);
    h->b_c3.upload(c3, s);
    h->b_in.build(st_in, ln_in, sg_in, ds_in, s);
    h->b_out.build(st_out, ln_out, sg_out, ds_out, s);
    inst.clear();
    h->lv = std::move(merged);
    h->saddle = false;
    h->pinned = -1;
    h->n_dof = 3 * h->lv[0].n;
    const size_t nd = static_cast<size_t>(h->n_dof);
    h->b_b.alloc(nd);
    h->b_x.alloc(nd);
    h->kr.alloc(nd);
    h->kz.alloc(nd);
    h->kp.alloc(nd);
    h->kq.alloc(nd);
    h->kw.alloc(nd);
    h->partial.alloc(static_cast<size_t>(std::max(1024 * 128, row_blocks(h->lv[0].n, 64))));
    if (p.precision != AMG_PREC_FP64) {
        // FP32 finest / BF16 (FP32) coarse copies of the merged levels; the
        // systems ending on a level keep their FP64 inverses
        SetupPhase ph(h, "reduced_copies");
        build_mixed(h);
    }
    h->tune_flush.release();
    h->sc.alloc(SC_COUNT);
    if (!h->h_sc) AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->h_sc), SC_COUNT * sizeof(double)));
    AMG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- batched FGMRES
// Per-system norms of a merged level-0 vector (host result).
static void seg_norms(amg_ctx *h, const double *v, DevBuf<double> &partial, DevBuf<double> &hb, int kmax,
                      std::vector<double> &out) {
    const ChunkView t = h->b_chunks.view();
    launch_seg_multidot(v, 0, 1, v, t, partial.p, h->stream);
    launch_seg_reduce(partial.p, t.n, 1, h->nsys, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p, kmax, h->stream);
    std::vector<double> tmp(static_cast<size_t>(h->nsys) * kmax);
    AMG_HIP(hipMemcpyAsync(tmp.data(), hb.p, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    AMG_HIP(hipStreamSynchronize(h->stream));
    out.resize(h->nsys);
    for (int i = 0; i < h->nsys; ++i) out[i] = std::sqrt(tmp[static_cast<size_t>(i) * kmax]);
}

// Right-preconditioned FGMRES(m), one Krylov process per system, advanced in
// lockstep: every launch serves all systems; a system that has converged
// stops taking Arnoldi steps (its columns are left out of its update) while
// the others continue. Orthogonalisation as in solve_fgmres (classical
// Gram-Schmidt with delayed reorthogonalisation, one pass of dots and one
// update per step, Hessenberg columns completed one step late or, when a
// system's provisional estimate meets the tolerance or the cycle ends, by one
// more pass over that system's chunks of the basis).
int solve_fgmres_batched(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int ns = h->nsys;
    const int64_t n = h->n_dof;
    const int m = std::max(1, h->prm.restart);
    if (h->gm_m != m) {
        h->gm_V.alloc(static_cast<size_t>(m + 1) * n);
        h->gm_Z.alloc(static_cast<size_t>(m) * n);
        h->gm_m = m;
    }
    const ChunkView t = h->b_chunks.view();
    // per system: the dots of a step (2 (m + 2)), then gamma, d, eta
    const int stride = 2 * (m + 2) + 4;
    DevBuf<double> partial(static_cast<size_t>(2 * (m + 2)) * std::max(1, t.n)),
        hb(static_cast<size_t>(ns) * stride), coef(ns), ycoef(static_cast<size_t>(ns) * m);
    DevBuf<int> cnt(ns), want(ns);
    double *V = h->gm_V.p, *Z = h->gm_Z.p;
    // per system: H rotated columns (row-major q * m + c), Hr raw columns
    // (column c at c * (m + 1)), rotations, g, pending scales eta
    const size_t hsz = static_cast<size_t>(m + 1) * m;
    std::vector<double> H(ns * hsz), Hr(ns * hsz), cs(static_cast<size_t>(ns) * m), sn(static_cast<size_t>(ns) * m),
        g(static_cast<size_t>(ns) * (m + 1)), eta(static_cast<size_t>(ns) * (m + 1), 1.0), hcol(m + 2),
        estl(ns, 1.0);
    // the step's dots land in pinned host memory (asynchronous copies, so
    // that the next step's preconditioner can be enqueued before the wait)
    const size_t nh = static_cast<size_t>(ns) * stride;
    if (h->gm_hpin_n < nh) {
        if (h->gm_hpin) AMG_HIP(hipHostFree(h->gm_hpin));
        h->gm_hpin = nullptr;
        AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->gm_hpin), nh * sizeof(double)));
        h->gm_hpin_n = nh;
    }
    double *hp = h->gm_hpin;
    if (!h->sc_ready) AMG_HIP(hipEventCreateWithFlags(&h->sc_ready, hipEventDisableTiming));
    std::vector<double> beta, r0;
    std::vector<int> status(ns, AMG_NOT_CONVERGED), iters(ns, 0), jcnt(ns, 0), wanth(ns, 0);
    std::vector<char> active(ns, 0), running(ns, 0), done(static_cast<size_t>(ns) * m, 0);
    std::vector<double> hc(ns);
    system_residual(h, b, x, V);
    seg_norms(h, V, partial, hb, stride, r0);
    beta = r0;
    for (int i = 0; i < ns; ++i) {
        if (!(r0[i] == r0[i])) status[i] = AMG_DIVERGED;
        else if (r0[i] == 0.0) status[i] = AMG_OK;
        else active[i] = 1;
    }
    auto any = [&](const std::vector<char> &v) { return std::any_of(v.begin(), v.end(), [](char c) { return c != 0; }); };
    // system i: rotations 0..c-1 on raw column c, rotation c, g; returns the
    // residual estimate after c + 1 columns (commit) or only that estimate
    auto rotate = [&](int i, int c, bool commit) {
        const double *raw = &Hr[i * hsz + static_cast<size_t>(c) * (m + 1)];
        double *csi = &cs[static_cast<size_t>(i) * m], *sni = &sn[static_cast<size_t>(i) * m];
        double *gi = &g[static_cast<size_t>(i) * (m + 1)];
        for (int q = 0; q <= c + 1; ++q) hcol[q] = raw[q];
        for (int q = 0; q < c; ++q) {
            const double tq = csi[q] * hcol[q] + sni[q] * hcol[q + 1];
            hcol[q + 1] = -sni[q] * hcol[q] + csi[q] * hcol[q + 1];
            hcol[q] = tq;
        }
        const double den = std::hypot(hcol[c], hcol[c + 1]);
        if (!commit) return den > 0.0 ? std::fabs(hcol[c + 1] / den * gi[c]) / r0[i] : 0.0;
        csi[c] = den > 0.0 ? hcol[c] / den : 1.0;
        sni[c] = den > 0.0 ? hcol[c + 1] / den : 0.0;
        hcol[c] = den;
        gi[c + 1] = -sni[c] * gi[c];
        gi[c] = csi[c] * gi[c];
        double *Hi = &H[i * hsz];
        for (int q = 0; q <= c; ++q) Hi[static_cast<size_t>(q) * m + c] = hcol[q];
        return std::fabs(gi[c + 1]) / r0[i];
    };
    // a completed column's test: false when system i stops taking steps
    auto judge = [&](int i, double est, bool breakdown) {
        estl[i] = est;
        if (!(est == est) || est > 1e3) {
            status[i] = AMG_DIVERGED;
            running[i] = 0;
            active[i] = 0;
            return false;
        }
        if (est <= tol || breakdown) {
            running[i] = 0;
            return false;
        }
        return true;
    };
    int it = 0;
    while (any(active) && it < maxit) {
        for (int i = 0; i < ns; ++i) hc[i] = active[i] && beta[i] > 0.0 ? 1.0 / beta[i] : 0.0;
        AMG_HIP(hipMemcpyAsync(coef.p, hc.data(), ns * sizeof(double), hipMemcpyHostToDevice, h->stream));
        launch_seg_scale(V, V, coef.p, t, h->stream);
        std::fill(g.begin(), g.end(), 0.0);
        std::fill(done.begin(), done.end(), 0);
        for (int i = 0; i < ns; ++i) {
            g[static_cast<size_t>(i) * (m + 1)] = active[i] ? beta[i] : 0.0;
            running[i] = active[i];
            jcnt[i] = 0;
        }
        bool ahead = false;  // this step's preconditioner already enqueued
        for (int j = 0; j < m && any(running) && it < maxit; ++j, ++it) {
            double *vj = V + static_cast<int64_t>(j) * n, *w = V + static_cast<int64_t>(j + 1) * n;
            double *zj = Z + static_cast<int64_t>(j) * n;
            if (!ahead) precondition_any(h, vj, zj);
            ahead = false;
            system_matvec(h, zj, w);
            const int k = j + 2;
            launch_seg_multidot2(V, n, k, vj, w, t, partial.p, h->stream);
            launch_seg_reduce(partial.p, t.n, 2 * k, ns, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p, stride,
                              h->stream);
            launch_seg_dcgs2_update(V, n, j, hb.p, stride, t, j > 0, h->stream);
            AMG_HIP(hipMemcpyAsync(hp, hb.p, nh * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            AMG_HIP(hipEventRecord(h->sc_ready, h->stream));
            // the pending vectors u_{j+1} are final for step j + 1: their
            // preconditioner goes ahead of the host's wait while every
            // running system's last estimate is far from the tolerance
            {
                double emin = 1e300;
                for (int i = 0; i < ns; ++i)
                    if (running[i]) emin = std::min(emin, estl[i]);
                if (j + 1 < m && it + 1 < maxit && emin > KRYLOV_AHEAD * tol) {
                    precondition_any(h, w, Z + static_cast<int64_t>(j + 1) * n);
                    ahead = true;
                }
            }
            AMG_HIP(hipEventSynchronize(h->sc_ready));
            const bool last = j + 1 == m || it + 1 >= maxit;
            bool cleanup = false;
            for (int i = 0; i < ns; ++i) {
                wanth[i] = 0;
                if (!running[i]) continue;
                const double *hi = &hp[static_cast<size_t>(i) * stride];
                const double *dA = hi, *dB = hi + k;
                const double gam = hi[2 * k], d = hi[2 * k + 1], et = hi[2 * k + 2];
                double *ei = &eta[static_cast<size_t>(i) * (m + 1)];
                char *di = &done[static_cast<size_t>(i) * m];
                if (j > 0 && !di[j - 1]) {
                    // u_j = V s + gamma v_j completes column j - 1
                    double *c1 = &Hr[i * hsz + static_cast<size_t>(j - 1) * (m + 1)];
                    for (int q = 0; q < j; ++q) c1[q] += ei[j] * dA[q];
                    c1[j] = ei[j] * gam;
                    di[j - 1] = 1;
                    jcnt[i] = j;
                    if (!judge(i, rotate(i, j - 1, true), gam == 0.0)) continue;
                }
                double *cj = &Hr[i * hsz + static_cast<size_t>(j) * (m + 1)];
                for (int q = 0; q < j; ++q) cj[q] = dB[q];
                cj[j] = d;
                cj[j + 1] = et;
                ei[j + 1] = et;
                wanth[i] = last || et == 0.0 || rotate(i, j, false) <= tol;
                cleanup |= wanth[i] != 0;
            }
            if (cleanup) {
                // complete column j of the flagged systems: V_{0..j} . u_{j+1}, |u_{j+1}|^2
                AMG_HIP(hipMemcpyAsync(want.p, wanth.data(), ns * sizeof(int), hipMemcpyHostToDevice, h->stream));
                launch_seg_multidot_masked(V, n, k, w, t, want.p, partial.p, h->stream);
                launch_seg_reduce(partial.p, t.n, k, ns, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p, stride,
                                  h->stream);
                AMG_HIP(hipMemcpyAsync(hp, hb.p, nh * sizeof(double), hipMemcpyDeviceToHost, h->stream));
                AMG_HIP(hipStreamSynchronize(h->stream));
                for (int i = 0; i < ns; ++i) {
                    if (!wanth[i]) continue;
                    const double *si = &hp[static_cast<size_t>(i) * stride];
                    const double et = eta[static_cast<size_t>(i) * (m + 1) + j + 1];
                    double *cj = &Hr[i * hsz + static_cast<size_t>(j) * (m + 1)];
                    double ss = 0.0;
                    for (int q = 0; q <= j; ++q) {
                        ss += si[q] * si[q];
                        cj[q] += et * si[q];
                    }
                    const double g2 = si[j + 1] - ss;
                    cj[j + 1] = et * (g2 > 0.0 ? std::sqrt(g2) : 0.0);
                    done[static_cast<size_t>(i) * m + j] = 1;
                    jcnt[i] = j + 1;
                    judge(i, rotate(i, j, true), cj[j + 1] == 0.0);
                }
            }
        }
        for (int i = 0; i < ns; ++i) iters[i] += jcnt[i];
        // x_i += Z y_i with y_i = R_i^{-1} g_i over the system's own columns
        std::vector<double> Y(static_cast<size_t>(ns) * m, 0.0);
        for (int i = 0; i < ns; ++i) {
            const int ji = jcnt[i];
            const double *Hi = &H[static_cast<size_t>(i) * (m + 1) * m];
            const double *gi = &g[static_cast<size_t>(i) * (m + 1)];
            double *yi = &Y[static_cast<size_t>(i) * m];
            for (int q = ji - 1; q >= 0; --q) {
                double sv = gi[q];
                for (int k = q + 1; k < ji; ++k) sv -= Hi[static_cast<size_t>(q) * m + k] * yi[k];
                yi[q] = Hi[static_cast<size_t>(q) * m + q] != 0.0 ? sv / Hi[static_cast<size_t>(q) * m + q] : 0.0;
            }
        }
        AMG_HIP(hipMemcpyAsync(ycoef.p, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
        AMG_HIP(hipMemcpyAsync(cnt.p, jcnt.data(), ns * sizeof(int), hipMemcpyHostToDevice, h->stream));
        launch_seg_multi_add(Z, n, ycoef.p, m, cnt.p, x, t, h->stream);
        system_residual(h, b, x, V);
        seg_norms(h, V, partial, hb, stride, beta);
        for (int i = 0; i < ns; ++i)
            if (active[i] && beta[i] / r0[i] <= tol) {
                status[i] = AMG_OK;
                active[i] = 0;
            }
    }
    system_residual(h, b, x, h->kw.p);
    std::vector<double> fin;
    seg_norms(h, h->kw.p, partial, hb, stride, fin);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = AMG_OK;
    for (int j = 0; j < ns; ++j) {
        const double rel = r0[j] > 0.0 ? fin[j] / r0[j] : 0.0;
        int st = status[j];
        if (st == AMG_OK && !(rel == rel)) st = AMG_DIVERGED;
        if (res) {
            amg_result &o = res[h->b_order[j]];
            o.iters = iters[j];
            o.status = st;
            o.relres = rel;
            o.solve_ms = ms;
        }
        worst = std::max(worst, st);
    }
    profile_collect(h);
    return worst;
}

// AMG-preconditioned CG on every system of an SPD batch, in lockstep: one
// launch per operation serves all systems, and each system keeps its own
// step lengths, residual norm, stopping test and iteration count (a system
// that has converged, broken down or diverged takes zero steps from then
// on; its iterate stays). Two host synchronisations per iteration: <p, Ap>,
// then ||r|| and <r, z> in one pass. With the flexible variant (FCG(1), for
// the reduced-precision cycle, as solve_fcg): alpha = <p, r> / <p, Ap> and
// p = z - (<z, q_prev> / <p_prev, q_prev>) p_prev, two synchronisations per
// iteration (<p, Ap> with <p, r>; ||r|| with the next <z, q_prev>) while
// every running system is far from the tolerance, three near it.
int solve_pcg_batched(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int ns = h->nsys;
    const int64_t n = h->n_dof;
    hipStream_t s = h->stream;
    const ChunkView t = h->b_chunks.view();
    double *r = h->kr.p, *z = h->kz.p, *pv = h->kp.p, *q = h->kq.p;
    DevBuf<double> partial(static_cast<size_t>(2) * std::max(1, t.n)), hb(static_cast<size_t>(2) * ns), da(ns),
        dm(ns), dbeta(ns), dones(ns);
    std::vector<double> hv(static_cast<size_t>(2) * ns), r0(ns), rz(ns), alpha(ns, 0.0), malpha(ns, 0.0),
        beta(ns, 0.0), ones(ns, 1.0), pq(ns);
    std::vector<int> status(ns, AMG_NOT_CONVERGED), iters(ns, 0);
    std::vector<char> active(ns, 0);
    // k = 1: <a, c> per system; k = 2: <a, a> and <a, c>
    auto dots = [&](const double *a, const double *c, int k) {
        if (k == 1)
            launch_seg_multidot(a, 0, 1, c, t, partial.p, s);
        else
            launch_seg_multidot2(a, 0, 1, a, c, t, partial.p, s);
        launch_seg_reduce(partial.p, t.n, k, ns, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p, k, s);
        AMG_HIP(hipMemcpyAsync(hv.data(), hb.p, static_cast<size_t>(k) * ns * sizeof(double), hipMemcpyDeviceToHost,
                               s));
        AMG_HIP(hipStreamSynchronize(s));
    };
    // <v, a> and <v, c> per system
    auto dots_pair = [&](const double *v, const double *a, const double *c) {
        launch_seg_multidot2(v, 0, 1, a, c, t, partial.p, s);
        launch_seg_reduce(partial.p, t.n, 2, ns, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p, 2, s);
        AMG_HIP(hipMemcpyAsync(hv.data(), hb.p, 2 * static_cast<size_t>(ns) * sizeof(double), hipMemcpyDeviceToHost,
                               s));
        AMG_HIP(hipStreamSynchronize(s));
    };
    auto put = [&](DevBuf<double> &d, const std::vector<double> &v) {
        AMG_HIP(hipMemcpyAsync(d.p, v.data(), ns * sizeof(double), hipMemcpyHostToDevice, s));
    };
    auto any_active = [&] { return std::any_of(active.begin(), active.end(), [](char c) { return c != 0; }); };
    put(dones, ones);
    system_residual(h, b, x, r);
    dots(r, r, 1);
    for (int i = 0; i < ns; ++i) {
        r0[i] = std::sqrt(hv[i]);
        if (!(r0[i] == r0[i])) status[i] = AMG_DIVERGED;
        else if (r0[i] == 0.0) status[i] = AMG_OK;
        else active[i] = 1;
    }
    const bool flexible = h->prm.krylov == AMG_KRYLOV_FCG;
    // FCG: while every running system's last relative residual is above
    // KRYLOV_AHEAD * tol, the next preconditioner application goes ahead of
    // the stopping test's read, and <z, q_prev> comes back in that read
    double relmin = 1.0;
    bool ahead = false;
    std::vector<double> zq(ns);
    for (int it = 0; flexible && any_active() && it < maxit; ++it) {
        if (!ahead) precondition(h, r, z);
        if (it == 0) {
            launch_copy(pv, z, n, s);
        } else {
            if (ahead)
                std::copy(zq.begin(), zq.end(), hv.begin());
            else
                dots(z, q, 1);  // <z, q_prev>
            for (int i = 0; i < ns; ++i) beta[i] = active[i] && pq[i] > 0.0 ? -hv[i] / pq[i] : 0.0;
            put(dbeta, beta);
            launch_seg_axpby(z, pv, dones.p, dbeta.p, t, s);  // p = z + beta p
        }
        apply_level(h, 0, pv, q);
        dots_pair(pv, q, r);  // <p, q>, <p, r>
        for (int i = 0; i < ns; ++i) {
            pq[i] = hv[2 * i];
            alpha[i] = 0.0;
            if (!active[i]) continue;
            if (!(pq[i] > 0.0) || !(hv[2 * i + 1] == hv[2 * i + 1])) {
                status[i] = AMG_BREAKDOWN;
                active[i] = 0;
                continue;
            }
            alpha[i] = hv[2 * i + 1] / pq[i];
            ++iters[i];
        }
        for (int i = 0; i < ns; ++i) malpha[i] = -alpha[i];
        put(da, alpha);
        put(dm, malpha);
        launch_seg_axpby(pv, x, da.p, dones.p, t, s);  // x += alpha p
        launch_seg_axpby(q, r, dm.p, dones.p, t, s);   // r -= alpha q
        ahead = it + 1 < maxit && relmin > KRYLOV_AHEAD * tol;
        if (ahead) {
            // <r, r> into hb[0, ns), then z and <z, q> into hb[ns, 2 ns): one read
            launch_seg_multidot(r, 0, 1, r, t, partial.p, s);
            launch_seg_reduce(partial.p, t.n, 1, ns, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p, 1, s);
            precondition(h, r, z);
            launch_seg_multidot(z, 0, 1, q, t, partial.p, s);
            launch_seg_reduce(partial.p, t.n, 1, ns, h->b_c0.p, h->b_c1.p, h->b_c2.p, h->b_c3.p, hb.p + ns, 1, s);
            AMG_HIP(hipMemcpyAsync(hv.data(), hb.p, 2 * static_cast<size_t>(ns) * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
            AMG_HIP(hipStreamSynchronize(s));
            std::copy(hv.begin() + ns, hv.begin() + 2 * ns, zq.begin());
        } else {
            dots(r, r, 1);
        }
        relmin = 1e300;
        for (int i = 0; i < ns; ++i) {
            if (!active[i]) continue;
            const double rel = std::sqrt(hv[i]) / r0[i];
            if (!(rel == rel) || rel > 1e3) {
                status[i] = AMG_DIVERGED;
                active[i] = 0;
            } else if (rel <= tol) {
                status[i] = AMG_OK;
                active[i] = 0;
            } else {
                relmin = std::min(relmin, rel);
            }
        }
    }
    if (!flexible && any_active()) {
        precondition(h, r, z);
        launch_copy(pv, z, n, s);
        dots(r, z, 1);
        for (int i = 0; i < ns; ++i) rz[i] = hv[i];
    }
    int it = 0;
    while (!flexible && any_active() && it < maxit) {
        apply_level(h, 0, pv, q);
        dots(pv, q, 1);
        for (int i = 0; i < ns; ++i) {
            pq[i] = hv[i];
            alpha[i] = 0.0;
            if (!active[i]) continue;
            if (!(pq[i] > 0.0) || !(rz[i] == rz[i])) {
                status[i] = AMG_BREAKDOWN;
                active[i] = 0;
                continue;
            }
            alpha[i] = rz[i] / pq[i];
            ++iters[i];
        }
        for (int i = 0; i < ns; ++i) malpha[i] = -alpha[i];
        put(da, alpha);
        put(dm, malpha);
        launch_seg_axpby(pv, x, da.p, dones.p, t, s);  // x += alpha p
        launch_seg_axpby(q, r, dm.p, dones.p, t, s);   // r -= alpha q
        ++it;
        precondition(h, r, z);
        dots(r, z, 2);
        for (int i = 0; i < ns; ++i) {
            beta[i] = 0.0;
            if (!active[i]) continue;
            const double rel = std::sqrt(hv[2 * i]) / r0[i];
            if (!(rel == rel) || rel > 1e3) {
                status[i] = AMG_DIVERGED;
                active[i] = 0;
            } else if (rel <= tol) {
                status[i] = AMG_OK;
                active[i] = 0;
            } else {
                beta[i] = hv[2 * i + 1] / rz[i];
                rz[i] = hv[2 * i + 1];
            }
        }
        put(dbeta, beta);
        launch_seg_axpby(z, pv, dones.p, dbeta.p, t, s);  // p = z + beta p
    }
    // the true residual of every system
    system_residual(h, b, x, h->kw.p);
    dots(h->kw.p, h->kw.p, 1);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = AMG_OK;
    for (int j = 0; j < ns; ++j) {
        const double rel = r0[j] > 0.0 ? std::sqrt(hv[j]) / r0[j] : 0.0;
        int st = status[j];
        if (st == AMG_OK && !(rel == rel)) st = AMG_DIVERGED;
        if (res) {
            amg_result &o = res[h->b_order[j]];
            o.iters = iters[j];
            o.status = st;
            o.relres = rel;
            o.solve_ms = ms;
        }
        worst = std::max(worst, st);
    }
    profile_collect(h);
    return worst;
}

}  // namespace amgp2
