// C ABI entry points (include/amg_p2.h). Every call catches library errors
// and returns an AMG_* code; the message is kept per thread for
// amg_last_error().
#include <cmath>
#include <cstring>

#include "context.h"

namespace amgp2 {
static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }
}  // namespace amgp2

using namespace amgp2;

amg_ctx::~amg_ctx() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto &pe : pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    if (sc_ready) (void)hipEventDestroy(sc_ready);
    if (gm_hpin) (void)hipHostFree(gm_hpin);
    if (h_sc) (void)hipHostFree(h_sc);
}

// A system given in device memory (amg_system::memory == AMG_MEM_DEVICE),
// copied to host vectors in stream order; sys then points at them.
struct StagedSystem {
    std::vector<int32_t> arp, acol, brp, bcol, crp, ccol;
    std::vector<double> aval, bval, cval;
    amg_system sys{};
};

static void require_device(const void *p, const char *name) {
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) (void)hipGetLastError();
    AMG_REQUIRE(e == hipSuccess && (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged), AMG_EINVAL,
                std::string("amg_setup: ") + name + " is not device memory (memory = AMG_MEM_DEVICE)");
}

template <typename T>
static void fetch(std::vector<T> &dst, const T *src, int64_t n, const char *name, hipStream_t s) {
    dst.resize(static_cast<size_t>(std::max<int64_t>(n, 0)));
    if (n <= 0) return;
    require_device(src, name);
    AMG_HIP(hipMemcpyAsync(dst.data(), src, static_cast<size_t>(n) * sizeof(T), hipMemcpyDeviceToHost, s));
}

static void stage_system(const amg_system &in, hipStream_t s, StagedSystem &out) {
    out.sys = in;
    out.sys.memory = AMG_MEM_HOST;
    const int64_t n = static_cast<int64_t>(in.n_lin) + in.n_quad;
    AMG_REQUIRE(n > 0 && in.n_lin >= 0 && in.n_quad >= 0 && in.n_pres >= 0 && (in.bs == 1 || in.bs == 3),
                AMG_EINVAL, "amg_setup: invalid sizes");
    AMG_REQUIRE(in.A_rowptr && in.A_col && in.A_val, AMG_EINVAL, "amg_setup: A is missing");
    // row pointers first: their last entries give the array lengths
    fetch(out.arp, in.A_rowptr, n + 1, "A_rowptr", s);
    const bool has_b = in.n_pres > 0 && in.B_rowptr && in.B_col && in.B_val;
    const bool has_c = in.n_pres > 0 && in.C_rowptr && in.C_col && in.C_val;
    if (has_b) fetch(out.brp, in.B_rowptr, static_cast<int64_t>(in.n_pres) + 1, "B_rowptr", s);
    if (has_c) fetch(out.crp, in.C_rowptr, static_cast<int64_t>(in.n_pres) + 1, "C_rowptr", s);
    AMG_HIP(hipStreamSynchronize(s));
    const int64_t na = out.arp[n], nb = has_b ? out.brp[in.n_pres] : 0, nc = has_c ? out.crp[in.n_pres] : 0;
    AMG_REQUIRE(na >= 0 && nb >= 0 && nc >= 0, AMG_EINVAL, "amg_setup: negative entry count in a row pointer");
    fetch(out.acol, in.A_col, na, "A_col", s);
    fetch(out.aval, in.A_val, na * in.bs * in.bs, "A_val", s);
    if (has_b) {
        fetch(out.bcol, in.B_col, nb, "B_col", s);
        fetch(out.bval, in.B_val, 3 * nb, "B_val", s);
    }
    if (has_c) {
        fetch(out.ccol, in.C_col, nc, "C_col", s);
        fetch(out.cval, in.C_val, nc, "C_val", s);
    }
    AMG_HIP(hipStreamSynchronize(s));
    // a zero-length array still needs a non-null host pointer for the checks
    for (auto *v : {&out.acol, &out.bcol, &out.ccol})
        if (v->empty()) v->push_back(0);
    for (auto *v : {&out.aval, &out.bval, &out.cval})
        if (v->empty()) v->push_back(0.0);
    out.sys.A_rowptr = out.arp.data();
    out.sys.A_col = out.acol.data();
    out.sys.A_val = out.aval.data();
    out.sys.B_rowptr = has_b ? out.brp.data() : nullptr;
    out.sys.B_col = has_b ? out.bcol.data() : nullptr;
    out.sys.B_val = has_b ? out.bval.data() : nullptr;
    out.sys.C_rowptr = has_c ? out.crp.data() : nullptr;
    out.sys.C_col = has_c ? out.ccol.data() : nullptr;
    out.sys.C_val = has_c ? out.cval.data() : nullptr;
}

template <typename F>
static int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return AMG_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return AMG_EHIP;
    }
}

extern "C" {

void amg_default_params(amg_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->smoother = AMG_SMOOTH_GS;
    p->pre = 1;
    p->post = 1;
    p->omega = 0.5;
    p->sgs_omega = 0.125;
    p->sgs_damping = 0.5;
    p->cycles = 1;
    p->nu = 1;
    p->max_levels = 10;
    p->coarse_max = 300;
    p->separate = 1;
    p->krylov = AMG_KRYLOV_PCG;
    p->restart = 100;
    p->precision = AMG_PREC_FP64;
    p->n_level_omega = 0;
    p->level_omega = nullptr;
    p->fuse_coarse = 1;
    p->autotune = 1;
    p->omega_model = nullptr;
    p->graph = 1;
    p->vanka_omega = 0.8;
    p->gs_post = 0;
}

int amg_setup(const amg_system *sys, const amg_params *params, amg_stream stream, amg_handle *out) {
    return guarded([&]() -> int {
        AMG_REQUIRE(out != nullptr, AMG_EINVAL, "amg_setup: null output handle");
        *out = nullptr;
        AMG_REQUIRE(params != nullptr, AMG_EINVAL, "amg_setup: null params");
        const amg_params &p = *params;
        AMG_REQUIRE(sys != nullptr, AMG_EINVAL, "amg_setup: null system");
        AMG_REQUIRE(sys->memory == AMG_MEM_HOST || sys->memory == AMG_MEM_DEVICE, AMG_EINVAL,
                    "amg_setup: memory must be AMG_MEM_HOST or AMG_MEM_DEVICE");
        StagedSystem staged;
        if (sys->memory == AMG_MEM_DEVICE) {
            stage_system(*sys, static_cast<hipStream_t>(stream), staged);
            sys = &staged.sys;
        }
        if (sys->n_pres > 0) {
            AMG_REQUIRE(p.smoother == AMG_SMOOTH_SGS || p.smoother == AMG_SMOOTH_BS ||
                            p.smoother == AMG_SMOOTH_VANKA,
                        AMG_EINVAL, "amg_setup: saddle point systems need the sGS, Braess-Sarazin or Vanka smoother");
            AMG_REQUIRE(p.smoother != AMG_SMOOTH_VANKA || p.precision == AMG_PREC_FP64, AMG_EUNSUPPORTED,
                        "amg_setup: the Vanka smoother runs in FP64");
            AMG_REQUIRE(p.krylov == AMG_KRYLOV_FGMRES || p.krylov == AMG_KRYLOV_NONE, AMG_EINVAL,
                        "amg_setup: saddle point systems need FGMRES or the stand-alone iteration");
            AMG_REQUIRE(p.precision == AMG_PREC_FP64 || p.krylov == AMG_KRYLOV_FGMRES, AMG_EINVAL,
                        "amg_setup: a reduced-precision saddle cycle needs the flexible GMRES outer loop");
        } else {
            AMG_REQUIRE(p.smoother == AMG_SMOOTH_JA || p.smoother == AMG_SMOOTH_GS, AMG_EINVAL,
                        "amg_setup: SPD systems need the JA or GS smoother");
        }
        AMG_REQUIRE(!p.omega_model || (p.smoother == AMG_SMOOTH_JA && sys->n_pres == 0), AMG_EINVAL,
                    "amg_setup: omega_model needs the JA smoother on an SPD system");
        AMG_REQUIRE(p.krylov != AMG_KRYLOV_FGMRES || p.restart >= 1, AMG_EINVAL, "amg_setup: restart < 1");
        AMG_REQUIRE(p.pre >= 0 && p.post >= 0 && p.cycles >= 1 && p.nu >= 1 && p.nu <= 2, AMG_EINVAL,
                    "amg_setup: invalid smoothing/cycle counts");
        AMG_REQUIRE(p.precision == AMG_PREC_FP64 || p.precision == AMG_PREC_MIXED || p.precision == AMG_PREC_FP32,
                    AMG_EINVAL, "amg_setup: unknown precision mode");
        AMG_REQUIRE(p.gs_post >= 0 && p.gs_post <= 2, AMG_EINVAL, "amg_setup: gs_post must be 0, 1 or 2");
        auto *h = new amg_ctx();
        h->prm = p;
        h->post_forward = p.gs_post == 2 || (p.gs_post == 0 && p.krylov == AMG_KRYLOV_NONE);
        h->prm.level_omega = nullptr;
        if (p.n_level_omega > 0 && p.level_omega)
            h->level_omega.assign(p.level_omega, p.level_omega + p.n_level_omega);
        h->stream = static_cast<hipStream_t>(stream);
        try {
            build_hierarchy(h, sys);
        } catch (...) {
            delete h;
            throw;
        }
        h->prm.omega_model = nullptr;  // only read during setup
        *out = h;
        return AMG_OK;
    });
}

static void check_params(const amg_params &p, bool saddle) {
    if (saddle) {
        AMG_REQUIRE(p.smoother == AMG_SMOOTH_SGS || p.smoother == AMG_SMOOTH_BS, AMG_EINVAL,
                    "amg_setup: saddle point systems need the sGS or Braess-Sarazin smoother");
        AMG_REQUIRE(p.krylov == AMG_KRYLOV_FGMRES || p.krylov == AMG_KRYLOV_NONE, AMG_EINVAL,
                    "amg_setup: saddle point systems need FGMRES or the stand-alone iteration");
        AMG_REQUIRE(p.precision == AMG_PREC_FP64 || p.krylov == AMG_KRYLOV_FGMRES, AMG_EINVAL,
                    "amg_setup: a reduced-precision saddle cycle needs the flexible GMRES outer loop");
    }
    AMG_REQUIRE(p.krylov != AMG_KRYLOV_FGMRES || p.restart >= 1, AMG_EINVAL, "amg_setup: restart < 1");
    AMG_REQUIRE(p.pre >= 0 && p.post >= 0 && p.cycles >= 1 && p.nu >= 1 && p.nu <= 2, AMG_EINVAL,
                "amg_setup: invalid smoothing/cycle counts");
    AMG_REQUIRE(p.gs_post >= 0 && p.gs_post <= 2, AMG_EINVAL, "amg_setup: gs_post must be 0, 1 or 2");
}

int amg_setup_batched(int32_t nsys, const amg_system *systems, const amg_params *params, amg_stream stream,
                      amg_handle *out) {
    return guarded([&]() -> int {
        AMG_REQUIRE(out != nullptr, AMG_EINVAL, "amg_setup_batched: null output handle");
        *out = nullptr;
        AMG_REQUIRE(systems && params && nsys >= 1, AMG_EINVAL, "amg_setup_batched: need systems and params");
        const amg_params &p = *params;
        // every system saddle (n_pres > 0) or every system SPD
        const bool spd = systems[0].n_pres == 0;
        for (int i = 1; i < nsys; ++i)
            AMG_REQUIRE((systems[i].n_pres == 0) == spd, AMG_EINVAL,
                        "amg_setup_batched: SPD and saddle point systems in one batch");
        check_params(p, !spd);
        if (spd) {
            AMG_REQUIRE(p.smoother == AMG_SMOOTH_JA || p.smoother == AMG_SMOOTH_GS, AMG_EINVAL,
                        "amg_setup_batched: SPD batches run the JA or GS smoother");
            AMG_REQUIRE(p.krylov == AMG_KRYLOV_PCG || p.krylov == AMG_KRYLOV_FCG, AMG_EINVAL,
                        "amg_setup_batched: SPD batches run PCG or FCG");
            AMG_REQUIRE(p.gs_post != 2, AMG_EINVAL, "amg_setup_batched: CG needs the symmetric cycle");
        } else {
            AMG_REQUIRE(p.krylov == AMG_KRYLOV_FGMRES, AMG_EINVAL, "amg_setup_batched: saddle batches run FGMRES");
            AMG_REQUIRE(p.smoother != AMG_SMOOTH_VANKA, AMG_EUNSUPPORTED,
                        "amg_setup_batched: batches run the sGS or Braess-Sarazin smoother");
        }
        AMG_REQUIRE(!p.omega_model, AMG_EINVAL, "amg_setup_batched: omega_model is for single SPD systems");
        std::vector<StagedSystem> staged;
        std::vector<amg_system> host_sys(systems, systems + nsys);
        for (int i = 0; i < nsys; ++i) {
            AMG_REQUIRE(systems[i].memory == AMG_MEM_HOST || systems[i].memory == AMG_MEM_DEVICE, AMG_EINVAL,
                        "amg_setup_batched: memory must be AMG_MEM_HOST or AMG_MEM_DEVICE");
            if (systems[i].memory == AMG_MEM_DEVICE) {
                if (staged.empty()) staged.resize(nsys);
                stage_system(systems[i], static_cast<hipStream_t>(stream), staged[i]);
                host_sys[i] = staged[i].sys;
            }
        }
        auto *h = new amg_ctx();
        h->prm = p;
        h->prm.level_omega = nullptr;
        h->prm.n_level_omega = 0;
        h->stream = static_cast<hipStream_t>(stream);
        try {
            if (spd)
                build_batch_spd(h, nsys, host_sys.data());
            else
                build_batch(h, nsys, host_sys.data());
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return AMG_OK;
    });
}

int amg_solve_batched(amg_handle h, const double *b, double *x, double tol, int32_t maxit, amg_stream stream,
                      amg_result *results) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && b && x, AMG_EINVAL, "amg_solve_batched: null argument");
        AMG_REQUIRE(h->nsys > 0, AMG_EINVAL, "amg_solve_batched: handle is not a batch (use amg_solve)");
        AMG_REQUIRE(tol > 0.0 && maxit >= 0, AMG_EINVAL, "amg_solve_batched: tol must be > 0, maxit >= 0");
        h->stream = static_cast<hipStream_t>(stream);
        launch_seg_copy(b, h->b_b.p, h->b_in.view(), h->b_in.dst.p, h->stream);
        launch_seg_copy(x, h->b_x.p, h->b_in.view(), h->b_in.dst.p, h->stream);
        const int st = h->saddle ? solve_fgmres_batched(h, h->b_b.p, h->b_x.p, tol, maxit, results)
                                 : solve_pcg_batched(h, h->b_b.p, h->b_x.p, tol, maxit, results);
        launch_seg_copy(h->b_x.p, x, h->b_out.view(), h->b_out.dst.p, h->stream);
        AMG_HIP(hipStreamSynchronize(h->stream));
        return st;
    });
}

int amg_batch_offsets(amg_handle h, int64_t *u_offset, int64_t *p_offset) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && u_offset && p_offset, AMG_EINVAL, "amg_batch_offsets: null argument");
        AMG_REQUIRE(h->nsys > 0, AMG_EINVAL, "amg_batch_offsets: handle is not a batch");
        for (int j = 0; j < h->nsys; ++j) {
            u_offset[h->b_order[j]] = h->b_uoff[j];
            p_offset[h->b_order[j]] = h->b_poff[j];
        }
        return AMG_OK;
    });
}

int amg_solve(amg_handle h, const double *b, double *x, double tol, int32_t maxit, amg_stream stream,
              amg_result *res) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && b && x, AMG_EINVAL, "amg_solve: null argument");
        AMG_REQUIRE(h->nsys == 0, AMG_EINVAL, "amg_solve: batch handle (use amg_solve_batched)");
        AMG_REQUIRE(tol > 0.0 && maxit >= 0, AMG_EINVAL, "amg_solve: tol must be > 0, maxit >= 0");
        h->stream = static_cast<hipStream_t>(stream);
        auto run = [&](amg_result *r) -> int {
            switch (h->prm.krylov) {
                case AMG_KRYLOV_PCG: return solve_pcg(h, b, x, tol, maxit, r);
                case AMG_KRYLOV_FCG: return solve_fcg(h, b, x, tol, maxit, r);
                case AMG_KRYLOV_NONE:
                    return h->saddle ? solve_stationary_saddle(h, b, x, tol, maxit, r)
                                     : solve_stationary(h, b, x, tol, maxit, r);
                case AMG_KRYLOV_FGMRES: return solve_fgmres(h, b, x, tol, maxit, r);
                default: throw Error(AMG_EINVAL, "amg_solve: unknown Krylov method");
            }
        };
        if (!h->learned) return run(res);
        // learned damping: the FP64 residual judges the weights; a solve that
        // breaks down, diverges or misses the tolerance is repeated from the
        // same initial guess with the caller's fixed weights, which stay
        amg_result first{};
        if (h->x0_save.n != static_cast<size_t>(h->n_dof)) h->x0_save.alloc(h->n_dof);
        launch_copy(h->x0_save.p, x, h->n_dof, h->stream);
        const int st = run(&first);
        if (st == AMG_OK) {
            if (res) *res = first;
            return st;
        }
        h->level_omega = h->fixed_omega;
        h->learned = false;
        h->omega_fallbacks += 1;
        for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
        h->graphs.clear();
        setup_tail(h);
        refresh_tail_f32(h);
        launch_copy(x, h->x0_save.p, h->n_dof, h->stream);
        amg_result second{};
        const int st2 = run(&second);
        second.iters += first.iters;
        second.solve_ms += first.solve_ms;
        if (res) *res = second;
        return st2;
    });
}

int amg_solve_multi(amg_handle h, int32_t nrhs, const double *B, double *X, double tol, int32_t maxit,
                    amg_stream stream, amg_result *results) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && B && X, AMG_EINVAL, "amg_solve_multi: null argument");
        AMG_REQUIRE(tol > 0.0 && maxit >= 0, AMG_EINVAL, "amg_solve_multi: tol must be > 0, maxit >= 0");
        h->stream = static_cast<hipStream_t>(stream);
        return solve_multi(h, nrhs, B, X, tol, maxit, results);
    });
}

int amg_precondition(amg_handle h, const double *r, double *z, amg_stream stream) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && r && z, AMG_EINVAL, "amg_precondition: null argument");
        h->stream = static_cast<hipStream_t>(stream);
        precondition_any(h, r, z);
        AMG_HIP(hipStreamSynchronize(h->stream));
        profile_collect(h);
        return AMG_OK;
    });
}

int amg_apply(amg_handle h, int32_t level, const double *x, double *y, amg_stream stream) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && x && y, AMG_EINVAL, "amg_apply: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL, "amg_apply: bad level");
        h->stream = static_cast<hipStream_t>(stream);
        if (h->saddle)
            saddle_apply(h, level, x, y);
        else
            apply_level(h, level, x, y);
        AMG_HIP(hipStreamSynchronize(h->stream));
        profile_collect(h);
        return AMG_OK;
    });
}

int amg_smooth(amg_handle h, int32_t level, const double *b, double *x, int32_t forward, amg_stream stream) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && b && x, AMG_EINVAL, "amg_smooth: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()) - 1, AMG_EINVAL,
                    "amg_smooth: level has no smoother (coarsest or out of range)");
        h->stream = static_cast<hipStream_t>(stream);
        // one step: temporarily force a single pre/post step, in the
        // direction asked for (colours ascending or descending)
        amg_params save = h->prm;
        const bool save_post = h->post_forward;
        h->prm.pre = h->prm.post = 1;
        h->post_forward = false;
        try {
            if (h->saddle)
                saddle_smooth(h, level, b, x);
            else
                smooth(h, level, b, x, forward != 0, false, false);
        } catch (...) {
            h->prm = save;
            h->post_forward = save_post;
            throw;
        }
        h->prm = save;
        h->post_forward = save_post;
        AMG_HIP(hipStreamSynchronize(h->stream));
        profile_collect(h);
        return AMG_OK;
    });
}

int amg_num_levels(amg_handle h) { return h ? static_cast<int>(h->lv.size()) : AMG_EINVAL; }

int amg_get_level_info(amg_handle h, int32_t level, amg_level_info *info) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && info, AMG_EINVAL, "amg_get_level_info: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL, "bad level");
        const Level &L = h->lv[level];
        std::memset(info, 0, sizeof(*info));
        info->n_lin = L.n_lin;
        info->n_quad = L.n_quad;
        info->n_pres = L.n_pres;
        info->bs = L.mode;
        info->nnz_A = L.pattern_nnz_A();
        info->nnz_B = L.pattern_nnz_B();
        info->kept_A = L.A.nnz;
        info->kept_B = L.B.nnz;
        info->nnz_C = L.C.nnz;
        info->nnz_P = L.coarsest ? 0 : L.P.nnz;
        info->n_colors = L.cptr.empty() ? 0 : static_cast<int>(L.cptr.size()) - 1;
        info->is_coarsest = L.coarsest ? 1 : 0;
        info->lanes_A = h->mixed ? L.mp.G : L.G;
        info->lanes_gs = h->mixed ? L.mp.Gg : L.Gg;
        info->trip_A = h->mixed ? L.mp.trip : L.trip;
        info->trip_gs = h->mixed ? L.mp.tripg : L.tripg;
        info->lanes64_A = L.G;
        info->trip64_A = L.trip;
        const int fs = h->tail_start >= 0 ? h->tail_start
                       : h->dense_start >= 0 ? h->dense_start
                                             : h->saddle_tail_from;
        info->fused = (fs >= 0 && level >= fs) ? 1 : 0;
        info->schur_levels = static_cast<int>(L.schur.lv.size());
        info->omega = jacobi_omega(h, level);
        info->gs_xcd = h->mixed ? L.mp.xcd : L.gs_xcd;
        info->nnz_S = L.schur.lv.empty() ? 0 : L.schur.lv[0].S.nnz;
        info->coarse_map = (level == h->dense_start) || (level == h->saddle_tail_from) ? 1 : 0;
        info->learned = h->learned ? 1 : 0;
        info->omega_max = level < static_cast<int>(h->omega_cap.size()) ? h->omega_cap[level] : 0.0;
        info->omega_fallbacks = h->omega_fallbacks;
        return AMG_OK;
    });
}

int amg_get_level_matrix(amg_handle h, int32_t level, int32_t which, int32_t *rowptr, int32_t *col, double *val) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && rowptr && col && val, AMG_EINVAL, "amg_get_level_matrix: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL, "bad level");
        const Level &L = h->lv[level];
        const DMat *m = nullptr;
        if (which == 0) m = L.A_pat.nnz > 0 ? &L.A_pat : &L.A;
        if (which == 1 && L.B.nnz > 0) m = L.B_pat.nnz > 0 ? &L.B_pat : &L.B;
        if (which == 2 && L.C.nnz > 0) m = &L.C;
        if (which == 3) {
            AMG_REQUIRE(!L.coarsest, AMG_EINVAL, "coarsest level has no prolongation");
            m = &L.P;
        }
        if (which == 4 && !L.schur.lv.empty()) m = &L.schur.lv[0].S;
        AMG_REQUIRE(m != nullptr, AMG_EUNSUPPORTED, "amg_get_level_matrix: operator not present");
        std::vector<int> rp = m->rowptr.download(h->stream), c = m->col.download(h->stream);
        std::vector<double> v = m->val.download(h->stream);
        std::memcpy(rowptr, rp.data(), rp.size() * sizeof(int));
        std::memcpy(col, c.data(), static_cast<size_t>(m->nnz) * sizeof(int));
        for (int64_t k = 0; k < m->nnz; ++k)
            for (int p = 0; p < m->np; ++p) val[k * m->np + p] = v[static_cast<size_t>(p) * m->nnz + k];
        return AMG_OK;
    });
}

int amg_get_level_colors(amg_handle h, int32_t level, int32_t *colors) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && colors, AMG_EINVAL, "amg_get_level_colors: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL, "bad level");
        const Level &L = h->lv[level];
        AMG_REQUIRE(!L.colour.empty(), AMG_EUNSUPPORTED, "no colouring on this level");
        std::memcpy(colors, L.colour.data(), L.colour.size() * sizeof(int));
        return AMG_OK;
    });
}

int amg_profile_enable(amg_handle h, int32_t enable) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h, AMG_EINVAL, "amg_profile_enable: null handle");
        profile_collect(h);
        h->prof = enable != 0;
        h->prof_finest_only = enable == 2;
        if (h->prof) h->stats.clear();
        return AMG_OK;
    });
}

int amg_profile_read(amg_handle h, const char *cls, int64_t *launches, double *total_ms, double *bytes) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && cls && launches && total_ms && bytes, AMG_EINVAL, "amg_profile_read: null argument");
        profile_collect(h);
        auto it = h->stats.find(cls);
        if (it == h->stats.end()) it = h->setup_stats.find(cls);
        if (it == h->setup_stats.end()) {
            *launches = 0;
            *total_ms = 0.0;
            *bytes = 0.0;
        } else {
            *launches = it->second.launches;
            *total_ms = it->second.ms;
            *bytes = it->second.bytes;
        }
        return AMG_OK;
    });
}

void amg_destroy(amg_handle h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    delete h;
}

// ---------------------------------------------------------------- learned damping
int amg_mlp_create(const float *params, amg_stream stream, amg_mlp_handle *out) {
    return guarded([&]() -> int {
        AMG_REQUIRE(params && out, AMG_EINVAL, "amg_mlp_create: null argument");
        *out = nullptr;
        auto *m = new amg_mlp();
        try {
            m->stream = static_cast<hipStream_t>(stream);
            m->theta.upload(params, MLP_NP, m->stream);
            m->m.alloc(MLP_NP);
            m->v.alloc(MLP_NP);
            m->m.zero(m->stream);
            m->v.zero(m->stream);
            m->grad.alloc(MLP_NP);
            m->loss.alloc(1);
            AMG_HIP(hipStreamSynchronize(m->stream));
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
        return AMG_OK;
    });
}

int amg_mlp_get_params(amg_mlp_handle m, float *params) {
    return guarded([&]() -> int {
        AMG_REQUIRE(m && params, AMG_EINVAL, "amg_mlp_get_params: null argument");
        AMG_HIP(hipMemcpyAsync(params, m->theta.p, MLP_NP * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        AMG_HIP(hipStreamSynchronize(m->stream));
        return AMG_OK;
    });
}

static void mlp_upload(amg_mlp *m, const float *X, const float *y, int n) {
    AMG_REQUIRE(X && n >= 1, AMG_EINVAL, "amg_mlp: need at least one feature row");
    m->w.reserve(n);
    AMG_HIP(hipMemcpyAsync(m->w.X.p, X, static_cast<size_t>(n) * MLP_NF * sizeof(float), hipMemcpyHostToDevice,
                           m->stream));
    if (y) AMG_HIP(hipMemcpyAsync(m->w.y.p, y, static_cast<size_t>(n) * sizeof(float), hipMemcpyHostToDevice, m->stream));
    AMG_HIP(hipStreamSynchronize(m->stream));  // the caller may free X and y on return
}

int amg_mlp_forward(amg_mlp_handle m, const float *X, int32_t n, float *omega) {
    return guarded([&]() -> int {
        AMG_REQUIRE(m && omega, AMG_EINVAL, "amg_mlp_forward: null argument");
        mlp_upload(m, X, nullptr, n);
        mlp_forward(m->theta.p, m->w.X.p, n, m->w, m->stream);
        AMG_HIP(hipMemcpyAsync(omega, m->w.om.p, n * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        AMG_HIP(hipStreamSynchronize(m->stream));
        return AMG_OK;
    });
}

int amg_mlp_gradient(amg_mlp_handle m, const float *X, const float *y, int32_t n, float *loss, float *grad) {
    return guarded([&]() -> int {
        AMG_REQUIRE(m && y && loss && grad, AMG_EINVAL, "amg_mlp_gradient: null argument");
        mlp_upload(m, X, y, n);
        mlp_forward(m->theta.p, m->w.X.p, n, m->w, m->stream);
        mlp_backward(m->theta.p, n, m->w, m->grad.p, m->loss.p, m->stream);
        AMG_HIP(hipMemcpyAsync(grad, m->grad.p, MLP_NP * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        AMG_HIP(hipMemcpyAsync(loss, m->loss.p, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        AMG_HIP(hipStreamSynchronize(m->stream));
        return AMG_OK;
    });
}

int amg_mlp_train(amg_mlp_handle m, const float *X, const float *y, int32_t n, int32_t steps, float lr,
                  float *loss_history) {
    return guarded([&]() -> int {
        AMG_REQUIRE(m && y, AMG_EINVAL, "amg_mlp_train: null argument");
        AMG_REQUIRE(steps >= 0 && lr > 0.0f, AMG_EINVAL, "amg_mlp_train: steps >= 0 and lr > 0 required");
        mlp_upload(m, X, y, n);
        DevBuf<float> hist(std::max(1, steps));
        const double b1 = 0.9, b2 = 0.999;
        for (int k = 0; k < steps; ++k) {
            const int t = ++m->t;
            mlp_forward(m->theta.p, m->w.X.p, n, m->w, m->stream);
            mlp_backward(m->theta.p, n, m->w, m->grad.p, hist.p + k, m->stream);
            mlp_adam(m->theta.p, m->grad.p, m->m.p, m->v.p, lr, static_cast<float>(b1), static_cast<float>(b2),
                     static_cast<float>(1.0 - std::pow(b1, t)), static_cast<float>(1.0 - std::pow(b2, t)), 1e-8f,
                     m->stream);
        }
        if (loss_history && steps > 0)
            AMG_HIP(hipMemcpyAsync(loss_history, hist.p, steps * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        AMG_HIP(hipStreamSynchronize(m->stream));
        return AMG_OK;
    });
}

void amg_mlp_destroy(amg_mlp_handle m) {
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    delete m;
}

int amg_set_launch_shape(amg_handle h, int32_t level, int32_t kernels, int32_t lanes, int32_t trip, int32_t xcd) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h != nullptr, AMG_EINVAL, "amg_set_launch_shape: null handle");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL,
                    "amg_set_launch_shape: bad level");
        AMG_REQUIRE(lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32 || lanes == 64, AMG_EINVAL,
                    "amg_set_launch_shape: lanes must be 4, 8, 16, 32 or 64");
        AMG_REQUIRE(trip == 1 || trip == 2 || trip == 4, AMG_EINVAL, "amg_set_launch_shape: trip must be 1, 2 or 4");
        AMG_REQUIRE(xcd == 0 || xcd == 1, AMG_EINVAL, "amg_set_launch_shape: xcd is 0 or 1");
        Level &L = h->lv[level];
        const bool sweep = kernels == AMG_SHAPE_SWEEP || kernels == AMG_SHAPE_SWEEP_RP;
        AMG_REQUIRE(sweep || xcd == 0, AMG_EINVAL, "amg_set_launch_shape: xcd applies to colour sweeps only");
        switch (kernels) {
            case AMG_SHAPE_NATURAL: L.G = lanes; L.trip = trip; break;
            case AMG_SHAPE_SWEEP: L.Gg = lanes; L.tripg = trip; L.gs_xcd = xcd; break;
            case AMG_SHAPE_NATURAL_RP:
            case AMG_SHAPE_SWEEP_RP:
                AMG_REQUIRE(h->mixed, AMG_EINVAL, "amg_set_launch_shape: no reduced-precision copy (FP64 hierarchy)");
                if (kernels == AMG_SHAPE_NATURAL_RP) {
                    L.mp.G = lanes;
                    L.mp.trip = trip;
                } else {
                    L.mp.Gg = lanes;
                    L.mp.tripg = trip;
                    L.mp.xcd = xcd;
                }
                break;
            case AMG_SHAPE_VANKA:
                AMG_REQUIRE(h->saddle && h->prm.smoother == AMG_SMOOTH_VANKA && !L.vanka.cptr.empty(), AMG_EINVAL,
                            "amg_set_launch_shape: no Vanka sweep on this level");
                AMG_REQUIRE(lanes >= 16 && (trip == 1 || trip == 2) && xcd == 0, AMG_EINVAL,
                            "amg_set_launch_shape: the Vanka residual takes 16, 32 or 64 lanes, trip 1 or 2, xcd 0");
                L.vanka.path = trip == 1 ? 2 : 3;
                L.vanka.rg = lanes;
                break;
            case AMG_SHAPE_VANKA_APPLY:
                AMG_REQUIRE(h->saddle && h->prm.smoother == AMG_SMOOTH_VANKA && !L.vanka.cptr.empty(), AMG_EINVAL,
                            "amg_set_launch_shape: no Vanka sweep on this level");
                AMG_REQUIRE(lanes >= 4 && lanes <= 16 && trip == 1 && xcd == 0, AMG_EINVAL,
                            "amg_set_launch_shape: 4, 8 or 16 wavefronts per Vanka correction tile, trip 1, xcd 0");
                L.vanka.path = 3;
                L.vanka.aw = lanes;
                break;
            default: throw Error(AMG_EINVAL, "amg_set_launch_shape: unknown kernel class");
        }
        for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
        h->graphs.clear();
        return AMG_OK;
    });
}

int amg_set_level_omega(amg_handle h, int32_t n, const double *omega) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && omega && n >= 1, AMG_EINVAL, "amg_set_level_omega: null argument or n < 1");
        AMG_REQUIRE(!h->saddle && h->prm.smoother == AMG_SMOOTH_JA, AMG_EINVAL,
                    "amg_set_level_omega: needs the JA smoother on an SPD system");
        for (int i = 0; i < n; ++i)
            AMG_REQUIRE(std::isfinite(omega[i]), AMG_EINVAL, "amg_set_level_omega: weight not finite");
        h->level_omega.assign(omega, omega + n);
        h->learned = false;  // the caller's weights from now on
        // recorded preconditioners hold the old weights
        for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
        h->graphs.clear();
        setup_tail(h);
        refresh_tail_f32(h);
        return AMG_OK;
    });
}

int amg_level_features(amg_handle h, int32_t level, double *features) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && features, AMG_EINVAL, "amg_level_features: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL, "bad level");
        const Level &L = h->lv[level];
        const DMat &A = L.A_pat.nnz > 0 ? L.A_pat : L.A;  // features are defined on the structural rows
        row_features(L.mode, L.n, A.rowptr.p, A.col.p, A.val.p, A.nnz, level, features, h->stream);
        return AMG_OK;
    });
}

int amg_level_features_noalloc(amg_handle h, int32_t level, double *features_dev, amg_stream stream) {
    return guarded([&]() -> int {
        AMG_REQUIRE(h && features_dev, AMG_EINVAL, "amg_level_features_noalloc: null argument");
        AMG_REQUIRE(level >= 0 && level < static_cast<int>(h->lv.size()), AMG_EINVAL, "bad level");
        const Level &L = h->lv[level];
        const DMat &A = L.A_pat.nnz > 0 ? L.A_pat : L.A;
        row_features_noalloc(L.mode, L.n, A.rowptr.p, A.col.p, A.val.p, A.nnz, level, features_scratch_address(),
                             features_dev, static_cast<hipStream_t>(stream));
        return AMG_OK;
    });
}

const char *amg_status_string(int status) {
    switch (status) {
        case AMG_OK: return "converged";
        case AMG_NOT_CONVERGED: return "not converged within maxit";
        case AMG_BREAKDOWN: return "Krylov breakdown";
        case AMG_DIVERGED: return "diverged (NaN/Inf or residual growth)";
        case AMG_EINVAL: return "invalid argument";
        case AMG_EHIP: return "HIP runtime error";
        case AMG_ENOMEM: return "out of memory";
        case AMG_EUNSUPPORTED: return "unsupported input or option";
        default: return "unknown status";
    }
}

const char *amg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
