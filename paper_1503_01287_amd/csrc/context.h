// The hierarchy held by an amg_handle and the routines that build and run it.
#pragma once

#include <chrono>
#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "host_setup.h"
#include "batch.h"
#include "kernels.h"
#include "learn.h"
#include "mixed.h"
#include "saddle.h"
#include "tail.h"
#include "vanka.h"

namespace amgp2 {

// Block-CSR operator on the device, values stored as planes (see kernels.h).
struct DMat {
    int nrows = 0, ncols = 0;
    int64_t nnz = 0;
    int np = 1;  // planes per entry: 9 (3x3), 3 (1x3 / 3x1), 1 (scalar)
    DevBuf<int> rowptr, col;
    DevBuf<double> val;
};

// Reduced-precision copy of a level for the mixed-precision cycle.
struct LevelMP {
    int kind = VAL_F32;            // value kind of A and its grouped copy
    int G = 16, Gg = 16;           // lanes per row of the reduced-precision A / grouped-A kernels
    int trip = 1, tripg = 1;       // their entries per lane and loop trip (1, 2, 4), chosen by the tuner
    int xcd = 0;                   // per-XCD contiguous rows in the colour sweeps (as Level::gs_xcd)
    DevBuf<float> a32, ag32;       // FP32 planes
    DevBuf<uint16_t> a16, ag16;    // BF16 planes (values / row scale)
    DevBuf<float> scale;           // BF16: scale of every scalar row
    DevBuf<float> dinv;            // FP32 inverted diagonal blocks
    DevBuf<float> pval, rval;      // FP32 transfer weights
    DevBuf<float> x, b, r, t;      // FP32 work vectors
    // saddle levels: FP32 planes of B, B^T, C, H, H^T and the smoothers' scalings
    DevBuf<float> sB, sBt, sC, sH, sHt, sgs, ahat;
    const void *aval() const { return kind == VAL_F32 ? static_cast<const void *>(a32.p) : a16.p; }
    const void *agval() const { return kind == VAL_F32 ? static_cast<const void *>(ag32.p) : ag16.p; }
    int vbytes() const { return kind == VAL_F32 ? 4 : 2; }
};

// Explicit inverses of the systems that end on a level: the coarsest level of
// one hierarchy, or, in a batch, every instance whose own hierarchy ends on
// this level (see DenseSegView).
struct DenseSegs {
    int count = 0, rows = 0;
    std::vector<int> h_m, h_uoff, h_nu, h_poff;
    std::vector<int64_t> h_moff;
    DevBuf<int64_t> moff;
    DevBuf<int> rstart, uoff, nu, poff;
    DevBuf<double> inv;
    DevBuf<float> inv32;  // FP32 copy for FP32 cycles (assembled maps only)
    double bytes = 0.0;  // matrix bytes read per application
    void add(int m, int uoff_, int nu_, int poff_) {
        h_moff.push_back(h_moff.empty() ? 0 : h_moff.back() + static_cast<int64_t>(h_m.back()) * h_m.back());
        h_m.push_back(m);
        h_uoff.push_back(uoff_);
        h_nu.push_back(nu_);
        h_poff.push_back(poff_);
    }
    void finalize(hipStream_t s);  // upload the tables, allocate inv
    void make_f32(hipStream_t s);  // inv32 from inv (FP32 cycles then read it)
    DenseSegView view() const {
        DenseSegView v;
        v.count = count;
        v.rows = rows;
        v.moff = moff.p;
        v.rstart = rstart.p;
        v.uoff = uoff.p;
        v.nu = nu.p;
        v.poff = poff.p;
        v.inv = inv.p;
        v.inv32 = inv32.n ? inv32.p : nullptr;
        return v;
    }
};

// One level of the scalar hierarchy of a Braess-Sarazin Schur complement
// S = C + B A_hat^{-1} B^T (natural row order, rows grouped by colour
// through `rowid`).
struct SchurLevel {
    DMat S;
    int nA = 0;                  // leading rows that are smoothed (the rest: dseg)
    DenseSegs dseg;
    std::vector<int> blk_off, blk_rows;  // the systems' row ranges (one block outside batches)
    DevBuf<double> dinv;         // 1 / S_ii
    std::vector<int> cptr;       // rows of colour c: rowid[cptr[c] .. cptr[c+1])
    DevBuf<int> rowid;
    DMat Sg;                     // the smoothed rows of S in the order rowid (colour sweeps)
    DevBuf<double> x, b, r;
    DevBuf<float> s32, sg32, dinv32, x32, b32, r32;  // reduced-precision cycle
    int G = 8;
};

// Scalar AMG for S_l: S_l, H_l^T S_l H_l, ... down to the saddle coarsest
// level, whose Schur matrix is inverted densely.
struct SchurHier {
    std::vector<SchurLevel> lv;
    DevBuf<double> inv;
    int m = 0;
    // the cycle from Schur level dense_from down, assembled per system as an
    // explicit operator (one GEMV instead of the colour sweeps); -1: none
    int dense_from = -1;
    DenseSegs tdense;
};

// Multiplicative Vanka data of a saddle level: patch node lists, the patches
// ordered by colour (rows order[cptr[c] .. cptr[c+1]) of colour c) and the
// patches' inverted local matrices.
struct VankaData {
    int npatch = 0, max_nodes = 0;
    double inv_bytes = 0.0;        // the patch inverses, read once per sweep
    DevBuf<int> pptr, pnode, order;
    DevBuf<int64_t> moff;
    DevBuf<double> inv;
    std::vector<int> cptr;
    // sweep form (chosen at setup): 0 one kernel per colour; 1 residuals,
    // then corrections over 64-row tiles; 2 residuals spread over rows,
    // partial corrections over 64-row x cc-column tiles, then their sum;
    // 3 residuals spread over rows, then corrections over 64-row tiles
    int path = 0;
    DevBuf<int64_t> roff;          // residual buffer offsets (paths 1, 2, 3)
    DevBuf<double> rbuf;
    DevBuf<int> tpre;              // per-colour prefix of the 64-row tiles
    std::vector<int> ntiles;       // 64-row tiles per colour
    int cc = 256;                  // path 2: columns per chunk
    DevBuf<int> upre;              // path 2: per-colour prefix of the 2-D tiles
    std::vector<int> nunits;       // path 2: 2-D tiles per colour
    DevBuf<int64_t> poff;          // path 2: partial buffer offsets
    DevBuf<double> pbuf;
    int rg = 16;                   // paths 2, 3: lanes per residual row (16, 32 or 64)
    int aw = 4;                    // path 3: wavefronts per 64-row correction tile (4, 8 or 16)
    // paths 2 and 3, for rg = 16, 32, 64 (index rg_index): per-colour prefix of the
    // residual's units (256 / rg node rows each) and units per colour
    DevBuf<int> rpre[3];
    std::vector<int> nrunits[3];
    static int rg_index(int rg) { return rg == 16 ? 0 : (rg == 32 ? 1 : 2); }
};

struct Level {
    int n_lin = 0, n_quad = 0, n = 0, n_pres = 0;
    int mode = 3;             // 3: 3x3 blocks; 1: scalar operator applied per component
    bool coarsest = false;
    DMat A;                   // natural node order
    HostCSR hpat;             // structural pattern of A (host)
    // smoother data
    DevBuf<double> dinv;      // inverted diagonal blocks, planes of stride n
    std::vector<int> colour;  // per node
    std::vector<int> cptr;    // grouped rows of colour c: [cptr[c], cptr[c+1])
    std::vector<int64_t> colour_nnz;  // stored entries in the rows of colour c
    DMat Ag;                  // rows of A grouped by colour
    DevBuf<int> g_rowid;      // node of grouped row g
    DevBuf<int> d_cptr;       // cptr on the device (tail kernel)
    // transfer between this level and the next coarser one
    DMat P, R;                // P: n x n_c scalar, R = P^T
    HostCSR hP;
    // work vectors (3n doubles each)
    DevBuf<double> x, b, r, t;
    int G = 16, Gg = 16, Gp = 4, Gr = 8;  // lanes per row: A, grouped A, P, R
    int gs_xcd = 0;           // colour sweeps with one contiguous eighth of the rows per XCD
    int trip = 1, tripg = 1;  // entries per lane and loop trip, 1, 2 or 4 (natural-order / colour kernels)
    LevelMP mp;               // mixed-precision copy (AMG_PREC_MIXED / FP32)
    // saddle point levels (n_pres > 0); vectors are [u (3n); p (n_pres)]
    DMat B, Bt, C;            // B: n_pres x n (1x3), Bt: n x n_pres (3x1), C: n_pres^2 (may be empty)
    // structural A and B where their numerically zero blocks were dropped
    // from A and B after setup (empty otherwise): export and row features;
    // a merged batch level keeps only the members' structural counts
    DMat A_pat, B_pat;
    int64_t nnz_pat_A = 0, nnz_pat_B = 0;
    int64_t pattern_nnz_A() const { return A_pat.nnz > 0 ? A_pat.nnz : nnz_pat_A > 0 ? nnz_pat_A : A.nnz; }
    int64_t pattern_nnz_B() const { return B_pat.nnz > 0 ? B_pat.nnz : nnz_pat_B > 0 ? nnz_pat_B : B.nnz; }
    DMat H, Ht;               // pressure prolongation to this level and its transpose
    DevBuf<double> sgs_scale; // sGS: 1 / diag(B M_A^{-1} B^T + C)
    DevBuf<double> bs_ahat;   // BS: 1 / (2 a_ii) per velocity unknown
    // leading velocity nodes / pressure nodes that are smoothed and coarsened
    // (all of them except on a coarsest level; in a batch, the instances
    // whose hierarchy continues below); the others are solved by dseg
    int nA = 0, npA = 0;
    DenseSegs dseg;
    // the systems on this level (one outside batches), in vector order:
    // first node, nodes, first pressure, pressures
    std::vector<int> sys_noff, sys_n, sys_poff, sys_np;
    SchurHier schur;          // BS: scalar hierarchy of this level's Schur complement
    VankaData vanka;          // multiplicative Vanka patches
    int Gb = 16, Gbt = 16, Gh = 4, Ght = 8;
    int64_t vlen() const { return 3 * static_cast<int64_t>(n) + n_pres; }
};

// Chunk table of a batch vector (see ChunkView); dst: second start per chunk
// for copies between layouts.
struct ChunkTable {
    int n = 0;
    DevBuf<int64_t> start, dst;
    DevBuf<int> len, seg;
    void build(const std::vector<int64_t> &st, const std::vector<int> &ln, const std::vector<int> &sg,
               const std::vector<int64_t> &ds, hipStream_t s) {
        n = static_cast<int>(st.size());
        start.upload(st, s);
        len.upload(ln, s);
        seg.upload(sg, s);
        if (!ds.empty()) dst.upload(ds, s);
    }
    ChunkView view() const {
        ChunkView v;
        v.n = n;
        v.start = start.p;
        v.len = len.p;
        v.seg = seg.p;
        return v;
    }
};

// Work of amg_solve_multi (blocks of K right-hand sides), kept between calls
// with the same K: per-level block vectors (FP64 or FP32 cycle), the outer
// Krylov blocks, dot partials and pinned slots for per-column coefficients.
struct MultiLevelWork {
    DevBuf<double> x, b, r, t;
    DevBuf<float> x32, b32, r32, t32;
};

struct MultiWork {
    static constexpr int SLOTS = 16;
    int K = 0;
    std::vector<MultiLevelWork> lv;
    DevBuf<double> B, X, R, Z, P, Q, partial, dots, coef;
    double *h_coef = nullptr, *h_dots = nullptr;
    int used = 0;
    MultiWork() = default;
    MultiWork(const MultiWork &) = delete;
    MultiWork &operator=(const MultiWork &) = delete;
    ~MultiWork() {
        if (h_coef) (void)hipHostFree(h_coef);
        if (h_dots) (void)hipHostFree(h_dots);
    }
};

struct ProfStat {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
};

struct amg_ctx_impl;

}  // namespace amgp2

struct amg_ctx {
    amg_params prm{};
    std::vector<double> level_omega;
    // learned damping: the network's weights are in use (set at setup); the
    // caller's fixed weights they replaced (fallback), and each level's
    // bound OMEGA_CAP_FACTOR * 2 / lambda_max(D^{-1} A_l) (JA hierarchies)
    // the learned weights are kept under
    bool learned = false;
    std::vector<double> fixed_omega;
    std::vector<double> omega_cap;
    int omega_fallbacks = 0;       // solves that fell back to the fixed weights
    amgp2::DevBuf<double> x0_save; // initial guess of a learned-weight solve
    hipStream_t stream = nullptr;
    std::vector<amgp2::Level> lv;
    // coarsest level: explicit dense inverse
    amgp2::DevBuf<double> coarse_inv;
    int coarse_m = 0, coarse_nc = 1;
    // single-workgroup tail: levels tail_start.. run in one kernel (-1: none)
    int tail_start = -1;
    amgp2::TailArgs tail_args;
    amgp2::DevBuf<amgp2::TailLevel> tail_levels;
    int tail_lds = 0;
    double tail_bytes = 0.0;
    // the V-cycle from level dense_start (>= 1) down, as an explicit
    // operator x = T b (tail_m x tail_m, applied to tail_nc components)
    int dense_start = -1;
    amgp2::DevBuf<double> tail_dense;
    int tail_m = 0, tail_nc = 1;
    // post-smoothing Gauss-Seidel sweeps forward (the stand-alone form, see
    // amg_params::gs_post) instead of backward (the symmetric cycle)
    bool post_forward = false;
    // reduced-precision cycle (precision != AMG_PREC_FP64)
    bool mixed = false;
    amgp2::DevBuf<float> tail_dense32;     // FP32 cycles
    amgp2::DevBuf<uint16_t> tail_dense16;  // FP32/BF16 cycles (coarse levels in BF16)
    int tail_ld = 0;                       // row stride of those copies (multiple of 8, zeros past tail_m)
    // setup-time tuners: a buffer larger than the 256 MB Infinity Cache,
    // written before every timed repetition (released after setup)
    amgp2::DevBuf<double> tune_flush;
    // saddle point system
    bool saddle = false;
    // the saddle V-cycle from level saddle_tail_from (>= 1) down, entered
    // from a zero guess, as one explicit map per system (-1: none)
    int saddle_tail_from = -1;
    amgp2::DenseSegs saddle_tail;
    int pinned = -1;                  // coarsest unknown pinned to zero (pressure kernel), -1 none
    // flexible GMRES workspace: V ((m+1) x n), Z (m x n), device scalars
    amgp2::DevBuf<double> gm_V, gm_Z, gm_h, gm_y, gm_part;
    int gm_m = 0;
    // pinned host copies of an FGMRES step's dots (asynchronous copies, so
    // that the next step's preconditioner can be enqueued before the wait)
    double *gm_hpin = nullptr;
    size_t gm_hpin_n = 0;
    // batch of independent saddle systems merged level by level (nsys > 0):
    // merged position q holds caller system b_order[q]; systems are ordered
    // by decreasing depth so that those still coarsening on a level lead it
    int nsys = 0;
    bool batch_member = false;  // a system's own hierarchy, built to be merged into a batch
    std::vector<int> b_order;
    std::vector<int64_t> b_uoff, b_poff, b_nu, b_np;  // per merged position, level-0 vector
    amgp2::ChunkTable b_chunks;                       // level-0 vector, by system
    amgp2::DevBuf<int> b_c0, b_c1, b_c2, b_c3;        // chunk runs of each system
    amgp2::ChunkTable b_in, b_out;                    // caller layout <-> merged layout
    amgp2::DevBuf<double> b_b, b_x;                   // merged-layout right-hand side / iterate
    // recorded preconditioner applications (HIP graphs) and staging vectors
    struct GraphEntry {
        const double *r;
        double *z;
        bool filled;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    amgp2::DevBuf<double> g_in, g_out;
    // Krylov workspace
    amgp2::DevBuf<double> kr, kz, kp, kq, kw;
    amgp2::MultiWork multi;  // amg_solve_multi
    amgp2::DevBuf<double> partial, sc;
    double *h_sc = nullptr;  // pinned host copy of the scalars
    hipEvent_t sc_ready = nullptr;  // that copy has landed (overlapped stopping tests)
    int n_dof = 0;           // length of a solve vector
    // profiling
    bool prof = false;
    bool prof_finest_only = false;
    struct Pending {
        std::string cls;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    std::map<std::string, amgp2::ProfStat> stats;
    // setup phases (always recorded, never cleared): "setup.<phase>" with
    // host wall time per phase; the Galerkin numeric kernels also with their
    // HIP-event time and algorithmic bytes ("setup.spgemm_numeric")
    std::map<std::string, amgp2::ProfStat> setup_stats;
    ~amg_ctx();
};

namespace amgp2 {

void build_hierarchy(amg_ctx *h, const amg_system *sys);
void build_mixed(amg_ctx *h);
void build_saddle_mp(amg_ctx *h);
void precondition_mp(amg_ctx *h, const double *r, double *z);
// saddle point path
void saddle_setup_level(amg_ctx *h, Level &L);
void setup_schur(amg_ctx *h, int l);
void setup_vanka(amg_ctx *h, int l);
void setup_schur_dense(amg_ctx *h, int l);
void setup_saddle_tail(amg_ctx *h);
VankaView vanka_view(Level &L);
// JA damping per level from the network of prm.omega_model (fallback: prm.omega)
void predict_level_omega(amg_ctx *h);
// every JA level's bound OMEGA_CAP_FACTOR * 2 / lambda_max(D^{-1} A_l), and
// learned weights lowered to it: a symmetric V-cycle with damped block Jacobi
// is positive definite only for weights below 2 / lambda_max; the estimate
// (a Rayleigh quotient after 100 power iterations) approaches lambda_max from
// below, hence the margin
constexpr double OMEGA_CAP_FACTOR = 0.95;
void cap_learned_omega(amg_ctx *h);
// estimate of lambda_max(D^{-1} A_l) by power iteration (FP64, on the device)
double lambda_max_dinv_a(amg_ctx *h, Level &L);
double jacobi_omega(const amg_ctx *h, int l);
// (re)build the fused coarse end of the SPD V-cycle from the current weights
void setup_tail(amg_ctx *h);
// lanes per row for a row kernel from the mean entries per row (4..64)
int lanes_for(int64_t nnz, int nrows);
// setup-time tuner of a level's FP64 kernels (lanes, loop form, XCD placement)
// natural_only: the natural-order kernels only (not the colour sweeps)
void autotune_level(amg_ctx *h, Level &L, bool natural_only = false);
// first level covered by the SPD hierarchy's assembled coarse end, or -1
int dense_tail_level(const amg_ctx *h);
// evict the GPU caches before a tuner's timed run: inside a cycle a level's
// operator is read after the finer levels' passes have replaced it in the
// caches, so the tuners time kernels on cold data
void evict_caches(amg_ctx *h);
// q.Sg from q.S, q.rowid and q.cptr
void group_schur_rows(SchurLevel &q, hipStream_t s);
// FP32 copy of the assembled coarse-end operator (reduced-precision cycle)
void refresh_tail_f32(amg_ctx *h);
void saddle_precondition(amg_ctx *h, const double *r, double *z);
void system_matvec(amg_ctx *h, const double *x, double *y);
void system_residual(amg_ctx *h, const double *b, const double *x, double *r);
int solve_fgmres(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
int solve_stationary_saddle(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
void precondition_any(amg_ctx *h, const double *r, double *z);
// Krylov loops enqueue the next preconditioner application ahead of the
// host's wait for an iteration's scalars while the last relative residual
// estimate is above KRYLOV_AHEAD * tol (several iterations from the
// tolerance at these convergence rates); the application only writes its
// output, so a solve that stops there loses nothing but its GPU time.
constexpr double KRYLOV_AHEAD = 50.0;
void precondition_staged(amg_ctx *h, const double *r, double *z);
// batches
void build_batch(amg_ctx *h, int nsys, const amg_system *sys);
// batches of SPD systems (every n_pres = 0): the merged FP64 hierarchy and
// its lockstep PCG
void build_batch_spd(amg_ctx *h, int nsys, const amg_system *sys);
int solve_pcg_batched(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
int solve_fgmres_batched(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
void saddle_apply(amg_ctx *h, int l, const double *x, double *y);
void saddle_smooth(amg_ctx *h, int l, const double *b, double *x);
void vcycle(amg_ctx *h, int l, const double *b, double *x);
void precondition(amg_ctx *h, const double *r, double *z);
void apply_level(amg_ctx *h, int l, const double *x, double *y);
void smooth(amg_ctx *h, int l, const double *b, double *x, bool pre, bool zero_init, bool filled);
int solve_pcg(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
int solve_fcg(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
int solve_stationary(amg_ctx *h, const double *b, double *x, double tol, int maxit, amg_result *res);
// K right-hand sides at once (SPD, PCG or FCG); B, X: nrhs vectors one after another
int solve_multi(amg_ctx *h, int nrhs, const double *B, double *X, double tol, int maxit, amg_result *res);
double true_relres(amg_ctx *h, const double *b, const double *x, double r0norm);

// Wall time of a setup phase (the stream synchronised at the end) added to
// h->setup_stats["setup." + name].
struct SetupPhase {
    amg_ctx *h;
    std::string name;
    std::chrono::steady_clock::time_point t0;
    SetupPhase(amg_ctx *hh, const char *n) : h(hh), name(std::string("setup.") + n), t0(std::chrono::steady_clock::now()) {}
    ~SetupPhase() {
        (void)hipStreamSynchronize(h->stream);
        ProfStat &st = h->setup_stats[name];
        st.launches += 1;
        st.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

// profiling helpers (no-ops unless enabled)
struct ProfScope {
    amg_ctx *h;
    size_t idx;
    ProfScope(amg_ctx *h, const std::string &cls, double bytes);
    ~ProfScope();
};
void profile_collect(amg_ctx *h);

}  // namespace amgp2
