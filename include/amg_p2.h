/*
 * amg_p2.h -- C ABI of the MI355X (gfx950) algebraic multigrid library for
 * hierarchical quadratic finite element systems.
 *
 * Method: H. Yang, "An algebraic multigrid method for quadratic finite element
 * equations of elliptic and saddle point systems in 3D", arXiv:1503.01287.
 *
 *   amg_setup  builds the multigrid hierarchy of Section 3.2: separate
 *              coarse/fine splits of the linear-node graph (pattern of K_ll)
 *              and the quadratic-node graph (pattern of K_qq), block-diagonal
 *              prolongation P = diag(I, J) (saddle: diag(I, J, H)) and
 *              Galerkin coarse operators P^T K_l P computed on the GPU.
 *   amg_solve  runs the AMG-preconditioned Krylov method of Sections 3.1 and
 *              4: Algorithm 1 (the basic AMG iteration, V-cycle for nu = 1)
 *              as the preconditioner of CG (SPD systems, equation for A u = f
 *              in Section 2.4) or of flexible GMRES (saddle point systems
 *              [[A, B^T], [B, -C]] [u; p] = [f; g], Section 2.4).
 *
 * Conventions for every entry point
 *  - Status: 0 on success, > 0 a solver outcome (AMG_NOT_CONVERGED, ...),
 *    < 0 an error (invalid argument, HIP failure, out of memory, unsupported
 *    input). amg_last_error() returns a text for the last error of the
 *    calling thread. No entry point aborts the process.
 *  - Index type: int32 (row pointers, column indices).
 *  - Node vectors: every velocity/displacement node carries 3 components,
 *    stored interleaved (x[3*i + c]); pressure vectors carry one value per
 *    pressure node; a saddle vector is [u (3*N values); p (Np values)].
 *  - Node order: linear nodes (mesh vertices) first, then quadratic nodes
 *    (mesh edges), as in the DOF vector [u_l; u_q] of Section 2.4.
 *  - Streams: a stream argument is a hipStream_t (NULL = legacy default
 *    stream). All device work is ordered on it; the call returns after the
 *    work it needs on the host is complete (see each call).
 *  - Ownership: the library copies whatever it keeps; it never retains a
 *    caller pointer after a call returns. Handles are freed by amg_destroy.
 *  - Threading: a handle may be used by one host thread at a time.
 */
#ifndef AMG_P2_H
#define AMG_P2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amg_ctx *amg_handle;
typedef struct amg_mlp *amg_mlp_handle; /* damping-weight network */
typedef void *amg_stream; /* hipStream_t */

/* ---- status codes ---------------------------------------------------- */
#define AMG_OK 0
#define AMG_NOT_CONVERGED 1 /* maxit reached before tol */
#define AMG_BREAKDOWN 2     /* Krylov breakdown (e.g. <p, A p> <= 0 in CG) */
#define AMG_DIVERGED 3      /* NaN/Inf or relative residual above 1e3 */
#define AMG_EINVAL (-1)
#define AMG_EHIP (-2)
#define AMG_ENOMEM (-3)
#define AMG_EUNSUPPORTED (-4)

/* ---- smoothers (Section 3.3) ----------------------------------------- */
#define AMG_SMOOTH_JA 0  /* damped block Jacobi ("JA-m-m-omega")            */
#define AMG_SMOOTH_GS 1  /* block Gauss-Seidel by colours ("GS-m-m")        */
#define AMG_SMOOTH_SGS 2 /* segregated Gauss-Seidel / Uzawa ("sGS-m-m")     */
#define AMG_SMOOTH_BS 3  /* Braess-Sarazin ("Braess-Sarazin-m-m")           */
#define AMG_SMOOTH_VANKA 4 /* multiplicative Vanka ("Vanka-m-m"), FP64, not
                              in batches: one patch per pressure DOF with the
                              velocity nodes of its row of B; local saddle
                              matrices inverted at setup; patches processed
                              colour by colour                                */

/* ---- outer iterations ------------------------------------------------ */
#define AMG_KRYLOV_PCG 0    /* preconditioned CG, FP64 (SPD)                 */
#define AMG_KRYLOV_FCG 1    /* flexible CG (one-term), FP64 outer loop (SPD) */
#define AMG_KRYLOV_FGMRES 2 /* right-preconditioned flexible GMRES(m)        */
#define AMG_KRYLOV_NONE 3   /* stand-alone AMG: repeated Algorithm 1         */

/* ---- arithmetic of the preconditioner -------------------------------- */
#define AMG_PREC_FP64 0  /* every level in FP64                               */
#define AMG_PREC_MIXED 1 /* FP32 cycle vectors, FP32 finest operator, BF16
                            coarse operators with per-row FP32 scales; outer
                            Krylov loop, its dots and the coarsest solve FP64.
                            Use a flexible outer method (FCG or FGMRES).      */
#define AMG_PREC_FP32 2  /* as AMG_PREC_MIXED with every operator in FP32    */
/* Saddle point systems: the same modes apply to A; B, B^T, C, the transfers,
 * the smoothers' scalings and the Braess-Sarazin Schur hierarchies are FP32
 * in both reduced modes; the explicit inverses of the systems that end on a
 * level stay FP64 (FP64 accumulation). Requires AMG_KRYLOV_FGMRES. */

/*
 * The linear system (Section 2.4). The pointers are host pointers, or device
 * pointers under memory = AMG_MEM_DEVICE; the library copies the data.
 *
 * A (velocity/displacement block): square over N = n_lin + n_quad nodes, CSR
 *   over nodes with sorted column indices and every diagonal entry present.
 *   bs = 3: each entry is a 3x3 block, A_val holds 9 doubles per entry in
 *           row-major order (A_val[9*k + 3*r + c]).
 *   bs = 1: A = A_s (x) I_3 (the vector Laplacian); A_val holds one double per
 *           entry, applied to each of the 3 components.
 *   The pattern is the STRUCTURAL pattern (all node pairs coupled through an
 *   element); entries whose value is zero must be kept, because coarsening
 *   uses the connectivity graph of the matrix (Section 3.2).
 * B (saddle only, n_pres > 0): n_pres rows (pressure nodes = mesh vertices,
 *   the same order as the linear velocity nodes, so n_pres == n_lin) times N
 *   node columns, 1x3 blocks (B_val[3*k + c]). Requires bs = 3.
 * C (saddle only, optional): n_pres x n_pres scalar CSR; NULL pointers mean
 *   C = 0 (Stokes, Section 2.4).
 * pressure_kernel: 1 when constant pressures lie in the kernel (velocity
 *   Dirichlet data on the whole boundary, C = 0); the coarsest solve then
 *   pins its last pressure unknown.
 * memory: where the nine arrays live. AMG_MEM_HOST (0, the default of a
 *   zero-initialised struct): host memory. AMG_MEM_DEVICE (1): device memory
 *   of the current device (hipMalloc'd or managed); the setup reads them in
 *   stream order on its stream (work the caller queued on that stream before
 *   the call is complete first) and copies them to the host for its
 *   host-side passes (coarse/fine splits, colouring, checks) before
 *   uploading its own copy, so the caller may free or overwrite them once the
 *   setup has returned. A pointer that is not device memory under
 *   AMG_MEM_DEVICE is rejected with AMG_EINVAL.
 */
typedef struct {
    int32_t n_lin, n_quad, n_pres;
    int32_t bs;
    const int32_t *A_rowptr, *A_col;
    const double *A_val;
    const int32_t *B_rowptr, *B_col;
    const double *B_val;
    const int32_t *C_rowptr, *C_col;
    const double *C_val;
    int32_t pressure_kernel;
    int32_t memory; /* AMG_MEM_HOST or AMG_MEM_DEVICE */
} amg_system;

#define AMG_MEM_HOST 0
#define AMG_MEM_DEVICE 1

/*
 * Parameters. amg_default_params fills the paper's defaults: GS-1-1, JA damping
 * 0.5 (Section 4.2), sGS omega 0.125 with block-Jacobi damping 0.5 (Sections
 * 3.3 and 4.4), one V-cycle per preconditioner application, separated
 * coarsening, coarsening until at most 300 unknowns or 10 levels, PCG, FP64.
 */
typedef struct {
    int32_t smoother;     /* AMG_SMOOTH_*                                    */
    int32_t pre, post;    /* m_pre, m_post of Algorithm 1                    */
    double omega;         /* JA damping                                      */
    double sgs_omega;     /* sGS pressure parameter omega                    */
    double sgs_damping;   /* sGS M_A: damped block Jacobi damping            */
    int32_t cycles;       /* Algorithm 1 applications per preconditioning    */
    int32_t nu;           /* recursive calls per level: 1 = V, 2 = W         */
    int32_t max_levels;   /* including the finest                            */
    int32_t coarse_max;   /* stop when a level has <= this many unknowns     */
    int32_t separate;     /* 1 = the paper's separated linear/quadratic
                             graphs, 0 = one graph over all nodes            */
    int32_t krylov;       /* AMG_KRYLOV_*                                    */
    int32_t restart;      /* FGMRES restart length                           */
    int32_t precision;    /* AMG_PREC_*                                      */
    int32_t n_level_omega;        /* > 0: per-level JA damping follows     */
    const double *level_omega;    /* host, n_level_omega values (copied)   */
    int32_t fuse_coarse;  /* 1 (default): the coarse end of a V-cycle runs as
                             one kernel (an explicit operator assembled at
                             setup, one per system for saddle systems and
                             batches, or a single-workgroup kernel); 0: one
                             launch per operation. Same arithmetic, up to
                             rounding order.                                  */
    int32_t autotune;     /* 1 (default): time the row kernels' lanes-per-row
                             choices on each level at setup, and time the
                             saddle coarse-end candidates (fuse_coarse);
                             0: no setup choice depends on timing (heuristic
                             launch shapes, no assembled saddle coarse end),
                             so two setups of the same input give the same
                             bits. Solves on one hierarchy always repeat
                             bit for bit (fixed summation orders).           */
    amg_mlp_handle omega_model; /* JA only, SPD only, NULL (default) = off:
                             the damping of every non-coarsest level is the
                             network's prediction from that level's row
                             features (amg_level_features); a prediction
                             that is not finite or not inside (0.2, 1.2)
                             falls back to omega / level_omega, and a
                             learned weight above the level's bound
                             0.95 * 2 / lambda_max(D^{-1} A_l) is lowered to
                             it (amg_level_info.omega_max). The FP64
                             residual judges the weights: an amg_solve that
                             breaks down, diverges or misses the tolerance
                             is repeated from its initial guess with the
                             fixed weights, which then stay (iterations and
                             time of both attempts are reported). Only read
                             during amg_setup.                               */
    int32_t graph;        /* 1 (default): each preconditioner application is
                             recorded once into a HIP graph and replayed
                             (same kernels, same order, same results); 0:
                             launched one by one. Profiling runs unrecorded. */
    double vanka_omega;   /* Vanka damping of the local corrections (0.8)  */
    int32_t gs_post;      /* direction of the post-smoothing Gauss-Seidel
                             sweeps (SPD systems): 0 (default) backward under
                             a Krylov method - a symmetric cycle, which CG
                             needs - and forward in the stand-alone solver,
                             the form the stand-alone tables of Section 4
                             follow; 1 always backward; 2 always forward.
                             A forward post-smoother runs the coarse end
                             level by level (no assembled coarse end).      */
} amg_params;

typedef struct {
    int32_t iters;     /* outer iterations performed                         */
    int32_t status;    /* AMG_OK / AMG_NOT_CONVERGED / AMG_BREAKDOWN / ...   */
    double relres;     /* true relative residual ||b - K x|| / ||b - K x0||  */
    double solve_ms;   /* wall time of the solve on the host clock           */
} amg_result;

typedef struct {
    int32_t n_lin, n_quad, n_pres; /* nodes on the level                      */
    int32_t bs;                    /* 3 or 1                                   */
    int64_t nnz_A, nnz_B, nnz_C;   /* entries (blocks) of the structural
                                      pattern, as amg_get_level_matrix
                                      returns them                            */
    int64_t nnz_P;                 /* entries of the scalar prolongation to
                                      this level from the next coarser one
                                      (0 on the coarsest level)               */
    int32_t n_colors;              /* Gauss-Seidel colours (0 if not built)    */
    int32_t is_coarsest;
    int32_t lanes_A, lanes_gs;     /* lanes per row chosen for the level's
                                      natural-order and colour-sweep kernels
                                      (of the reduced-precision copies when
                                      precision is not FP64)                 */
    int32_t fused;                 /* 1 if a V-cycle reaching this level runs
                                      it inside the fused coarse kernel       */
    double omega;                  /* JA damping used on this level          */
    int32_t schur_levels;          /* Braess-Sarazin: levels of the scalar
                                      hierarchy of this level's Schur
                                      complement (0 if not built)             */
    int64_t nnz_S;                 /* entries of that Schur complement S_l   */
    int32_t gs_xcd;                /* 1 if the colour sweeps give each XCD one
                                      contiguous eighth of a colour's rows    */
    int32_t trip_A, trip_gs;       /* entries per lane and loop trip of those
                                      kernels: 1, 2 or 4                      */
    int32_t lanes64_A, trip64_A;   /* the FP64 natural-order kernels' lanes
                                      and entries per trip (the outer Krylov
                                      operator also in reduced-precision
                                      solves)                                 */
    int64_t kept_A, kept_B;        /* entries the smoothers and solve kernels
                                      stream: the structural ones less the
                                      numerically zero off-diagonal blocks,
                                      dropped once the setup's pattern-based
                                      steps are done (Dirichlet couplings,
                                      couplings that vanish on the mesh)     */
    int32_t coarse_map;            /* 1 on the first level of the assembled
                                      coarse end: a V-cycle that enters this
                                      level from a zero guess applies the
                                      explicit map x = T b of the cycle from
                                      here down (FP64 assembly; streamed as
                                      BF16 in the FP32/BF16 cycle, each entry
                                      rounded to nearest even, and as FP32 in
                                      the FP32 cycle); 0 elsewhere          */
    int32_t learned;               /* 1 while the JA weights are the damping
                                      network's (0 after a fallback or
                                      amg_set_level_omega)                   */
    double omega_max;              /* JA smoother (SPD): the bound learned
                                      weights are kept under,
                                      0.95 * 2 / lambda_max(D^{-1} A_l) with
                                      lambda_max estimated by 100 power
                                      iterations (a symmetric V-cycle with
                                      damped block Jacobi is positive
                                      definite only for omega below
                                      2 / lambda_max); fixed weights are not
                                      changed; 0 for other smoothers          */
    int32_t omega_fallbacks;       /* solves repeated with the fixed weights
                                      because the learned ones failed        */
} amg_level_info;

/* Fill *p with the defaults listed above. */
void amg_default_params(amg_params *p);

/* Build the hierarchy for *sys (Section 3.2). Device work runs on `stream`;
 * returns after setup is complete. On success *out owns all device memory of
 * the hierarchy. Errors: AMG_EINVAL (inconsistent sizes, missing diagonal,
 * unsorted columns), AMG_EUNSUPPORTED (a coarse row beyond the Galerkin
 * kernel's capacity), AMG_ENOMEM, AMG_EHIP. */
int amg_setup(const amg_system *sys, const amg_params *params, amg_stream stream, amg_handle *out);

/* Solve K x = b to ||b - K x_k|| <= tol ||b - K x_0|| (Section 4's stopping
 * rule, Euclidean norm of the whole residual). b and x are DEVICE pointers of
 * 3N (+ n_pres) doubles; x holds x_0 on entry and the solution on return.
 * maxit bounds the outer iterations. Returns the solver status (also stored
 * in res->status, with iterations and the true relative residual). Blocks
 * until the solve has finished. */
int amg_solve(amg_handle h, const double *b, double *x, double tol, int32_t maxit,
              amg_stream stream, amg_result *res);

/* Several right-hand sides on one SPD hierarchy (PCG or FCG, any precision,
 * JA or GS): K x_r = b_r for r < nrhs, 1 <= nrhs <= 8. Every operator,
 * transfer and coarse-end pass of the V-cycle and of the outer operator reads
 * its matrix once for all right-hand sides (blocks of 2, 4 or 8; a block
 * beyond nrhs carries zero right-hand sides, which take no iterations);
 * each right-hand side keeps its own Krylov scalars, stopping test
 * (||b_r - K x_r|| <= tol ||b_r - K x_r,0||) and iteration count, and one
 * that has converged keeps its iterate while the others continue. The
 * arithmetic per right-hand side is amg_solve's up to the order of the
 * floating-point sums; the learned-damping fallback of amg_solve is not
 * applied here. B, X: DEVICE arrays of nrhs vectors one after another (each
 * laid out as amg_solve's b, x); X holds the initial guesses on entry.
 * results: HOST array of nrhs (solve_ms is the whole call's). Returns the
 * worst status. Errors: AMG_EINVAL for a saddle point system or batch
 * handle, another outer method, nrhs outside 1..8. */
int amg_solve_multi(amg_handle h, int32_t nrhs, const double *B, double *X, double tol, int32_t maxit,
                    amg_stream stream, amg_result *results);

/* z = M^{-1} r: `cycles` applications of Algorithm 1 from a zero initial
 * guess on the finest level (the preconditioner used inside amg_solve).
 * r, z: device pointers, same layout as amg_solve's b and x. FP64 in and
 * out; under AMG_PREC_MIXED the cycle itself runs in the mixed arithmetic. */
int amg_precondition(amg_handle h, const double *r, double *z, amg_stream stream);

/* y = K_l x on hierarchy level l (device pointers, level-l layout). */
int amg_apply(amg_handle h, int32_t level, const double *x, double *y, amg_stream stream);

/* One smoothing step S_l(x, b) of the configured smoother on level l, in
 * place on x (device pointers). forward = 1 for a pre-smoothing step (colours
 * ascending), 0 for a post-smoothing step (colours descending). */
int amg_smooth(amg_handle h, int32_t level, const double *b, double *x, int32_t forward,
               amg_stream stream);

int amg_num_levels(amg_handle h);
int amg_get_level_info(amg_handle h, int32_t level, amg_level_info *info);

/* Copy a level operator to HOST arrays sized from amg_get_level_info:
 * which = 0: A (rowptr n+1, col nnz_A, val nnz_A*bs*bs), 1: B (1x3 blocks),
 * 2: C, 3: P (scalar prolongation from level+1 to level, n rows),
 * 4: the Braess-Sarazin Schur complement S_l = C + B (2 diag A)^{-1} B^T
 *    (n_pres rows, nnz_S scalar entries; Section 3.3). */
int amg_get_level_matrix(amg_handle h, int32_t level, int32_t which, int32_t *rowptr,
                         int32_t *col, double *val);

/* Colour of every node of level l (host array of n_lin + n_quad int32). */
int amg_get_level_colors(amg_handle h, int32_t level, int32_t *colors);

/* Launch shape of level l's row kernels, replacing the setup tuner's choice
 * (for tests that run every variant; results agree up to rounding order).
 * kernels: AMG_SHAPE_NATURAL the FP64 natural-order kernels (residual,
 * Jacobi, operator, the outer Krylov operator on level 0), AMG_SHAPE_SWEEP
 * the FP64 colour sweeps, AMG_SHAPE_NATURAL_RP / AMG_SHAPE_SWEEP_RP the same
 * kernels of the reduced-precision copies. lanes: lanes of the 64-wide
 * wavefront per row, one of 4, 8, 16, 32, 64. trip: entries per lane and
 * loop trip, 1, 2 or 4 (a lane's entries of one trip have their loads in
 * flight together; the sums do not depend on it; the prolongation kernels
 * always take 1). xcd (colour sweeps only): 1 = each XCD takes one
 * contiguous eighth of a colour's rows, 0 = round-robin placement.
 * AMG_SHAPE_VANKA (Vanka smoother, any level but the coarsest): the
 * level's sweeps compute the patch residuals with `lanes` lanes per row
 * (16, 32 or 64), then, for trip 1, partial corrections over 64-row x
 * chunk tiles of the patch inverses and their sum in chunk order, for
 * trip 2, the corrections over 64-row tiles of the inverses (xcd 0).
 * AMG_SHAPE_VANKA_APPLY: the latter form, with `lanes` = 4, 8 or 16
 * wavefronts per 64-row tile splitting its columns (trip 1, xcd 0).
 * Recorded preconditioner graphs are dropped (they hold the old shapes).
 * Errors: AMG_EINVAL for a bad level, kernel class, lane count, trip or flag, or a
 * reduced-precision class on an FP64 hierarchy. */
#define AMG_SHAPE_NATURAL 0
#define AMG_SHAPE_SWEEP 1
#define AMG_SHAPE_NATURAL_RP 2
#define AMG_SHAPE_SWEEP_RP 3
#define AMG_SHAPE_VANKA 4
#define AMG_SHAPE_VANKA_APPLY 5
int amg_set_launch_shape(amg_handle h, int32_t level, int32_t kernels, int32_t lanes, int32_t trip, int32_t xcd);

/* ---- batches of independent systems ------------------------------------
 * Many solves of uneven size in one set of launches (addition X2). Each
 * system gets the hierarchy amg_setup would build for it alone; the
 * hierarchies are merged level by level into one block-diagonal hierarchy
 * (systems ordered by decreasing depth, so those still coarsening on a level
 * lead it and those ending on it are solved by their explicit inverses),
 * and every kernel of a cycle serves the whole batch. Every system of a
 * batch is a saddle point system, or every one is SPD:
 *  - saddle point systems: flexible GMRES with per-system inner products,
 *    Hessenberg matrices and convergence tests (sGS or Braess-Sarazin
 *    smoother; any precision mode);
 *  - SPD systems (n_pres = 0, one bs for all): preconditioned CG (PCG) or
 *    its flexible form (FCG, for the reduced-precision cycles) with
 *    per-system step lengths, residual norms and convergence tests, in
 *    lockstep (JA or GS smoother, V or W cycles; any precision mode: the
 *    merged levels get the FP32 / BF16 copies of a single system, and
 *    systems ending on a level keep their FP64 inverses; the coarse levels
 *    run level by level: fuse_coarse is a single-system feature). Errors:
 *    AMG_EINVAL for mixed kinds or bs, another Krylov method or smoother,
 *    or gs_post = 2.
 * Both take host or device arrays (amg_system::memory).
 */
int amg_setup_batched(int32_t nsys, const amg_system *systems, const amg_params *params, amg_stream stream,
                      amg_handle *out);
/* b, x: DEVICE arrays holding the systems one after another in the order
 * given to amg_setup_batched, each as [u (3 N_i); p (Np_i)] (SPD: u); x is the initial
 * guess on entry and the solution on return. results: HOST array of nsys
 * (per-system iterations, status, true relative residual; solve_ms is the
 * whole batch's). Returns the worst status. */
int amg_solve_batched(amg_handle h, const double *b, double *x, double tol, int32_t maxit, amg_stream stream,
                      amg_result *results);
/* Offsets of system i's velocity and pressure values in the merged level-0
 * vector [u (all systems); p (all systems)] that amg_precondition and
 * amg_apply use on a batch handle (pressure offsets relative to the start
 * of the pressure block). HOST arrays of nsys. */
int amg_batch_offsets(amg_handle h, int64_t *u_offset, int64_t *p_offset);

/* ---- learned Jacobi damping -------------------------------------------
 * Not in the paper, which damps block Jacobi with a fixed 0.5 (Section 4.2):
 * a multilayer perceptron 8 -> 32 -> 32 -> 1 (tanh hidden units, output
 * omega = 0.2 + sigmoid(z) in (0.2, 1.2)) maps eight statistics of the rows
 * of A_l to a damping weight for level l. Training (full-batch Adam on the
 * mean squared error to target weights) and inference run on the GPU in FP32.
 *
 * Parameters are AMG_MLP_PARAMS floats in the order W1 (32x8 row-major), b1
 * (32), W2 (32x32 row-major), b2 (32), W3 (32), b3 (1). Feature and target
 * arrays are HOST arrays: X is n x AMG_MLP_FEATURES row-major, y has n values.
 */
#define AMG_MLP_FEATURES 8
#define AMG_MLP_PARAMS 1377

/* Create a network from host parameters (copied); Adam state starts at zero.
 * Work is ordered on `stream`. */
int amg_mlp_create(const float *params, amg_stream stream, amg_mlp_handle *out);
int amg_mlp_get_params(amg_mlp_handle m, float *params);
/* omega[i] for every feature row (host arrays, n >= 1). */
int amg_mlp_forward(amg_mlp_handle m, const float *X, int32_t n, float *omega);
/* Mean squared error to y and its gradient (AMG_MLP_PARAMS floats). */
int amg_mlp_gradient(amg_mlp_handle m, const float *X, const float *y, int32_t n, float *loss, float *grad);
/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning
 * rate lr) continuing the handle's step count; loss_history (host, may be
 * NULL) receives the loss before every step. */
int amg_mlp_train(amg_mlp_handle m, const float *X, const float *y, int32_t n, int32_t steps, float lr,
                  float *loss_history);
void amg_mlp_destroy(amg_mlp_handle m);

/* Replace the JA damping of every level after setup (level l uses
 * omega[min(l, n - 1)]); rebuilds the fused coarse end of the cycle, which
 * holds the weights. JA smoother, SPD systems only. */
int amg_set_level_omega(amg_handle h, int32_t n, const double *omega);

/* The network's input for level l of an SPD hierarchy (host array of 8):
 * over the scalar rows of A_l (row r of node i; a bs = 1 operator stands for
 * A_s (x) I_3), with d the diagonal entry and a_j the other stored entries,
 * rho = sum |a_j| / |d|, sigma = (d + sum a_j) / d, tau = sqrt(sum a_j^2) / |d|
 * (all 0 for a zero diagonal), nz = stored scalars of the row:
 *   [mean rho, max rho, std rho, mean sigma, mean tau, mean nz / 64,
 *    l / 10, log10(3 N_l) / 7]. */
int amg_level_features(amg_handle h, int32_t level, double *features);

/* amg_level_features for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid allocation):
 * the same eight features of level l, written to features_dev, a DEVICE
 * array of 8 doubles, on `stream` without allocating and without a host
 * synchronisation (the call returns once the work is enqueued). The partial
 * sums live in a fixed 1 MiB device array of the library, one per GPU, held
 * until the process ends; the level may have at most 6,710,272 scalar rows
 * (3 N_l for 3x3 blocks, N_l for bs = 1), else AMG_EINVAL. Every call on one
 * GPU shares that array: calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller. Values agree with
 * amg_level_features up to the last bit of the square root and logarithm. */
int amg_level_features_noalloc(amg_handle h, int32_t level, double *features_dev, amg_stream stream);

/* Per-kernel timing of the hot loops with HIP events recorded on the
 * library's launch stream (the stream of the call that launches them).
 * enable = 1 times every launch, enable = 2 only the finest level's launches
 * (fewer events in flight), 0 stops; a nonzero value clears the counters. */
int amg_profile_enable(amg_handle h, int32_t enable);
/* Kernel classes "<op>.L<level>" with op one of spmv, gs, jacobi, jacobi0,
 * resid, restrict, prolong; plus "coarse" and "blas". Returns launches,
 * total ms and algorithmic bytes (bytes the operation must move at least:
 * every stored entry and index once, every vector once).
 * Setup phases are always recorded (never cleared): "setup.<phase>" with
 * phase one of upload, coarsen (graphs, independent sets, interpolation;
 * host), galerkin (the Galerkin products), omega_network, drop_zeros,
 * smoother (diagonal inverses, colouring, colour-grouped copies, saddle
 * scalings), autotune, coarsest (dense inverse), omega_bound, schur,
 * schur_map, vanka, coarse_map, reduced_copies, saddle_map, merge
 * (batches): calls and wall ms. A batch sets its systems up concurrently on
 * several host threads: "setup.systems" is the wall ms of that step and
 * "setup.systems.<phase>" the systems' own phases, summed over them.
 * "setup.spgemm_numeric": the Galerkin numeric kernels' HIP-event ms and
 * algorithmic bytes (both factors and the product's pattern read once, its
 * values written once). */
int amg_profile_read(amg_handle h, const char *kernel_class, int64_t *launches, double *total_ms,
                     double *bytes);

void amg_destroy(amg_handle h);
const char *amg_status_string(int status);
const char *amg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMG_P2_H */
