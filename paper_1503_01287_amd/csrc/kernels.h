// Device kernels of the AMG library (gfx950, wave64) and their launchers.
//
// Storage of a block-CSR operator on the device ("planes"): the k-th entry of
// a block of shape br x bc is stored in plane p = r*bc + c at val[p*nnz + k].
// A wavefront reading the same plane for consecutive entries issues fully
// coalesced loads (8 bytes per lane), which is what the memory-bound row
// kernels below are built around.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

// Operation applied at the end of a row kernel, after the G lanes of a row
// group have reduced s = (A x)_i (3 components).
enum RowOp : int {
    OP_SPMV = 0,      // y_i = s
    OP_SPMV_ADD = 1,  // y_i += s                         (prolongation x += P e)
    OP_RESID = 2,     // y_i = b_i - s                    (residual)
    OP_JACOBI = 3,    // y_i = x_i + omega D_i^{-1}(b_i - s)   (damped block Jacobi)
    OP_GS = 4,        // x_i += D_i^{-1}(b_i - s), in place   (Gauss-Seidel, one colour)
    OP_SPMV_DOT = 5,  // y_i = s and a block partial of <x, y>
};

struct RowArgs {
    int nrows = 0;                  // rows handled by this launch
    const int *rowptr = nullptr;    // CSR row pointers (of the launch's row range)
    const int *col = nullptr;
    const double *val = nullptr;    // planes
    int64_t nnz = 0;                // plane stride
    const int *rowid = nullptr;     // output/input node of row g (nullptr: g)
    const double *x = nullptr;      // vector the operator multiplies
    const double *b = nullptr;      // right-hand side (RESID, JACOBI, GS)
    double *y = nullptr;            // output (for GS: the vector updated in place)
    const double *dinv = nullptr;   // inverted diagonal blocks, planes of stride dinv_n
    int64_t dinv_n = 0;
    double omega = 1.0;
    double *partial = nullptr;      // per-block partial sums (SPMV_DOT)
    double *zero_out = nullptr;     // if set: zero_out_i = 0 for every row i written
    int xcd_chunks = 0;             // 1: each XCD takes one contiguous eighth of the rows
    int trip = 1;                   // entries per lane and loop trip: 1, 2 or 4 (OP_SPMV_ADD: 1)
};

// mode: 3 = 3x3 blocks; 1 = scalar entries applied to 3-component vectors.
// G: lanes per row (4, 8, 16, 32, 64).
void launch_row(int mode, RowOp op, int G, const RowArgs &a, hipStream_t s);

// Number of blocks the row kernel uses (size of the partial-sum buffer).
int row_blocks(int nrows, int G);

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w runs on
// XCD w mod 8). With a grid padded to a multiple of 8, this maps the
// workgroups of XCD k to the k-th contiguous eighth of the logical blocks, so
// that each XCD's L2 holds the vector entries of one region of the mesh.
__device__ __forceinline__ int64_t xcd_chunk_block() {
    return static_cast<int64_t>(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
}

// ---------------------------------------------------------------- vectors
void launch_fill(double *x, double v, int64_t n, hipStream_t s);
void launch_fill_hash(double *x, int64_t n, uint32_t seed, hipStream_t s);
void launch_copy(double *dst, const double *src, int64_t n, hipStream_t s);
// planes[p * nnz + k] = aos[k * np + p] (blocks stored entry by entry -> planes)
void launch_aos_to_planes(const double *aos, int np, int64_t nnz, double *planes, hipStream_t s);
// x_i = D_i^{-1} b_i for the nodes rowid[0..nrows) (first colour of a
// Gauss-Seidel sweep from x = 0); dinv planes of stride n
void launch_diag_solve(int mode, int nrows, const int *rowid, const double *dinv, int64_t n, const double *b,
                       double *x, hipStream_t s);
// x = omega D^{-1} b (first Jacobi step from x = 0) on nodes 0 .. nnodes-1;
// dinv: inverted diagonal blocks, planes dn apart
void launch_jacobi_zero(int mode, int64_t nnodes, const double *dinv, int64_t dn, const double *b, double omega,
                        double *x, hipStream_t s);
// per-block partial sums of <a, b> over n doubles; returns the number of blocks
int launch_dot_partial(const double *a, const double *b, int64_t n, double *partial, hipStream_t s);
int dot_blocks(int64_t n);

// Scalars of the Krylov drivers live in a small device array.
enum Scalar : int {
    SC_RZ = 0, SC_PQ, SC_ALPHA, SC_BETA, SC_RR, SC_TMP, SC_RZ_OLD, SC_PR, SC_COUNT
};
// Sum partial[0..np) into sc[dst] in a fixed order (deterministic), then
// derive the Krylov step scalars from it:
enum ReducePost : int {
    RED_NONE = 0,
    RED_CG_ALPHA,   // dst = PQ:  alpha = rz / pq
    RED_CG_BETA,    // dst = TMP: beta = tmp / rz, rz = tmp
    RED_FCG_BETA,   // dst = TMP: beta = -tmp / pq_prev
    RED_FCG_ALPHA,  // dst = PR:  alpha = pr / pq, pq_prev = pq
};
void launch_reduce(const double *partial, int np, double *sc, int dst, hipStream_t s, int post = RED_NONE);
// x += alpha p; r -= alpha q; partial of <r, r>; zero[i] = 0 if zero != nullptr
int launch_cg_update(double *x, double *r, const double *p, const double *q, const double *sc,
                     int64_t n, double *partial, double *zero, hipStream_t s);
// p = z + beta p  (beta from sc)
void launch_cg_direction(double *p, const double *z, const double *sc, int64_t n, hipStream_t s);
// y = a x + b y with host scalars
void launch_axpby(double *y, const double *x, double a, double b, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- dense
// Y[i*nc + c] = sum_j M[i*m + j] * X[j*nc + c]  (m x m matrix, nc components)
void launch_dense_gemv(const double *M, int m, int nc, const double *X, double *Y, hipStream_t s);

// ---------------------------------------------------------------- setup
// Inverted diagonal blocks (3x3 or scalar) of a square block-CSR matrix,
// written as planes of stride n. Fails (flag set) if a diagonal is missing.
void launch_diag_inverse(int mode, int n, const int *rowptr, const int *col, const double *val,
                         int64_t nnz, double *dinv, int *flag, hipStream_t s);
// Gather rows order[g] of (rowptr, col, val; planes nnz apart) into the
// grouped copy (g_rowptr, g_col, g_val; planes g_nnz apart).
void launch_gather_rows(int np, int nrows, const int *order, const int *rowptr, const int *col,
                        const double *val, int64_t nnz, const int *g_rowptr, int *g_col,
                        double *g_val, int64_t g_nnz, hipStream_t s);

// Dropping numerically zero entries (all planes zero; the diagonal of a
// square operator is always kept): count per row, then the kept entries in
// their order into (c_rowptr, c_col, c_val) with c_nnz entries.
void launch_count_kept(int np, int nrows, bool square, const int *rowptr, const int *col, const double *val,
                       int64_t nnz, int *count, hipStream_t s);
void launch_compact_rows(int np, int nrows, bool square, const int *rowptr, const int *col, const double *val,
                         int64_t nnz, const int *c_rowptr, int *c_col, double *c_val, int64_t c_nnz,
                         hipStream_t s);

// Galerkin SpGEMM C = X Y on node patterns (setup's hot loop).
// Symbolic phases use a hash set in LDS per wavefront; numeric phases let
// each lane own one output entry and sum its products in a fixed order, so
// the result is deterministic.
constexpr int SPGEMM_HASH = 2048;  // LDS hash slots per wavefront
void launch_spgemm_count(int nrows, const int *xr, const int *xc, const int *yr, const int *yc,
                         int *count, int *overflow, hipStream_t s);
void launch_spgemm_fill(int nrows, const int *xr, const int *xc, const int *yr, const int *yc,
                        const int *cr, int *cc, hipStream_t s);
// X has np planes (blocks), Y is scalar
void launch_spgemm_numeric_bx(int np, int nrows, const int *xr, const int *xc, const double *xv,
                              int64_t xnnz, const int *yr, const int *yc, const double *yv,
                              const int *cr, const int *cc, double *cv, int64_t cnnz, hipStream_t s);
// LDS-staged numeric phase, same sums in the same order (by: X scalar and Y
// in planes, else X in planes and Y scalar); *overflow (device) is set when
// a Y row alone exceeds the staging capacity: then run the kernels above
bool launch_spgemm_numeric_lds(bool by, int np, int nrows, const int *xr, const int *xc, const double *xv,
                               int64_t xnnz, const int *yr, const int *yc, const double *yv, int64_t ynnz,
                               const int *cr, const int *cc, double *cv, int64_t cnnz, int *overflow,
                               hipStream_t s);
// X is scalar, Y has np planes (Y rows sorted)
void launch_spgemm_numeric_by(int np, int nrows, const int *xr, const int *xc, const double *xv,
                              const int *yr, const int *yc, const double *yv, int64_t ynnz,
                              const int *cr, const int *cc, double *cv, int64_t cnnz, hipStream_t s);

}  // namespace amgp2
