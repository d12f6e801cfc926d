// Descriptors of the levels handled by the single-workgroup tail kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

struct TailLevel {
    int n = 0;          // nodes
    int ncolors = 0;    // Gauss-Seidel colours (0 for Jacobi / coarsest)
    int lds_off = 0;    // offset (doubles) of x, b, r (3n each) in LDS
    int nc = 0;         // nodes of the next coarser level
    const int *cptr = nullptr;  // colour ranges of the grouped rows
    const int *g_rowptr = nullptr, *g_col = nullptr;
    const double *g_val = nullptr;
    int64_t g_nnz = 0;
    const int *g_rowid = nullptr;
    const int *a_rowptr = nullptr, *a_col = nullptr;
    const double *a_val = nullptr;
    int64_t a_nnz = 0;
    const double *dinv = nullptr;
    const int *r_rowptr = nullptr, *r_col = nullptr;  // restriction (nc rows)
    const double *r_val = nullptr;
    const int *p_rowptr = nullptr, *p_col = nullptr;  // prolongation (n rows)
    const double *p_val = nullptr;
    double omega = 0.5;
};

struct TailArgs {
    int nlev = 0;        // tail levels, the last one the coarsest
    int smoother = 1;    // AMG_SMOOTH_JA or AMG_SMOOTH_GS
    int pre = 1, post = 1;
    int x_in_zero = 1;   // 1: the first tail level starts from x = 0
    const TailLevel *lv = nullptr;  // device array of nlev descriptors
    const double *cinv = nullptr;   // coarsest explicit inverse (cm x cm)
    int cm = 0, cnc = 1;
    const double *b_in = nullptr;   // right-hand side of the first tail level
    double *x_out = nullptr;        // its solution (also the initial guess if !x_in_zero)
    // unit_rhs = 1: workgroup j solves for the j-th unit right-hand side
    // (mode 3: e_j over the 3n unknowns; mode 1: component 0 of node j) and
    // writes its result as column j of the row-major m x m matrix x_out
    int unit_rhs = 0;
    int m = 0;
    int unit_base = 0;   // workgroup j handles unit right-hand side unit_base + j
    // if set, workgroup j keeps its level vectors at gscratch + j * gstride
    // (doubles) instead of LDS
    double *gscratch = nullptr;
    int64_t gstride = 0;
};

constexpr int TAIL_LDS_MAX = 64 * 1024;   // bytes of LDS the tail may use
constexpr int64_t TAIL_NNZ_MAX = 40000;   // stored entries of the first tail level
constexpr int TAIL_DENSE_MAX = 9000;      // largest tail operator kept as an explicit matrix

// grid = 1 for a solve, grid = m with unit_rhs = 1 to assemble the operator
void launch_tail(int mode, const TailArgs &a, int lds_bytes, int grid, hipStream_t s);

}  // namespace amgp2
