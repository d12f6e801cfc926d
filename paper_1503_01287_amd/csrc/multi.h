// Blocks of right-hand sides that share one SPD hierarchy: every operator,
// transfer and coarse-end pass reads its matrix once for K right-hand sides.
// Vectors are interleaved per node: value (node i, component c, right-hand
// side r) at ((3 i + c) K + r), so the gather of a column reads 3 K
// contiguous values.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

constexpr int MULTI_MAX_K = 8;  // right-hand sides per block (K in {2, 4, 8})

enum MOp : int { M_SPMV = 0, M_SPMV_ADD = 1, M_RESID = 2, M_JACOBI = 3, M_GS = 4 };
// value kinds: FP64 values with FP64 vectors; FP32 or BF16 (+ FP32 row
// scale) values with FP32 vectors
enum MKind : int { MK_F64 = 0, MK_F32 = 1, MK_BF16 = 2 };

struct MRowArgs {
    int nrows = 0;
    const int *rowptr = nullptr;
    const int *col = nullptr;
    const void *val = nullptr;     // planes (double, float or bf16)
    const float *rscale = nullptr; // BF16: scale of each scalar row (3 per node for 3x3 blocks)
    int64_t nnz = 0;
    const int *rowid = nullptr;    // node of row g (nullptr: g)
    const void *x = nullptr;       // interleaved vectors (double or float)
    const void *b = nullptr;
    void *y = nullptr;             // output; GS: updated in place (aliases x)
    const void *dinv = nullptr;    // inverted diagonal blocks, planes of stride dinv_n (double or float)
    int64_t dinv_n = 0;
    double omega = 1.0;
    void *zero_out = nullptr;      // if set: zero_out at every written (node, component, rhs) = 0
};

// mode 3: 3x3 blocks; mode 1: scalar applied to 3 components; K in {2, 4, 8},
// and 16 for scalar FP64 operators (mode 1, MK_F64)
void launch_mrow(int mode, int op, int kind, int K, const MRowArgs &a, hipStream_t s);
// x = omega D^{-1} b over all nodes (first Jacobi step from zero); T: double (kind F64) or float
void launch_mjacobi_zero(int mode, int kind, int K, int64_t nn, const void *dinv, const void *b, double omega,
                         void *x, hipStream_t s);
// x_i = D_i^{-1} b_i for the nodes rowid[0..nrows) (first colour of a sweep from zero)
void launch_mdiag_solve(int mode, int kind, int K, int nrows, const int *rowid, const void *dinv, int64_t n,
                        const void *b, void *x, hipStream_t s);
// Y (m x nc) = M (m x m, rows ld values apart) X (m x nc): mkind 0 FP64 M with
// double X, Y; 1 FP32 M, 2 BF16 M with float X, Y
void launch_mdense(int mkind, const void *M, int m, int ld, int nc, const void *X, void *Y, hipStream_t s);
// Krylov vector work on interleaved FP64 blocks of n_dof x K values
// out[p * K + r] = <a_p, b_p> over right-hand side r, for the np pairs (np <= 3), fixed order
int mdot_blocks(int64_t nd);
void launch_mdot(int np, int K, int64_t nd, const double *const *a, const double *const *b, double *partial,
                 double *out, hipStream_t s);
// y[i K + r] = cy[r] y[i K + r] + cx[r] x[i K + r] (coefficient arrays on the device)
void launch_mlincomb(int K, int64_t nd, double *y, const double *cy, const double *x, const double *cx,
                     hipStream_t s);
// between the caller's layout (nvec <= K vectors of nd one after another) and
// the interleaved block (columns nvec..K-1 zero going in, dropped coming out)
void launch_interleave(int K, int nvec, int64_t nd, const double *src, double *dst, bool to_interleaved,
                       hipStream_t s);

}  // namespace amgp2
