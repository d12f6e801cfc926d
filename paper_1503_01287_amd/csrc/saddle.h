// Kernels of the saddle-point path: the off-diagonal blocks B (pressure x
// velocity, 1x3 blocks), B^T (3x1 blocks) and C (scalar), the segregated
// Gauss-Seidel (Uzawa) smoother's updates, the Braess-Sarazin smoother's
// diagonal solves, and the batched inner products of flexible GMRES.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

enum BlkOp : int {
    BLK_SPMV = 0,   // y = s
    BLK_ADD = 1,    // y += s
    BLK_SUB = 2,    // y -= s
    BLK_RESID = 3,  // y = b - s
    BLK_SGS_P = 4,  // (1x3 rows of B) y_p += omega * dscale_p * (s - b_p)
    BLK_ADD_SCALED = 5,  // (3x1 rows of B^T) y_o += dscale_o * (b_o + s_o), per component o
};

// T = double (FP64 path) or float (reduced-precision cycle: FP32 values,
// vectors and accumulation)
template <typename T>
struct BlkArgsT {
    int nrows = 0;
    const int *rowptr = nullptr, *col = nullptr;
    const T *val = nullptr;   // planes: br*bc
    int64_t nnz = 0;
    const T *x = nullptr;     // bc components per column node
    const T *b = nullptr;     // br components per row
    T *y = nullptr;
    const T *dscale = nullptr;
    T omega = 1;
    // optional scalar operator on the same rows (1x3 B rows only, with
    // BLK_RESID or BLK_SPMV): y_i = (result) + c_sign (C c_x)_i, the C row
    // read by the same lanes after the B row
    const int *c_rowptr = nullptr, *c_col = nullptr;
    const T *c_val = nullptr;
    const T *c_x = nullptr;
    T c_sign = 1;
    // BLK_SGS_P, BLK_ADD_SCALED: y starts from zero (y is written, not read)
    int y_zero = 0;
};
using BlkArgs = BlkArgsT<double>;
using BlkArgsF = BlkArgsT<float>;

// y = -x
template <typename T>
void launch_neg(int64_t n, const T *x, T *y, hipStream_t s);

// br, bc in {1, 3}; G lanes per row
template <typename T>
void launch_blk(int br, int bc, int op, int G, const BlkArgsT<T> &a, hipStream_t s);

// sGS velocity step on the first n nodes: t_i = damping * D_i^{-1} r_i;
// u_i += t_i, or u_i = t_i when u starts from zero (u_zero: u is not read)
// (3x3 blocks, dinv planes of stride ld >= n)
template <typename T>
void launch_sgs_u(int64_t n, int64_t ld, const T *dinv, const T *r, T damping, T *t, T *u, bool u_zero,
                  hipStream_t s);
// sGS pressure scaling 1 / (damping * sum_k b_k^T D_{col k}^{-1} b_k + C_pp)
void launch_sgs_scale(int np, const int *brow, const int *bcol, const double *bval, int64_t bnnz,
                      const double *dinv, int64_t nv, double damping, const int *crow, const int *ccol,
                      const double *cval, int64_t cnnz, double *out, hipStream_t s);
// y_i = d_i * x_i (elementwise) / y_i = d_i * (x_i - z_i)
template <typename T>
void launch_scale(int64_t n, const T *d, const T *x, T *y, hipStream_t s);
void launch_scale_diff(int64_t n, const double *d, const double *x, const double *z, double *y, hipStream_t s);
// 1 / (2 a_ii) for every velocity unknown (Braess-Sarazin's A_hat = 2 diag(A))
void launch_bs_diag(int n, const int *rowptr, const int *col, const double *val, int64_t nnz, double *out,
                    hipStream_t s);

// Braess-Sarazin Schur complement on a given (sorted) pattern:
// S_pq = sum_k sum_c B_pk[c] d[3k+c] B^T_kq[c] + C_pq (C optional, its
// pattern contained in S's). One lane per output entry, fixed summation order.
void launch_schur_numeric(int np, const int *brow, const int *bcol, const double *bval, int64_t bnnz,
                          const int *btrow, const int *btcol, const double *btval, int64_t btnnz, const double *d,
                          const int *crow, const int *ccol, const double *cval, const int *srow, const int *scol,
                          double *sval, hipStream_t s);
// scalar Gauss-Seidel update of the rows of one colour of S, grouped: row g
// (g < nrows) has entries rowptr[g] .. rowptr[g+1] of col/val and node
// i = rowid[g]: x_i = dinv_i (b_i - sum_{j != i} S_ij x_j)
template <typename T>
void launch_scalar_gs(int nrows, const int *rowptr, const int *col, const T *val, const int *rowid, const T *dinv,
                      const T *b, T *x, int G, hipStream_t s);
// u += d .* w
template <typename T>
void launch_add_scaled(int64_t n, const T *d, const T *w, T *u, hipStream_t s);
// y = a x + b y
void launch_axpby_f(float *y, const float *x, float a, float b, int64_t n, hipStream_t s);

// Explicit inverses of the systems that end on a level ("dense segments"):
// segment s is an m_s x m_s row-major inverse at inv + moff[s] acting on the
// vector made of nu_s values at u + uoff[s] followed by np_s values at
// p + poff[s] (m_s = nu_s + np_s). rstart holds the prefix sums of m_s.
struct DenseSegView {
    int count = 0, rows = 0;
    const int64_t *moff = nullptr;
    const int *rstart = nullptr, *uoff = nullptr, *nu = nullptr, *poff = nullptr;
    const double *inv = nullptr;
    const float *inv32 = nullptr;  // FP32 copy of inv, or null
};
// y = M_s x on every segment (x and y: u parts xu/yu, p parts xp/yp); the
// accumulation is FP64; FP32 vectors use the FP32 copy of the matrices when
// there is one (assembled coarse-end maps), else the FP64 matrices
template <typename T>
void launch_dense_segs(const DenseSegView &d, const T *xu, const T *xp, T *yu, T *yp, hipStream_t s);

// x = sum over segments s with m_s > j of the unit vector of the segment's
// row j: xu[uoff[s] + j] for j < nu[s], else xp[poff[s] + j - nu[s]]
void launch_segment_units(const DenseSegView &d, int j, double *xu, double *xp, hipStream_t s);
// column j of every segment's matrix (row-major) from x, rows read as in
// launch_segment_units: M_s[i][j] = x(row i of segment s)
void launch_segment_store_column(const DenseSegView &d, int j, const double *xu, const double *xp, double *inv,
                                 hipStream_t s);
// The same for blocks of C columns over pressure-only segments (nu = 0):
// vectors row-major with C columns (segment s's row i, column c at
// (poff_s + i) C + c). Units: x[(poff_s + j0 + c) C + c] = 1 for j0 + c <
// m_s; store: M_s[i][j0 + c] from column c; y = M_s x on every segment, FP64.
void launch_segment_units_block(const DenseSegView &d, int j0, int C, double *x, hipStream_t s);
void launch_segment_store_block(const DenseSegView &d, int j0, int C, const double *x, double *inv, hipStream_t s);
void launch_dense_segs_block(const DenseSegView &d, int C, const double *x, double *y, hipStream_t s);

// FGMRES inner products: h[i] = <V_i, w> for i < k (V_i = V + i * ld) as
// block partials partial[i * nb + block] (nb = multidot_blocks(n), the
// buffer holds k * nb values); returns nb
int launch_multidot(const double *V, int64_t ld, int k, const double *w, int64_t n, double *partial,
                    hipStream_t s);
int multidot_blocks(int64_t n);
// the same for two right-hand sides in one pass over the basis:
// partial[(r * k + i) * nb + block] holds <V_i, a> (r = 0) and <V_i, b>
// (r = 1); the buffer holds 2 k nb values
int launch_multidot2(const double *V, int64_t ld, int k, const double *a, const double *b, int64_t n,
                     double *partial, hipStream_t s);
// h[i] = sum of partial[i * nb ...] for i < k
void launch_multidot_reduce(const double *partial, int nb, int k, double *h, hipStream_t s);
// Delayed reorthogonalisation step on basis slots j (pending vector) and
// j + 1 (new vector) from the reduced dots h[0 .. 2(j + 2)) of
// launch_multidot2(V, ld, j + 2, V_j, V_{j+1}); writes gamma, d, eta to
// h[2(j + 2) ..] (see k_dcgs2_update)
void launch_dcgs2_update(double *V, int64_t ld, int j, double *h, int64_t n, bool reorth, hipStream_t s);
// x += sum_i y[i] Z_i  (y on the device)
void launch_multi_add(const double *Z, int64_t ld, int k, const double *y, double *x, int64_t n,
                      hipStream_t s);
// y = a * x (device scalar a = 1 / sc[idx])
void launch_scale_by_inverse(const double *x, double *y, int64_t n, const double *sc, int idx, hipStream_t s);

}  // namespace amgp2
