// Reduced-precision copies of the hierarchy for the mixed-precision cycle:
// FP32 vectors, FP32 or BF16 operator values (BF16 with one FP32 scale per
// scalar row, so the stored diagonal is exactly 1), FP32 transfer operators
// and inverted diagonal blocks. Index arrays are shared with the FP64 copy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

enum ValKind : int { VAL_F32 = 0, VAL_BF16 = 1 };

struct RowArgsMP {
    int nrows = 0;
    const int *rowptr = nullptr;
    const int *col = nullptr;
    const void *val = nullptr;      // planes of float or bf16 (uint16)
    const float *rscale = nullptr;  // BF16: scale of scalar row (3 per node for 3x3 blocks)
    int64_t nnz = 0;
    const int *rowid = nullptr;
    const float *x = nullptr;
    const float *b = nullptr;
    float *y = nullptr;
    const float *dinv = nullptr;
    int64_t dinv_n = 0;
    float omega = 1.f;
    float *zero_out = nullptr;
    int xcd_chunks = 0;             // as RowArgs::xcd_chunks
    int trip = 1;                   // OP_RESID / OP_JACOBI / OP_GS: 1, 2 or 4 entries per lane and trip
};

// Same operations as launch_row (OP_SPMV, OP_SPMV_ADD, OP_RESID, OP_JACOBI,
// OP_GS) on FP32 vectors with FP32 accumulation.
void launch_row_mp(int mode, int op, int G, int kind, const RowArgsMP &a, hipStream_t s);

// conversions
void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
void launch_to_f64(const float *src, double *dst, int64_t n, hipStream_t s);
void launch_fill_f32(float *x, float v, int64_t n, hipStream_t s);
void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s);
// row scales |a_ii| (per scalar row) from the FP64 diagonal blocks
void launch_row_scales(int mode, int n, const int *rowptr, const int *col, const double *val, int64_t nnz,
                       float *scale, hipStream_t s);
// planes: FP64 -> FP32, or FP64 -> BF16 divided by the scale of the entry's
// scalar row (rowid maps grouped rows to nodes, may be null)
void launch_planes_f32(const double *src, float *dst, int64_t count, hipStream_t s);
void launch_planes_bf16(int mode, int nrows, const int *rowptr, const int *rowid, const double *src,
                        int64_t nnz, const float *scale, uint16_t *dst, hipStream_t s);
// x = omega D^{-1} b over nodes [0, nn) (dinv planes dn apart) / x_i =
// D_i^{-1} b_i over rowid
void launch_jacobi_zero_mp(int mode, int64_t nn, int64_t dn, const float *dinv, const float *b, float omega,
                           float *x, hipStream_t s);
void launch_diag_solve_mp(int mode, int nrows, const int *rowid, const float *dinv, int64_t n, const float *b,
                          float *x, hipStream_t s);
// Y = M X with an FP32 or BF16 dense matrix (m x m, rows ld values apart, ld
// a multiple of 8 with zeros past m), nc = 1 or 3 components; M and X
// 16-byte aligned
void launch_dense_gemv_f32(const float *M, int m, int ld, int nc, const float *X, float *Y, hipStream_t s);
void launch_dense_gemv_bf16(const uint16_t *M, int m, int ld, int nc, const float *X, float *Y, hipStream_t s);
// dst = FP32 (kind VAL_F32) or BF16 (VAL_BF16, rounded once, ties to even)
// copy of the FP64 m x m src with rows ld values apart and zeros past m
void launch_dense_copy(const double *src, int m, int ld, int kind, void *dst, hipStream_t s);
// BF16 (round to nearest even) copy of FP64 values
void launch_to_bf16(const double *src, uint16_t *dst, int64_t n, hipStream_t s);

}  // namespace amgp2
