// Kernels of the mixed-precision cycle: the row kernels of k_row.hip on FP32
// vectors with FP32 or BF16 (+ per-row FP32 scale) operator values, and the
// conversions that build those copies. A 3x3 block costs 40 bytes in FP32
// and 22 bytes in BF16 (76 in FP64), so the bandwidth-bound passes move
// 1.9x / 3.5x fewer bytes.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "mixed.h"

namespace amgp2 {

constexpr int MBLOCK = 256;

__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }

// FP64 -> BF16, rounded once to the nearest value with 8 significant bits
// (ties to even) straight from the FP64 value: the low 45 of FP64's 52
// fraction bits are dropped with round-half-even, and the result, which has
// 8 significant bits and an exponent inside FP32's normal range for the
// scaled operator values, converts to FP32 exactly; its high 16 bits are the
// BF16 value. (Rounding through FP32 first would round twice.)
__device__ __forceinline__ uint16_t f64_to_bf16(double d) {
    uint64_t u = static_cast<uint64_t>(__double_as_longlong(d));
    if ((u & 0x7fffffffffffffffull) > 0x7ff0000000000000ull) return 0x7fc0;  // NaN
    u += 0x00000fffffffffffull + ((u >> 45) & 1ull);
    u &= ~0x00001fffffffffffull;
    const float f = static_cast<float>(__longlong_as_double(static_cast<long long>(u)));
    return static_cast<uint16_t>(__float_as_uint(f) >> 16);
}

template <int G>
__device__ __forceinline__ float group_sum_f(float v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

template <int KIND>
__device__ __forceinline__ float ld(const void *p, int64_t idx) {
    if constexpr (KIND == VAL_F32)
        return static_cast<const float *>(p)[idx];
    else
        return bf16_to_f32(static_cast<const uint16_t *>(p)[idx]);
}

// s += A_k x_j for entry k (a 3x3 block of nine planes, or a scalar that
// multiplies every component)
template <int MODE, int KIND>
__device__ __forceinline__ void acc_entry(const void *val, int64_t nz, int k, float x0, float x1, float x2,
                                          float &s0, float &s1, float &s2) {
    if constexpr (MODE == 3) {
        s0 += ld<KIND>(val, k) * x0 + ld<KIND>(val, nz + k) * x1 + ld<KIND>(val, 2 * nz + k) * x2;
        s1 += ld<KIND>(val, 3 * nz + k) * x0 + ld<KIND>(val, 4 * nz + k) * x1 + ld<KIND>(val, 5 * nz + k) * x2;
        s2 += ld<KIND>(val, 6 * nz + k) * x0 + ld<KIND>(val, 7 * nz + k) * x1 + ld<KIND>(val, 8 * nz + k) * x2;
    } else {
        const float v = ld<KIND>(val, k);
        s0 += v * x0;
        s1 += v * x1;
        s2 += v * x2;
    }
}

// U entries per lane and loop trip as in k_row (the same result for every U)
template <int MODE, int G, int OP, int KIND, int U>
__global__ void __launch_bounds__(MBLOCK) k_row_mp(const RowArgsMP a) {
    const int64_t blk = a.xcd_chunks ? xcd_chunk_block() : static_cast<int64_t>(blockIdx.x);
    const int64_t t = blk * MBLOCK + threadIdx.x;
    const int g = static_cast<int>(t / G);
    const int lane = static_cast<int>(t % G);
    const bool active = g < a.nrows;
    constexpr bool NEEDS_B = OP == OP_RESID || OP == OP_JACOBI || OP == OP_GS;
    constexpr bool NEEDS_D = OP == OP_JACOBI || OP == OP_GS;
    constexpr bool NEEDS_OWN = OP == OP_SPMV_ADD || OP == OP_JACOBI || OP == OP_GS;
    // Row-local operands of the epilogue (right-hand side, inverted diagonal
    // block, own entry, BF16 row scales) are loaded before the row's matrix
    // entries so that their latency overlaps the row instead of following
    // the group reduction.
    const int i = active ? (a.rowid ? a.rowid[g] : g) : 0;
    const bool ep = active && lane < 3;
    const int c = ep ? lane : 0;
    float b0 = 0.f, b1 = 0.f, b2 = 0.f, d0 = 0.f, d1 = 0.f, d2 = 0.f, own = 0.f;
    float q0 = 1.f, q1 = 1.f, q2 = 1.f;
    if (ep) {
        if constexpr (NEEDS_B) {
            b0 = a.b[3 * i];
            b1 = a.b[3 * i + 1];
            b2 = a.b[3 * i + 2];
        }
        if constexpr (NEEDS_D) {
            if constexpr (MODE == 3) {
                const float *D = a.dinv + i;
                const int64_t dn = a.dinv_n;
                d0 = D[(3 * c) * dn];
                d1 = D[(3 * c + 1) * dn];
                d2 = D[(3 * c + 2) * dn];
            } else {
                d0 = a.dinv[i];
            }
        }
        if constexpr (NEEDS_OWN) own = OP == OP_JACOBI ? a.x[3 * i + c] : a.y[3 * i + c];
        if constexpr (KIND == VAL_BF16) {
            if constexpr (MODE == 3) {
                q0 = a.rscale[3 * i];
                q1 = a.rscale[3 * i + 1];
                q2 = a.rscale[3 * i + 2];
            } else {
                q0 = q1 = q2 = a.rscale[i];
            }
        }
    }
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    if (active) {
        const int beg = a.rowptr[g], end = a.rowptr[g + 1];
        const int64_t nz = a.nnz;
        if constexpr (U == 1) {
            for (int k = beg + lane; k < end; k += G) {
                const int j = a.col[k];
                const float x0 = a.x[3 * j], x1 = a.x[3 * j + 1], x2 = a.x[3 * j + 2];
                acc_entry<MODE, KIND>(a.val, nz, k, x0, x1, x2, s0, s1, s2);
            }
        } else {
            for (int k = beg + lane; k < end; k += U * G) {
                int j[U];
#pragma unroll
                for (int u = 0; u < U; ++u) j[u] = k + u * G < end ? a.col[k + u * G] : -1;
                float xv[U][3];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int jj = j[u] >= 0 ? j[u] : 0;
                    if (j[u] >= 0) {
                        xv[u][0] = a.x[3 * jj];
                        xv[u][1] = a.x[3 * jj + 1];
                        xv[u][2] = a.x[3 * jj + 2];
                    } else {
                        xv[u][0] = xv[u][1] = xv[u][2] = 0.f;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j[u] >= 0)
                        acc_entry<MODE, KIND>(a.val, nz, k + u * G, xv[u][0], xv[u][1], xv[u][2], s0, s1, s2);
            }
        }
    }
    s0 = group_sum_f<G>(s0);
    s1 = group_sum_f<G>(s1);
    s2 = group_sum_f<G>(s2);
    if (!ep) return;
    if constexpr (KIND == VAL_BF16) {
        s0 *= q0;
        s1 *= q1;
        s2 *= q2;
    }
    const float sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
    if (a.zero_out) a.zero_out[3 * i + c] = 0.f;
    if constexpr (OP == OP_SPMV) {
        a.y[3 * i + c] = sc;
    } else if constexpr (OP == OP_SPMV_ADD) {
        a.y[3 * i + c] = own + sc;
    } else if constexpr (OP == OP_RESID) {
        a.y[3 * i + c] = (c == 0 ? b0 : (c == 1 ? b1 : b2)) - sc;
    } else {
        const float r0 = b0 - s0, r1 = b1 - s1, r2 = b2 - s2;
        float d;
        if constexpr (MODE == 3)
            d = d0 * r0 + d1 * r1 + d2 * r2;
        else
            d = d0 * (c == 0 ? r0 : (c == 1 ? r1 : r2));
        if constexpr (OP == OP_JACOBI)
            a.y[3 * i + c] = own + a.omega * d;
        else  // OP_GS: in place (a.y aliases a.x)
            a.y[3 * i + c] = own + d;
    }
}

template <int MODE, int G, int KIND>
static void launch_mp_g(int op, const RowArgsMP &a, hipStream_t s) {
    int nb = ceil_div(static_cast<int64_t>(a.nrows) * G, MBLOCK);
    if (nb == 0) return;
    if (a.xcd_chunks) nb = (nb + 7) / 8 * 8;
    AMG_REQUIRE(a.trip == 1 || a.trip == 2 || a.trip == 4, AMG_EINVAL,
                "mixed row kernel: 1, 2 or 4 entries per trip");
#define AMG_MP_CASE(OPC)                                                             \
    case OPC:                                                                        \
        if (a.trip == 4) k_row_mp<MODE, G, OPC, KIND, 4><<<nb, MBLOCK, 0, s>>>(a);   \
        else if (a.trip == 2) k_row_mp<MODE, G, OPC, KIND, 2><<<nb, MBLOCK, 0, s>>>(a); \
        else k_row_mp<MODE, G, OPC, KIND, 1><<<nb, MBLOCK, 0, s>>>(a);               \
        break;
    switch (op) {
        case OP_SPMV: k_row_mp<MODE, G, OP_SPMV, KIND, 1><<<nb, MBLOCK, 0, s>>>(a); break;
        case OP_SPMV_ADD: k_row_mp<MODE, G, OP_SPMV_ADD, KIND, 1><<<nb, MBLOCK, 0, s>>>(a); break;
        AMG_MP_CASE(OP_RESID)
        AMG_MP_CASE(OP_JACOBI)
        AMG_MP_CASE(OP_GS)
        default: throw Error(AMG_EINVAL, "mixed row kernel: unsupported operation");
    }
#undef AMG_MP_CASE
    AMG_CHECK_LAUNCH();
}

template <int MODE, int KIND>
static void launch_mp_m(int op, int G, const RowArgsMP &a, hipStream_t s) {
    switch (G) {
        case 4: launch_mp_g<MODE, 4, KIND>(op, a, s); break;
        case 8: launch_mp_g<MODE, 8, KIND>(op, a, s); break;
        case 16: launch_mp_g<MODE, 16, KIND>(op, a, s); break;
        case 32: launch_mp_g<MODE, 32, KIND>(op, a, s); break;
        case 64: launch_mp_g<MODE, 64, KIND>(op, a, s); break;
        default: throw Error(AMG_EINVAL, "mixed row kernel: unsupported group size");
    }
}

void launch_row_mp(int mode, int op, int G, int kind, const RowArgsMP &a, hipStream_t s) {
    if (mode == 3) {
        if (kind == VAL_F32) launch_mp_m<3, VAL_F32>(op, G, a, s);
        else launch_mp_m<3, VAL_BF16>(op, G, a, s);
    } else {
        if (kind == VAL_F32) launch_mp_m<1, VAL_F32>(op, G, a, s);
        else launch_mp_m<1, VAL_BF16>(op, G, a, s);
    }
}

// ---------------------------------------------------------------- conversions
static int grid_n(int64_t n) {
    int64_t nb = (n + MBLOCK - 1) / MBLOCK;
    if (nb > 8192) nb = 8192;
    return static_cast<int>(nb < 1 ? 1 : nb);
}

__global__ void k_to_f32(const double *src, float *dst, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * MBLOCK)
        dst[i] = static_cast<float>(src[i]);
}
__global__ void k_to_f64(const float *src, double *dst, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * MBLOCK)
        dst[i] = static_cast<double>(src[i]);
}
__global__ void k_fill_f32(float *x, float v, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * MBLOCK)
        x[i] = v;
}
__global__ void k_copy_f32(float *d, const float *src, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * MBLOCK)
        d[i] = src[i];
}

void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_to_f32<<<grid_n(n), MBLOCK, 0, s>>>(src, dst, n);
    AMG_CHECK_LAUNCH();
}
void launch_to_f64(const float *src, double *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_to_f64<<<grid_n(n), MBLOCK, 0, s>>>(src, dst, n);
    AMG_CHECK_LAUNCH();
}
void launch_fill_f32(float *x, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_f32<<<grid_n(n), MBLOCK, 0, s>>>(x, v, n);
    AMG_CHECK_LAUNCH();
}
void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_copy_f32<<<grid_n(n), MBLOCK, 0, s>>>(dst, src, n);
    AMG_CHECK_LAUNCH();
}
void launch_planes_f32(const double *src, float *dst, int64_t count, hipStream_t s) {
    launch_to_f32(src, dst, count, s);
}

template <int MODE>
__global__ void k_row_scales(int n, const int *rowptr, const int *col, const double *val, int64_t nnz,
                             float *scale) {
    const int i = blockIdx.x * MBLOCK + threadIdx.x;
    if (i >= n) return;
    int kd = -1;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (col[k] == i) { kd = k; break; }
    for (int r = 0; r < MODE; ++r) {
        double d = kd >= 0 ? fabs(val[static_cast<int64_t>(r * MODE + r) * nnz + kd]) : 0.0;
        if (d == 0.0) {
            // no usable diagonal: the row's largest magnitude
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
                for (int c = 0; c < MODE; ++c) d = fmax(d, fabs(val[static_cast<int64_t>(r * MODE + c) * nnz + k]));
            if (d == 0.0) d = 1.0;
        }
        scale[MODE * i + r] = static_cast<float>(d);
    }
}

void launch_row_scales(int mode, int n, const int *rowptr, const int *col, const double *val, int64_t nnz,
                       float *scale, hipStream_t s) {
    if (n <= 0) return;
    if (mode == 3)
        k_row_scales<3><<<ceil_div(n, MBLOCK), MBLOCK, 0, s>>>(n, rowptr, col, val, nnz, scale);
    else
        k_row_scales<1><<<ceil_div(n, MBLOCK), MBLOCK, 0, s>>>(n, rowptr, col, val, nnz, scale);
    AMG_CHECK_LAUNCH();
}

// one wavefront per row: entry k of (grouped) row g belongs to node rowid[g]
template <int MODE>
__global__ void k_planes_bf16(int nrows, const int *rowptr, const int *rowid, const double *src, int64_t nnz,
                              const float *scale, uint16_t *dst) {
    const int g = blockIdx.x * (MBLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= nrows) return;
    const int i = rowid ? rowid[g] : g;
    for (int k = rowptr[g] + lane; k < rowptr[g + 1]; k += 64) {
#pragma unroll
        for (int p = 0; p < MODE * MODE; ++p) {
            const int r = p / MODE;
            const double v = src[static_cast<int64_t>(p) * nnz + k] / static_cast<double>(scale[MODE * i + r]);
            dst[static_cast<int64_t>(p) * nnz + k] = f64_to_bf16(v);
        }
    }
}

void launch_planes_bf16(int mode, int nrows, const int *rowptr, const int *rowid, const double *src, int64_t nnz,
                        const float *scale, uint16_t *dst, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(nrows, MBLOCK / 64);
    if (mode == 3)
        k_planes_bf16<3><<<nb, MBLOCK, 0, s>>>(nrows, rowptr, rowid, src, nnz, scale, dst);
    else
        k_planes_bf16<1><<<nb, MBLOCK, 0, s>>>(nrows, rowptr, rowid, src, nnz, scale, dst);
    AMG_CHECK_LAUNCH();
}

// x = omega D^{-1} b on rows [0, nn); dn is the plane stride of dinv
template <int MODE>
__global__ void k_jacobi_zero_mp(int64_t nn, int64_t dn, const float *dinv, const float *b, float omega, float *x) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x;
    if (t >= 3 * nn) return;
    const int64_t i = t / 3;
    const int c = static_cast<int>(t % 3);
    float d;
    if constexpr (MODE == 3)
        d = dinv[(3 * c) * dn + i] * b[3 * i] + dinv[(3 * c + 1) * dn + i] * b[3 * i + 1] +
            dinv[(3 * c + 2) * dn + i] * b[3 * i + 2];
    else
        d = dinv[i] * b[t];
    x[t] = omega * d;
}

void launch_jacobi_zero_mp(int mode, int64_t nn, int64_t dn, const float *dinv, const float *b, float omega,
                           float *x, hipStream_t s) {
    if (nn <= 0) return;
    AMG_REQUIRE(dn >= nn, AMG_EINVAL, "jacobi_zero_mp: plane stride below the row count");
    const int nb = ceil_div(3 * nn, MBLOCK);
    if (mode == 3)
        k_jacobi_zero_mp<3><<<nb, MBLOCK, 0, s>>>(nn, dn, dinv, b, omega, x);
    else
        k_jacobi_zero_mp<1><<<nb, MBLOCK, 0, s>>>(nn, dn, dinv, b, omega, x);
    AMG_CHECK_LAUNCH();
}

template <int MODE>
__global__ void k_diag_solve_mp(int nrows, const int *rowid, const float *dinv, int64_t n, const float *b, float *x) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x;
    if (t >= 3 * static_cast<int64_t>(nrows)) return;
    const int i = rowid[t / 3];
    const int c = static_cast<int>(t % 3);
    if constexpr (MODE == 3)
        x[3 * i + c] = dinv[(3 * c) * n + i] * b[3 * i] + dinv[(3 * c + 1) * n + i] * b[3 * i + 1] +
                       dinv[(3 * c + 2) * n + i] * b[3 * i + 2];
    else
        x[3 * i + c] = dinv[i] * b[3 * i + c];
}

void launch_diag_solve_mp(int mode, int nrows, const int *rowid, const float *dinv, int64_t n, const float *b,
                          float *x, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(3 * static_cast<int64_t>(nrows), MBLOCK);
    if (mode == 3)
        k_diag_solve_mp<3><<<nb, MBLOCK, 0, s>>>(nrows, rowid, dinv, n, b, x);
    else
        k_diag_solve_mp<1><<<nb, MBLOCK, 0, s>>>(nrows, rowid, dinv, n, b, x);
    AMG_CHECK_LAUNCH();
}

// y = M x for a dense m x m operator applied to nc (1 or 3) components, M in
// FP32 or BF16 with rows ld values apart (ld a multiple of 8, the values
// past m zero), FP32 accumulation, one wavefront per row. A lane reads 16
// bytes of the row (4 FP32 or 8 BF16 values) and the matching entries of x
// as 16-byte loads per chunk, two chunks per trip.
template <int KIND, int NC>
__global__ void __launch_bounds__(MBLOCK) k_dense_gemv_mp(const void *M, int m, int ld, const float *X, float *Y) {
    constexpr int CV = KIND == VAL_F32 ? 4 : 8;  // values per 16-byte chunk
    constexpr int VB = KIND == VAL_F32 ? 4 : 2;  // bytes per value
    const int row = blockIdx.x * (MBLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const unsigned char *Mr = static_cast<const unsigned char *>(M) + static_cast<int64_t>(row) * ld * VB;
    float acc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = 0.f;
    for (int c0 = CV * lane; c0 < m; c0 += 2 * 64 * CV) {
        uint4 w[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = c0 + h * 64 * CV;
            if (c < m) w[h] = *reinterpret_cast<const uint4 *>(Mr + static_cast<int64_t>(c) * VB);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = c0 + h * 64 * CV;
            if (c >= m) continue;
            const uint32_t u[4] = {w[h].x, w[h].y, w[h].z, w[h].w};
            float v[CV];
#pragma unroll
            for (int e = 0; e < CV; ++e) {
                if constexpr (KIND == VAL_F32)
                    v[e] = __uint_as_float(u[e]);
                else
                    v[e] = __uint_as_float((e & 1) ? (u[e >> 1] & 0xffff0000u) : (u[e >> 1] << 16));
            }
            if (c + CV <= m) {
                float xv[CV * NC];
                const float4 *xp = reinterpret_cast<const float4 *>(X + static_cast<int64_t>(c) * NC);
#pragma unroll
                for (int t = 0; t < CV * NC / 4; ++t) {
                    const float4 f = xp[t];
                    xv[4 * t] = f.x;
                    xv[4 * t + 1] = f.y;
                    xv[4 * t + 2] = f.z;
                    xv[4 * t + 3] = f.w;
                }
#pragma unroll
                for (int e = 0; e < CV; ++e)
#pragma unroll
                    for (int q = 0; q < NC; ++q) acc[q] += v[e] * xv[e * NC + q];
            } else {
#pragma unroll
                for (int e = 0; e < CV; ++e)
                    if (c + e < m)
#pragma unroll
                        for (int q = 0; q < NC; ++q) acc[q] += v[e] * X[static_cast<int64_t>(c + e) * NC + q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = group_sum_f<64>(acc[q]);
    if (lane < NC) {
        float out = acc[0];
#pragma unroll
        for (int q = 1; q < NC; ++q)
            if (lane == q) out = acc[q];
        Y[static_cast<int64_t>(row) * NC + lane] = out;
    }
}

template <int KIND>
static void launch_dense_mp(const void *M, int m, int ld, int nc, const float *X, float *Y, hipStream_t s) {
    if (m <= 0) return;
    AMG_REQUIRE(nc == 1 || nc == 3, AMG_EINVAL, "dense GEMV: 1 or 3 components");
    AMG_REQUIRE(ld >= m && ld % 8 == 0, AMG_EINVAL, "dense GEMV: row stride must be >= m and a multiple of 8");
    AMG_REQUIRE((reinterpret_cast<uintptr_t>(M) | reinterpret_cast<uintptr_t>(X)) % 16 == 0, AMG_EINVAL,
                "dense GEMV: operator and input must be 16-byte aligned");
    if (nc == 1)
        k_dense_gemv_mp<KIND, 1><<<ceil_div(m, MBLOCK / 64), MBLOCK, 0, s>>>(M, m, ld, X, Y);
    else
        k_dense_gemv_mp<KIND, 3><<<ceil_div(m, MBLOCK / 64), MBLOCK, 0, s>>>(M, m, ld, X, Y);
    AMG_CHECK_LAUNCH();
}

void launch_dense_gemv_f32(const float *M, int m, int ld, int nc, const float *X, float *Y, hipStream_t s) {
    launch_dense_mp<VAL_F32>(M, m, ld, nc, X, Y, s);
}

void launch_dense_gemv_bf16(const uint16_t *M, int m, int ld, int nc, const float *X, float *Y, hipStream_t s) {
    launch_dense_mp<VAL_BF16>(M, m, ld, nc, X, Y, s);
}

// dst (rows ld apart, zero past m) = rounded copy of the FP64 m x m src
template <int KIND>
__global__ void k_dense_copy(const double *src, int m, int ld, void *dst) {
    const int64_t n = static_cast<int64_t>(m) * ld;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * MBLOCK) {
        const int64_t r = i / ld;
        const int c = static_cast<int>(i - r * ld);
        const double v = c < m ? src[r * m + c] : 0.0;
        if constexpr (KIND == VAL_F32)
            static_cast<float *>(dst)[i] = static_cast<float>(v);
        else
            static_cast<uint16_t *>(dst)[i] = f64_to_bf16(v);
    }
}

void launch_dense_copy(const double *src, int m, int ld, int kind, void *dst, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(m) * ld;
    if (n <= 0) return;
    const int nb = static_cast<int>(std::min<int64_t>(4096, (n + MBLOCK - 1) / MBLOCK));
    if (kind == VAL_F32)
        k_dense_copy<VAL_F32><<<nb, MBLOCK, 0, s>>>(src, m, ld, dst);
    else
        k_dense_copy<VAL_BF16><<<nb, MBLOCK, 0, s>>>(src, m, ld, dst);
    AMG_CHECK_LAUNCH();
}

__global__ void k_to_bf16(const double *src, uint16_t *dst, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * MBLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * MBLOCK)
        dst[i] = f64_to_bf16(src[i]);
}

void launch_to_bf16(const double *src, uint16_t *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = std::min<int64_t>(4096, (n + MBLOCK - 1) / MBLOCK);
    k_to_bf16<<<static_cast<int>(nb), MBLOCK, 0, s>>>(src, dst, n);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
