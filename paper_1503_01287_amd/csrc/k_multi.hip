// Kernels for blocks of K right-hand sides on one SPD hierarchy (multi.h):
// the row kernels of k_row.hip / k_mixed.hip with K interleaved vectors, so
// each stored entry (and its column index) is read once for all K, the
// dense coarse-end GEMV with K columns, and the Krylov vector work with one
// scalar per right-hand side.
#include <type_traits>

#include "common.h"
#include "multi.h"

namespace amgp2 {

constexpr int TB = 256;

template <int VK>
using vec_t = typename std::conditional<VK == MK_F64, double, float>::type;

template <int VK>
__device__ __forceinline__ vec_t<VK> ldv(const void *p, int64_t idx) {
    if constexpr (VK == MK_F64)
        return static_cast<const double *>(p)[idx];
    else if constexpr (VK == MK_F32)
        return static_cast<const float *>(p)[idx];
    else
        return __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t *>(p)[idx]) << 16);
}

template <int G, typename T>
__device__ __forceinline__ T gsum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// One group of G = E K lanes per row. Lane (e, r) = (lane / K, lane % K)
// walks the row's entries e, e + E, ... for right-hand side r, U entries per
// trip (their column indices, then their values and gathers, in flight
// together; entries past the row's end are skipped): the K lanes of one
// entry slot read its column index and values at the same addresses and the
// 3 K contiguous values of x at that column together (x at column j,
// component c, right-hand side r sits at (3 j + c) K + r). The 3 sums of
// every lane are reduced over the E slots in a fixed butterfly order, and the
// slot-0 lanes write their right-hand side's 3 outputs of the row.
template <int MODE, int E, int U, int OP, int VK, int K>
__global__ void __launch_bounds__(TB) k_mrow(const MRowArgs a) {
    using T = vec_t<VK>;
    constexpr int G = E * K;
    static_assert(G <= 64 && (64 % G) == 0, "a row group stays inside one wavefront");
    const int64_t t = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    const int g = static_cast<int>(t / G), lane = static_cast<int>(t % G);
    if (g >= a.nrows) return;  // whole groups leave together (G divides 64)
    const int e = lane / K, r = lane % K;
    const int i = a.rowid ? a.rowid[g] : g;
    const T *x = static_cast<const T *>(a.x);
    const T *b = static_cast<const T *>(a.b);
    T *y = static_cast<T *>(a.y);
    const T *D = static_cast<const T *>(a.dinv);
    const int64_t o0 = static_cast<int64_t>(3) * i * K + r;  // output (i, 0, r); (i, c, r) at o0 + c K
    constexpr bool NEEDS_B = OP == M_RESID || OP == M_JACOBI || OP == M_GS;
    constexpr bool NEEDS_D = OP == M_JACOBI || OP == M_GS;
    // the epilogue's row operands, loaded before the row's entries so that
    // their latency overlaps the row
    T b0 = T(0), b1 = T(0), b2 = T(0), w0 = T(0), w1 = T(0), w2 = T(0);
    T dm[MODE == 3 ? 9 : 1];
#pragma unroll
    for (int q = 0; q < (MODE == 3 ? 9 : 1); ++q) dm[q] = T(0);
    float q0 = 1.f, q1 = 1.f, q2 = 1.f;
    if (e == 0) {
        if constexpr (NEEDS_B) {
            b0 = b[o0];
            b1 = b[o0 + K];
            b2 = b[o0 + 2 * K];
        }
        if constexpr (NEEDS_D) {
            if constexpr (MODE == 3) {
#pragma unroll
                for (int q = 0; q < 9; ++q) dm[q] = D[q * a.dinv_n + i];
            } else {
                dm[0] = D[i];
            }
        }
        if constexpr (OP == M_SPMV_ADD || OP == M_GS || OP == M_JACOBI) {
            const T *own = OP == M_JACOBI ? x : y;
            w0 = own[o0];
            w1 = own[o0 + K];
            w2 = own[o0 + 2 * K];
        }
        if constexpr (VK == MK_BF16) {
            if constexpr (MODE == 3) {
                q0 = a.rscale[3 * i];
                q1 = a.rscale[3 * i + 1];
                q2 = a.rscale[3 * i + 2];
            } else {
                q0 = q1 = q2 = a.rscale[i];
            }
        }
    }
    T s0 = T(0), s1 = T(0), s2 = T(0);
    const int beg = a.rowptr[g], end = a.rowptr[g + 1];
    const int64_t nz = a.nnz;
    constexpr int NV = MODE == 3 ? 9 : 1;
    for (int k = beg + e; k < end; k += U * E) {
        int j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = k + u * E < end ? a.col[k + u * E] : -1;
        T v[U][NV], xv[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j[u] >= 0) {
#pragma unroll
                for (int q = 0; q < NV; ++q) v[u][q] = ldv<VK>(a.val, q * nz + k + u * E);
                const T *xj = x + static_cast<int64_t>(3) * j[u] * K + r;
                xv[u][0] = xj[0];
                xv[u][1] = xj[K];
                xv[u][2] = xj[2 * K];
            } else {
#pragma unroll
                for (int q = 0; q < NV; ++q) v[u][q] = T(0);
                xv[u][0] = xv[u][1] = xv[u][2] = T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (MODE == 3) {
                s0 += v[u][0] * xv[u][0] + v[u][1] * xv[u][1] + v[u][2] * xv[u][2];
                s1 += v[u][3] * xv[u][0] + v[u][4] * xv[u][1] + v[u][5] * xv[u][2];
                s2 += v[u][6] * xv[u][0] + v[u][7] * xv[u][1] + v[u][8] * xv[u][2];
            } else {
                s0 += v[u][0] * xv[u][0];
                s1 += v[u][0] * xv[u][1];
                s2 += v[u][0] * xv[u][2];
            }
        }
    }
    // over the entry slots: lanes of one right-hand side differ by multiples of K
#pragma unroll
    for (int o = G / 2; o >= K; o >>= 1) {
        s0 += __shfl_xor(s0, o, G);
        s1 += __shfl_xor(s1, o, G);
        s2 += __shfl_xor(s2, o, G);
    }
    if (e != 0) return;
    if constexpr (VK == MK_BF16) {
        s0 *= q0;
        s1 *= q1;
        s2 *= q2;
    }
    if (a.zero_out) {
        T *z = static_cast<T *>(a.zero_out);
        z[o0] = T(0);
        z[o0 + K] = T(0);
        z[o0 + 2 * K] = T(0);
    }
    T y0, y1, y2;
    if constexpr (OP == M_SPMV) {
        y0 = s0;
        y1 = s1;
        y2 = s2;
    } else if constexpr (OP == M_SPMV_ADD) {
        y0 = w0 + s0;
        y1 = w1 + s1;
        y2 = w2 + s2;
    } else if constexpr (OP == M_RESID) {
        y0 = b0 - s0;
        y1 = b1 - s1;
        y2 = b2 - s2;
    } else {
        const T r0 = b0 - s0, r1 = b1 - s1, r2 = b2 - s2;
        T d0, d1, d2;
        if constexpr (MODE == 3) {
            d0 = dm[0] * r0 + dm[1] * r1 + dm[2] * r2;
            d1 = dm[3] * r0 + dm[4] * r1 + dm[5] * r2;
            d2 = dm[6] * r0 + dm[7] * r1 + dm[8] * r2;
        } else {
            d0 = dm[0] * r0;
            d1 = dm[0] * r1;
            d2 = dm[0] * r2;
        }
        if constexpr (OP == M_JACOBI) {
            const T om = static_cast<T>(a.omega);
            y0 = w0 + om * d0;
            y1 = w1 + om * d1;
            y2 = w2 + om * d2;
        } else {  // M_GS, in place
            y0 = w0 + d0;
            y1 = w1 + d1;
            y2 = w2 + d2;
        }
    }
    y[o0] = y0;
    y[o0 + K] = y1;
    y[o0 + 2 * K] = y2;
}

// 16 lanes per row (E = 16 / K entry slots), 4 entries per slot and trip for
// scalar entries, 2 for 3x3 blocks: the fastest of the shapes measured on
// the 48^3 Laplacian's finest operator with 8 right-hand sides (E in 1..16,
// U in 1..8; 2- and 4-wide vector gathers per lane and per-XCD row chunks
// were slower)
template <int MODE, int OP, int VK, int K>
static void mrow_launch(const MRowArgs &a, hipStream_t s) {
    constexpr int G = 16, E = G / K, U = MODE == 3 ? 2 : 4;
    const int nb = ceil_div(static_cast<int64_t>(a.nrows) * G, TB);
    if (nb == 0) return;
    k_mrow<MODE, E, U, OP, VK, K><<<nb, TB, 0, s>>>(a);
}

template <int MODE, int VK, int K>
static void mrow_op(int op, const MRowArgs &a, hipStream_t s) {
    switch (op) {
        case M_SPMV: mrow_launch<MODE, M_SPMV, VK, K>(a, s); break;
        case M_SPMV_ADD: mrow_launch<MODE, M_SPMV_ADD, VK, K>(a, s); break;
        case M_RESID: mrow_launch<MODE, M_RESID, VK, K>(a, s); break;
        case M_JACOBI: mrow_launch<MODE, M_JACOBI, VK, K>(a, s); break;
        case M_GS: mrow_launch<MODE, M_GS, VK, K>(a, s); break;
        default: throw Error(AMG_EINVAL, "multi row kernel: unknown operation");
    }
}

template <int MODE, int VK>
static void mrow_k(int op, int K, const MRowArgs &a, hipStream_t s) {
    switch (K) {
        case 2: mrow_op<MODE, VK, 2>(op, a, s); break;
        case 4: mrow_op<MODE, VK, 4>(op, a, s); break;
        case 8: mrow_op<MODE, VK, 8>(op, a, s); break;
        case 16:
            // (one entry slot per row: the scalar FP64 operators of the
            // setup's blocked map assembly)
            if constexpr (MODE == 1 && VK == MK_F64) {
                mrow_op<MODE, VK, 16>(op, a, s);
                break;
            }
            [[fallthrough]];
        default: throw Error(AMG_EINVAL, "multi row kernel: K must be 2, 4 or 8 (16: scalar FP64 operators)");
    }
}

template <int MODE>
static void mrow_kind(int op, int kind, int K, const MRowArgs &a, hipStream_t s) {
    switch (kind) {
        case MK_F64: mrow_k<MODE, MK_F64>(op, K, a, s); break;
        case MK_F32: mrow_k<MODE, MK_F32>(op, K, a, s); break;
        case MK_BF16: mrow_k<MODE, MK_BF16>(op, K, a, s); break;
        default: throw Error(AMG_EINVAL, "multi row kernel: unknown value kind");
    }
}

void launch_mrow(int mode, int op, int kind, int K, const MRowArgs &a, hipStream_t s) {
    if (a.nrows <= 0) return;
    if (mode == 3)
        mrow_kind<3>(op, kind, K, a, s);
    else
        mrow_kind<1>(op, kind, K, a, s);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- diagonal solves
// one thread per (node, component, rhs)
template <int MODE, typename T>
__global__ void k_mdiag(int nrows, const int *rowid, const T *dinv, int64_t n, const T *b, T omega, int K, T *x) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (t >= static_cast<int64_t>(3) * K * nrows) return;
    const int64_t g = t / (3 * K);
    const int rem = static_cast<int>(t - g * 3 * K);
    const int c = rem / K, r = rem % K;
    const int64_t i = rowid ? rowid[g] : g;
    const int64_t base = 3 * i * K;
    T d;
    if constexpr (MODE == 3)
        d = dinv[(3 * c) * n + i] * b[base + r] + dinv[(3 * c + 1) * n + i] * b[base + K + r] +
            dinv[(3 * c + 2) * n + i] * b[base + 2 * K + r];
    else
        d = dinv[i] * b[base + c * K + r];
    x[base + c * K + r] = omega * d;
}

template <typename T>
static void mdiag(int mode, int K, int nrows, const int *rowid, const void *dinv, int64_t n, const void *b,
                  double omega, void *x, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(static_cast<int64_t>(3) * K * nrows, TB);
    if (mode == 3)
        k_mdiag<3, T><<<nb, TB, 0, s>>>(nrows, rowid, static_cast<const T *>(dinv), n, static_cast<const T *>(b),
                                         static_cast<T>(omega), K, static_cast<T *>(x));
    else
        k_mdiag<1, T><<<nb, TB, 0, s>>>(nrows, rowid, static_cast<const T *>(dinv), n, static_cast<const T *>(b),
                                         static_cast<T>(omega), K, static_cast<T *>(x));
    AMG_CHECK_LAUNCH();
}

void launch_mjacobi_zero(int mode, int kind, int K, int64_t nn, const void *dinv, const void *b, double omega,
                         void *x, hipStream_t s) {
    if (kind == MK_F64)
        mdiag<double>(mode, K, static_cast<int>(nn), nullptr, dinv, nn, b, omega, x, s);
    else
        mdiag<float>(mode, K, static_cast<int>(nn), nullptr, dinv, nn, b, omega, x, s);
}

void launch_mdiag_solve(int mode, int kind, int K, int nrows, const int *rowid, const void *dinv, int64_t n,
                        const void *b, void *x, hipStream_t s) {
    if (kind == MK_F64)
        mdiag<double>(mode, K, nrows, rowid, dinv, n, b, 1.0, x, s);
    else
        mdiag<float>(mode, K, nrows, rowid, dinv, n, b, 1.0, x, s);
}

// ---------------------------------------------------------------- dense coarse end
// Y = M X with NC columns (M's rows ld values apart): one wavefront per row
// of M, lane j walks columns j, j + 64, ... and keeps NC partial sums
template <int MK, int NC>
__global__ void __launch_bounds__(TB) k_mdense(const void *M, int m, int ld, const void *Xv, void *Yv) {
    using T = vec_t<MK>;
    const int row = blockIdx.x * (TB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const T *X = static_cast<const T *>(Xv);
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = T(0);
    const int64_t base = static_cast<int64_t>(row) * ld;
    for (int j = lane; j < m; j += 64) {
        const T v = ldv<MK>(M, base + j);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += v * X[static_cast<int64_t>(j) * NC + c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = gsum<64>(acc[c]);
    T *Y = static_cast<T *>(Yv);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (lane == c) Y[static_cast<int64_t>(row) * NC + c] = acc[c];
}

template <int MK>
static void mdense_nc(const void *M, int m, int ld, int nc, const void *X, void *Y, hipStream_t s) {
    const int nb = ceil_div(m, TB / 64);
    switch (nc) {
        case 2: k_mdense<MK, 2><<<nb, TB, 0, s>>>(M, m, ld, X, Y); break;
        case 4: k_mdense<MK, 4><<<nb, TB, 0, s>>>(M, m, ld, X, Y); break;
        case 6: k_mdense<MK, 6><<<nb, TB, 0, s>>>(M, m, ld, X, Y); break;
        case 8: k_mdense<MK, 8><<<nb, TB, 0, s>>>(M, m, ld, X, Y); break;
        case 12: k_mdense<MK, 12><<<nb, TB, 0, s>>>(M, m, ld, X, Y); break;
        case 24: k_mdense<MK, 24><<<nb, TB, 0, s>>>(M, m, ld, X, Y); break;
        default: throw Error(AMG_EINVAL, "multi dense kernel: unsupported column count");
    }
}

void launch_mdense(int mkind, const void *M, int m, int ld, int nc, const void *X, void *Y, hipStream_t s) {
    if (m <= 0) return;
    AMG_REQUIRE(ld >= m, AMG_EINVAL, "multi dense kernel: row stride below m");
    switch (mkind) {
        case MK_F64: mdense_nc<MK_F64>(M, m, ld, nc, X, Y, s); break;
        case MK_F32: mdense_nc<MK_F32>(M, m, ld, nc, X, Y, s); break;
        default: mdense_nc<MK_BF16>(M, m, ld, nc, X, Y, s); break;
    }
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- Krylov vectors
constexpr int MDOT_MAX_BLOCKS = 1024;

int mdot_blocks(int64_t nd) {
    const int64_t nb = (nd + TB - 1) / TB;
    return static_cast<int>(nb < MDOT_MAX_BLOCKS ? (nb > 0 ? nb : 1) : MDOT_MAX_BLOCKS);
}

struct DotPtrs {
    const double *a[3];
    const double *b[3];
};

// per block: sums over the dofs d = t, t + stride, ... (a fixed assignment),
// then a fixed-order tree over the block; partial[blk * np K + p K + r]
template <int NP, int K>
__global__ void __launch_bounds__(TB) k_mdot(DotPtrs q, int64_t nd, double *partial) {
    __shared__ double red[NP * K][TB / 64];
    double acc[NP][K];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < K; ++r) acc[p][r] = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * TB;
    for (int64_t d = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x; d < nd; d += stride)
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < K; ++r) acc[p][r] += q.a[p][d * K + r] * q.b[p][d * K + r];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const double v = gsum<64>(acc[p][r]);
            if (lane == 0) red[p * K + r][w] = v;
        }
    __syncthreads();
    if (threadIdx.x < NP * K) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < TB / 64; ++u) v += red[threadIdx.x][u];
        partial[static_cast<int64_t>(blockIdx.x) * NP * K + threadIdx.x] = v;
    }
}

// out[o] = sum of partial[blk][o] over the nb blocks: one workgroup per
// output; thread u sums blocks u, u + TB, ... in order, then a fixed-order
// tree over the workgroup
__global__ void __launch_bounds__(TB) k_mdot_reduce(const double *partial, int nb, int no, double *out) {
    __shared__ double red[TB / 64];
    const int o = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += TB) v += partial[static_cast<int64_t>(b) * no + o];
    v = gsum<64>(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w = 0.0;
#pragma unroll
        for (int u = 0; u < TB / 64; ++u) w += red[u];
        out[o] = w;
    }
}

template <int NP>
static void mdot_np(int K, int nb, const DotPtrs &q, int64_t nd, double *partial, hipStream_t s) {
    switch (K) {
        case 2: k_mdot<NP, 2><<<nb, TB, 0, s>>>(q, nd, partial); break;
        case 4: k_mdot<NP, 4><<<nb, TB, 0, s>>>(q, nd, partial); break;
        case 8: k_mdot<NP, 8><<<nb, TB, 0, s>>>(q, nd, partial); break;
        default: throw Error(AMG_EINVAL, "multi dot: K must be 2, 4 or 8");
    }
}

void launch_mdot(int np, int K, int64_t nd, const double *const *a, const double *const *b, double *partial,
                 double *out, hipStream_t s) {
    AMG_REQUIRE(np >= 1 && np <= 3, AMG_EINVAL, "multi dot: 1 to 3 pairs");
    DotPtrs q{};
    for (int p = 0; p < np; ++p) {
        q.a[p] = a[p];
        q.b[p] = b[p];
    }
    const int nb = mdot_blocks(nd);
    switch (np) {
        case 1: mdot_np<1>(K, nb, q, nd, partial, s); break;
        case 2: mdot_np<2>(K, nb, q, nd, partial, s); break;
        default: mdot_np<3>(K, nb, q, nd, partial, s); break;
    }
    AMG_CHECK_LAUNCH();
    const int no = np * K;
    k_mdot_reduce<<<no, TB, 0, s>>>(partial, nb, no, out);
    AMG_CHECK_LAUNCH();
}

__global__ void k_mlincomb(int K, int64_t n, double *y, const double *cy, const double *x, const double *cx) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * TB) {
        const int r = static_cast<int>(e % K);
        y[e] = cy[r] * y[e] + cx[r] * x[e];
    }
}

static int grid_e(int64_t n) {
    int64_t nb = (n + TB - 1) / TB;
    return static_cast<int>(nb > 8192 ? 8192 : (nb > 0 ? nb : 1));
}

void launch_mlincomb(int K, int64_t nd, double *y, const double *cy, const double *x, const double *cx,
                     hipStream_t s) {
    if (nd <= 0) return;
    k_mlincomb<<<grid_e(nd * K), TB, 0, s>>>(K, nd * K, y, cy, x, cx);
    AMG_CHECK_LAUNCH();
}

// the caller's nvec vectors <-> the interleaved block of K >= nvec (the
// block's other columns are zero going in, dropped coming out)
__global__ void k_interleave(int K, int nvec, int64_t nd, const double *src, double *dst, int to) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x; e < nd * K;
         e += static_cast<int64_t>(gridDim.x) * TB) {
        const int64_t d = e / K;
        const int r = static_cast<int>(e - d * K);
        if (to)
            dst[e] = r < nvec ? src[static_cast<int64_t>(r) * nd + d] : 0.0;
        else if (r < nvec)
            dst[static_cast<int64_t>(r) * nd + d] = src[e];
    }
}

void launch_interleave(int K, int nvec, int64_t nd, const double *src, double *dst, bool to_interleaved,
                       hipStream_t s) {
    if (nd <= 0) return;
    k_interleave<<<grid_e(nd * K), TB, 0, s>>>(K, nvec, nd, src, dst, to_interleaved ? 1 : 0);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
