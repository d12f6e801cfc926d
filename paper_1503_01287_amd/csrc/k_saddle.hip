// Saddle-point kernels (see saddle.h). Like the velocity row kernels these
// are bandwidth bound: B holds 1x3 blocks (28 bytes per entry in FP64), C
// scalars (12 bytes); the vectors they gather are small.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "saddle.h"

namespace amgp2 {

constexpr int SB = 256;

template <int G, typename T>
__device__ __forceinline__ T gsum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

template <typename T, int BR, int BC, int G, int OP>
__global__ void __launch_bounds__(SB) k_blk(const BlkArgsT<T> a) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x;
    const int i = static_cast<int>(t / G);
    const int lane = static_cast<int>(t % G);
    const bool active = i < a.nrows;
    // the epilogue's row-local operands are loaded before the row's entries
    // so that their latency overlaps the row
    const bool ep = active && lane < BR;
    const int64_t o = static_cast<int64_t>(BR) * i + (ep ? lane : 0);
    T bo = T(0), yo = T(0), ds = T(0);
    if (ep) {
        if constexpr (OP == BLK_RESID || OP == BLK_SGS_P) bo = a.b[o];
        if constexpr (OP == BLK_ADD || OP == BLK_SUB) yo = a.y[o];
        if constexpr (OP == BLK_SGS_P) yo = a.y_zero ? T(0) : a.y[o];
        if constexpr (OP == BLK_SGS_P) ds = a.dscale[i];
        if constexpr (OP == BLK_ADD_SCALED) {
            bo = a.b[o];
            yo = a.y_zero ? T(0) : a.y[o];
            ds = a.dscale[o];
        }
    }
    T s[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) s[r] = T(0);
    if (active) {
        const int64_t nz = a.nnz;
        const int beg = a.rowptr[i], end = a.rowptr[i + 1];
        for (int k = beg + lane; k < end; k += G) {
            const int j = a.col[k];
            T xv[BC];
#pragma unroll
            for (int c = 0; c < BC; ++c) xv[c] = a.x[BC * j + c];
#pragma unroll
            for (int r = 0; r < BR; ++r)
#pragma unroll
                for (int c = 0; c < BC; ++c) s[r] += a.val[(r * BC + c) * nz + k] * xv[c];
        }
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) s[r] = gsum<G>(s[r]);
    // the fused scalar C row (a uniform choice over the grid)
    T sc = T(0);
    if constexpr (BR == 1 && (OP == BLK_RESID || OP == BLK_SPMV)) {
        if (a.c_rowptr) {
            if (active) {
                const int cb = a.c_rowptr[i], ce = a.c_rowptr[i + 1];
                for (int k = cb + lane; k < ce; k += G) sc += a.c_val[k] * a.c_x[a.c_col[k]];
            }
            sc = gsum<G>(sc);
        }
    }
    if (!ep) return;
    const int r = lane;
    T sv = s[0];
#pragma unroll
    for (int q = 1; q < BR; ++q)
        if (r == q) sv = s[q];
    if constexpr (OP == BLK_SPMV) {
        T v = sv;
        if constexpr (BR == 1)
            if (a.c_rowptr) v = v + a.c_sign * sc;
        a.y[o] = v;
    } else if constexpr (OP == BLK_ADD) {
        a.y[o] = yo + sv;
    } else if constexpr (OP == BLK_SUB) {
        a.y[o] = yo - sv;
    } else if constexpr (OP == BLK_RESID) {
        T v = bo - sv;
        if constexpr (BR == 1)
            if (a.c_rowptr) v = v + a.c_sign * sc;
        a.y[o] = v;
    } else if constexpr (OP == BLK_ADD_SCALED) {
        a.y[o] = yo + ds * (bo + sv);
    } else {
        a.y[o] = yo + a.omega * ds * (sv - bo);
    }
}

template <typename T, int BR, int BC, int G>
static void launch_blk_g(int op, const BlkArgsT<T> &a, hipStream_t s) {
    const int nb = ceil_div(static_cast<int64_t>(a.nrows) * G, SB);
    if (nb == 0) return;
    AMG_REQUIRE(!a.c_rowptr || (BR == 1 && (op == BLK_RESID || op == BLK_SPMV) && a.c_col && a.c_val && a.c_x),
                AMG_EINVAL, "block kernel: a fused C row needs 1-row blocks and BLK_RESID or BLK_SPMV");
    switch (op) {
        case BLK_SPMV: k_blk<T, BR, BC, G, BLK_SPMV><<<nb, SB, 0, s>>>(a); break;
        case BLK_ADD: k_blk<T, BR, BC, G, BLK_ADD><<<nb, SB, 0, s>>>(a); break;
        case BLK_SUB: k_blk<T, BR, BC, G, BLK_SUB><<<nb, SB, 0, s>>>(a); break;
        case BLK_RESID: k_blk<T, BR, BC, G, BLK_RESID><<<nb, SB, 0, s>>>(a); break;
        case BLK_SGS_P:
            if constexpr (BR == 1) {
                k_blk<T, BR, BC, G, BLK_SGS_P><<<nb, SB, 0, s>>>(a);
                break;
            }
            throw Error(AMG_EINVAL, "block kernel: BLK_SGS_P needs 1-row blocks");
        case BLK_ADD_SCALED:
            if constexpr (BR == 3 && BC == 1) {
                k_blk<T, BR, BC, G, BLK_ADD_SCALED><<<nb, SB, 0, s>>>(a);
                break;
            }
            throw Error(AMG_EINVAL, "block kernel: BLK_ADD_SCALED needs 3x1 blocks");
        default: throw Error(AMG_EINVAL, "block kernel: unsupported operation");
    }
    AMG_CHECK_LAUNCH();
}

template <typename T, int BR, int BC>
static void launch_blk_m(int op, int G, const BlkArgsT<T> &a, hipStream_t s) {
    switch (G) {
        case 4: launch_blk_g<T, BR, BC, 4>(op, a, s); break;
        case 8: launch_blk_g<T, BR, BC, 8>(op, a, s); break;
        case 16: launch_blk_g<T, BR, BC, 16>(op, a, s); break;
        case 32: launch_blk_g<T, BR, BC, 32>(op, a, s); break;
        case 64: launch_blk_g<T, BR, BC, 64>(op, a, s); break;
        default: throw Error(AMG_EINVAL, "block kernel: unsupported group size");
    }
}

template <typename T>
void launch_blk(int br, int bc, int op, int G, const BlkArgsT<T> &a, hipStream_t s) {
    if (br == 1 && bc == 3) launch_blk_m<T, 1, 3>(op, G, a, s);
    else if (br == 3 && bc == 1) launch_blk_m<T, 3, 1>(op, G, a, s);
    else if (br == 1 && bc == 1) launch_blk_m<T, 1, 1>(op, G, a, s);
    else if (br == 3 && bc == 3) launch_blk_m<T, 3, 3>(op, G, a, s);
    else throw Error(AMG_EINVAL, "block kernel: unsupported block shape");
}
template void launch_blk<double>(int, int, int, int, const BlkArgsT<double> &, hipStream_t);
template void launch_blk<float>(int, int, int, int, const BlkArgsT<float> &, hipStream_t);

template <typename T>
__global__ void k_sgs_u(int64_t n, int64_t ld, const T *dinv, const T *r, T damping, T *t, T *u, bool u_zero) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x;
    if (q >= 3 * n) return;
    const int64_t i = q / 3;
    const int c = static_cast<int>(q % 3);
    const T d = dinv[(3 * c) * ld + i] * r[3 * i] + dinv[(3 * c + 1) * ld + i] * r[3 * i + 1] +
                dinv[(3 * c + 2) * ld + i] * r[3 * i + 2];
    const T v = damping * d;
    t[q] = v;
    u[q] = u_zero ? v : u[q] + v;
}

template <typename T>
void launch_sgs_u(int64_t n, int64_t ld, const T *dinv, const T *r, T damping, T *t, T *u, bool u_zero,
                  hipStream_t s) {
    if (n <= 0) return;
    k_sgs_u<T><<<ceil_div(3 * n, SB), SB, 0, s>>>(n, ld, dinv, r, damping, t, u, u_zero);
    AMG_CHECK_LAUNCH();
}
template void launch_sgs_u<double>(int64_t, int64_t, const double *, const double *, double, double *, double *,
                                   bool, hipStream_t);
template void launch_sgs_u<float>(int64_t, int64_t, const float *, const float *, float, float *, float *, bool,
                                  hipStream_t);

__global__ void k_sgs_scale(int np, const int *brow, const int *bcol, const double *bval, int64_t bnnz,
                            const double *dinv, int64_t nv, double damping, const int *crow, const int *ccol,
                            const double *cval, double *out) {
    const int p = blockIdx.x * SB + threadIdx.x;
    if (p >= np) return;
    double acc = 0.0;
    for (int k = brow[p]; k < brow[p + 1]; ++k) {
        const int j = bcol[k];
        const double b0 = bval[k], b1 = bval[bnnz + k], b2 = bval[2 * bnnz + k];
        const double bb[3] = {b0, b1, b2};
        for (int r = 0; r < 3; ++r) {
            const double dr = dinv[(3 * r) * nv + j] * b0 + dinv[(3 * r + 1) * nv + j] * b1 + dinv[(3 * r + 2) * nv + j] * b2;
            acc += bb[r] * dr;
        }
    }
    acc *= damping;
    if (crow) {
        for (int k = crow[p]; k < crow[p + 1]; ++k)
            if (ccol[k] == p) acc += cval[k];
    }
    out[p] = acc != 0.0 ? 1.0 / acc : 0.0;
}

void launch_sgs_scale(int np, const int *brow, const int *bcol, const double *bval, int64_t bnnz,
                      const double *dinv, int64_t nv, double damping, const int *crow, const int *ccol,
                      const double *cval, int64_t cnnz, double *out, hipStream_t s) {
    (void)cnnz;
    if (np <= 0) return;
    k_sgs_scale<<<ceil_div(np, SB), SB, 0, s>>>(np, brow, bcol, bval, bnnz, dinv, nv, damping, crow, ccol, cval,
                                                 out);
    AMG_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_scale(int64_t n, const T *d, const T *x, T *y) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * SB)
        y[i] = d[i] * x[i];
}
__global__ void k_scale_diff(int64_t n, const double *d, const double *x, const double *z, double *y) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * SB)
        y[i] = d[i] * (x[i] - z[i]);
}

static int grid_s(int64_t n) {
    int64_t nb = (n + SB - 1) / SB;
    if (nb > 4096) nb = 4096;
    return static_cast<int>(nb < 1 ? 1 : nb);
}

template <typename T>
void launch_scale(int64_t n, const T *d, const T *x, T *y, hipStream_t s) {
    if (n <= 0) return;
    k_scale<T><<<grid_s(n), SB, 0, s>>>(n, d, x, y);
    AMG_CHECK_LAUNCH();
}
template void launch_scale<double>(int64_t, const double *, const double *, double *, hipStream_t);
template void launch_scale<float>(int64_t, const float *, const float *, float *, hipStream_t);
void launch_scale_diff(int64_t n, const double *d, const double *x, const double *z, double *y, hipStream_t s) {
    if (n <= 0) return;
    k_scale_diff<<<grid_s(n), SB, 0, s>>>(n, d, x, z, y);
    AMG_CHECK_LAUNCH();
}

__global__ void k_bs_diag(int n, const int *rowptr, const int *col, const double *val, int64_t nnz, double *out) {
    const int i = blockIdx.x * SB + threadIdx.x;
    if (i >= n) return;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        if (col[k] == i) {
            for (int c = 0; c < 3; ++c) {
                const double a = val[static_cast<int64_t>(4 * c) * nnz + k];
                out[3 * i + c] = a != 0.0 ? 1.0 / (2.0 * a) : 0.0;
            }
            return;
        }
    }
    for (int c = 0; c < 3; ++c) out[3 * i + c] = 0.0;
}

void launch_bs_diag(int n, const int *rowptr, const int *col, const double *val, int64_t nnz, double *out,
                    hipStream_t s) {
    if (n <= 0) return;
    k_bs_diag<<<ceil_div(n, SB), SB, 0, s>>>(n, rowptr, col, val, nnz, out);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- Braess-Sarazin
// one wavefront per Schur row p; lanes own the row's output entries
__global__ void __launch_bounds__(SB) k_schur_numeric(int np, const int *brow, const int *bcol, const double *bval,
                                                      int64_t bnnz, const int *btrow, const int *btcol,
                                                      const double *btval, int64_t btnnz, const double *d,
                                                      const int *crow, const int *ccol, const double *cval,
                                                      const int *srow, const int *scol, double *sval) {
    const int p = blockIdx.x * (SB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= np) return;
    for (int q = srow[p] + lane; q < srow[p + 1]; q += 64) {
        const int Q = scol[q];
        double acc = 0.0;
        for (int k = brow[p]; k < brow[p + 1]; ++k) {
            const int j = bcol[k];
            int lo = btrow[j], hi = btrow[j + 1] - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = btcol[mid];
                if (c == Q) {
                    for (int cc = 0; cc < 3; ++cc)
                        acc += bval[cc * bnnz + k] * d[3 * j + cc] * btval[cc * btnnz + mid];
                    break;
                }
                if (c < Q) lo = mid + 1;
                else hi = mid - 1;
            }
        }
        if (crow) {
            int lo = crow[p], hi = crow[p + 1] - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = ccol[mid];
                if (c == Q) {
                    acc += cval[mid];
                    break;
                }
                if (c < Q) lo = mid + 1;
                else hi = mid - 1;
            }
        }
        sval[q] = acc;
    }
}

void launch_schur_numeric(int np, const int *brow, const int *bcol, const double *bval, int64_t bnnz,
                          const int *btrow, const int *btcol, const double *btval, int64_t btnnz, const double *d,
                          const int *crow, const int *ccol, const double *cval, const int *srow, const int *scol,
                          double *sval, hipStream_t s) {
    if (np <= 0) return;
    k_schur_numeric<<<ceil_div(np, SB / 64), SB, 0, s>>>(np, brow, bcol, bval, bnnz, btrow, btcol, btval, btnnz,
                                                          d, crow, ccol, cval, srow, scol, sval);
    AMG_CHECK_LAUNCH();
}

template <typename T, int G>
__global__ void __launch_bounds__(SB) k_scalar_gs(int nrows, const int *rowptr, const int *col, const T *val,
                                                  const int *rowid, const T *dinv, const T *b, T *x) {
    // rows of one colour grouped (row g of the launch: entries rowptr[g] ..
    // rowptr[g+1], node rowid[g]); the row pointers and the row id load
    // together, the right-hand side and diagonal with the row's entries
    const int64_t t = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x;
    const int g = static_cast<int>(t / G);
    const int lane = static_cast<int>(t % G);
    const bool active = g < nrows;
    T s = T(0), bi = T(0), di = T(0);
    int i = 0;
    if (active) {
        i = rowid[g];
        const int beg = rowptr[g], end = rowptr[g + 1];
        if (lane == 0) {
            bi = b[i];
            di = dinv[i];
        }
        for (int k = beg + lane; k < end; k += G) {
            const int j = col[k];
            const T v = val[k], xj = x[j];
            s += j != i ? v * xj : T(0);
        }
    }
    s = gsum<G>(s);
    if (!active || lane != 0) return;
    x[i] = (bi - s) * di;
}

template <typename T>
void launch_scalar_gs(int nrows, const int *rowptr, const int *col, const T *val, const int *rowid, const T *dinv,
                      const T *b, T *x, int G, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(static_cast<int64_t>(nrows) * G, SB);
    switch (G) {
        case 4: k_scalar_gs<T, 4><<<nb, SB, 0, s>>>(nrows, rowptr, col, val, rowid, dinv, b, x); break;
        case 8: k_scalar_gs<T, 8><<<nb, SB, 0, s>>>(nrows, rowptr, col, val, rowid, dinv, b, x); break;
        case 16: k_scalar_gs<T, 16><<<nb, SB, 0, s>>>(nrows, rowptr, col, val, rowid, dinv, b, x); break;
        case 32: k_scalar_gs<T, 32><<<nb, SB, 0, s>>>(nrows, rowptr, col, val, rowid, dinv, b, x); break;
        default: k_scalar_gs<T, 64><<<nb, SB, 0, s>>>(nrows, rowptr, col, val, rowid, dinv, b, x); break;
    }
    AMG_CHECK_LAUNCH();
}
template void launch_scalar_gs<double>(int, const int *, const int *, const double *, const int *, const double *,
                                       const double *, double *, int, hipStream_t);
template void launch_scalar_gs<float>(int, const int *, const int *, const float *, const int *, const float *,
                                      const float *, float *, int, hipStream_t);

template <typename T>
__global__ void k_add_scaled(int64_t n, const T *d, const T *w, T *u) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * SB)
        u[i] += d[i] * w[i];
}

template <typename T>
__global__ void k_neg(int64_t n, const T *x, T *y) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * SB)
        y[i] = -x[i];
}

template <typename T>
void launch_neg(int64_t n, const T *x, T *y, hipStream_t s) {
    if (n <= 0) return;
    k_neg<T><<<grid_s(n), SB, 0, s>>>(n, x, y);
    AMG_CHECK_LAUNCH();
}
template void launch_neg<double>(int64_t, const double *, double *, hipStream_t);
template void launch_neg<float>(int64_t, const float *, float *, hipStream_t);

template <typename T>
void launch_add_scaled(int64_t n, const T *d, const T *w, T *u, hipStream_t s) {
    if (n <= 0) return;
    k_add_scaled<T><<<grid_s(n), SB, 0, s>>>(n, d, w, u);
    AMG_CHECK_LAUNCH();
}
template void launch_add_scaled<double>(int64_t, const double *, const double *, double *, hipStream_t);
template void launch_add_scaled<float>(int64_t, const float *, const float *, float *, hipStream_t);

__global__ void k_axpby_f(float *y, const float *x, float a, float b, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * SB)
        y[i] = a * x[i] + b * y[i];
}

void launch_axpby_f(float *y, const float *x, float a, float b, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_axpby_f<<<grid_s(n), SB, 0, s>>>(y, x, a, b, n);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- dense segments
// one wavefront per output row over all segments; lanes stride the columns;
// FP64 inverse and accumulation whatever the vector type
template <typename T, typename M>
__global__ void __launch_bounds__(SB) k_dense_segs(const DenseSegView d, const M *mat, const T *xu, const T *xp,
                                                   T *yu, T *yp) {
    const int r = blockIdx.x * (SB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= d.rows) return;
    int lo = 0, hi = d.count - 1;
    while (lo < hi) {  // last segment with rstart <= r
        const int mid = (lo + hi + 1) >> 1;
        if (d.rstart[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const int sg = lo;
    const int m = d.rstart[sg + 1] - d.rstart[sg];
    const int i = r - d.rstart[sg];
    const int nu = d.nu[sg];
    const T *xus = xu + d.uoff[sg], *xps = xp + d.poff[sg];
    const M *row = mat + d.moff[sg] + static_cast<int64_t>(i) * m;
    double acc = 0.0;
    // four entries per lane and trip keep four row loads in flight
    int j = lane;
    for (; j + 192 < m; j += 256) {
        const double a0 = row[j], a1 = row[j + 64], a2 = row[j + 128], a3 = row[j + 192];
        const int j1 = j + 64, j2 = j + 128, j3 = j + 192;
        acc += a0 * static_cast<double>(j < nu ? xus[j] : xps[j - nu]);
        acc += a1 * static_cast<double>(j1 < nu ? xus[j1] : xps[j1 - nu]);
        acc += a2 * static_cast<double>(j2 < nu ? xus[j2] : xps[j2 - nu]);
        acc += a3 * static_cast<double>(j3 < nu ? xus[j3] : xps[j3 - nu]);
    }
    for (; j < m; j += 64) acc += static_cast<double>(row[j]) * static_cast<double>(j < nu ? xus[j] : xps[j - nu]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) {
        if (i < nu) yu[d.uoff[sg] + i] = static_cast<T>(acc);
        else yp[d.poff[sg] + i - nu] = static_cast<T>(acc);
    }
}

template <typename T>
void launch_dense_segs(const DenseSegView &d, const T *xu, const T *xp, T *yu, T *yp, hipStream_t s) {
    if (d.count <= 0 || d.rows <= 0) return;
    const int nb = ceil_div(d.rows, SB / 64);
    if (std::is_same<T, float>::value && d.inv32)
        k_dense_segs<T, float><<<nb, SB, 0, s>>>(d, d.inv32, xu, xp, yu, yp);
    else
        k_dense_segs<T, double><<<nb, SB, 0, s>>>(d, d.inv, xu, xp, yu, yp);
    AMG_CHECK_LAUNCH();
}
template void launch_dense_segs<double>(const DenseSegView &, const double *, const double *, double *, double *,
                                        hipStream_t);
template void launch_dense_segs<float>(const DenseSegView &, const float *, const float *, float *, float *,
                                       hipStream_t);

// one thread per segment
__global__ void k_segment_units(const DenseSegView d, int j, double *xu, double *xp) {
    const int sg = blockIdx.x * SB + threadIdx.x;
    if (sg >= d.count) return;
    if (j >= d.rstart[sg + 1] - d.rstart[sg]) return;
    const int nu = d.nu[sg];
    if (j < nu) xu[d.uoff[sg] + j] = 1.0;
    else xp[d.poff[sg] + j - nu] = 1.0;
}

void launch_segment_units(const DenseSegView &d, int j, double *xu, double *xp, hipStream_t s) {
    if (d.count <= 0) return;
    k_segment_units<<<ceil_div(d.count, SB), SB, 0, s>>>(d, j, xu, xp);
    AMG_CHECK_LAUNCH();
}

// one workgroup per segment
__global__ void k_segment_store_column(const DenseSegView d, int j, const double *xu, const double *xp,
                                       double *inv) {
    const int sg = blockIdx.x;
    const int m = d.rstart[sg + 1] - d.rstart[sg];
    if (j >= m) return;
    const int nu = d.nu[sg];
    for (int i = threadIdx.x; i < m; i += SB)
        inv[d.moff[sg] + static_cast<int64_t>(i) * m + j] = i < nu ? xu[d.uoff[sg] + i] : xp[d.poff[sg] + i - nu];
}

void launch_segment_store_column(const DenseSegView &d, int j, const double *xu, const double *xp, double *inv,
                                 hipStream_t s) {
    if (d.count <= 0) return;
    k_segment_store_column<<<d.count, SB, 0, s>>>(d, j, xu, xp, inv);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- blocks of columns
// For pressure-only segments (nu = 0, as in the Schur maps): vectors of C
// columns, row-major (row i of segment s, column c at (poff_s + i) C + c).

// x[(poff_s + j0 + c) C + c] = 1 for every segment s and c < C with
// j0 + c < m_s (x zero elsewhere beforehand)
__global__ void k_segment_units_block(const DenseSegView d, int j0, int C, double *x) {
    const int sg = blockIdx.x;
    const int m = d.rstart[sg + 1] - d.rstart[sg];
    for (int c = threadIdx.x; c < C; c += SB) {
        const int j = j0 + c;
        if (j < m) x[static_cast<int64_t>(d.poff[sg] + j) * C + c] = 1.0;
    }
}

void launch_segment_units_block(const DenseSegView &d, int j0, int C, double *x, hipStream_t s) {
    if (d.count <= 0) return;
    k_segment_units_block<<<d.count, SB, 0, s>>>(d, j0, C, x);
    AMG_CHECK_LAUNCH();
}

// columns j0 .. j0 + C - 1 of every segment's matrix (row-major):
// M_s[i][j0 + c] = x[(poff_s + i) C + c]
__global__ void k_segment_store_block(const DenseSegView d, int j0, int C, const double *x, double *inv) {
    const int sg = blockIdx.x;
    const int m = d.rstart[sg + 1] - d.rstart[sg];
    const int64_t mc = static_cast<int64_t>(m) * C;
    for (int64_t e = threadIdx.x; e < mc; e += SB) {
        const int i = static_cast<int>(e / C), c = static_cast<int>(e % C);
        const int j = j0 + c;
        if (j < m) inv[d.moff[sg] + static_cast<int64_t>(i) * m + j] = x[static_cast<int64_t>(d.poff[sg] + i) * C + c];
    }
}

void launch_segment_store_block(const DenseSegView &d, int j0, int C, const double *x, double *inv, hipStream_t s) {
    if (d.count <= 0) return;
    k_segment_store_block<<<d.count, SB, 0, s>>>(d, j0, C, x, inv);
    AMG_CHECK_LAUNCH();
}

// y = M_s x on every segment for C columns: one wavefront per segment row,
// lanes over the columns, FP64
__global__ void __launch_bounds__(SB) k_dense_segs_block(const DenseSegView d, int C, const double *x, double *y) {
    const int r = blockIdx.x * (SB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= d.rows) return;
    int lo = 0, hi = d.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.rstart[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const int sg = lo;
    const int m = d.rstart[sg + 1] - d.rstart[sg];
    const int i = r - d.rstart[sg];
    const double *row = d.inv + d.moff[sg] + static_cast<int64_t>(i) * m;
    const int64_t p0 = d.poff[sg];
    for (int c = lane; c < C; c += 64) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += row[j] * x[(p0 + j) * C + c];
        y[(p0 + i) * C + c] = acc;
    }
}

void launch_dense_segs_block(const DenseSegView &d, int C, const double *x, double *y, hipStream_t s) {
    if (d.count <= 0 || d.rows <= 0) return;
    k_dense_segs_block<<<ceil_div(d.rows, SB / 64), SB, 0, s>>>(d, C, x, y);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- FGMRES
// Workgroup (c, g) dots the chunk c of the NR right-hand sides (MD_CHUNK
// entries each, held in registers) with the same chunk of the basis vectors
// g * MD_VEC .. g * MD_VEC + MD_VEC - 1: one pass over the right-hand sides
// per group instead of one per vector, every basis chunk read once for all
// right-hand sides, and one block reduction for the whole group. Right-hand
// side r's dot with vector q goes to partial[(r * k + q) * nb + c].
constexpr int MD_PER = 4;
constexpr int MD_CHUNK = MD_PER * SB;
constexpr int MD_VEC = 8;

template <int NR>
__global__ void __launch_bounds__(SB) k_multidot(const double *V, int64_t ld, int k, const double *w0,
                                                 const double *w1, int64_t n, double *partial) {
    __shared__ double red[NR * MD_VEC][SB / 64];
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * MD_CHUNK;
    const int j0 = blockIdx.y * MD_VEC;
    const int nv = min(MD_VEC, k - j0);
    double wv[NR][MD_PER];
#pragma unroll
    for (int e = 0; e < MD_PER; ++e) {
        const int64_t t = s0 + threadIdx.x + e * SB;
        wv[0][e] = t < n ? w0[t] : 0.0;
        if (NR == 2) wv[NR - 1][e] = t < n ? w1[t] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < MD_VEC; ++q) {
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = 0.0;
        if (q < nv) {
            const double *v = V + (j0 + q) * ld;
#pragma unroll
            for (int e = 0; e < MD_PER; ++e) {
                const int64_t t = s0 + threadIdx.x + e * SB;
                if (t < n) {
                    const double vt = v[t];
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r] += vt * wv[r][e];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double a = gsum<64>(acc[r]);
            if ((threadIdx.x & 63) == 0) red[r * MD_VEC + q][threadIdx.x >> 6] = a;
        }
    }
    __syncthreads();
    if (threadIdx.x < NR * nv) {
        const int r = threadIdx.x / nv, q = threadIdx.x % nv;
        double s = 0.0;
        for (int b = 0; b < SB / 64; ++b) s += red[r * MD_VEC + q][b];
        partial[(static_cast<int64_t>(r) * k + j0 + q) * gridDim.x + blockIdx.x] = s;
    }
}

int multidot_blocks(int64_t n) { return static_cast<int>(std::max<int64_t>(1, (n + MD_CHUNK - 1) / MD_CHUNK)); }

int launch_multidot(const double *V, int64_t ld, int k, const double *w, int64_t n, double *partial,
                    hipStream_t s) {
    if (k <= 0) return 0;
    const int nb = multidot_blocks(n);
    k_multidot<1><<<dim3(nb, ceil_div(k, MD_VEC)), SB, 0, s>>>(V, ld, k, w, w, n, partial);
    AMG_CHECK_LAUNCH();
    return nb;
}

int launch_multidot2(const double *V, int64_t ld, int k, const double *a, const double *b, int64_t n,
                     double *partial, hipStream_t s) {
    if (k <= 0) return 0;
    const int nb = multidot_blocks(n);
    k_multidot<2><<<dim3(nb, ceil_div(k, MD_VEC)), SB, 0, s>>>(V, ld, k, a, b, n, partial);
    AMG_CHECK_LAUNCH();
    return nb;
}

__global__ void k_multidot_reduce(const double *partial, int nb, int k, double *h) {
    // one wavefront per vector
    const int i = blockIdx.x * (SB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= k) return;
    double acc = 0.0;
    for (int b = lane; b < nb; b += 64) acc += partial[static_cast<int64_t>(i) * nb + b];
    acc = gsum<64>(acc);
    if (lane == 0) h[i] = acc;
}

void launch_multidot_reduce(const double *partial, int nb, int k, double *h, hipStream_t s) {
    if (k <= 0) return;
    k_multidot_reduce<<<ceil_div(k, SB / 64), SB, 0, s>>>(partial, nb, k, h);
    AMG_CHECK_LAUNCH();
}

// One step of classical Gram-Schmidt with delayed reorthogonalisation.
// Basis slot j holds the pending vector u (orthogonalised once against
// V_0..V_{j-1}), slot j + 1 the new vector w. With k = j + 2, h[0..k) are
// the dots V_i . u and h[k..2k) the dots V_i . w (i <= j + 1). The update
// finishes u: v_j = (u - sum_{i<j} s_i V_i) / gamma, s_i = V_i . u,
// gamma^2 = u . u - |s|^2 (skipped when reorth is 0: v_j is final already),
// and orthogonalises w once against V_0..V_{j-1}, v_j:
// w' = w - sum_{i<j} c_i V_i - d v_j with c_i = V_i . w,
// d = v_j . w = (u . w - s . c) / gamma, then scales it by
// eta = sqrt(w . w - |c|^2 - d^2) (Pythagoras; any positive scale serves,
// as the next step measures the new pending vector exactly, so a
// cancelled estimate falls back to 1e-2 |w|). gamma, d and eta are written
// to h[2k], h[2k + 1], h[2k + 2].
template <bool REORTH>
__global__ void __launch_bounds__(SB) k_dcgs2_update(double *V, int64_t ld, int j, double *h, int64_t n) {
    const int k = j + 2;
    const double *dA = h, *dB = h + k;
    double ss = 0.0, sc = 0.0, cc = 0.0;
    for (int i = 0; i < j; ++i) {
        if (REORTH) {
            ss += dA[i] * dA[i];
            sc += dA[i] * dB[i];
        }
        cc += dB[i] * dB[i];
    }
    double gam = 1.0;
    if (REORTH) {
        const double g2 = dA[j] - ss;
        gam = g2 > 0.0 ? sqrt(g2) : 0.0;
    }
    const double gs = gam > 0.0 ? gam : 1.0;
    const double d = REORTH ? (dB[j] - sc) / gs : dB[j];
    const double omega = dB[j + 1];
    const double eta = sqrt(fmax(omega - cc - d * d, 1e-4 * omega));
    const double ig = 1.0 / gs, ie = eta > 0.0 ? 1.0 / eta : 1.0;
    double *vj = V + static_cast<int64_t>(j) * ld, *w = V + static_cast<int64_t>(j + 1) * ld;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; t < n;
         t += static_cast<int64_t>(gridDim.x) * SB) {
        double as = 0.0, ac = 0.0;
#pragma unroll 8
        for (int i = 0; i < j; ++i) {
            const double v = V[static_cast<int64_t>(i) * ld + t];
            if (REORTH) as += dA[i] * v;
            ac += dB[i] * v;
        }
        double u = vj[t];
        if (REORTH) {
            u = (u - as) * ig;
            vj[t] = u;
        }
        w[t] = (w[t] - ac - d * u) * ie;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        h[2 * k] = gam;
        h[2 * k + 1] = d;
        h[2 * k + 2] = eta;
    }
}

void launch_dcgs2_update(double *V, int64_t ld, int j, double *h, int64_t n, bool reorth, hipStream_t s) {
    if (n <= 0) return;
    if (reorth)
        k_dcgs2_update<true><<<grid_s(n), SB, 0, s>>>(V, ld, j, h, n);
    else
        k_dcgs2_update<false><<<grid_s(n), SB, 0, s>>>(V, ld, j, h, n);
    AMG_CHECK_LAUNCH();
}

__global__ void k_multi_add(const double *Z, int64_t ld, int k, const double *y, double *x, int64_t n) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; t < n;
         t += static_cast<int64_t>(gridDim.x) * SB) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += y[i] * Z[static_cast<int64_t>(i) * ld + t];
        x[t] += s;
    }
}

void launch_multi_add(const double *Z, int64_t ld, int k, const double *y, double *x, int64_t n, hipStream_t s) {
    if (k <= 0 || n <= 0) return;
    k_multi_add<<<grid_s(n), SB, 0, s>>>(Z, ld, k, y, x, n);
    AMG_CHECK_LAUNCH();
}

__global__ void k_scale_by_inverse(const double *x, double *y, int64_t n, const double *sc, int idx) {
    const double a = 1.0 / sc[idx];
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * SB + threadIdx.x; t < n;
         t += static_cast<int64_t>(gridDim.x) * SB)
        y[t] = a * x[t];
}

void launch_scale_by_inverse(const double *x, double *y, int64_t n, const double *sc, int idx, hipStream_t s) {
    if (n <= 0) return;
    k_scale_by_inverse<<<grid_s(n), SB, 0, s>>>(x, y, n, sc, idx);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
