// Galerkin coarse operators A_{l+1} = P^T (A_l P) on the GPU (Section 3.2:
// coarse matrices by Galerkin projection with the block-diagonal
// prolongation). Two sparse products, each in a symbolic and a numeric phase:
//   symbolic: one wavefront per output row inserts the candidate column
//             indices into a hash set held in LDS (open addressing, bounded
//             probing), counts them, then compacts and ranks them so that each
//             output row is sorted;
//   numeric:  each lane owns one output entry (row, J) and accumulates its
//             products in a fixed order (deterministic result, no atomics).
// The structural pattern is produced whatever the values are, so explicit
// zeros survive as the coarsening requires.
#include "common.h"
#include "kernels.h"

namespace amgp2 {

constexpr int SBLOCK = 256;
constexpr int WAVES = SBLOCK / 64;
constexpr int HS = SPGEMM_HASH;
static_assert((HS & (HS - 1)) == 0, "hash size must be a power of two");
constexpr int HBITS = 11;
static_assert((1 << HBITS) == HS, "hash bits");

__device__ __forceinline__ int hslot(int key) {
    return static_cast<int>((static_cast<unsigned>(key) * 2654435761u) >> (32 - HBITS));
}

// Insert every candidate column of output row `row` into tab; returns via
// cnt the number of distinct keys; sets *overflow when a probe sequence ran
// through the whole table.
__device__ __forceinline__ void insert_row(int row, int lane, const int *xr, const int *xc, const int *yr,
                                           const int *yc, int *tab, int *cnt, int *overflow) {
    for (int k = xr[row] + lane; k < xr[row + 1]; k += 64) {
        const int j = xc[k];
        for (int m = yr[j]; m < yr[j + 1]; ++m) {
            const int key = yc[m];
            int h = hslot(key);
            bool done = false;
            for (int probe = 0; probe < HS; ++probe) {
                const int prev = atomicCAS(&tab[h], -1, key);
                if (prev == -1) {
                    atomicAdd(cnt, 1);
                    done = true;
                    break;
                }
                if (prev == key) {
                    done = true;
                    break;
                }
                h = (h + 1) & (HS - 1);
            }
            if (!done) atomicOr(overflow, 1);
        }
    }
}

__global__ void __launch_bounds__(SBLOCK) k_spgemm_count(int nrows, const int *xr, const int *xc,
                                                         const int *yr, const int *yc, int *count,
                                                         int *overflow) {
    __shared__ int tab[WAVES][HS];
    __shared__ int cnt[WAVES];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * WAVES + w;
    for (int s = lane; s < HS; s += 64) tab[w][s] = -1;
    if (lane == 0) cnt[w] = 0;
    __syncthreads();
    if (row < nrows) insert_row(row, lane, xr, xc, yr, yc, tab[w], &cnt[w], overflow);
    __syncthreads();
    if (row < nrows && lane == 0) {
        count[row] = cnt[w];
        if (cnt[w] > (HS * 3) / 4) atomicOr(overflow, 2);
    }
}

__global__ void __launch_bounds__(SBLOCK) k_spgemm_fill(int nrows, const int *xr, const int *xc,
                                                        const int *yr, const int *yc, const int *cr,
                                                        int *cc) {
    __shared__ int tab[WAVES][HS];
    __shared__ int lst[WAVES][HS];
    __shared__ int cnt[WAVES], cnt2[WAVES], ovf[WAVES];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * WAVES + w;
    for (int s = lane; s < HS; s += 64) tab[w][s] = -1;
    if (lane == 0) {
        cnt[w] = 0;
        cnt2[w] = 0;
        ovf[w] = 0;
    }
    __syncthreads();
    if (row < nrows) insert_row(row, lane, xr, xc, yr, yc, tab[w], &cnt[w], &ovf[w]);
    __syncthreads();
    if (row < nrows) {
        for (int s = lane; s < HS; s += 64) {
            const int v = tab[w][s];
            if (v >= 0) lst[w][atomicAdd(&cnt2[w], 1)] = v;
        }
    }
    __syncthreads();
    if (row < nrows) {
        const int n = cnt2[w];
        const int base = cr[row];
        for (int e = lane; e < n; e += 64) {
            const int v = lst[w][e];
            int rank = 0;
            for (int f = 0; f < n; ++f) rank += lst[w][f] < v;
            cc[base + rank] = v;
        }
    }
}

void launch_spgemm_count(int nrows, const int *xr, const int *xc, const int *yr, const int *yc,
                         int *count, int *overflow, hipStream_t s) {
    if (nrows <= 0) return;
    k_spgemm_count<<<ceil_div(nrows, WAVES), SBLOCK, 0, s>>>(nrows, xr, xc, yr, yc, count, overflow);
    AMG_CHECK_LAUNCH();
}

void launch_spgemm_fill(int nrows, const int *xr, const int *xc, const int *yr, const int *yc,
                        const int *cr, int *cc, hipStream_t s) {
    if (nrows <= 0) return;
    k_spgemm_fill<<<ceil_div(nrows, WAVES), SBLOCK, 0, s>>>(nrows, xr, xc, yr, yc, cr, cc);
    AMG_CHECK_LAUNCH();
}

// C = X Y with X in planes (np) and Y scalar: lane owns output (row, J) and
// sums X_rk * Y_kJ over the entries k of X's row in order.
template <int NP>
__global__ void __launch_bounds__(SBLOCK) k_spgemm_num_bx(int nrows, const int *xr, const int *xc,
                                                          const double *xv, int64_t xnnz, const int *yr,
                                                          const int *yc, const double *yv, const int *cr,
                                                          const int *cc, double *cv, int64_t cnnz) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * WAVES + w;
    if (row >= nrows) return;
    const int xb = xr[row], xe = xr[row + 1];
    for (int q = cr[row] + lane; q < cr[row + 1]; q += 64) {
        const int J = cc[q];
        double acc[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[p] = 0.0;
        for (int k = xb; k < xe; ++k) {
            const int j = xc[k];
            for (int m = yr[j]; m < yr[j + 1]; ++m) {
                if (yc[m] == J) {
                    const double wgt = yv[m];
#pragma unroll
                    for (int p = 0; p < NP; ++p) acc[p] += wgt * xv[p * xnnz + k];
                }
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) cv[p * cnnz + q] = acc[p];
    }
}

// C = X Y with X scalar and Y in planes (np), Y rows sorted: lane owns
// output (row, J) and sums X_rk * Y_kJ with a binary search in Y's row k.
template <int NP>
__global__ void __launch_bounds__(SBLOCK) k_spgemm_num_by(int nrows, const int *xr, const int *xc,
                                                          const double *xv, const int *yr, const int *yc,
                                                          const double *yv, int64_t ynnz, const int *cr,
                                                          const int *cc, double *cv, int64_t cnnz) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * WAVES + w;
    if (row >= nrows) return;
    const int xb = xr[row], xe = xr[row + 1];
    for (int q = cr[row] + lane; q < cr[row + 1]; q += 64) {
        const int J = cc[q];
        double acc[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[p] = 0.0;
        for (int k = xb; k < xe; ++k) {
            const int i = xc[k];
            int lo = yr[i], hi = yr[i + 1] - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = yc[mid];
                if (c == J) {
                    const double wgt = xv[k];
#pragma unroll
                    for (int p = 0; p < NP; ++p) acc[p] += wgt * yv[p * ynnz + mid];
                    break;
                }
                if (c < J)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) cv[p * cnnz + q] = acc[p];
    }
}

void launch_spgemm_numeric_bx(int np, int nrows, const int *xr, const int *xc, const double *xv,
                              int64_t xnnz, const int *yr, const int *yc, const double *yv, const int *cr,
                              const int *cc, double *cv, int64_t cnnz, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(nrows, WAVES);
    switch (np) {
        case 1: k_spgemm_num_bx<1><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, xnnz, yr, yc, yv, cr, cc, cv, cnnz); break;
        case 3: k_spgemm_num_bx<3><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, xnnz, yr, yc, yv, cr, cc, cv, cnnz); break;
        case 9: k_spgemm_num_bx<9><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, xnnz, yr, yc, yv, cr, cc, cv, cnnz); break;
        default: throw Error(AMG_EINVAL, "spgemm: unsupported block shape");
    }
    AMG_CHECK_LAUNCH();
}

void launch_spgemm_numeric_by(int np, int nrows, const int *xr, const int *xc, const double *xv,
                              const int *yr, const int *yc, const double *yv, int64_t ynnz, const int *cr,
                              const int *cc, double *cv, int64_t cnnz, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(nrows, WAVES);
    switch (np) {
        case 1: k_spgemm_num_by<1><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, yr, yc, yv, ynnz, cr, cc, cv, cnnz); break;
        case 3: k_spgemm_num_by<3><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, yr, yc, yv, ynnz, cr, cc, cv, cnnz); break;
        case 9: k_spgemm_num_by<9><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, yr, yc, yv, ynnz, cr, cc, cv, cnnz); break;
        default: throw Error(AMG_EINVAL, "spgemm: unsupported block shape");
    }
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
