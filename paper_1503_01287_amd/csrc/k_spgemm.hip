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

// ---------------------------------------------------------------- numeric, LDS-staged
// The same sums in the same order as the kernels above, with the dependent
// loads taken out of each lane's inner loop: one wavefront per output row
// stages a chunk of the row's products in LDS (all lanes load in parallel,
// an in-wave prefix sum places them), then every lane scans the staged
// list for the output entries it owns. Each output is still summed over
// k ascending (and, for X Y with Y scalar, over Y's row in order), so the
// result is bit-for-bit the one-lane-per-entry kernels'.
constexpr int NCAP = 1024;  // staged products per wavefront
constexpr int NT = 4;       // output entries per lane kept in registers (256 per row per pass)

// wavefront inclusive prefix sum
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// C = X Y, X in planes (np), Y scalar (an interpolation: few entries per row)
template <int NP>
__global__ void __launch_bounds__(SBLOCK) k_spgemm_num_bx_lds(int nrows, const int *xr, const int *xc,
                                                              const double *xv, int64_t xnnz, const int *yr,
                                                              const int *yc, const double *yv, const int *cr,
                                                              const int *cc, double *cv, int64_t cnnz,
                                                              int *overflow) {
    __shared__ int s_col[WAVES][NCAP];
    __shared__ int s_k[WAVES][NCAP];
    __shared__ double s_w[WAVES][NCAP];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * WAVES + w;
    if (row >= nrows) return;  // whole wavefronts leave; only wave-level syncs below
    const int xb = xr[row], xe = xr[row + 1];
    for (int q0 = cr[row]; q0 < cr[row + 1]; q0 += 64 * NT) {
        int J[NT];
        double acc[NT][NP];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int q = q0 + lane + 64 * t;
            J[t] = q < cr[row + 1] ? cc[q] : -1;
#pragma unroll
            for (int p = 0; p < NP; ++p) acc[t][p] = 0.0;
        }
        for (int k0 = xb; k0 < xe;) {
            const int k = k0 + lane;
            int yb = 0, cnt = 0;
            if (k < xe) {
                const int j = xc[k];
                yb = yr[j];
                cnt = yr[j + 1] - yb;
            }
            const int incl = wave_incl_scan(cnt, lane);
            // the leading lanes whose products fit (incl grows with the lane)
            const unsigned long long fit = __ballot(k < xe && incl <= NCAP);
            const int take = __popcll(fit);
            if (take == 0) {  // one Y row alone exceeds the staging capacity
                if (lane == 0) atomicOr(overflow, 1);
                return;
            }
            const int total = __shfl(incl, take - 1, 64);
            if (lane < take)
                for (int m = 0, e = incl - cnt; m < cnt; ++m, ++e) {
                    s_col[w][e] = yc[yb + m];
                    s_w[w][e] = yv[yb + m];
                    s_k[w][e] = k;
                }
            wave_sync();
            for (int e = 0; e < total; ++e) {
                const int col = s_col[w][e];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    if (col == J[t]) {
                        const double wgt = s_w[w][e];
                        const int kk = s_k[w][e];
#pragma unroll
                        for (int p = 0; p < NP; ++p) acc[t][p] += wgt * xv[p * xnnz + kk];
                    }
            }
            wave_sync();
            k0 += take;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int q = q0 + lane + 64 * t;
            if (q < cr[row + 1])
#pragma unroll
                for (int p = 0; p < NP; ++p) cv[p * cnnz + q] = acc[t][p];
        }
    }
}

// C = X Y, X scalar, Y in planes (np) with sorted rows: the column lists of
// the Y rows a chunk of X's row touches are staged, and each lane finds its
// output column in them by binary search in LDS
template <int NP>
__global__ void __launch_bounds__(SBLOCK) k_spgemm_num_by_lds(int nrows, const int *xr, const int *xc,
                                                              const double *xv, const int *yr, const int *yc,
                                                              const double *yv, int64_t ynnz, const int *cr,
                                                              const int *cc, double *cv, int64_t cnnz,
                                                              int *overflow) {
    __shared__ int s_col[WAVES][2 * NCAP];
    __shared__ int s_beg[WAVES][64], s_cnt[WAVES][64], s_yb[WAVES][64];
    __shared__ double s_x[WAVES][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * WAVES + w;
    if (row >= nrows) return;
    const int xb = xr[row], xe = xr[row + 1];
    for (int q0 = cr[row]; q0 < cr[row + 1]; q0 += 64 * NT) {
        int J[NT];
        double acc[NT][NP];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int q = q0 + lane + 64 * t;
            J[t] = q < cr[row + 1] ? cc[q] : -1;
#pragma unroll
            for (int p = 0; p < NP; ++p) acc[t][p] = 0.0;
        }
        for (int k0 = xb; k0 < xe;) {
            const int k = k0 + lane;
            int yb = 0, cnt = 0;
            double xk = 0.0;
            if (k < xe) {
                const int i = xc[k];
                xk = xv[k];
                yb = yr[i];
                cnt = yr[i + 1] - yb;
            }
            const int incl = wave_incl_scan(cnt, lane);
            const unsigned long long fit = __ballot(k < xe && incl <= 2 * NCAP);
            const int take = __popcll(fit);
            if (take == 0) {
                if (lane == 0) atomicOr(overflow, 1);
                return;
            }
            if (lane < take) {
                const int e0 = incl - cnt;
                s_beg[w][lane] = e0;
                s_cnt[w][lane] = cnt;
                s_yb[w][lane] = yb;
                s_x[w][lane] = xk;
                for (int m = 0; m < cnt; ++m) s_col[w][e0 + m] = yc[yb + m];
            }
            wave_sync();
            for (int u = 0; u < take; ++u) {
                const int beg = s_beg[w][u], n = s_cnt[w][u];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (J[t] < 0) continue;
                    int lo = 0, hi = n - 1;
                    while (lo <= hi) {
                        const int mid = (lo + hi) >> 1;
                        const int c = s_col[w][beg + mid];
                        if (c == J[t]) {
                            const double wgt = s_x[w][u];
                            const int64_t m = s_yb[w][u] + mid;
#pragma unroll
                            for (int p = 0; p < NP; ++p) acc[t][p] += wgt * yv[p * ynnz + m];
                            break;
                        }
                        if (c < J[t])
                            lo = mid + 1;
                        else
                            hi = mid - 1;
                    }
                }
            }
            wave_sync();
            k0 += take;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int q = q0 + lane + 64 * t;
            if (q < cr[row + 1])
#pragma unroll
                for (int p = 0; p < NP; ++p) cv[p * cnnz + q] = acc[t][p];
        }
    }
}

bool launch_spgemm_numeric_lds(bool by, int np, int nrows, const int *xr, const int *xc, const double *xv,
                               int64_t xnnz, const int *yr, const int *yc, const double *yv, int64_t ynnz,
                               const int *cr, const int *cc, double *cv, int64_t cnnz, int *overflow,
                               hipStream_t s) {
    if (nrows <= 0) return true;
    const int nb = ceil_div(nrows, WAVES);
#define AMG_NUM(NPV)                                                                                         \
    if (by)                                                                                                \
        k_spgemm_num_by_lds<NPV><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, yr, yc, yv, ynnz, cr, cc, cv, cnnz, \
                                                      overflow);                                           \
    else                                                                                                   \
        k_spgemm_num_bx_lds<NPV><<<nb, SBLOCK, 0, s>>>(nrows, xr, xc, xv, xnnz, yr, yc, yv, cr, cc, cv, cnnz, \
                                                      overflow);
    switch (np) {
        case 1: AMG_NUM(1) break;
        case 3: AMG_NUM(3) break;
        case 9: AMG_NUM(9) break;
        default: throw Error(AMG_EINVAL, "spgemm: unsupported block shape");
    }
#undef AMG_NUM
    AMG_CHECK_LAUNCH();
    return true;
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
