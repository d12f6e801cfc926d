// The coarse end of Algorithm 1 in one workgroup.
//
// On the smallest levels every operation of the V-cycle is a few hundred rows:
// launched one by one, each Gauss-Seidel colour, residual, restriction and
// prolongation would cost a full dispatch (about 4.5 us on gfx950, the
// latency floor of a kernel) for well under a microsecond of work. Here one
// workgroup of 1024 threads runs the whole remaining V-cycle, from the
// pre-smoothing of the first tail level down to the coarsest solve and back
// up: the level vectors live in LDS, colours and phases are separated by
// workgroup barriers, and the operators stream from L2.
#include "common.h"
#include "kernels.h"
#include "tail.h"

namespace amgp2 {

constexpr int TBLOCK = 1024;
constexpr int TWAVES = TBLOCK / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// s = (A x)_g for one row, the 64 lanes of the calling wave cooperating;
// x is a 3-component vector in LDS. Every lane returns the full sums.
template <int MODE>
__device__ __forceinline__ void row_apply(const int *rowptr, const int *col, const double *val, int64_t nnz,
                                          int g, const double *x, int lane, double &s0, double &s1,
                                          double &s2) {
    s0 = s1 = s2 = 0.0;
    for (int k = rowptr[g] + lane; k < rowptr[g + 1]; k += 64) {
        const int j = col[k];
        const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
        if constexpr (MODE == 3) {
            const double *v = val + k;
            s0 += v[0] * x0 + v[nnz] * x1 + v[2 * nnz] * x2;
            s1 += v[3 * nnz] * x0 + v[4 * nnz] * x1 + v[5 * nnz] * x2;
            s2 += v[6 * nnz] * x0 + v[7 * nnz] * x1 + v[8 * nnz] * x2;
        } else {
            const double v = val[k];
            s0 += v * x0;
            s1 += v * x1;
            s2 += v * x2;
        }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
}

// component c of D_i^{-1} (r0, r1, r2)
template <int MODE>
__device__ __forceinline__ double dinv_apply(const double *dinv, int n, int i, int c, double r0, double r1,
                                             double r2) {
    if constexpr (MODE == 3) {
        return dinv[(3 * c) * n + i] * r0 + dinv[(3 * c + 1) * n + i] * r1 + dinv[(3 * c + 2) * n + i] * r2;
    } else {
        return dinv[i] * (c == 0 ? r0 : (c == 1 ? r1 : r2));
    }
}

template <int MODE>
__device__ void tail_gs(const TailLevel &L, double *x, const double *b, bool forward, int wave, int lane) {
    for (int q = 0; q < L.ncolors; ++q) {
        const int c = forward ? q : L.ncolors - 1 - q;
        for (int g = L.cptr[c] + wave; g < L.cptr[c + 1]; g += TWAVES) {
            double s0, s1, s2;
            row_apply<MODE>(L.g_rowptr, L.g_col, L.g_val, L.g_nnz, g, x, lane, s0, s1, s2);
            if (lane < 3) {
                const int i = L.g_rowid[g];
                const double r0 = b[3 * i] - s0, r1 = b[3 * i + 1] - s1, r2 = b[3 * i + 2] - s2;
                x[3 * i + lane] += dinv_apply<MODE>(L.dinv, L.n, i, lane, r0, r1, r2);
            }
        }
        __syncthreads();
    }
}

template <int MODE>
__device__ void tail_residual(const TailLevel &L, const double *x, const double *b, double *r, int wave,
                              int lane) {
    for (int i = wave; i < L.n; i += TWAVES) {
        double s0, s1, s2;
        row_apply<MODE>(L.a_rowptr, L.a_col, L.a_val, L.a_nnz, i, x, lane, s0, s1, s2);
        if (lane < 3) r[3 * i + lane] = b[3 * i + lane] - (lane == 0 ? s0 : (lane == 1 ? s1 : s2));
    }
    __syncthreads();
}

// damped block Jacobi: x <- x + omega D^{-1} (b - A x)
template <int MODE>
__device__ void tail_jacobi(const TailLevel &L, double *x, const double *b, double *r, bool from_zero,
                            int wave, int lane) {
    const int tid = threadIdx.x;
    if (from_zero) {
        for (int t = tid; t < 3 * L.n; t += TBLOCK) {
            const int i = t / 3, c = t % 3;
            x[t] = L.omega * dinv_apply<MODE>(L.dinv, L.n, i, c, b[3 * i], b[3 * i + 1], b[3 * i + 2]);
        }
        __syncthreads();
        return;
    }
    tail_residual<MODE>(L, x, b, r, wave, lane);
    for (int t = tid; t < 3 * L.n; t += TBLOCK) {
        const int i = t / 3, c = t % 3;
        x[t] += L.omega * dinv_apply<MODE>(L.dinv, L.n, i, c, r[3 * i], r[3 * i + 1], r[3 * i + 2]);
    }
    __syncthreads();
}

template <int MODE>
__device__ void tail_smooth(const TailArgs &a, const TailLevel &L, double *x, const double *b, double *r,
                            bool pre, bool x_zero, int wave, int lane) {
    const int steps = pre ? a.pre : a.post;
    for (int k = 0; k < steps; ++k) {
        if (a.smoother == AMG_SMOOTH_JA)
            tail_jacobi<MODE>(L, x, b, r, x_zero && k == 0, wave, lane);
        else
            tail_gs<MODE>(L, x, b, pre, wave, lane);
    }
}

template <int MODE>
__global__ void __launch_bounds__(TBLOCK) k_tail(const TailArgs a) {
    extern __shared__ double lds_buf[];
    // level vectors: in LDS, or (when assembling a tail too large for LDS)
    // in this workgroup's slice of a global scratch buffer
    double *lds = a.gscratch ? a.gscratch + static_cast<int64_t>(blockIdx.x) * a.gstride : lds_buf;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const TailLevel *lv = a.lv;
    {
        const TailLevel &L = lv[0];
        double *x = lds + L.lds_off, *b = x + 3 * L.n;
        const int uj = a.unit_base + static_cast<int>(blockIdx.x);
        const int unit = a.unit_rhs ? (MODE == 3 ? uj : 3 * uj) : -1;
        for (int t = tid; t < 3 * L.n; t += TBLOCK) {
            b[t] = a.unit_rhs ? (t == unit ? 1.0 : 0.0) : a.b_in[t];
            x[t] = (a.x_in_zero || a.unit_rhs) ? 0.0 : a.x_out[t];
        }
        __syncthreads();
    }
    // down: smoothing, residual, restriction
    for (int l = 0; l + 1 < a.nlev; ++l) {
        const TailLevel &L = lv[l];
        const TailLevel &C = lv[l + 1];
        double *x = lds + L.lds_off, *b = x + 3 * L.n, *r = b + 3 * L.n;
        tail_smooth<MODE>(a, L, x, b, r, true, l > 0 || a.x_in_zero, wave, lane);
        tail_residual<MODE>(L, x, b, r, wave, lane);
        double *xc = lds + C.lds_off, *bc = xc + 3 * C.n;
        for (int t = tid; t < 3 * C.n; t += TBLOCK) {
            const int J = t / 3, c = t % 3;
            double s = 0.0;
            for (int k = L.r_rowptr[J]; k < L.r_rowptr[J + 1]; ++k) s += L.r_val[k] * r[3 * L.r_col[k] + c];
            bc[t] = s;
            xc[t] = 0.0;
        }
        __syncthreads();
    }
    // coarsest: x = A_L^{-1} b with the explicit inverse
    {
        const TailLevel &L = lv[a.nlev - 1];
        double *x = lds + L.lds_off, *b = x + 3 * L.n;
        for (int row = wave; row < a.cm; row += TWAVES) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            const double *M = a.cinv + static_cast<int64_t>(row) * a.cm;
            for (int j = lane; j < a.cm; j += 64) {
                const double v = M[j];
                s0 += v * b[j * a.cnc];
                if (a.cnc > 1) {
                    s1 += v * b[j * a.cnc + 1];
                    s2 += v * b[j * a.cnc + 2];
                }
            }
            s0 = wave_sum(s0);
            s1 = wave_sum(s1);
            s2 = wave_sum(s2);
            if (lane < a.cnc) x[row * a.cnc + lane] = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
        }
        __syncthreads();
    }
    // up: prolongation and post-smoothing
    for (int l = a.nlev - 2; l >= 0; --l) {
        const TailLevel &L = lv[l];
        const TailLevel &C = lv[l + 1];
        double *x = lds + L.lds_off, *b = x + 3 * L.n, *r = b + 3 * L.n;
        const double *xc = lds + C.lds_off;
        for (int t = tid; t < 3 * L.n; t += TBLOCK) {
            const int I = t / 3, c = t % 3;
            double s = 0.0;
            for (int k = L.p_rowptr[I]; k < L.p_rowptr[I + 1]; ++k) s += L.p_val[k] * xc[3 * L.p_col[k] + c];
            x[t] += s;
        }
        __syncthreads();
        tail_smooth<MODE>(a, L, x, b, r, false, false, wave, lane);
    }
    {
        const TailLevel &L = lv[0];
        const double *x = lds + L.lds_off;
        if (a.unit_rhs) {
            const int64_t j = a.unit_base + static_cast<int64_t>(blockIdx.x);
            if constexpr (MODE == 3) {
                for (int i = tid; i < 3 * L.n; i += TBLOCK) a.x_out[static_cast<int64_t>(i) * a.m + j] = x[i];
            } else {
                for (int i = tid; i < L.n; i += TBLOCK) a.x_out[static_cast<int64_t>(i) * a.m + j] = x[3 * i];
            }
        } else {
            for (int t = tid; t < 3 * L.n; t += TBLOCK) a.x_out[t] = x[t];
        }
    }
}

void launch_tail(int mode, const TailArgs &a, int lds_bytes, int grid, hipStream_t s) {
    if (mode == 3)
        k_tail<3><<<grid, TBLOCK, lds_bytes, s>>>(a);
    else
        k_tail<1><<<grid, TBLOCK, lds_bytes, s>>>(a);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
