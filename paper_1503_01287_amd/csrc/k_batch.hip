// Segmented vector kernels of a batch (see batch.h). One workgroup per chunk;
// every reduction runs in a fixed order, so results are deterministic.
#include "batch.h"
#include "common.h"

namespace amgp2 {

constexpr int CB = 256;
constexpr int PER = BATCH_CHUNK / CB;

__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < CB / 64; ++w) t += red[w];
    return t;
}

// Workgroup (c, g) dots chunk c of the NR right-hand sides (held in
// registers) with the same chunk of basis vectors g * SMD_VEC ..
// g * SMD_VEC + SMD_VEC - 1: every basis chunk is read once for all
// right-hand sides and one block reduction serves the whole group. Right-
// hand side r's dot with vector j goes to partial[(r * k + j) * n_chunks + c].
// With `want`, chunks of systems s with want[s] == 0 are skipped (their
// partial entries are left as they were).
constexpr int SMD_VEC = 8;

template <int NR>
__global__ void __launch_bounds__(CB) k_seg_multidot(const double *V, int64_t ld, int k, const double *w0,
                                                     const double *w1, const ChunkView t, const int *want,
                                                     double *partial) {
    __shared__ double red[NR * SMD_VEC][CB / 64];
    const int c = blockIdx.x;
    if (want && !want[t.seg[c]]) return;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    const int j0 = blockIdx.y * SMD_VEC;
    const int nv = min(SMD_VEC, k - j0);
    double wv[NR][PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int i = threadIdx.x + e * CB;
        wv[0][e] = i < len ? w0[s0 + i] : 0.0;
        if (NR == 2) wv[NR - 1][e] = i < len ? w1[s0 + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < SMD_VEC; ++q) {
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = 0.0;
        if (q < nv) {
            const double *v = V + (j0 + q) * ld + s0;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int i = threadIdx.x + e * CB;
                if (i < len) {
                    const double vi = v[i];
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r] += vi * wv[r][e];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double a = acc[r];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
            if ((threadIdx.x & 63) == 0) red[r * SMD_VEC + q][threadIdx.x >> 6] = a;
        }
    }
    __syncthreads();
    if (threadIdx.x < NR * nv) {
        const int r = threadIdx.x / nv, q = threadIdx.x % nv;
        double a = 0.0;
        for (int w = 0; w < CB / 64; ++w) a += red[r * SMD_VEC + q][w];
        partial[(static_cast<int64_t>(r) * k + j0 + q) * t.n + c] = a;
    }
}

void launch_seg_multidot(const double *V, int64_t ld, int k, const double *w, const ChunkView &t, double *partial,
                         hipStream_t s) {
    launch_seg_multidot_masked(V, ld, k, w, t, nullptr, partial, s);
}

void launch_seg_multidot_masked(const double *V, int64_t ld, int k, const double *w, const ChunkView &t,
                                const int *want, double *partial, hipStream_t s) {
    if (t.n <= 0 || k <= 0) return;
    k_seg_multidot<1><<<dim3(t.n, ceil_div(k, SMD_VEC)), CB, 0, s>>>(V, ld, k, w, w, t, want, partial);
    AMG_CHECK_LAUNCH();
}

void launch_seg_multidot2(const double *V, int64_t ld, int k, const double *a, const double *b, const ChunkView &t,
                          double *partial, hipStream_t s) {
    if (t.n <= 0 || k <= 0) return;
    k_seg_multidot<2><<<dim3(t.n, ceil_div(k, SMD_VEC)), CB, 0, s>>>(V, ld, k, a, b, t, nullptr, partial);
    AMG_CHECK_LAUNCH();
}

// The delayed-reorthogonalisation step of every system (see
// launch_seg_dcgs2_update): chunk c takes its system's dots from
// h + seg * stride.
template <bool REORTH>
__global__ void __launch_bounds__(CB) k_seg_dcgs2_update(double *V, int64_t ld, int j, double *h, int stride,
                                                         const ChunkView t) {
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    double *hs = h + static_cast<int64_t>(t.seg[c]) * stride;
    const int k = j + 2;
    const double *dA = hs, *dB = hs + k;
    double ss = 0.0, sc = 0.0, cc = 0.0;
    for (int q = 0; q < j; ++q) {
        if (REORTH) {
            ss += dA[q] * dA[q];
            sc += dA[q] * dB[q];
        }
        cc += dB[q] * dB[q];
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
    // basis vectors outer, the thread's PER entries inner: PER independent
    // loads in flight per vector
    double as[PER], ac[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) as[e] = ac[e] = 0.0;
    for (int q = 0; q < j; ++q) {
        const double sq = REORTH ? dA[q] : 0.0, cq = dB[q];
        const double *v = V + q * ld + s0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int i = threadIdx.x + e * CB;
            if (i < len) {
                const double vi = v[i];
                if (REORTH) as[e] += sq * vi;
                ac[e] += cq * vi;
            }
        }
    }
    double *vj = V + static_cast<int64_t>(j) * ld + s0, *w = V + static_cast<int64_t>(j + 1) * ld + s0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int i = threadIdx.x + e * CB;
        if (i >= len) continue;
        double u = vj[i];
        if (REORTH) {
            u = (u - as[e]) * ig;
            vj[i] = u;
        }
        w[i] = (w[i] - ac[e] - d * u) * ie;
    }
    // every chunk of the system writes the same three values; the dots
    // read above lie below them
    if (threadIdx.x == 0) {
        hs[2 * k] = gam;
        hs[2 * k + 1] = d;
        hs[2 * k + 2] = eta;
    }
}

void launch_seg_dcgs2_update(double *V, int64_t ld, int j, double *h, int stride, const ChunkView &t, bool reorth,
                             hipStream_t s) {
    if (t.n <= 0) return;
    if (reorth)
        k_seg_dcgs2_update<true><<<t.n, CB, 0, s>>>(V, ld, j, h, stride, t);
    else
        k_seg_dcgs2_update<false><<<t.n, CB, 0, s>>>(V, ld, j, h, stride, t);
    AMG_CHECK_LAUNCH();
}

// one workgroup per (system, column)
__global__ void __launch_bounds__(CB) k_seg_reduce(const double *partial, int n, int k, const int *c0,
                                                   const int *c1, const int *c2, const int *c3, double *h,
                                                   int kmax) {
    __shared__ double red[CB / 64];
    const int i = blockIdx.x / k, j = blockIdx.x % k;
    const double *p = partial + static_cast<int64_t>(j) * n;
    double a = 0.0;
    for (int c = c0[i] + threadIdx.x; c < c1[i]; c += CB) a += p[c];
    for (int c = c2[i] + threadIdx.x; c < c3[i]; c += CB) a += p[c];
    a = block_sum(a, red);
    if (threadIdx.x == 0) h[static_cast<int64_t>(i) * kmax + j] = a;
}

void launch_seg_reduce(const double *partial, int n, int k, int nsys, const int *c0, const int *c1, const int *c2,
                       const int *c3, double *h, int kmax, hipStream_t s) {
    if (nsys <= 0 || k <= 0) return;
    k_seg_reduce<<<nsys * k, CB, 0, s>>>(partial, n, k, c0, c1, c2, c3, h, kmax);
    AMG_CHECK_LAUNCH();
}

__global__ void __launch_bounds__(CB) k_seg_scale(const double *x, double *y, const double *coef, const ChunkView t) {
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    const double a = coef[t.seg[c]];
    for (int i = threadIdx.x; i < len; i += CB) y[s0 + i] = a * x[s0 + i];
}

void launch_seg_scale(const double *x, double *y, const double *coef, const ChunkView &t, hipStream_t s) {
    if (t.n <= 0) return;
    k_seg_scale<<<t.n, CB, 0, s>>>(x, y, coef, t);
    AMG_CHECK_LAUNCH();
}

// y = a[seg] x + b[seg] y
__global__ void __launch_bounds__(CB) k_seg_axpby(const double *x, double *y, const double *a, const double *b,
                                                  const ChunkView t) {
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    const double ca = a[t.seg[c]], cb = b[t.seg[c]];
    for (int i = threadIdx.x; i < len; i += CB) y[s0 + i] = ca * x[s0 + i] + cb * y[s0 + i];
}

void launch_seg_axpby(const double *x, double *y, const double *a, const double *b, const ChunkView &t,
                      hipStream_t s) {
    if (t.n <= 0) return;
    k_seg_axpby<<<t.n, CB, 0, s>>>(x, y, a, b, t);
    AMG_CHECK_LAUNCH();
}

__global__ void __launch_bounds__(CB) k_seg_multi_add(const double *Z, int64_t ld, const double *y, int kmax,
                                                      const int *cnt, double *x, const ChunkView t) {
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    const int sg = t.seg[c];
    const int k = cnt[sg];
    const double *ys = y + static_cast<int64_t>(sg) * kmax;
    for (int i = threadIdx.x; i < len; i += CB) {
        double a = x[s0 + i];
        for (int j = 0; j < k; ++j) a += ys[j] * Z[j * ld + s0 + i];
        x[s0 + i] = a;
    }
}

void launch_seg_multi_add(const double *Z, int64_t ld, const double *y, int kmax, const int *cnt, double *x,
                          const ChunkView &t, hipStream_t s) {
    if (t.n <= 0) return;
    k_seg_multi_add<<<t.n, CB, 0, s>>>(Z, ld, y, kmax, cnt, x, t);
    AMG_CHECK_LAUNCH();
}

__global__ void __launch_bounds__(CB) k_seg_copy(const double *src, double *dst, const ChunkView t,
                                                 const int64_t *dstart) {
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c], d0 = dstart[c];
    const int len = t.len[c];
    for (int i = threadIdx.x; i < len; i += CB) dst[d0 + i] = src[s0 + i];
}

void launch_seg_copy(const double *src, double *dst, const ChunkView &t, const int64_t *dstart, hipStream_t s) {
    if (t.n <= 0) return;
    k_seg_copy<<<t.n, CB, 0, s>>>(src, dst, t, dstart);
    AMG_CHECK_LAUNCH();
}

__global__ void k_copy_shift_i32(const int *src, int64_t n, int add, int *dst) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * CB + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * CB)
        dst[k] = (src ? src[k] : 0) + add;
}

void launch_copy_shift_i32(const int *src, int64_t n, int add, int *dst, hipStream_t s) {
    if (n <= 0) return;
    const int nb = static_cast<int>(std::min<int64_t>(4096, (n + CB - 1) / CB));
    k_copy_shift_i32<<<nb, CB, 0, s>>>(src, n, add, dst);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
