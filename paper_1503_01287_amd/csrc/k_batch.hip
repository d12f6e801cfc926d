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

__global__ void __launch_bounds__(CB) k_seg_multidot(const double *V, int64_t ld, int k, const double *w,
                                                     const ChunkView t, double *partial) {
    __shared__ double red[CB / 64];
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    double wv[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int i = threadIdx.x + e * CB;
        wv[e] = i < len ? w[s0 + i] : 0.0;
    }
    for (int j = 0; j < k; ++j) {
        const double *v = V + j * ld + s0;
        double a = 0.0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int i = threadIdx.x + e * CB;
            if (i < len) a += v[i] * wv[e];
        }
        a = block_sum(a, red);
        if (threadIdx.x == 0) partial[static_cast<int64_t>(j) * t.n + c] = a;
    }
}

void launch_seg_multidot(const double *V, int64_t ld, int k, const double *w, const ChunkView &t, double *partial,
                         hipStream_t s) {
    if (t.n <= 0 || k <= 0) return;
    k_seg_multidot<<<t.n, CB, 0, s>>>(V, ld, k, w, t, partial);
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

__global__ void __launch_bounds__(CB) k_seg_multi_axpy(const double *V, int64_t ld, int k, const double *h,
                                                       int kmax, double *w, const ChunkView t, int scaled) {
    const int c = blockIdx.x;
    const int64_t s0 = t.start[c];
    const int len = t.len[c];
    const double *hs = h + static_cast<int64_t>(t.seg[c]) * kmax;
    double inv = 1.0;
    if (scaled) {
        const double hn = hs[k + 1];
        inv = hn > 0.0 ? 1.0 / hn : 1.0;
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int i = threadIdx.x + e * CB;
        if (i >= len) continue;
        double a = w[s0 + i];
        for (int j = 0; j < k; ++j) a -= hs[j] * V[j * ld + s0 + i];
        w[s0 + i] = a * inv;
    }
}

void launch_seg_multi_axpy(const double *V, int64_t ld, int k, const double *h, int kmax, double *w,
                           const ChunkView &t, hipStream_t s) {
    if (t.n <= 0 || k <= 0) return;
    k_seg_multi_axpy<<<t.n, CB, 0, s>>>(V, ld, k, h, kmax, w, t, 0);
    AMG_CHECK_LAUNCH();
}

// one thread per system: hn = sqrt(h[k] - sum_{j<k} h[j]^2) into h[k + 1]
__global__ void k_seg_pythagoras(double *h, int k, int kmax, int nsys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsys) return;
    double *hs = h + static_cast<int64_t>(i) * kmax;
    double hsq = hs[k];
    for (int j = 0; j < k; ++j) hsq -= hs[j] * hs[j];
    hs[k + 1] = sqrt(fmax(hsq, 0.0));
}

void launch_seg_multi_axpy_normalize(const double *V, int64_t ld, int k, double *h, int kmax, double *w,
                                     const ChunkView &t, int nsys, hipStream_t s) {
    if (t.n <= 0 || nsys <= 0) return;
    k_seg_pythagoras<<<ceil_div(nsys, CB), CB, 0, s>>>(h, k, kmax, nsys);
    AMG_CHECK_LAUNCH();
    k_seg_multi_axpy<<<t.n, CB, 0, s>>>(V, ld, k, h, kmax, w, t, 1);
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

}  // namespace amgp2
