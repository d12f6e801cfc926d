// Row-statistics features and the damping-weight network (see learn.h).
// Reductions run in a fixed order (per-block tree, then one block over the
// partials; per-parameter gradient sums over the samples in order), so the
// results are deterministic.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "learn.h"

namespace amgp2 {

constexpr int LB = 256;

static int ceil_div_i(int64_t a, int b) { return static_cast<int>((a + b - 1) / b); }

// ------------------------------------------------------------ features
// Per scalar row: rho = sum_{off} |a| / |d|, sigma = (d + sum_{off} a) / d,
// tau = sqrt(sum_{off} a^2) / |d|, nz = stored scalars of the row.
// PASS 0 accumulates (rho, sigma, tau, nz, max rho); PASS 1 (rho - mean)^2.
// mean_sum: when not null, the mean of rho is mean_sum[0] / rows (the pass-0
// sum left on the device), else mean_rho.
template <int MODE, int PASS>
__global__ void __launch_bounds__(LB) k_row_stats(int rows, const int *rowptr, const int *col, const double *val,
                                                   int64_t nnz, double mean_rho, const double *mean_sum,
                                                   double *partial) {
    if (mean_sum) mean_rho = mean_sum[0] / rows;
    constexpr int NV = PASS == 0 ? 5 : 1;
    __shared__ double red[NV][LB];
    const int q = blockIdx.x * LB + threadIdx.x;
    double v[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = 0.0;
    if (q < rows) {
        const int i = MODE == 3 ? q / 3 : q;
        const int r = MODE == 3 ? q % 3 : 0;
        double d = 0.0, sabs = 0.0, ssum = 0.0, ssq = 0.0;
        const int b = rowptr[i], e = rowptr[i + 1];
        for (int k = b; k < e; ++k) {
            const int j = col[k];
#pragma unroll
            for (int c = 0; c < MODE; ++c) {
                const double a = val[static_cast<int64_t>(r * MODE + c) * nnz + k];
                if (j == i && c == r) {
                    d = a;
                } else {
                    sabs += fabs(a);
                    ssum += a;
                    ssq += a * a;
                }
            }
        }
        double rho = 0.0, sigma = 0.0, tau = 0.0;
        if (d != 0.0) {
            rho = sabs / fabs(d);
            sigma = (d + ssum) / d;
            tau = sqrt(ssq) / fabs(d);
        }
        // a scalar operator applied per component stands for 3 stored scalars per entry
        const double nz = 3.0 * (e - b);
        if constexpr (PASS == 0) {
            v[0] = rho;
            v[1] = sigma;
            v[2] = tau;
            v[3] = nz;
            v[4] = rho;
        } else {
            v[0] = (rho - mean_rho) * (rho - mean_rho);
        }
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = LB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                if (PASS == 0 && c == 4)
                    red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + o]);
                else
                    red[c][threadIdx.x] += red[c][threadIdx.x + o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < NV) partial[static_cast<int64_t>(blockIdx.x) * NV + threadIdx.x] = red[threadIdx.x][0];
}

// out[c] = sum (or max for c == 4 of pass 0) over the nb partials, fixed order
template <int NV>
__global__ void __launch_bounds__(LB) k_stats_reduce(const double *partial, int nb, double *out) {
    __shared__ double red[NV][LB];
    double v[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = 0.0;
    for (int b = threadIdx.x; b < nb; b += LB)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const double x = partial[static_cast<int64_t>(b) * NV + c];
            v[c] = (NV == 5 && c == 4) ? fmax(v[c], x) : v[c] + x;
        }
#pragma unroll
    for (int c = 0; c < NV; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = LB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
#pragma unroll
            for (int c = 0; c < NV; ++c)
                red[c][threadIdx.x] = (NV == 5 && c == 4) ? fmax(red[c][threadIdx.x], red[c][threadIdx.x + o])
                                                          : red[c][threadIdx.x] + red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < NV) out[threadIdx.x] = red[threadIdx.x][0];
}

template <int PASS>
static void stats_pass(int mode, int rows, const int *rowptr, const int *col, const double *val, int64_t nnz,
                       double mean, const double *mean_sum, double *partial, int nb, hipStream_t s) {
    if (mode == 3)
        k_row_stats<3, PASS><<<nb, LB, 0, s>>>(rows, rowptr, col, val, nnz, mean, mean_sum, partial);
    else
        k_row_stats<1, PASS><<<nb, LB, 0, s>>>(rows, rowptr, col, val, nnz, mean, mean_sum, partial);
    AMG_CHECK_LAUNCH();
}

void row_features(int mode, int n, const int *rowptr, const int *col, const double *val, int64_t nnz, int level,
                  double *f, hipStream_t s) {
    AMG_REQUIRE(mode == 1 || mode == 3, AMG_EINVAL, "row_features: mode must be 1 or 3");
    AMG_REQUIRE(n > 0, AMG_EINVAL, "row_features: empty level");
    const int rows = mode * n;
    const int nb = ceil_div_i(rows, LB);
    DevBuf<double> partial(static_cast<size_t>(nb) * 5), out(5);
    stats_pass<0>(mode, rows, rowptr, col, val, nnz, 0.0, nullptr, partial.p, nb, s);
    k_stats_reduce<5><<<1, LB, 0, s>>>(partial.p, nb, out.p);
    AMG_CHECK_LAUNCH();
    std::vector<double> a = out.download(s);
    const double mean = a[0] / rows;
    stats_pass<1>(mode, rows, rowptr, col, val, nnz, mean, nullptr, partial.p, nb, s);
    k_stats_reduce<1><<<1, LB, 0, s>>>(partial.p, nb, out.p);
    AMG_CHECK_LAUNCH();
    std::vector<double> b = out.download(s);
    f[0] = mean;
    f[1] = a[4];
    f[2] = std::sqrt(b[0] / rows);
    f[3] = a[1] / rows;
    f[4] = a[2] / rows;
    f[5] = a[3] / rows / 64.0;
    f[6] = level / 10.0;
    f[7] = std::log10(3.0 * n) / 7.0;
}

// ------------------------------------------------------------ features without allocation
// The same two passes with every intermediate in a fixed device array of the
// library (`scratch`, one copy per GPU for the life of the process) instead
// of buffers allocated per call, and the eight features written to the
// device: [0, 8) the reductions (pass-0 sums and maximum, pass-1 sum),
// [8, 8 + 5 nb) the per-block partials. Nothing in it needs clearing: each
// call writes every value it reads.
constexpr int64_t FEAT_SCRATCH_DOUBLES = 131072;  // 1 MiB
constexpr int64_t FEAT_PARTIAL_OFF = 8;
constexpr int FEAT_MAX_BLOCKS = static_cast<int>((FEAT_SCRATCH_DOUBLES - FEAT_PARTIAL_OFF) / 5);
static __device__ __align__(256) double scratch[FEAT_SCRATCH_DOUBLES];

int features_noalloc_max_rows() { return FEAT_MAX_BLOCKS * LB; }

// out[0..8) from the reductions, the same expressions as row_features' host part
__global__ void k_features_final(const double *red, int rows, int n, int level, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double mean = red[0] / rows;
    out[0] = mean;
    out[1] = red[4];
    out[2] = sqrt(red[5] / rows);
    out[3] = red[1] / rows;
    out[4] = red[2] / rows;
    out[5] = red[3] / rows / 64.0;
    out[6] = level / 10.0;
    out[7] = log10(3.0 * n) / 7.0;
}

void row_features_noalloc(int mode, int n, const int *rowptr, const int *col, const double *val, int64_t nnz,
                          int level, double *scratch_dev, double *f_dev, hipStream_t s) {
    AMG_REQUIRE(mode == 1 || mode == 3, AMG_EINVAL, "row_features: mode must be 1 or 3");
    AMG_REQUIRE(n > 0, AMG_EINVAL, "row_features: empty level");
    const int64_t rows64 = static_cast<int64_t>(mode) * n;
    AMG_REQUIRE(rows64 <= features_noalloc_max_rows(), AMG_EINVAL,
                "amg_level_features_noalloc: level has " + std::to_string(rows64) +
                    " scalar rows, more than the fixed scratch array serves (" +
                    std::to_string(features_noalloc_max_rows()) + ")");
    const int rows = static_cast<int>(rows64);
    const int nb = ceil_div_i(rows, LB);
    double *red = scratch_dev;
    double *partial = scratch_dev + FEAT_PARTIAL_OFF;
    stats_pass<0>(mode, rows, rowptr, col, val, nnz, 0.0, nullptr, partial, nb, s);
    k_stats_reduce<5><<<1, LB, 0, s>>>(partial, nb, red);
    AMG_CHECK_LAUNCH();
    stats_pass<1>(mode, rows, rowptr, col, val, nnz, 0.0, red, partial, nb, s);
    k_stats_reduce<1><<<1, LB, 0, s>>>(partial, nb, red + 5);
    AMG_CHECK_LAUNCH();
    k_features_final<<<1, 64, 0, s>>>(red, rows, n, level, f_dev);
    AMG_CHECK_LAUNCH();
}

// Device address of `scratch` on the current device: looked up once per
// device with that device current (each GPU holds its own copy of the array
// at its own address; the array's name is not a device address in host code).
double *features_scratch_address() {
    static std::mutex mu;
    static double *addr[64] = {};
    int d = 0;
    AMG_HIP(hipGetDevice(&d));
    AMG_REQUIRE(d >= 0 && d < 64, AMG_EINVAL, "features scratch: device index beyond 63");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[d]) {
        void *p = nullptr;
        AMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        AMG_REQUIRE(p != nullptr, AMG_EHIP, "features scratch: no device address");
        addr[d] = static_cast<double *>(p);
    }
    return addr[d];
}

// ------------------------------------------------------------ network
void MlpWork::reserve(int n) {
    if (n <= cap) return;
    X.alloc(static_cast<size_t>(n) * MLP_NF);
    y.alloc(n);
    H1.alloc(static_cast<size_t>(n) * MLP_NH);
    H2.alloc(static_cast<size_t>(n) * MLP_NH);
    S.alloc(n);
    om.alloc(n);
    D1.alloc(static_cast<size_t>(n) * MLP_NH);
    D2.alloc(static_cast<size_t>(n) * MLP_NH);
    D3.alloc(n);
    err2.alloc(n);
    cap = n;
}

// one thread per sample
__global__ void __launch_bounds__(LB) k_mlp_forward(const float *__restrict__ th, const float *__restrict__ X, int n,
                                                     float *H1, float *H2, float *S, float *om) {
    const int s = blockIdx.x * LB + threadIdx.x;
    if (s >= n) return;
    float x[MLP_NF], h1[MLP_NH], h2[MLP_NH];
#pragma unroll
    for (int k = 0; k < MLP_NF; ++k) x[k] = X[s * MLP_NF + k];
#pragma unroll
    for (int j = 0; j < MLP_NH; ++j) {
        float a = th[MLP_OB1 + j];
#pragma unroll
        for (int k = 0; k < MLP_NF; ++k) a += th[MLP_OW1 + j * MLP_NF + k] * x[k];
        h1[j] = tanhf(a);
        H1[s * MLP_NH + j] = h1[j];
    }
#pragma unroll 4
    for (int j = 0; j < MLP_NH; ++j) {
        float a = th[MLP_OB2 + j];
#pragma unroll
        for (int k = 0; k < MLP_NH; ++k) a += th[MLP_OW2 + j * MLP_NH + k] * h1[k];
        h2[j] = tanhf(a);
        H2[s * MLP_NH + j] = h2[j];
    }
    float z = th[MLP_OB3];
#pragma unroll
    for (int j = 0; j < MLP_NH; ++j) z += th[MLP_OW3 + j] * h2[j];
    const float sg = 1.0f / (1.0f + expf(-z));
    S[s] = sg;
    om[s] = MLP_OMEGA_MIN + MLP_OMEGA_SPAN * sg;
}

// per sample: dL/dz and the pre-activation deltas of both hidden layers
__global__ void __launch_bounds__(LB) k_mlp_delta(const float *__restrict__ th, const float *H1, const float *H2,
                                                   const float *S, const float *om, const float *y, int n, float *D1,
                                                   float *D2, float *D3, float *err2) {
    const int s = blockIdx.x * LB + threadIdx.x;
    if (s >= n) return;
    const float e = om[s] - y[s];
    err2[s] = e * e;
    const float sg = S[s];
    const float dz = (2.0f / n) * e * MLP_OMEGA_SPAN * sg * (1.0f - sg);
    D3[s] = dz;
    float d2[MLP_NH];
#pragma unroll
    for (int j = 0; j < MLP_NH; ++j) {
        const float h = H2[s * MLP_NH + j];
        d2[j] = dz * th[MLP_OW3 + j] * (1.0f - h * h);
        D2[s * MLP_NH + j] = d2[j];
    }
#pragma unroll 4
    for (int k = 0; k < MLP_NH; ++k) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < MLP_NH; ++j) a += d2[j] * th[MLP_OW2 + j * MLP_NH + k];
        const float h = H1[s * MLP_NH + k];
        D1[s * MLP_NH + k] = a * (1.0f - h * h);
    }
}

// one thread per parameter, sum over the samples in order
__global__ void __launch_bounds__(LB) k_mlp_grad(const float *X, const float *H1, const float *H2, const float *D1,
                                                  const float *D2, const float *D3, int n, float *g) {
    const int p = blockIdx.x * LB + threadIdx.x;
    if (p >= MLP_NP) return;
    float acc = 0.0f;
    if (p < MLP_OB1) {
        const int j = p / MLP_NF, k = p % MLP_NF;
        for (int s = 0; s < n; ++s) acc += D1[s * MLP_NH + j] * X[s * MLP_NF + k];
    } else if (p < MLP_OW2) {
        const int j = p - MLP_OB1;
        for (int s = 0; s < n; ++s) acc += D1[s * MLP_NH + j];
    } else if (p < MLP_OB2) {
        const int q = p - MLP_OW2, j = q / MLP_NH, k = q % MLP_NH;
        for (int s = 0; s < n; ++s) acc += D2[s * MLP_NH + j] * H1[s * MLP_NH + k];
    } else if (p < MLP_OW3) {
        const int j = p - MLP_OB2;
        for (int s = 0; s < n; ++s) acc += D2[s * MLP_NH + j];
    } else if (p < MLP_OB3) {
        const int j = p - MLP_OW3;
        for (int s = 0; s < n; ++s) acc += D3[s] * H2[s * MLP_NH + j];
    } else {
        for (int s = 0; s < n; ++s) acc += D3[s];
    }
    g[p] = acc;
}

// mean of err2 over n samples (one block, fixed order)
__global__ void __launch_bounds__(LB) k_mean(const float *v, int n, float *out) {
    __shared__ float red[LB];
    float a = 0.0f;
    for (int i = threadIdx.x; i < n; i += LB) a += v[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = LB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / n;
}

__global__ void __launch_bounds__(LB) k_adam(float *th, const float *g, float *m, float *v, float lr, float b1,
                                              float b2, float c1, float c2, float eps) {
    const int p = blockIdx.x * LB + threadIdx.x;
    if (p >= MLP_NP) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    th[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

void mlp_forward(const float *theta, const float *X, int n, MlpWork &w, hipStream_t s) {
    if (n <= 0) return;
    k_mlp_forward<<<ceil_div_i(n, LB), LB, 0, s>>>(theta, X, n, w.H1.p, w.H2.p, w.S.p, w.om.p);
    AMG_CHECK_LAUNCH();
}

void mlp_backward(const float *theta, int n, MlpWork &w, float *grad, float *loss_dev, hipStream_t s) {
    AMG_REQUIRE(n > 0, AMG_EINVAL, "mlp: empty batch");
    k_mlp_delta<<<ceil_div_i(n, LB), LB, 0, s>>>(theta, w.H1.p, w.H2.p, w.S.p, w.om.p, w.y.p, n, w.D1.p, w.D2.p,
                                                 w.D3.p, w.err2.p);
    AMG_CHECK_LAUNCH();
    k_mean<<<1, LB, 0, s>>>(w.err2.p, n, loss_dev);
    AMG_CHECK_LAUNCH();
    k_mlp_grad<<<ceil_div_i(MLP_NP, LB), LB, 0, s>>>(w.X.p, w.H1.p, w.H2.p, w.D1.p, w.D2.p, w.D3.p, n, grad);
    AMG_CHECK_LAUNCH();
}

void mlp_adam(float *theta, const float *grad, float *m, float *v, float lr, float beta1, float beta2, float c1,
              float c2, float eps, hipStream_t s) {
    k_adam<<<ceil_div_i(MLP_NP, LB), LB, 0, s>>>(theta, grad, m, v, lr, beta1, beta2, c1, c2, eps);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
