// Multiplicative Vanka kernels (see vanka.h): local-matrix assembly, batched
// Gauss-Jordan inversion and the coloured patch update. One workgroup per
// patch; local DOF a < 3 n_P is component a % 3 of node a / 3 of the patch,
// a = 3 n_P is the patch's pressure.
#include "common.h"
#include "vanka.h"

namespace amgp2 {

constexpr int VB = 256;

// position of column c in the sorted row [b, e) of idx, or -1
__device__ __forceinline__ int find_col(const int *idx, int b, int e, int c) {
    int lo = b, hi = e - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = idx[mid];
        if (v == c) return mid;
        if (v < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

__global__ void __launch_bounds__(VB) k_vanka_assemble(const VankaView v) {
    extern __shared__ int nodes[];
    const int i = blockIdx.x;
    const int p0 = v.pptr[i], nn = v.pptr[i + 1] - p0;
    for (int k = threadIdx.x; k < nn; k += VB) nodes[k] = v.pnode[p0 + k];
    __syncthreads();
    const int m = 3 * nn + 1;
    double *M = v.inv + v.moff[i];
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(m) * m; e += VB) {
        const int a = static_cast<int>(e % m), bcol = static_cast<int>(e / m);  // column-major
        double val = 0.0;
        const bool ap = a == 3 * nn, bp = bcol == 3 * nn;
        if (!ap && !bp) {
            const int ua = nodes[a / 3], ub = nodes[bcol / 3];
            const int q = find_col(v.acol, v.arow[ua], v.arow[ua + 1], ub);
            if (q >= 0) val = v.aval[static_cast<int64_t>((a % 3) * 3 + bcol % 3) * v.annz + q];
        } else if (!ap && bp) {  // B^T(u_a, i)[c_a]
            const int ua = nodes[a / 3];
            const int q = find_col(v.btcol, v.btrow[ua], v.btrow[ua + 1], i);
            if (q >= 0) val = v.btval[static_cast<int64_t>(a % 3) * v.btnnz + q];
        } else if (ap && !bp) {  // B(i, u_b)[c_b] = B^T(u_b, i)[c_b]
            const int ub = nodes[bcol / 3];
            const int q = find_col(v.btcol, v.btrow[ub], v.btrow[ub + 1], i);
            if (q >= 0) val = v.btval[static_cast<int64_t>(bcol % 3) * v.btnnz + q];
        } else if (v.crow) {     // -C(i, i)
            const int q = find_col(v.ccol, v.crow[i], v.crow[i + 1], i);
            if (q >= 0) val = -v.cval[q];
        }
        M[e] = val;
    }
}

void launch_vanka_assemble(const VankaView &v, int max_nodes, hipStream_t s) {
    if (v.npatch <= 0) return;
    k_vanka_assemble<<<v.npatch, VB, max_nodes * sizeof(int), s>>>(v);
    AMG_CHECK_LAUNCH();
}

// In-place Gauss-Jordan inversion with partial (row) pivoting of one
// column-major m x m matrix per workgroup; row swaps are undone as column
// swaps at the end.
__global__ void __launch_bounds__(VB) k_vanka_invert(const VankaView v, int *flag) {
    extern __shared__ unsigned char smem[];
    __shared__ double rv[VB];
    __shared__ int ri[VB];
    const int i = blockIdx.x;
    const int m = 3 * (v.pptr[i + 1] - v.pptr[i]) + 1;
    double *f = reinterpret_cast<double *>(smem);
    int *perm = reinterpret_cast<int *>(f + m);
    double *M = v.inv + v.moff[i];
    auto E = [&](int r, int c) -> double & { return M[static_cast<int64_t>(c) * m + r]; };
    for (int k = 0; k < m; ++k) {
        double best = -1.0;
        int bi = k;
        for (int r = k + threadIdx.x; r < m; r += VB) {
            const double a = fabs(E(r, k));
            if (a > best) {
                best = a;
                bi = r;
            }
        }
        rv[threadIdx.x] = best;
        ri[threadIdx.x] = bi;
        __syncthreads();
        for (int o = VB / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                const double b2 = rv[threadIdx.x + o];
                const int i2 = ri[threadIdx.x + o];
                if (b2 > rv[threadIdx.x] || (b2 == rv[threadIdx.x] && i2 < ri[threadIdx.x])) {
                    rv[threadIdx.x] = b2;
                    ri[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        const int piv = ri[0];
        const bool zero = rv[0] == 0.0;
        __syncthreads();
        if (zero) {
            if (threadIdx.x == 0) atomicOr(flag, 1);
            return;  // uniform across the workgroup
        }
        if (threadIdx.x == 0) perm[k] = piv;
        if (piv != k)
            for (int c = threadIdx.x; c < m; c += VB) {
                const double t = E(k, c);
                E(k, c) = E(piv, c);
                E(piv, c) = t;
            }
        __syncthreads();
        const double p = E(k, k);
        for (int r = threadIdx.x; r < m; r += VB) f[r] = E(r, k);
        __syncthreads();
        for (int r = threadIdx.x; r < m; r += VB) E(r, k) = r == k ? 1.0 : 0.0;
        __syncthreads();
        for (int c = threadIdx.x; c < m; c += VB) E(k, c) /= p;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < static_cast<int64_t>(m) * m; e += VB) {
            const int r = static_cast<int>(e % m), c = static_cast<int>(e / m);
            if (r != k) E(r, c) -= f[r] * E(k, c);
        }
        __syncthreads();
    }
    for (int k = m - 1; k >= 0; --k) {
        const int q = perm[k];
        if (q != k)
            for (int r = threadIdx.x; r < m; r += VB) {
                const double t = E(r, k);
                E(r, k) = E(r, q);
                E(r, q) = t;
            }
        __syncthreads();
    }
}

void launch_vanka_invert(const VankaView &v, int max_m, int *flag, hipStream_t s) {
    if (v.npatch <= 0) return;
    k_vanka_invert<<<v.npatch, VB, static_cast<size_t>(max_m) * (sizeof(double) + sizeof(int)), s>>>(v, flag);
    AMG_CHECK_LAUNCH();
}

// One colour of the multiplicative sweep, 1,024 threads per patch (a colour
// holds only a few hundred patches, so each needs many waves in flight):
// residual on the patch (VG lanes per node row, 64 rows at a time, over the
// node's A and B^T rows), correction with the patch's inverse (row tiles of
// 64 VR rows, the 16 wavefronts spread over tiles and column groups, partial
// sums added in LDS in a fixed order), update in place.
constexpr int VG = 16;
constexpr int VR = 4;     // rows per lane and pass in the apply
constexpr int VCB = 1024; // threads per patch: the ~m / 3 node rows of a patch at once
constexpr int VNW = VCB / 64;

__global__ void __launch_bounds__(VCB) k_vanka_colour(const VankaView v, const int *order, const double *b,
                                                      double *x, double omega) {
    extern __shared__ unsigned char smem[];
    const int i = order[blockIdx.x];
    const int p0 = v.pptr[i], nn = v.pptr[i + 1] - p0;
    const int m = 3 * nn + 1;
    double *r = reinterpret_cast<double *>(smem);
    double *part = r + m;                       // NG x m partial products (NG m <= m + 64 VR VNW)
    int *nodes = reinterpret_cast<int *>(part + m + 64 * VR * VNW);
    for (int k = threadIdx.x; k < nn; k += VCB) nodes[k] = v.pnode[p0 + k];
    __syncthreads();
    const int64_t nu = 3 * static_cast<int64_t>(v.n);
    const double *p = x + nu;
    const int grp = threadIdx.x / VG, lane = threadIdx.x % VG;
    for (int k = grp; k <= nn; k += VCB / VG) {
        if (k < nn) {
            const int u = nodes[k];
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int q = v.arow[u] + lane; q < v.arow[u + 1]; q += VG) {
                const int j = v.acol[q];
                const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
                s0 += v.aval[0 * v.annz + q] * x0 + v.aval[1 * v.annz + q] * x1 + v.aval[2 * v.annz + q] * x2;
                s1 += v.aval[3 * v.annz + q] * x0 + v.aval[4 * v.annz + q] * x1 + v.aval[5 * v.annz + q] * x2;
                s2 += v.aval[6 * v.annz + q] * x0 + v.aval[7 * v.annz + q] * x1 + v.aval[8 * v.annz + q] * x2;
            }
            for (int q = v.btrow[u] + lane; q < v.btrow[u + 1]; q += VG) {
                const double pq = p[v.btcol[q]];
                s0 += v.btval[q] * pq;
                s1 += v.btval[v.btnnz + q] * pq;
                s2 += v.btval[2 * v.btnnz + q] * pq;
            }
#pragma unroll
            for (int o = VG / 2; o > 0; o >>= 1) {
                s0 += __shfl_xor(s0, o, VG);
                s1 += __shfl_xor(s1, o, VG);
                s2 += __shfl_xor(s2, o, VG);
            }
            if (lane == 0) {
                r[3 * k] = b[3 * u] - s0;
                r[3 * k + 1] = b[3 * u + 1] - s1;
                r[3 * k + 2] = b[3 * u + 2] - s2;
            }
        } else {
            // pressure row: g_i - B_i u + C_i p
            double s = 0.0;
            for (int q = v.brow[i] + lane; q < v.brow[i + 1]; q += VG) {
                const int j = v.bcol[q];
                s += v.bval[q] * x[3 * j] + v.bval[v.bnnz + q] * x[3 * j + 1] + v.bval[2 * v.bnnz + q] * x[3 * j + 2];
            }
            if (v.crow)
                for (int q = v.crow[i] + lane; q < v.crow[i + 1]; q += VG) s -= v.cval[q] * p[v.ccol[q]];
#pragma unroll
            for (int o = VG / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, VG);
            if (lane == 0) r[3 * nn] = b[nu + i] - s;
        }
    }
    __syncthreads();
    const double *M = v.inv + v.moff[i];
    const int wave = threadIdx.x >> 6, wl = threadIdx.x & 63;
    // RT tiles of 64 * VR rows; the waves of a tile split the columns into NG groups
    const int RT = (m + 64 * VR - 1) / (64 * VR);
    const int NG = RT >= VNW ? 1 : VNW / RT;
    const int grpc = wave % NG;
    const int c0 = grpc * m / NG, c1 = (grpc + 1) * m / NG;
    for (int tile = wave / NG; tile < RT; tile += VNW / NG) {
        const int a0 = tile * 64 * VR;
        double acc[VR];
#pragma unroll
        for (int t = 0; t < VR; ++t) acc[t] = 0.0;
        // four columns' loads in flight per lane before their products are
        // added (still in column order)
        int c = c0;
        for (; c + 4 <= c1; c += 4) {
            double mv[4][VR], rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                rv[u] = r[c + u];
                const double *col = M + static_cast<int64_t>(c + u) * m;
#pragma unroll
                for (int t = 0; t < VR; ++t) {
                    const int a = a0 + wl + 64 * t;
                    mv[u][t] = a < m ? col[a] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < VR; ++t)
                    if (a0 + wl + 64 * t < m) acc[t] += mv[u][t] * rv[u];
        }
        for (; c < c1; ++c) {
            const double rc = r[c];
            const double *col = M + static_cast<int64_t>(c) * m;
#pragma unroll
            for (int t = 0; t < VR; ++t) {
                const int a = a0 + wl + 64 * t;
                if (a < m) acc[t] += col[a] * rc;
            }
        }
#pragma unroll
        for (int t = 0; t < VR; ++t) {
            const int a = a0 + wl + 64 * t;
            if (a < m) part[grpc * m + a] = acc[t];
        }
    }
    __syncthreads();
    for (int a = threadIdx.x; a < m; a += VCB) {
        double sum = 0.0;
        const int RT = (m + 64 * VR - 1) / (64 * VR);
        const int NG = RT >= VNW ? 1 : VNW / RT;
        for (int g = 0; g < NG; ++g) sum += part[g * m + a];
        const double d = omega * sum;
        if (a < 3 * nn) x[3 * static_cast<int64_t>(nodes[a / 3]) + a % 3] += d;
        else x[nu + i] += d;
    }
}

void launch_vanka_colour(const VankaView &v, const int *order, int count, int max_nodes, const double *b,
                         double *x, double omega, hipStream_t s) {
    if (count <= 0) return;
    const int max_m = 3 * max_nodes + 1;
    const size_t lds = static_cast<size_t>(2 * max_m + 64 * VR * VNW) * sizeof(double) + max_nodes * sizeof(int);
    k_vanka_colour<<<count, VCB, lds, s>>>(v, order, b, x, omega);
    AMG_CHECK_LAUNCH();
}

// Residual of every patch of a colour into rbuf (same arithmetic as the
// fused kernel's first phase).
__global__ void __launch_bounds__(VCB) k_vanka_resid(const VankaView v, const int *order, const int64_t *roff,
                                                     double *rbuf, const double *b, const double *x) {
    extern __shared__ int snodes[];
    const int i = order[blockIdx.x];
    const int p0 = v.pptr[i], nn = v.pptr[i + 1] - p0;
    for (int k = threadIdx.x; k < nn; k += VCB) snodes[k] = v.pnode[p0 + k];
    __syncthreads();
    double *r = rbuf + roff[i];
    const int64_t nu = 3 * static_cast<int64_t>(v.n);
    const double *p = x + nu;
    const int grp = threadIdx.x / VG, lane = threadIdx.x % VG;
    for (int k = grp; k <= nn; k += VCB / VG) {
        if (k < nn) {
            const int u = snodes[k];
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int q = v.arow[u] + lane; q < v.arow[u + 1]; q += VG) {
                const int j = v.acol[q];
                const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
                s0 += v.aval[0 * v.annz + q] * x0 + v.aval[1 * v.annz + q] * x1 + v.aval[2 * v.annz + q] * x2;
                s1 += v.aval[3 * v.annz + q] * x0 + v.aval[4 * v.annz + q] * x1 + v.aval[5 * v.annz + q] * x2;
                s2 += v.aval[6 * v.annz + q] * x0 + v.aval[7 * v.annz + q] * x1 + v.aval[8 * v.annz + q] * x2;
            }
            for (int q = v.btrow[u] + lane; q < v.btrow[u + 1]; q += VG) {
                const double pq = p[v.btcol[q]];
                s0 += v.btval[q] * pq;
                s1 += v.btval[v.btnnz + q] * pq;
                s2 += v.btval[2 * v.btnnz + q] * pq;
            }
#pragma unroll
            for (int o = VG / 2; o > 0; o >>= 1) {
                s0 += __shfl_xor(s0, o, VG);
                s1 += __shfl_xor(s1, o, VG);
                s2 += __shfl_xor(s2, o, VG);
            }
            if (lane == 0) {
                r[3 * k] = b[3 * u] - s0;
                r[3 * k + 1] = b[3 * u + 1] - s1;
                r[3 * k + 2] = b[3 * u + 2] - s2;
            }
        } else {
            double s = 0.0;
            for (int q = v.brow[i] + lane; q < v.brow[i + 1]; q += VG) {
                const int j = v.bcol[q];
                s += v.bval[q] * x[3 * j] + v.bval[v.bnnz + q] * x[3 * j + 1] + v.bval[2 * v.bnnz + q] * x[3 * j + 2];
            }
            if (v.crow)
                for (int q = v.crow[i] + lane; q < v.crow[i + 1]; q += VG) s -= v.cval[q] * p[v.ccol[q]];
#pragma unroll
            for (int o = VG / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, VG);
            if (lane == 0) r[3 * nn] = b[nu + i] - s;
        }
    }
}

// 64 rows of one patch's correction per workgroup: lane = row, the NW
// wavefronts take 1 / NW of the columns each, partial sums added in LDS in
// wavefront order.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_vanka_apply(const VankaView v, const int *order, const int *tpre,
                                                         int count, const int64_t *roff, const double *rbuf,
                                                         double *x, double omega) {
    __shared__ double part[NW][64];
    int lo = 0, hi = count - 1;
    const int t = blockIdx.x;
    while (lo < hi) {  // last patch whose first tile is <= t
        const int mid = (lo + hi + 1) >> 1;
        if (tpre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int i = order[lo];
    const int p0 = v.pptr[i], nn = v.pptr[i + 1] - p0;
    const int m = 3 * nn + 1;
    const int a = (t - tpre[lo]) * 64 + (threadIdx.x & 63);
    const int wave = threadIdx.x >> 6;
    const double *r = rbuf + roff[i];
    const double *M = v.inv + v.moff[i];
    const int c0 = wave * m / NW, c1 = (wave + 1) * m / NW;
    double acc = 0.0;
    if (a < m) {
        int c = c0;
        for (; c + 8 <= c1; c += 8) {  // eight column loads in flight per lane
            double mv[8], rv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                mv[u] = M[static_cast<int64_t>(c + u) * m + a];
                rv[u] = r[c + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += mv[u] * rv[u];
        }
        for (; c < c1; ++c) acc += M[static_cast<int64_t>(c) * m + a] * r[c];
    }
    part[wave][threadIdx.x & 63] = acc;
    __syncthreads();
    if (wave != 0 || a >= m) return;
    const int l = threadIdx.x;
    double sum = part[0][l];
#pragma unroll
    for (int w = 1; w < NW; ++w) sum += part[w][l];
    const double d = omega * sum;
    if (a < 3 * nn) x[3 * static_cast<int64_t>(v.pnode[p0 + a / 3]) + a % 3] += d;
    else x[3 * static_cast<int64_t>(v.n) + i] += d;
}

// Partial corrections of one colour's large patches, tiled in two dimensions
// so that a colour of few, large patches still fills the GPU: workgroup u
// takes 64 rows (row tile rt) and a chunk of cc columns (chunk q) of one
// patch's inverse (upre: prefix of the units ceil(m_i / 64) ceil(m_i / cc)
// over the colour's patches, rt fastest); its 4 wavefronts take a quarter of
// the chunk each, eight column loads in flight per lane, and their sums are
// added in a fixed order into pbuf (chunk q of patch i at pbuf + poff[i] +
// q m_i).
__global__ void __launch_bounds__(VB) k_vanka_apply_part(const VankaView v, const int *order, const int *upre,
                                                         int count, int cc, const int64_t *roff, const double *rbuf,
                                                         const int64_t *poff, double *pbuf) {
    __shared__ double part[4][64];
    int lo = 0, hi = count - 1;
    const int u = blockIdx.x;
    while (lo < hi) {  // last patch whose first unit is <= u
        const int mid = (lo + hi + 1) >> 1;
        if (upre[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    const int i = order[lo];
    const int m = 3 * (v.pptr[i + 1] - v.pptr[i]) + 1;
    const int RT = (m + 63) / 64;
    const int local = u - upre[lo];
    const int rt = local % RT, q = local / RT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int a = rt * 64 + lane;
    const int c0 = q * cc, c1 = min(m, c0 + cc);
    const int w0 = c0 + wave * (c1 - c0) / 4, w1 = c0 + (wave + 1) * (c1 - c0) / 4;
    const double *r = rbuf + roff[i];
    const double *M = v.inv + v.moff[i];
    double acc = 0.0;
    if (a < m) {
        int c = w0;
        for (; c + 8 <= w1; c += 8) {
            double mv[8], rv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                mv[t] = M[static_cast<int64_t>(c + t) * m + a];
                rv[t] = r[c + t];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) acc += mv[t] * rv[t];
        }
        for (; c < w1; ++c) acc += M[static_cast<int64_t>(c) * m + a] * r[c];
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && a < m) pbuf[poff[i] + static_cast<int64_t>(q) * m + a] = ((part[0][lane] + part[1][lane]) +
                                                                               part[2][lane]) + part[3][lane];
}

// x_P += omega (sum of the chunks' partials, in chunk order) over 64-row tiles
// (tpre: prefix of ceil(m_i / 64) over the colour's patches)
__global__ void __launch_bounds__(64) k_vanka_reduce(const VankaView v, const int *order, const int *tpre,
                                                     int count, int cc, const int64_t *poff, const double *pbuf,
                                                     double *x, double omega) {
    int lo = 0, hi = count - 1;
    const int t = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tpre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int i = order[lo];
    const int p0 = v.pptr[i], nn = v.pptr[i + 1] - p0;
    const int m = 3 * nn + 1;
    const int a = (t - tpre[lo]) * 64 + threadIdx.x;
    if (a >= m) return;
    const int kc = (m + cc - 1) / cc;
    double sum = 0.0;
    for (int q = 0; q < kc; ++q) sum += pbuf[poff[i] + static_cast<int64_t>(q) * m + a];
    const double d = omega * sum;
    if (a < 3 * nn) x[3 * static_cast<int64_t>(v.pnode[p0 + a / 3]) + a % 3] += d;
    else x[3 * static_cast<int64_t>(v.n) + i] += d;
}

// Residuals of one colour's patches, VB / G node rows (G lanes each) per
// workgroup so that a colour of few, large patches still spreads over the
// GPU (rpre: prefix of ceil((n_P + 1) / (VB / G)) over the colour's
// patches; the last row of a patch is its pressure row); with G = 16 the
// same arithmetic as k_vanka_resid, wider groups for the long rows of
// coarse levels.
template <int G>
__global__ void __launch_bounds__(VB) k_vanka_resid_rows(const VankaView v, const int *order, const int *rpre,
                                                         int count, const int64_t *roff, double *rbuf,
                                                         const double *b, const double *x) {
    constexpr int VRW = VB / G;  // node rows per workgroup
    int lo = 0, hi = count - 1;
    const int t = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rpre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int i = order[lo];
    const int p0 = v.pptr[i], nn = v.pptr[i + 1] - p0;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int k = (t - rpre[lo]) * VRW + grp;
    if (k > nn) return;  // whole G-lane groups leave together
    double *r = rbuf + roff[i];
    const int64_t nu = 3 * static_cast<int64_t>(v.n);
    const double *p = x + nu;
    if (k < nn) {
        const int u = v.pnode[p0 + k];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = v.arow[u] + lane; q < v.arow[u + 1]; q += G) {
            const int j = v.acol[q];
            const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
            s0 += v.aval[0 * v.annz + q] * x0 + v.aval[1 * v.annz + q] * x1 + v.aval[2 * v.annz + q] * x2;
            s1 += v.aval[3 * v.annz + q] * x0 + v.aval[4 * v.annz + q] * x1 + v.aval[5 * v.annz + q] * x2;
            s2 += v.aval[6 * v.annz + q] * x0 + v.aval[7 * v.annz + q] * x1 + v.aval[8 * v.annz + q] * x2;
        }
        for (int q = v.btrow[u] + lane; q < v.btrow[u + 1]; q += G) {
            const double pq = p[v.btcol[q]];
            s0 += v.btval[q] * pq;
            s1 += v.btval[v.btnnz + q] * pq;
            s2 += v.btval[2 * v.btnnz + q] * pq;
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o, G);
            s1 += __shfl_xor(s1, o, G);
            s2 += __shfl_xor(s2, o, G);
        }
        if (lane == 0) {
            r[3 * k] = b[3 * u] - s0;
            r[3 * k + 1] = b[3 * u + 1] - s1;
            r[3 * k + 2] = b[3 * u + 2] - s2;
        }
    } else {
        double s = 0.0;
        for (int q = v.brow[i] + lane; q < v.brow[i + 1]; q += G) {
            const int j = v.bcol[q];
            s += v.bval[q] * x[3 * j] + v.bval[v.bnnz + q] * x[3 * j + 1] + v.bval[2 * v.bnnz + q] * x[3 * j + 2];
        }
        if (v.crow)
            for (int q = v.crow[i] + lane; q < v.crow[i + 1]; q += G) s -= v.cval[q] * p[v.ccol[q]];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (lane == 0) r[3 * nn] = b[nu + i] - s;
    }
}

static void resid_rows(const VankaView &v, const int *order, const int *rpre, int count, int nrunits, int rg,
                       const int64_t *roff, double *rbuf, const double *b, const double *x, hipStream_t s) {
    switch (rg) {
        case 16: k_vanka_resid_rows<16><<<nrunits, VB, 0, s>>>(v, order, rpre, count, roff, rbuf, b, x); break;
        case 32: k_vanka_resid_rows<32><<<nrunits, VB, 0, s>>>(v, order, rpre, count, roff, rbuf, b, x); break;
        case 64: k_vanka_resid_rows<64><<<nrunits, VB, 0, s>>>(v, order, rpre, count, roff, rbuf, b, x); break;
        default: throw Error(AMG_EINVAL, "Vanka residual: 16, 32 or 64 lanes per row");
    }
    AMG_CHECK_LAUNCH();
}

void launch_vanka_colour_rows(const VankaView &v, const int *order, const int *tpre, const int *rpre, int count,
                              int ntiles, int nrunits, int rg, int aw, const int64_t *roff, double *rbuf,
                              const double *b, double *x, double omega, hipStream_t s) {
    if (count <= 0) return;
    resid_rows(v, order, rpre, count, nrunits, rg, roff, rbuf, b, x, s);
    switch (aw) {
        case 4: k_vanka_apply<4><<<ntiles, 256, 0, s>>>(v, order, tpre, count, roff, rbuf, x, omega); break;
        case 8: k_vanka_apply<8><<<ntiles, 512, 0, s>>>(v, order, tpre, count, roff, rbuf, x, omega); break;
        case 16: k_vanka_apply<16><<<ntiles, 1024, 0, s>>>(v, order, tpre, count, roff, rbuf, x, omega); break;
        default: throw Error(AMG_EINVAL, "Vanka corrections: 4, 8 or 16 wavefronts per tile");
    }
    AMG_CHECK_LAUNCH();
}

void launch_vanka_colour_tiled(const VankaView &v, const int *order, const int *tpre, const int *upre,
                               const int *rpre, int count, int ntiles, int nunits, int nrunits, int cc, int rg,
                               const int64_t *roff, double *rbuf, const int64_t *poff, double *pbuf, const double *b,
                               double *x, double omega, hipStream_t s) {
    if (count <= 0) return;
    resid_rows(v, order, rpre, count, nrunits, rg, roff, rbuf, b, x, s);
    k_vanka_apply_part<<<nunits, VB, 0, s>>>(v, order, upre, count, cc, roff, rbuf, poff, pbuf);
    AMG_CHECK_LAUNCH();
    k_vanka_reduce<<<ntiles, 64, 0, s>>>(v, order, tpre, count, cc, poff, pbuf, x, omega);
    AMG_CHECK_LAUNCH();
}

void launch_vanka_colour_split(const VankaView &v, const int *order, const int *tpre, int count, int ntiles,
                               int max_nodes, const int64_t *roff, double *rbuf, const double *b, double *x,
                               double omega, hipStream_t s) {
    if (count <= 0) return;
    k_vanka_resid<<<count, VCB, max_nodes * sizeof(int), s>>>(v, order, roff, rbuf, b, x);
    AMG_CHECK_LAUNCH();
    k_vanka_apply<4><<<ntiles, 256, 0, s>>>(v, order, tpre, count, roff, rbuf, x, omega);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
