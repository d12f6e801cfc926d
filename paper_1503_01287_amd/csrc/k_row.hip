// Row kernels (SpMV, residual, damped block Jacobi, coloured block
// Gauss-Seidel, restriction, prolongation), Krylov vector kernels, the
// coarsest-level dense solve and smoother setup kernels. gfx950, wave64.
//
// All of these are bound by HBM bandwidth: a 3x3 FP64 block costs 76 bytes
// (72 value bytes + a 4-byte column index) for 18 flops. The row kernels give
// each matrix row a group of G lanes; lane t of the group walks the row's
// entries t, t+G, ..., so each plane load of the group is one contiguous
// segment, and the 3 partial sums are reduced across the group with
// cross-lane shuffles.
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace amgp2 {

constexpr int BLOCK = 256;

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Sum over the NT threads of a block (deterministic order); result in thread 0.
template <int NT = BLOCK>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[NT / 64];
    v = group_sum<64>(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) t += red[i];
    }
    return t;
}

// s += A_k x_j for entry k (a 3x3 block of nine planes, or a scalar that
// multiplies every component)
template <int MODE>
__device__ __forceinline__ void acc_entry(const double *val, int64_t nz, int k, double x0, double x1, double x2,
                                          double &s0, double &s1, double &s2) {
    if constexpr (MODE == 3) {
        const double *v = val + k;
        s0 += v[0] * x0 + v[nz] * x1 + v[2 * nz] * x2;
        s1 += v[3 * nz] * x0 + v[4 * nz] * x1 + v[5 * nz] * x2;
        s2 += v[6 * nz] * x0 + v[7 * nz] * x1 + v[8 * nz] * x2;
    } else {
        const double v = val[k];
        s0 += v * x0;
        s1 += v * x1;
        s2 += v * x2;
    }
}

// U entries per lane and loop trip (1, 2 or 4): the trip's column indices,
// then its gathers of x and its values, are in flight together; entries past
// the row's end are skipped. Each lane still adds its entries in increasing
// order, so the result does not depend on U.
template <int MODE, int G, int OP, int U>
__global__ void __launch_bounds__(BLOCK) k_row(const RowArgs a) {
    // Workgroups are dispatched round-robin over the 8 XCDs, so consecutive
    // row blocks run on different XCDs at the same time and the whole chip
    // streams through one region of the matrix. Contiguous ranges per XCD
    // (xcd_chunks) are chosen by the setup-time tuner where they pay: they
    // keep each XCD's gathers of x inside its own L2.
    const int64_t blk = a.xcd_chunks ? xcd_chunk_block() : static_cast<int64_t>(blockIdx.x);
    const int64_t t = blk * BLOCK + threadIdx.x;
    const int g = static_cast<int>(t / G);
    const int lane = static_cast<int>(t % G);
    const bool active = g < a.nrows;
    constexpr bool NEEDS_B = OP == OP_RESID || OP == OP_JACOBI || OP == OP_GS;
    constexpr bool NEEDS_D = OP == OP_JACOBI || OP == OP_GS;
    constexpr bool NEEDS_OWN = OP == OP_SPMV_ADD || OP == OP_JACOBI || OP == OP_GS || OP == OP_SPMV_DOT;
    // Row-local operands of the epilogue are loaded first so that their
    // latency overlaps the row's matrix loads instead of following them.
    const int i = active ? (a.rowid ? a.rowid[g] : g) : 0;
    const bool ep = active && lane < 3;
    const int c = ep ? lane : 0;
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0, own = 0.0;
    if (ep) {
        if constexpr (NEEDS_B) {
            b0 = a.b[3 * i];
            b1 = a.b[3 * i + 1];
            b2 = a.b[3 * i + 2];
        }
        if constexpr (NEEDS_D) {
            if constexpr (MODE == 3) {
                const double *D = a.dinv + i;
                const int64_t dn = a.dinv_n;
                d0 = D[(3 * c) * dn];
                d1 = D[(3 * c + 1) * dn];
                d2 = D[(3 * c + 2) * dn];
            } else {
                d0 = a.dinv[i];
            }
        }
        if constexpr (NEEDS_OWN) own = (OP == OP_SPMV_ADD || OP == OP_GS) ? a.y[3 * i + c] : a.x[3 * i + c];
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (active) {
        const int beg = a.rowptr[g], end = a.rowptr[g + 1];
        const int64_t nz = a.nnz;
        if constexpr (U == 1) {
            for (int k = beg + lane; k < end; k += G) {
                const int j = a.col[k];
                const double x0 = a.x[3 * j], x1 = a.x[3 * j + 1], x2 = a.x[3 * j + 2];
                acc_entry<MODE>(a.val, nz, k, x0, x1, x2, s0, s1, s2);
            }
        } else {
            for (int k = beg + lane; k < end; k += U * G) {
                int j[U];
#pragma unroll
                for (int u = 0; u < U; ++u) j[u] = k + u * G < end ? a.col[k + u * G] : -1;
                double xv[U][3];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int jj = j[u] >= 0 ? j[u] : 0;
                    if (j[u] >= 0) {
                        xv[u][0] = a.x[3 * jj];
                        xv[u][1] = a.x[3 * jj + 1];
                        xv[u][2] = a.x[3 * jj + 2];
                    } else {
                        xv[u][0] = xv[u][1] = xv[u][2] = 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j[u] >= 0) acc_entry<MODE>(a.val, nz, k + u * G, xv[u][0], xv[u][1], xv[u][2], s0, s1, s2);
            }
        }
    }
    s0 = group_sum<G>(s0);
    s1 = group_sum<G>(s1);
    s2 = group_sum<G>(s2);

    if constexpr (OP == OP_SPMV_DOT) {
        double cd = 0.0;
        if (ep) {
            const double sv = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
            a.y[3 * i + lane] = sv;
            cd = own * sv;
        }
        const double tot = block_sum(cd);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = tot;
        return;
    }
    if (!ep) return;
    const double sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
    if (a.zero_out) a.zero_out[3 * i + c] = 0.0;
    if constexpr (OP == OP_SPMV) {
        a.y[3 * i + c] = sc;
    } else if constexpr (OP == OP_SPMV_ADD) {
        a.y[3 * i + c] = own + sc;
    } else if constexpr (OP == OP_RESID) {
        a.y[3 * i + c] = (c == 0 ? b0 : (c == 1 ? b1 : b2)) - sc;
    } else {
        const double r0 = b0 - s0, r1 = b1 - s1, r2 = b2 - s2;
        double d;
        if constexpr (MODE == 3) {
            d = d0 * r0 + d1 * r1 + d2 * r2;
        } else {
            d = d0 * (c == 0 ? r0 : (c == 1 ? r1 : r2));
        }
        if constexpr (OP == OP_JACOBI) {
            a.y[3 * i + c] = own + a.omega * d;
        } else {  // OP_GS: in place (a.y aliases a.x)
            a.y[3 * i + c] = own + d;
        }
    }
}

int row_blocks(int nrows, int G) { return ceil_div(static_cast<int64_t>(nrows) * G, BLOCK); }

template <int MODE, int G>
static void launch_row_g(RowOp op, const RowArgs &a, hipStream_t s) {
    int nb = row_blocks(a.nrows, G);
    if (nb == 0) return;
    if (a.xcd_chunks) {
        AMG_REQUIRE(op != OP_SPMV_DOT, AMG_EINVAL, "row kernel: XCD chunks with block partials");
        nb = (nb + 7) / 8 * 8;
    }
    AMG_REQUIRE(a.trip == 1 || a.trip == 2 || a.trip == 4, AMG_EINVAL, "row kernel: 1, 2 or 4 entries per trip");
#define AMG_ROW_CASE(OPC)                                                       \
    case OPC:                                                                   \
        if (a.trip == 4) k_row<MODE, G, OPC, 4><<<nb, BLOCK, 0, s>>>(a);         \
        else if (a.trip == 2) k_row<MODE, G, OPC, 2><<<nb, BLOCK, 0, s>>>(a);    \
        else k_row<MODE, G, OPC, 1><<<nb, BLOCK, 0, s>>>(a);                     \
        break;
    switch (op) {
        AMG_ROW_CASE(OP_SPMV)
        case OP_SPMV_ADD: k_row<MODE, G, OP_SPMV_ADD, 1><<<nb, BLOCK, 0, s>>>(a); break;
        AMG_ROW_CASE(OP_RESID)
        AMG_ROW_CASE(OP_JACOBI)
        AMG_ROW_CASE(OP_GS)
        AMG_ROW_CASE(OP_SPMV_DOT)
    }
#undef AMG_ROW_CASE
    AMG_CHECK_LAUNCH();
}

template <int MODE>
static void launch_row_m(RowOp op, int G, const RowArgs &a, hipStream_t s) {
    switch (G) {
        case 4: launch_row_g<MODE, 4>(op, a, s); break;
        case 8: launch_row_g<MODE, 8>(op, a, s); break;
        case 16: launch_row_g<MODE, 16>(op, a, s); break;
        case 32: launch_row_g<MODE, 32>(op, a, s); break;
        case 64: launch_row_g<MODE, 64>(op, a, s); break;
        default: throw Error(AMG_EINVAL, "row kernel: unsupported group size");
    }
}

void launch_row(int mode, RowOp op, int G, const RowArgs &a, hipStream_t s) {
    if (mode == 3)
        launch_row_m<3>(op, G, a, s);
    else
        launch_row_m<1>(op, G, a, s);
}

// ---------------------------------------------------------------- vectors
__global__ void k_fill(double *x, double v, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK)
        x[i] = v;
}

// x_i = a value in [-1, 1) from a hash of (i, seed): a fixed start vector
// with components along every eigenvector (power iterations)
__global__ void k_fill_hash(double *x, int64_t n, uint32_t seed) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK) {
        uint32_t h = static_cast<uint32_t>(i) * 0x9e3779b1u ^ seed;
        h ^= h >> 16;
        h *= 0x85ebca6bu;
        h ^= h >> 13;
        h *= 0xc2b2ae35u;
        h ^= h >> 16;
        x[i] = static_cast<double>(h) * (2.0 / 4294967296.0) - 1.0;
    }
}

static int grid_for(int64_t n) {
    int64_t nb = (n + BLOCK - 1) / BLOCK;
    if (nb > 4096) nb = 4096;
    return static_cast<int>(nb < 1 ? 1 : nb);
}

void launch_fill_hash(double *x, int64_t n, uint32_t seed, hipStream_t s) {
    if (n <= 0) return;
    k_fill_hash<<<grid_for(n), BLOCK, 0, s>>>(x, n, seed);
    AMG_CHECK_LAUNCH();
}

void launch_fill(double *x, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<<<grid_for(n), BLOCK, 0, s>>>(x, v, n);
    AMG_CHECK_LAUNCH();
}

__global__ void k_copy(double *d, const double *src, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK)
        d[i] = src[i];
}

// Pinned staging buffer pairs for copy_h2d, kept until the process ends:
// one per concurrent caller (the batch setup uploads its systems from
// several threads), created on first need. The events that order a pair's
// reuse inside one call are the call's own: an event last recorded on
// another caller's stream (which may since have been destroyed) is never
// waited on.
namespace {
struct Staging {
    char *pin[2] = {nullptr, nullptr};
};
constexpr size_t STAGING_CHUNK = 8u << 20;
std::mutex staging_mu;
std::vector<Staging *> staging_free;

Staging *staging_acquire() {
    {
        std::lock_guard<std::mutex> lock(staging_mu);
        if (!staging_free.empty()) {
            Staging *st = staging_free.back();
            staging_free.pop_back();
            return st;
        }
    }
    auto st = std::make_unique<Staging>();
    for (int i = 0; i < 2; ++i)
        AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&st->pin[i]), STAGING_CHUNK, hipHostMallocPortable));
    return st.release();
}

void staging_release(Staging *st) {
    std::lock_guard<std::mutex> lock(staging_mu);
    staging_free.push_back(st);
}
}  // namespace

void copy_h2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
    constexpr size_t SMALL = 1u << 18;
    if (bytes == 0) return;
    if (bytes <= SMALL) {
        AMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        AMG_HIP(hipStreamSynchronize(s));
        return;
    }
    // (declared before the staging pair: destroyed after its release, which
    // synchronises the stream first)
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } done;
    for (int i = 0; i < 2; ++i) AMG_HIP(hipEventCreateWithFlags(&done.e[i], hipEventDisableTiming));
    Staging *st = staging_acquire();
    struct Release {
        Staging *st;
        hipStream_t s;
        ~Release() {
            (void)hipStreamSynchronize(s);  // no DMA from the pair is left in flight
            staging_release(st);
        }
    } release{st, s};
    const char *from = static_cast<const char *>(src);
    char *to = static_cast<char *>(dst);
    bool live[2] = {false, false};
    int half = 0;
    for (size_t off = 0; off < bytes; off += STAGING_CHUNK, half ^= 1) {
        const size_t nb = std::min(STAGING_CHUNK, bytes - off);
        if (live[half]) AMG_HIP(hipEventSynchronize(done.e[half]));  // this half's previous DMA has finished
        std::memcpy(st->pin[half], from + off, nb);
        AMG_HIP(hipMemcpyAsync(to + off, st->pin[half], nb, hipMemcpyHostToDevice, s));
        AMG_HIP(hipEventRecord(done.e[half], s));
        live[half] = true;
    }
    AMG_HIP(hipStreamSynchronize(s));
}

// planes[p * nnz + k] = aos[k * np + p]
__global__ void k_aos_to_planes(const double *aos, int np, int64_t nnz, double *planes) {
    const int64_t total = nnz * np;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * BLOCK) {
        const int64_t k = t / np;
        const int p = static_cast<int>(t - k * np);
        planes[p * nnz + k] = aos[t];
    }
}

void launch_aos_to_planes(const double *aos, int np, int64_t nnz, double *planes, hipStream_t s) {
    if (nnz <= 0) return;
    k_aos_to_planes<<<grid_for(nnz * np), BLOCK, 0, s>>>(aos, np, nnz, planes);
    AMG_CHECK_LAUNCH();
}

void launch_copy(double *dst, const double *src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_copy<<<grid_for(n), BLOCK, 0, s>>>(dst, src, n);
    AMG_CHECK_LAUNCH();
}

template <int MODE>
__global__ void k_diag_solve(int nrows, const int *rowid, const double *dinv, int64_t n, const double *b,
                             double *x) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
    if (t >= 3 * static_cast<int64_t>(nrows)) return;
    const int i = rowid[t / 3];
    const int c = static_cast<int>(t % 3);
    if constexpr (MODE == 3) {
        x[3 * i + c] = dinv[(3 * c) * n + i] * b[3 * i] + dinv[(3 * c + 1) * n + i] * b[3 * i + 1] +
                       dinv[(3 * c + 2) * n + i] * b[3 * i + 2];
    } else {
        x[3 * i + c] = dinv[i] * b[3 * i + c];
    }
}

void launch_diag_solve(int mode, int nrows, const int *rowid, const double *dinv, int64_t n, const double *b,
                       double *x, hipStream_t s) {
    if (nrows <= 0) return;
    const int nb = ceil_div(3 * static_cast<int64_t>(nrows), BLOCK);
    if (mode == 3)
        k_diag_solve<3><<<nb, BLOCK, 0, s>>>(nrows, rowid, dinv, n, b, x);
    else
        k_diag_solve<1><<<nb, BLOCK, 0, s>>>(nrows, rowid, dinv, n, b, x);
    AMG_CHECK_LAUNCH();
}

template <int MODE>
__global__ void k_jacobi_zero(int64_t nn, int64_t dn, const double *dinv, const double *b, double omega,
                              double *x) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
    if (t >= 3 * nn) return;
    const int64_t i = t / 3;
    const int c = static_cast<int>(t % 3);
    double d;
    if constexpr (MODE == 3) {
        d = dinv[(3 * c) * dn + i] * b[3 * i] + dinv[(3 * c + 1) * dn + i] * b[3 * i + 1] +
            dinv[(3 * c + 2) * dn + i] * b[3 * i + 2];
    } else {
        d = dinv[i] * b[t];
    }
    x[t] = omega * d;
}

void launch_jacobi_zero(int mode, int64_t nn, const double *dinv, int64_t dn, const double *b, double omega,
                        double *x, hipStream_t s) {
    if (nn <= 0) return;
    const int nb = ceil_div(3 * nn, BLOCK);
    if (mode == 3)
        k_jacobi_zero<3><<<nb, BLOCK, 0, s>>>(nn, dn, dinv, b, omega, x);
    else
        k_jacobi_zero<1><<<nb, BLOCK, 0, s>>>(nn, dn, dinv, b, omega, x);
    AMG_CHECK_LAUNCH();
}

int dot_blocks(int64_t n) { return grid_for(n) > 1024 ? 1024 : grid_for(n); }

__global__ void k_dot_partial(const double *a, const double *b, int64_t n, double *partial) {
    double acc = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK)
        acc += a[i] * b[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

int launch_dot_partial(const double *a, const double *b, int64_t n, double *partial, hipStream_t s) {
    const int nb = dot_blocks(n);
    k_dot_partial<<<nb, BLOCK, 0, s>>>(a, b, n, partial);
    AMG_CHECK_LAUNCH();
    return nb;
}

constexpr int RBLOCK = 1024;

template <int POST>
__global__ void __launch_bounds__(RBLOCK) k_reduce(const double *partial, int np, double *sc, int dst) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += RBLOCK) acc += partial[i];
    const double t = block_sum<RBLOCK>(acc);
    if (threadIdx.x != 0) return;
    sc[dst] = t;
    if constexpr (POST == RED_CG_ALPHA) {
        sc[SC_ALPHA] = sc[SC_RZ] / t;
    } else if constexpr (POST == RED_CG_BETA) {
        sc[SC_BETA] = t / sc[SC_RZ];
        sc[SC_RZ] = t;
    } else if constexpr (POST == RED_FCG_BETA) {
        sc[SC_BETA] = -t / sc[SC_RZ_OLD];
    } else if constexpr (POST == RED_FCG_ALPHA) {
        sc[SC_ALPHA] = t / sc[SC_PQ];
        sc[SC_RZ_OLD] = sc[SC_PQ];
    }
}

void launch_reduce(const double *partial, int np, double *sc, int dst, hipStream_t s, int post) {
    switch (post) {
        case RED_NONE: k_reduce<RED_NONE><<<1, RBLOCK, 0, s>>>(partial, np, sc, dst); break;
        case RED_CG_ALPHA: k_reduce<RED_CG_ALPHA><<<1, RBLOCK, 0, s>>>(partial, np, sc, dst); break;
        case RED_CG_BETA: k_reduce<RED_CG_BETA><<<1, RBLOCK, 0, s>>>(partial, np, sc, dst); break;
        case RED_FCG_BETA: k_reduce<RED_FCG_BETA><<<1, RBLOCK, 0, s>>>(partial, np, sc, dst); break;
        case RED_FCG_ALPHA: k_reduce<RED_FCG_ALPHA><<<1, RBLOCK, 0, s>>>(partial, np, sc, dst); break;
        default: throw Error(AMG_EINVAL, "reduce: unknown post operation");
    }
    AMG_CHECK_LAUNCH();
}

__global__ void k_cg_update(double *x, double *r, const double *p, const double *q, const double *sc,
                            int64_t n, double *partial, double *zero) {
    const double al = sc[SC_ALPHA];
    double acc = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK) {
        x[i] += al * p[i];
        const double ri = r[i] - al * q[i];
        r[i] = ri;
        acc += ri * ri;
        if (zero) zero[i] = 0.0;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

int launch_cg_update(double *x, double *r, const double *p, const double *q, const double *sc,
                     int64_t n, double *partial, double *zero, hipStream_t s) {
    const int nb = dot_blocks(n);
    k_cg_update<<<nb, BLOCK, 0, s>>>(x, r, p, q, sc, n, partial, zero);
    AMG_CHECK_LAUNCH();
    return nb;
}

__global__ void k_cg_direction(double *p, const double *z, const double *sc, int64_t n) {
    const double be = sc[SC_BETA];
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK)
        p[i] = z[i] + be * p[i];
}

void launch_cg_direction(double *p, const double *z, const double *sc, int64_t n, hipStream_t s) {
    k_cg_direction<<<grid_for(n), BLOCK, 0, s>>>(p, z, sc, n);
    AMG_CHECK_LAUNCH();
}

__global__ void k_axpby(double *y, const double *x, double a, double b, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK)
        y[i] = a * x[i] + b * y[i];
}

void launch_axpby(double *y, const double *x, double a, double b, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_axpby<<<grid_for(n), BLOCK, 0, s>>>(y, x, a, b, n);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- dense
// One wavefront per output row; lanes stride over the columns.
__global__ void __launch_bounds__(BLOCK) k_dense_gemv(const double *M, int m, int nc, const double *X,
                                                      double *Y) {
    const int row = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const double *Mr = M + static_cast<int64_t>(row) * m;
    // four loads in flight per lane per trip
    int j = lane;
    for (; j + 192 < m; j += 256) {
        const double v0 = Mr[j], v1 = Mr[j + 64], v2 = Mr[j + 128], v3 = Mr[j + 192];
        if (nc == 1) {
            a0 += v0 * X[j] + v1 * X[j + 64] + v2 * X[j + 128] + v3 * X[j + 192];
        } else {
            a0 += v0 * X[3 * j] + v1 * X[3 * (j + 64)] + v2 * X[3 * (j + 128)] + v3 * X[3 * (j + 192)];
            a1 += v0 * X[3 * j + 1] + v1 * X[3 * (j + 64) + 1] + v2 * X[3 * (j + 128) + 1] +
                  v3 * X[3 * (j + 192) + 1];
            a2 += v0 * X[3 * j + 2] + v1 * X[3 * (j + 64) + 2] + v2 * X[3 * (j + 128) + 2] +
                  v3 * X[3 * (j + 192) + 2];
        }
    }
    for (; j < m; j += 64) {
        const double v = Mr[j];
        a0 += v * X[j * nc];
        if (nc > 1) {
            a1 += v * X[j * nc + 1];
            a2 += v * X[j * nc + 2];
        }
    }
    a0 = group_sum<64>(a0);
    a1 = group_sum<64>(a1);
    a2 = group_sum<64>(a2);
    if (lane < nc) Y[row * nc + lane] = lane == 0 ? a0 : (lane == 1 ? a1 : a2);
}

void launch_dense_gemv(const double *M, int m, int nc, const double *X, double *Y, hipStream_t s) {
    if (m <= 0) return;
    k_dense_gemv<<<ceil_div(m, BLOCK / 64), BLOCK, 0, s>>>(M, m, nc, X, Y);
    AMG_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- setup
template <int MODE>
__global__ void k_diag_inverse(int n, const int *rowptr, const int *col, const double *val, int64_t nnz,
                               double *dinv, int *flag) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    int k = -1;
    for (int q = rowptr[i]; q < rowptr[i + 1]; ++q)
        if (col[q] == i) { k = q; break; }
    if (k < 0) { atomicOr(flag, 1); return; }
    if constexpr (MODE == 1) {
        const double d = val[k];
        if (d == 0.0) atomicOr(flag, 2);
        dinv[i] = 1.0 / d;
    } else {
        double a[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) a[p] = val[p * nnz + k];
        // inverse by the adjugate: inv = adj(a) / det(a)
        const double c00 = a[4] * a[8] - a[5] * a[7];
        const double c01 = a[5] * a[6] - a[3] * a[8];
        const double c02 = a[3] * a[7] - a[4] * a[6];
        const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
        if (det == 0.0) { atomicOr(flag, 2); return; }
        const double id = 1.0 / det;
        double inv[9];
        inv[0] = c00 * id;
        inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
        inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
        inv[3] = c01 * id;
        inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
        inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
        inv[6] = c02 * id;
        inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
        inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
#pragma unroll
        for (int p = 0; p < 9; ++p) dinv[static_cast<int64_t>(p) * n + i] = inv[p];
    }
}

void launch_diag_inverse(int mode, int n, const int *rowptr, const int *col, const double *val,
                         int64_t nnz, double *dinv, int *flag, hipStream_t s) {
    if (n <= 0) return;
    if (mode == 3)
        k_diag_inverse<3><<<ceil_div(n, BLOCK), BLOCK, 0, s>>>(n, rowptr, col, val, nnz, dinv, flag);
    else
        k_diag_inverse<1><<<ceil_div(n, BLOCK), BLOCK, 0, s>>>(n, rowptr, col, val, nnz, dinv, flag);
    AMG_CHECK_LAUNCH();
}

// one wavefront per grouped row
__global__ void k_gather_rows(int np, int nrows, const int *order, const int *rowptr, const int *col,
                              const double *val, int64_t nnz, const int *g_rowptr, int *g_col,
                              double *g_val, int64_t g_nnz) {
    const int g = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= nrows) return;
    const int i = order[g];
    const int src = rowptr[i], len = rowptr[i + 1] - rowptr[i];
    const int dst = g_rowptr[g];
    for (int q = lane; q < len; q += 64) {
        g_col[dst + q] = col[src + q];
        for (int p = 0; p < np; ++p) g_val[p * g_nnz + dst + q] = val[p * nnz + src + q];
    }
}

void launch_gather_rows(int np, int nrows, const int *order, const int *rowptr, const int *col,
                        const double *val, int64_t nnz, const int *g_rowptr, int *g_col, double *g_val,
                        int64_t g_nnz, hipStream_t s) {
    if (nrows <= 0) return;
    k_gather_rows<<<ceil_div(nrows, BLOCK / 64), BLOCK, 0, s>>>(np, nrows, order, rowptr, col, val, nnz,
                                                                 g_rowptr, g_col, g_val, g_nnz);
    AMG_CHECK_LAUNCH();
}

// Entry k of row i is kept when it is the diagonal of a square operator or
// one of its np planes is nonzero.
__device__ inline bool kept_entry(int np, const double *val, int64_t nnz, int64_t k, bool diag) {
    if (diag) return true;
    for (int p = 0; p < np; ++p)
        if (val[p * nnz + k] != 0.0) return true;
    return false;
}

// One wavefront per row: the row's kept entries.
__global__ void k_count_kept(int np, int nrows, int square, const int *rowptr, const int *col, const double *val,
                             int64_t nnz, int *count) {
    const int i = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nrows) return;
    int c = 0;
    for (int k = rowptr[i] + lane; k < rowptr[i + 1]; k += 64)
        c += kept_entry(np, val, nnz, k, square && col[k] == i) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) count[i] = c;
}

// One wavefront per row: the kept entries in their order, placed by a
// prefix count over the wavefront's ballot.
__global__ void k_compact_rows(int np, int nrows, int square, const int *rowptr, const int *col, const double *val,
                               int64_t nnz, const int *c_rowptr, int *c_col, double *c_val, int64_t c_nnz) {
    const int i = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nrows) return;
    int dst = c_rowptr[i];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int k0 = rowptr[i]; k0 < rowptr[i + 1]; k0 += 64) {
        const int k = k0 + lane;
        const bool keep = k < rowptr[i + 1] && kept_entry(np, val, nnz, k, square && col[k] == i);
        const uint64_t mask = __ballot(keep);
        if (keep) {
            const int64_t d = dst + __popcll(mask & below);
            c_col[d] = col[k];
            for (int p = 0; p < np; ++p) c_val[p * c_nnz + d] = val[p * nnz + k];
        }
        dst += __popcll(mask);
    }
}

void launch_count_kept(int np, int nrows, bool square, const int *rowptr, const int *col, const double *val,
                       int64_t nnz, int *count, hipStream_t s) {
    if (nrows <= 0) return;
    k_count_kept<<<ceil_div(nrows, BLOCK / 64), BLOCK, 0, s>>>(np, nrows, square ? 1 : 0, rowptr, col, val, nnz,
                                                                count);
    AMG_CHECK_LAUNCH();
}

void launch_compact_rows(int np, int nrows, bool square, const int *rowptr, const int *col, const double *val,
                         int64_t nnz, const int *c_rowptr, int *c_col, double *c_val, int64_t c_nnz,
                         hipStream_t s) {
    if (nrows <= 0) return;
    k_compact_rows<<<ceil_div(nrows, BLOCK / 64), BLOCK, 0, s>>>(np, nrows, square ? 1 : 0, rowptr, col, val, nnz,
                                                                  c_rowptr, c_col, c_val, c_nnz);
    AMG_CHECK_LAUNCH();
}

}  // namespace amgp2
