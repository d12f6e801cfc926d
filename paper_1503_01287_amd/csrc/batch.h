// Batches of independent saddle point systems: segmented vector kernels over
// a table of chunks (each chunk lies inside one system's velocity or
// pressure range), used by the batched flexible GMRES and to move vectors
// between the caller's layout and the merged hierarchy's.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

constexpr int BATCH_CHUNK = 2048;

struct ChunkView {
    int n = 0;                        // chunks
    const int64_t *start = nullptr;   // first element of chunk c
    const int *len = nullptr;         // elements (<= BATCH_CHUNK)
    const int *seg = nullptr;         // system of chunk c (merged position)
};

// partial[j * n + c] = <V_j, w> over chunk c, j < k (V_j = V + j * ld)
void launch_seg_multidot(const double *V, int64_t ld, int k, const double *w, const ChunkView &t, double *partial,
                         hipStream_t s);
// the same for the chunks of the systems s with want[s] != 0 only
void launch_seg_multidot_masked(const double *V, int64_t ld, int k, const double *w, const ChunkView &t,
                                const int *want, double *partial, hipStream_t s);
// two right-hand sides in one pass over the basis: partial[(r * k + j) * n
// + c] holds <V_j, a> (r = 0) and <V_j, b> (r = 1) over chunk c
void launch_seg_multidot2(const double *V, int64_t ld, int k, const double *a, const double *b, const ChunkView &t,
                          double *partial, hipStream_t s);
// h[i * kmax + j] = sum of partial[j * n + c] over the chunks c of system i:
// [c0[i], c1[i]) then [c2[i], c3[i]) in order
void launch_seg_reduce(const double *partial, int n, int k, int nsys, const int *c0, const int *c1, const int *c2,
                       const int *c3, double *h, int kmax, hipStream_t s);
// Delayed reorthogonalisation step of every system on basis slots j
// (pending vector) and j + 1 (new vector), as launch_dcgs2_update, with
// system s's dots of launch_multidot2 over V_0..V_{j+1} at h + s * stride
// (2 (j + 2) values) and its gamma, d, eta written after them
void launch_seg_dcgs2_update(double *V, int64_t ld, int j, double *h, int stride, const ChunkView &t, bool reorth,
                             hipStream_t s);
// y = coef[seg] * x
void launch_seg_scale(const double *x, double *y, const double *coef, const ChunkView &t, hipStream_t s);
// y = a[seg] x + b[seg] y
void launch_seg_axpby(const double *x, double *y, const double *a, const double *b, const ChunkView &t,
                      hipStream_t s);
// x += sum_{j < cnt[seg]} y[seg * kmax + j] Z_j
void launch_seg_multi_add(const double *Z, int64_t ld, const double *y, int kmax, const int *cnt, double *x,
                          const ChunkView &t, hipStream_t s);
// dst[k] = src[k] + add for k < n (src null: dst[k] = add)
void launch_copy_shift_i32(const int *src, int64_t n, int add, int *dst, hipStream_t s);
// dst[dstart[c] + e] = src[start[c] + e] for e < len[c]
void launch_seg_copy(const double *src, double *dst, const ChunkView &t, const int64_t *dstart, hipStream_t s);

}  // namespace amgp2
