/* Sequential loops of the oracle (test infrastructure only; FP64, plain C).
 *
 * These are the parts of the method that are inherently ordered:
 *  - greedy maximal independent set for the coarse/fine split of a node graph
 *    (the reading of the C/F selection of Section 3.2: nodes visited in index
 *    order, an undecided node becomes coarse and its undecided neighbours fine);
 *  - greedy first-fit colouring of a node graph in index order;
 *  - one block Gauss-Seidel sweep over 3x3 node blocks in a given node order
 *    (Section 3.3's block Gauss-Seidel smoother).
 * Nothing here is shared with the GPU library.
 */
#include <stdint.h>
#include <stdlib.h>

/* state[i]: 1 = coarse, 2 = fine. Graph in CSR (self loops ignored).
 * Returns the number of coarse nodes. */
int64_t oracle_greedy_mis(int64_t n, const int64_t *indptr, const int64_t *indices, int8_t *state)
{
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) state[i] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (state[i] != 0) continue;
        state[i] = 1;
        ++nc;
        for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) {
            int64_t j = indices[k];
            if (j != i && state[j] == 0) state[j] = 2;
        }
    }
    return nc;
}

/* color[i] = smallest colour not used by an already coloured neighbour.
 * Returns the number of colours. */
int64_t oracle_greedy_colour(int64_t n, const int64_t *indptr, const int64_t *indices, int32_t *color)
{
    int64_t ncol = 0;
    int64_t cap = 64;
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * cap);
    for (int64_t c = 0; c < cap; ++c) mark[c] = -1;
    for (int64_t i = 0; i < n; ++i) color[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) {
            int64_t j = indices[k];
            if (j != i && color[j] >= 0) mark[color[j]] = i;
        }
        int64_t c = 0;
        while (c < cap && mark[c] == i) ++c;
        if (c == cap) {
            int64_t ncap = cap * 2;
            mark = (int64_t *)realloc(mark, sizeof(int64_t) * ncap);
            for (int64_t q = cap; q < ncap; ++q) mark[q] = -1;
            cap = ncap;
        }
        color[i] = (int32_t)c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(mark);
    return ncol;
}

/* One block Gauss-Seidel sweep, nodes visited in order[0..m):
 *   x_i <- A_ii^{-1} ( b_i - sum_{j != i} A_ij x_j )
 * A in block CSR with 3x3 row-major blocks, dinv the inverted diagonal blocks. */
void oracle_block_gs(int64_t m, const int64_t *order, const int64_t *indptr, const int64_t *indices,
                     const double *vals, const double *dinv, const double *b, double *x)
{
    for (int64_t q = 0; q < m; ++q) {
        int64_t i = order[q];
        double s0 = b[3 * i], s1 = b[3 * i + 1], s2 = b[3 * i + 2];
        for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) {
            int64_t j = indices[k];
            if (j == i) continue;
            const double *a = vals + 9 * k;
            double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
            s0 -= a[0] * x0 + a[1] * x1 + a[2] * x2;
            s1 -= a[3] * x0 + a[4] * x1 + a[5] * x2;
            s2 -= a[6] * x0 + a[7] * x1 + a[8] * x2;
        }
        const double *d = dinv + 9 * i;
        x[3 * i] = d[0] * s0 + d[1] * s1 + d[2] * s2;
        x[3 * i + 1] = d[3] * s0 + d[4] * s1 + d[5] * s2;
        x[3 * i + 2] = d[6] * s0 + d[7] * s1 + d[8] * s2;
    }
}

/* Scalar (1x1 block) variant, used for the pressure Schur complement. */
void oracle_scalar_gs(int64_t m, const int64_t *order, const int64_t *indptr, const int64_t *indices,
                      const double *vals, const double *b, double *x)
{
    for (int64_t q = 0; q < m; ++q) {
        int64_t i = order[q];
        double s = b[i], d = 0.0;
        for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) {
            int64_t j = indices[k];
            if (j == i) d = vals[k];
            else s -= vals[k] * x[j];
        }
        x[i] = s / d;
    }
}

/* One block Gauss-Seidel sweep in correction form, nodes visited in
 * order[0..m):  x_i <- x_i + D_i^{-1} ( b_i - sum_j A_ij x_j )  (j = i included).
 * With D_i = A_ii this is the sweep above; the reduced-precision reading of
 * the cycle uses it with the rounded operator A and D_i^{-1} inverted from
 * the unrounded diagonal blocks. */
void oracle_block_gs_update(int64_t m, const int64_t *order, const int64_t *indptr, const int64_t *indices,
                            const double *vals, const double *dinv, const double *b, double *x)
{
    for (int64_t q = 0; q < m; ++q) {
        int64_t i = order[q];
        double s0 = b[3 * i], s1 = b[3 * i + 1], s2 = b[3 * i + 2];
        for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) {
            int64_t j = indices[k];
            const double *a = vals + 9 * k;
            double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
            s0 -= a[0] * x0 + a[1] * x1 + a[2] * x2;
            s1 -= a[3] * x0 + a[4] * x1 + a[5] * x2;
            s2 -= a[6] * x0 + a[7] * x1 + a[8] * x2;
        }
        const double *d = dinv + 9 * i;
        x[3 * i] += d[0] * s0 + d[1] * s1 + d[2] * s2;
        x[3 * i + 1] += d[3] * s0 + d[4] * s1 + d[5] * s2;
        x[3 * i + 2] += d[6] * s0 + d[7] * s1 + d[8] * s2;
    }
}
