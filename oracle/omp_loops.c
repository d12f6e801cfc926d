/* Order-independent loops of the oracle on all host cores (test
 * infrastructure only; FP64, plain C with OpenMP).
 *
 * Used only to time the oracle on every host core beside its single-thread
 * timing. Each loop does the arithmetic of the oracle step it stands in for,
 * split over rows:
 *  - y = M x for a block CSR matrix (every row's sum over its entries in
 *    entry order, each block product summed over its columns first);
 *  - y = M x for a scalar CSR matrix (the transfers P and P^T);
 *  - one block Gauss-Seidel sweep by colours (Section 3.3's smoother on a
 *    coloured level): the colours one after another, the nodes of one colour
 *    in parallel. No two nodes of a colour are coupled, so every node reads
 *    the same neighbour values as in the sequential sweep over the same order
 *    and the result is the same bit for bit;
 *  - x + omega D^{-1} r for block Jacobi.
 * Nothing here is shared with the GPU library.
 */
#include <omp.h>
#include <stdint.h>

void omp_set_threads(int n) { omp_set_num_threads(n); }

int omp_threads(void) { return omp_get_max_threads(); }

void omp_bsr_matvec(int64_t nrows, int64_t br, int64_t bc, const int64_t *indptr, const int64_t *indices,
                    const double *vals, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        for (int64_t c = 0; c < br; ++c) {
            double s = 0.0;
            for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) {
                const double *a = vals + (k * br + c) * bc;
                const double *xj = x + indices[k] * bc;
                double t = 0.0;
                for (int64_t d = 0; d < bc; ++d) t += a[d] * xj[d];
                s += t;
            }
            y[i * br + c] = s;
        }
    }
}

void omp_csr_matvec(int64_t nrows, const int64_t *indptr, const int64_t *indices, const double *vals,
                    const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) s += vals[k] * x[indices[k]];
        y[i] = s;
    }
}

/* Colour c holds the nodes order[cstart[c] .. cstart[c+1]). */
void omp_block_gs_colours(int64_t ncolours, const int64_t *cstart, const int64_t *order, const int64_t *indptr,
                          const int64_t *indices, const double *vals, const double *dinv, const double *b,
                          double *x)
{
    for (int64_t c = 0; c < ncolours; ++c) {
#pragma omp parallel for schedule(static)
        for (int64_t q = cstart[c]; q < cstart[c + 1]; ++q) {
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
}

/* out_i = x_i + omega D_i^{-1} r_i over n nodes of 3x3 blocks */
void omp_block_jacobi(int64_t n, const double *dinv, const double *r, const double *x, double omega, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *d = dinv + 9 * i;
        const double *ri = r + 3 * i;
        for (int c = 0; c < 3; ++c)
            out[3 * i + c] = x[3 * i + c] + omega * (d[3 * c] * ri[0] + d[3 * c + 1] * ri[1] + d[3 * c + 2] * ri[2]);
    }
}
