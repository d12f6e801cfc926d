// Multiplicative Vanka smoother (Section 3.3): one patch per pressure DOF
// holding that DOF and the velocity nodes coupled to it through B; each
// patch's local saddle matrix is inverted once at setup (batched
// Gauss-Jordan, FP64) and a sweep applies x_P += omega K_P^{-1} (b - K x)_P
// patch by patch, colour by colour (patches of one colour share no node and
// are not coupled, so they update at the same time).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgp2 {

struct VankaView {
    int npatch = 0;
    const int *pptr = nullptr, *pnode = nullptr;  // patch i: velocity nodes pnode[pptr[i] .. pptr[i+1])
    const int64_t *moff = nullptr;                // inverse of patch i at inv + moff[i], m_i x m_i, column-major
    double *inv = nullptr;
    // the level's operators (planes)
    int n = 0;                                    // velocity nodes
    const int *arow = nullptr, *acol = nullptr;
    const double *aval = nullptr;
    int64_t annz = 0;
    const int *brow = nullptr, *bcol = nullptr;   // B (1x3)
    const double *bval = nullptr;
    int64_t bnnz = 0;
    const int *btrow = nullptr, *btcol = nullptr; // B^T (3x1)
    const double *btval = nullptr;
    int64_t btnnz = 0;
    const int *crow = nullptr, *ccol = nullptr;   // C (may be null)
    const double *cval = nullptr;
};

// local matrices [[A_P, B_P^T], [B_P, -C_ii]] of every patch, then their
// inverses in place; flag |= 1 on an exactly zero pivot
void launch_vanka_assemble(const VankaView &v, int max_nodes, hipStream_t s);
void launch_vanka_invert(const VankaView &v, int max_m, int *flag, hipStream_t s);
// one colour: the patches order[0 .. count); x = [u (3n); p]
void launch_vanka_colour(const VankaView &v, const int *order, int count, int max_nodes, const double *b,
                         double *x, double omega, hipStream_t s);
// the same colour in two kernels, for large patches: the patches' residuals
// into rbuf (patch i at rbuf + roff[i]), then the corrections with
// ceil(m_i / 64) workgroups per patch (tpre: prefix of those counts over the
// colour's patches, ntiles their total)
void launch_vanka_colour_split(const VankaView &v, const int *order, const int *tpre, int count, int ntiles,
                               int max_nodes, const int64_t *roff, double *rbuf, const double *b, double *x,
                               double omega, hipStream_t s);
// the residual spread as in the tiled form (rpre, nrunits, rg), then the
// corrections over 64-row tiles of every inverse as the two-kernel form
// (tpre, ntiles), aw (4, 8 or 16) wavefronts per tile splitting its columns
void launch_vanka_colour_rows(const VankaView &v, const int *order, const int *tpre, const int *rpre, int count,
                              int ntiles, int nrunits, int rg, int aw, const int64_t *roff, double *rbuf,
                              const double *b, double *x, double omega, hipStream_t s);
// the same colour in three kernels for colours of few, large patches: the
// residuals into rbuf, rg lanes per row (16, 32 or 64) and 256 / rg node
// rows per workgroup (rpre: prefix of ceil((n_P + 1) / (256 / rg)) over the
// colour's patches, nrunits their total),
// then partial corrections over 64-row x cc-column tiles of every inverse
// into pbuf (patch i's ceil(m_i / cc) chunks of m_i values at pbuf +
// poff[i]; upre: prefix of the tiles ceil(m_i / 64) ceil(m_i / cc) over the
// colour's patches, nunits their total), then the chunks summed in order
// into x over the 64-row tiles (tpre, ntiles)
void launch_vanka_colour_tiled(const VankaView &v, const int *order, const int *tpre, const int *upre,
                               const int *rpre, int count, int ntiles, int nunits, int nrunits, int cc, int rg,
                               const int64_t *roff, double *rbuf, const int64_t *poff, double *pbuf, const double *b,
                               double *x, double omega, hipStream_t s);

}  // namespace amgp2
