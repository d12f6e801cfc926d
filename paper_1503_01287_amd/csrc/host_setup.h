// Host-side parts of the hierarchy setup: graph extraction, coarse/fine
// splitting, interpolation, colouring and the coarsest dense inverse.
// These passes are sequential by definition (a greedy independent set and a
// greedy colouring in index order) and run once per level on index arrays.
#pragma once

#include <cstdint>
#include <vector>

namespace amgp2 {

struct HostCSR {
    int nrows = 0, ncols = 0;
    std::vector<int> rowptr, col;
    std::vector<double> val;  // empty for a pure pattern
    int64_t nnz() const { return static_cast<int64_t>(col.size()); }
};

// Graph of the node range [lo, hi) of a square pattern, self loops removed,
// indices shifted to start at 0.
HostCSR subgraph(const HostCSR &pattern, int lo, int hi);

// Greedy maximal independent set, nodes visited in index order: an undecided
// node becomes coarse (1), its undecided neighbours fine (0).
std::vector<char> greedy_independent_set(const HostCSR &graph);

// Interpolation of Section 3.2's reading: coarse node -> identity row, fine
// node -> equal weights 1/|C_i| on its coarse graph neighbours.
HostCSR averaging_interpolation(const HostCSR &graph, const std::vector<char> &coarse);

// [[A, 0], [0, B]] for two rectangular scalar matrices.
HostCSR block_diagonal(const HostCSR &a, const HostCSR &b);

HostCSR transpose(const HostCSR &a);

// Structural pattern of X Y (plus the pattern of `extra`, same shape, if
// given), rows sorted.
HostCSR pattern_product(const HostCSR &x, const HostCSR &y, const HostCSR *extra);

// Greedy first-fit colouring in index order over the whole pattern (self
// loops ignored). Returns the number of colours.
int greedy_colouring(const HostCSR &pattern, std::vector<int> &colour);

// Dense inverse of a row-major n x n matrix by LU with partial pivoting.
// Returns false if a pivot is exactly zero.
bool dense_inverse(std::vector<double> &a, int n);

}  // namespace amgp2
