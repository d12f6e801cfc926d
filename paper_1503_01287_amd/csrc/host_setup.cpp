#include "host_setup.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace amgp2 {

HostCSR subgraph(const HostCSR &p, int lo, int hi) {
    HostCSR g;
    g.nrows = g.ncols = hi - lo;
    g.rowptr.assign(g.nrows + 1, 0);
    g.col.reserve(static_cast<size_t>(p.rowptr[hi] - p.rowptr[lo]));
    for (int i = lo; i < hi; ++i) {
        for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) {
            const int j = p.col[k];
            if (j >= lo && j < hi && j != i) g.col.push_back(j - lo);
        }
        g.rowptr[i - lo + 1] = static_cast<int>(g.col.size());
    }
    return g;
}

std::vector<char> greedy_independent_set(const HostCSR &g) {
    // state: 0 undecided, 1 coarse, 2 fine
    std::vector<char> st(g.nrows, 0);
    for (int i = 0; i < g.nrows; ++i) {
        if (st[i]) continue;
        st[i] = 1;
        for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k)
            if (st[g.col[k]] == 0) st[g.col[k]] = 2;
    }
    std::vector<char> coarse(g.nrows);
    for (int i = 0; i < g.nrows; ++i) coarse[i] = st[i] == 1;
    return coarse;
}

HostCSR averaging_interpolation(const HostCSR &g, const std::vector<char> &coarse) {
    HostCSR P;
    P.nrows = g.nrows;
    std::vector<int> cidx(g.nrows, -1);
    int nc = 0;
    for (int i = 0; i < g.nrows; ++i)
        if (coarse[i]) cidx[i] = nc++;
    P.ncols = nc;
    P.rowptr.assign(g.nrows + 1, 0);
    std::vector<int> nb;
    for (int i = 0; i < g.nrows; ++i) {
        if (coarse[i]) {
            P.col.push_back(cidx[i]);
            P.val.push_back(1.0);
        } else {
            nb.clear();
            for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k)
                if (coarse[g.col[k]]) nb.push_back(cidx[g.col[k]]);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            // a maximal independent set leaves no fine node without a coarse neighbour
            const double w = nb.empty() ? 0.0 : 1.0 / static_cast<double>(nb.size());
            for (int c : nb) {
                P.col.push_back(c);
                P.val.push_back(w);
            }
        }
        P.rowptr[i + 1] = static_cast<int>(P.col.size());
    }
    return P;
}

HostCSR block_diagonal(const HostCSR &a, const HostCSR &b) {
    HostCSR c;
    c.nrows = a.nrows + b.nrows;
    c.ncols = a.ncols + b.ncols;
    c.rowptr = a.rowptr;
    c.col = a.col;
    c.val = a.val;
    const int off = static_cast<int>(a.col.size());
    for (int i = 0; i < b.nrows; ++i) c.rowptr.push_back(off + b.rowptr[i + 1]);
    for (int j : b.col) c.col.push_back(j + a.ncols);
    c.val.insert(c.val.end(), b.val.begin(), b.val.end());
    return c;
}

HostCSR transpose(const HostCSR &a) {
    HostCSR t;
    t.nrows = a.ncols;
    t.ncols = a.nrows;
    t.rowptr.assign(t.nrows + 1, 0);
    for (int j : a.col) ++t.rowptr[j + 1];
    std::partial_sum(t.rowptr.begin(), t.rowptr.end(), t.rowptr.begin());
    t.col.resize(a.col.size());
    t.val.resize(a.val.size());
    std::vector<int> next(t.rowptr.begin(), t.rowptr.end() - 1);
    for (int i = 0; i < a.nrows; ++i)
        for (int k = a.rowptr[i]; k < a.rowptr[i + 1]; ++k) {
            const int q = next[a.col[k]]++;
            t.col[q] = i;  // rows visited in order: each output row stays sorted
            if (!a.val.empty()) t.val[q] = a.val[k];
        }
    return t;
}

HostCSR pattern_product(const HostCSR &x, const HostCSR &y, const HostCSR *extra) {
    HostCSR c;
    c.nrows = x.nrows;
    c.ncols = y.ncols;
    c.rowptr.assign(c.nrows + 1, 0);
    std::vector<int> mark(std::max(1, c.ncols), -1), row;
    for (int i = 0; i < x.nrows; ++i) {
        row.clear();
        auto put = [&](int q) {
            if (mark[q] != i) {
                mark[q] = i;
                row.push_back(q);
            }
        };
        for (int k = x.rowptr[i]; k < x.rowptr[i + 1]; ++k) {
            const int j = x.col[k];
            for (int m = y.rowptr[j]; m < y.rowptr[j + 1]; ++m) put(y.col[m]);
        }
        if (extra)
            for (int k = extra->rowptr[i]; k < extra->rowptr[i + 1]; ++k) put(extra->col[k]);
        std::sort(row.begin(), row.end());
        c.col.insert(c.col.end(), row.begin(), row.end());
        c.rowptr[i + 1] = static_cast<int>(c.col.size());
    }
    return c;
}

int greedy_colouring(const HostCSR &p, std::vector<int> &colour) {
    colour.assign(p.nrows, -1);
    std::vector<int> seen;  // seen[c] == i: colour c used by a neighbour of i
    int ncol = 0;
    for (int i = 0; i < p.nrows; ++i) {
        for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) {
            const int j = p.col[k];
            if (j != i && colour[j] >= 0) {
                if (colour[j] >= static_cast<int>(seen.size())) seen.resize(colour[j] + 1, -1);
                seen[colour[j]] = i;
            }
        }
        int c = 0;
        while (c < static_cast<int>(seen.size()) && seen[c] == i) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

bool dense_inverse(std::vector<double> &a, int n) {
    std::vector<int> piv(n);
    // LU with partial pivoting, in place (row-major)
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::fabs(a[static_cast<size_t>(k) * n + k]);
        for (int i = k + 1; i < n; ++i) {
            const double v = std::fabs(a[static_cast<size_t>(i) * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(a[static_cast<size_t>(k) * n + j], a[static_cast<size_t>(p) * n + j]);
        const double d = a[static_cast<size_t>(k) * n + k];
        for (int i = k + 1; i < n; ++i) {
            double &l = a[static_cast<size_t>(i) * n + k];
            l /= d;
            for (int j = k + 1; j < n; ++j) a[static_cast<size_t>(i) * n + j] -= l * a[static_cast<size_t>(k) * n + j];
        }
    }
    // solve for the columns of the inverse: L U X = P I
    std::vector<double> inv(static_cast<size_t>(n) * n, 0.0), e(n);
    for (int c = 0; c < n; ++c) {
        std::fill(e.begin(), e.end(), 0.0);
        e[c] = 1.0;
        for (int k = 0; k < n; ++k) std::swap(e[k], e[piv[k]]);
        for (int i = 0; i < n; ++i) {
            double s = e[i];
            for (int j = 0; j < i; ++j) s -= a[static_cast<size_t>(i) * n + j] * e[j];
            e[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = e[i];
            for (int j = i + 1; j < n; ++j) s -= a[static_cast<size_t>(i) * n + j] * e[j];
            e[i] = s / a[static_cast<size_t>(i) * n + i];
        }
        for (int i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + c] = e[i];
    }
    a.swap(inv);
    return true;
}

}  // namespace amgp2
