// Incomplete Cholesky IC(0) of an operator in a multicolour order (the
// preconditioner the paper's Sec. 5 remarks use for the velocity systems),
// factorised on the host for one Dirichlet set and uploaded for the
// colour-by-colour triangular solves of the device.
//
// Order: greedy colouring of the graph of the matrix with the Dirichlet rows
// and columns removed (node i takes the smallest colour no lower-numbered
// neighbour has), then the nodes sorted by (colour, node).  Rows of one
// colour are not coupled, so each triangular solve is one parallel step per
// colour.  Factor: B = P A_D P^T (A_D the matrix with Dirichlet rows and
// columns replaced by the identity); L has the pattern of the lower triangle
// of B and (L L^T)_ij = B_ij there.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "hns_internal.h"

namespace hns {

namespace {

template <class F>
void parallel_rows(int64_t lo, int64_t hi, F &&f)
{
    const int64_t n = hi - lo;
    unsigned nt = std::max(1u, std::thread::hardware_concurrency());
    nt = (unsigned)std::min<int64_t>(nt, std::max<int64_t>(1, n / 2048));
    if (nt <= 1) {
        f(lo, hi);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t a = lo + t * chunk, b = std::min<int64_t>(hi, a + chunk);
        if (a >= b) break;
        th.emplace_back([&f, a, b] { f(a, b); });
    }
    for (auto &t : th) t.join();
}

}  // namespace

hns_status ic0_factor_host(const HostCSR &A, const uint8_t *bc, int bit, IC0Host &F)
{
    const int64_t n = A.n;
    auto dir = [&](int64_t i) { return bit >= 0 && bc && ((bc[i] >> bit) & 1u); };
    // colours
    std::vector<int32_t> color(n, 0);
    int ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t used = 0;
        if (!dir(i))
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
                const int32_t j = A.col[k];
                if (j < i && !dir(j) && color[j] < 64) used |= 1ull << color[j];
            }
        int c = 0;
        while (c < 64 && (used >> c) & 1ull) ++c;
        if (c >= 64) {
            set_error("IC(0): the matrix graph needs more than 64 colours");
            return HNS_ERR_INVALID;
        }
        color[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    // order
    F.n = n;
    F.ncolors = ncol;
    F.perm.assign(n, 0);
    F.cstart.assign(ncol + 1, 0);
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) F.cstart[color[i] + 1]++;
    for (int c = 0; c < ncol; ++c) F.cstart[c + 1] += F.cstart[c];
    {
        std::vector<int64_t> fill(F.cstart.begin(), F.cstart.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = fill[color[i]]++;
            F.perm[k] = (int32_t)i;
            iperm[i] = (int32_t)k;
        }
    }
    // strict lower pattern of B by permuted rows, ascending permuted columns
    F.lptr.assign(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = F.perm[r];
        int32_t cnt = 0;
        if (!dir(i))
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
                const int32_t j = A.col[k];
                if (!dir(j) && iperm[j] < r) ++cnt;
            }
        F.lptr[r + 1] = F.lptr[r] + cnt;
    }
    const int64_t nl = F.lptr[n];
    F.lcol.assign(nl, 0);
    F.lval.assign(nl, 0.0);
    F.diag.assign(n, 0.0);
    std::vector<double> bval(nl, 0.0), bdiag(n, 0.0);
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = F.perm[r];
        int64_t w = F.lptr[r];
        std::vector<std::pair<int32_t, double>> row;
        if (dir(i)) {
            bdiag[r] = 1.0;
            continue;
        }
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            if (j == i) bdiag[r] = A.val[k];
            else if (!dir(j) && iperm[j] < r) row.emplace_back(iperm[j], A.val[k]);
        }
        std::sort(row.begin(), row.end());
        for (auto &e : row) {
            F.lcol[w] = e.first;
            bval[w] = e.second;
            ++w;
        }
    }
    // values, colour by colour (rows of one colour only read earlier colours)
    bool bad = false;
    for (int c = 0; c < ncol && !bad; ++c) {
        std::vector<char> fail(1, 0);
        parallel_rows(F.cstart[c], F.cstart[c + 1], [&](int64_t lo, int64_t hi) {
            for (int64_t r = lo; r < hi; ++r) {
                const int64_t b0 = F.lptr[r], b1 = F.lptr[r + 1];
                for (int64_t t = b0; t < b1; ++t) {
                    const int32_t j = F.lcol[t];
                    double s = 0.0;
                    int64_t u = b0, v = F.lptr[j];
                    const int64_t vend = F.lptr[j + 1];
                    while (u < t && v < vend) {
                        if (F.lcol[u] == F.lcol[v]) {
                            s += F.lval[u] * F.lval[v];
                            ++u;
                            ++v;
                        } else if (F.lcol[u] < F.lcol[v]) {
                            ++u;
                        } else {
                            ++v;
                        }
                    }
                    F.lval[t] = (bval[t] - s) / F.diag[j];
                }
                double d = bdiag[r];
                for (int64_t t = b0; t < b1; ++t) d -= F.lval[t] * F.lval[t];
                if (!(d > 0.0) || !std::isfinite(d)) {
                    fail[0] = 1;
                    continue;
                }
                F.diag[r] = std::sqrt(d);
            }
        });
        bad = fail[0] != 0;
    }
    if (bad) {
        set_error("IC(0) breakdown: a pivot is not positive");
        return HNS_ERR_BREAKDOWN;
    }
    // the transpose (strict upper by permuted rows) for the backward solve
    F.uptr.assign(n + 1, 0);
    for (int64_t t = 0; t < nl; ++t) F.uptr[F.lcol[t] + 1]++;
    for (int64_t r = 0; r < n; ++r) F.uptr[r + 1] += F.uptr[r];
    F.ucol.assign(nl, 0);
    F.uval.assign(nl, 0.0);
    {
        std::vector<int64_t> fill(F.uptr.begin(), F.uptr.end() - 1);
        for (int64_t r = 0; r < n; ++r)
            for (int64_t t = F.lptr[r]; t < F.lptr[r + 1]; ++t) {
                const int64_t k = fill[F.lcol[t]]++;
                F.ucol[k] = (int32_t)r;
                F.uval[k] = F.lval[t];
            }
    }
    return HNS_OK;
}

}  // namespace hns
