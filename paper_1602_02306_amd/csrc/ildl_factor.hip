// Host-side ILDL(t) factorization for the factored absolute-value
// preconditioner of Section 6: P (A - tau I) P^T ~ L D L^T with Bunch-Kaufman
// 1x1 / 2x2 pivots and a drop tolerance t, T = P^T L^{-T} |D|^{-1} L^{-1} P.
//
// Sparse right-looking elimination on the active (Schur) matrix, kept with
// both triangles as sorted sparse rows:
//   - pivot: lambda = max_{i>k} |S_ik| (first such i = r); 1x1 at k when
//     lambda == 0, |S_kk| >= alpha lambda or |S_kk| sigma >= alpha lambda^2
//     (sigma = max_{i>=k, i!=r} |S_ir|); 1x1 after the interchange r <-> k when
//     |S_rr| >= alpha sigma; otherwise a 2x2 pivot after r <-> k+1;
//     alpha = (1 + sqrt 17) / 8 (Bunch & Kaufman's partial pivoting);
//   - multipliers l = S(:,k) / d, or [l1 l2] = [S(:,k) S(:,k+1)] D^{-1};
//   - each multiplier column is thinned: |l_i| < t * sum_i |l_i| -> 0;
//   - Schur update with the thinned multipliers, one value per unordered
//     pair {i, j}: (l_hi d) l_lo (1x1) or w1_hi l1_lo + w2_hi l2_lo with
//     w1 = l1 a + l2 b, w2 = l1 b + l2 c (2x2), hi = max(i, j), lo = min(i, j),
//     so the active matrix stays exactly symmetric.
// The matrix keeps its own order (no fill-reducing permutation); interchanges
// come from pivoting only.  Every entry receives its updates in step order,
// so the factor does not depend on how the sparse rows are stored.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ecount.h"
#include "ecount_internal.h"

#pragma clang fp contract(off)

namespace {

struct Row {
    std::vector<int32_t> c;   // sorted column indices (active columns only)
    std::vector<double> v;
};

constexpr double kAlphaBK = 0.6403882032022076;   // (1 + sqrt(17)) / 8

double row_get(const Row &r, int32_t col)
{
    auto it = std::lower_bound(r.c.begin(), r.c.end(), col);
    if (it == r.c.end() || *it != col) return 0.0;
    return r.v[it - r.c.begin()];
}

void row_erase(Row &r, int32_t col)
{
    auto it = std::lower_bound(r.c.begin(), r.c.end(), col);
    if (it == r.c.end() || *it != col) return;
    const size_t p = it - r.c.begin();
    r.c.erase(r.c.begin() + p);
    r.v.erase(r.v.begin() + p);
}

// r(cols[q]) -= delta[q] for sorted cols: a merge that inserts fill in order.
void row_sub(Row &r, const std::vector<int32_t> &cols, const std::vector<double> &delta,
             std::vector<int32_t> &tc, std::vector<double> &tv)
{
    tc.clear();
    tv.clear();
    size_t a = 0, b = 0;
    while (a < r.c.size() || b < cols.size()) {
        if (b == cols.size() || (a < r.c.size() && r.c[a] < cols[b])) {
            tc.push_back(r.c[a]);
            tv.push_back(r.v[a]);
            ++a;
        } else if (a == r.c.size() || cols[b] < r.c[a]) {
            tc.push_back(cols[b]);
            tv.push_back(0.0 - delta[b]);
            ++b;
        } else {
            tc.push_back(r.c[a]);
            tv.push_back(r.v[a] - delta[b]);
            ++a;
            ++b;
        }
    }
    r.c.swap(tc);
    r.v.swap(tv);
}

}  // namespace

struct ecnt_ildl_s {
    int64_t n = 0;
    std::vector<int32_t> perm;
    std::vector<int32_t> lrp, lci;   // strictly lower L by rows
    std::vector<double> lval;
    std::vector<double> dd, doff;
    int32_t bandwidth = 0, n2x2 = 0, nneg = 0;
};

namespace {

// Returns ECNT_OK, ECNT_ENOTHPD on a zero or singular pivot.
ecnt_status factor(ecnt_ildl_s &F, int64_t n, const int32_t *rp, const int32_t *ci,
                   const double *val, double tau, double t)
{
    std::vector<Row> S(n);
    for (int64_t r = 0; r < n; ++r) {
        Row &row = S[r];
        // duplicate column indices are summed, the shift goes on the diagonal
        std::vector<std::pair<int32_t, double>> e;
        e.reserve(rp[r + 1] - rp[r] + 1);
        for (int32_t p = rp[r]; p < rp[r + 1]; ++p) e.emplace_back(ci[p], val[p]);
        std::stable_sort(e.begin(), e.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        bool diag = false;
        for (size_t q = 0; q < e.size(); ++q) {
            if (!row.c.empty() && row.c.back() == e[q].first) {
                row.v.back() += e[q].second;
            } else {
                row.c.push_back(e[q].first);
                row.v.push_back(0.0 + e[q].second);
            }
        }
        for (size_t q = 0; q < row.c.size(); ++q)
            if (row.c[q] == r) {
                row.v[q] -= tau;
                diag = true;
            }
        if (!diag) {
            auto it = std::lower_bound(row.c.begin(), row.c.end(), (int32_t)r);
            const size_t p = it - row.c.begin();
            row.c.insert(row.c.begin() + p, (int32_t)r);
            row.v.insert(row.v.begin() + p, 0.0 - tau);
        }
    }
    // the pattern is made symmetric (explicit zeros where only one triangle
    // stores an entry), so that an interchange finds every row it touches
    {
        std::vector<std::vector<int32_t>> add(n);
        for (int64_t r = 0; r < n; ++r)
            for (int32_t c : S[r].c)
                if (!std::binary_search(S[c].c.begin(), S[c].c.end(), (int32_t)r))
                    add[c].push_back((int32_t)r);
        for (int64_t r = 0; r < n; ++r)
            for (int32_t c : add[r]) {
                auto it = std::lower_bound(S[r].c.begin(), S[r].c.end(), c);
                const size_t p = it - S[r].c.begin();
                S[r].c.insert(S[r].c.begin() + p, c);
                S[r].v.insert(S[r].v.begin() + p, 0.0);
            }
    }
    F.n = n;
    F.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) F.perm[i] = (int32_t)i;
    F.dd.assign(n, 0.0);
    F.doff.assign(n, 0.0);
    std::vector<std::vector<std::pair<int32_t, double>>> Lrows(n);   // (col, l) in column order
    std::vector<int32_t> tc, cols;
    std::vector<double> tv, delta, l1(n, 0.0), l2(n, 0.0);
    std::vector<int32_t> idx;
    std::vector<int32_t> touched;

    // symmetric interchange of active indices a and b
    auto swap_idx = [&](int32_t a, int32_t b) {
        if (a == b) return;
        std::swap(S[a], S[b]);
        std::swap(Lrows[a], Lrows[b]);
        std::swap(F.perm[a], F.perm[b]);
        touched.clear();
        for (int32_t c : S[a].c) touched.push_back(c);
        for (int32_t c : S[b].c) touched.push_back(c);
        std::sort(touched.begin(), touched.end());
        touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
        for (int32_t x : touched) {
            Row &row = S[x];
            const double va = row_get(row, a), vb = row_get(row, b);
            const bool ha = std::binary_search(row.c.begin(), row.c.end(), a);
            const bool hb = std::binary_search(row.c.begin(), row.c.end(), b);
            row_erase(row, a);
            row_erase(row, b);
            auto put = [&](int32_t col, double v) {
                auto it = std::lower_bound(row.c.begin(), row.c.end(), col);
                const size_t p = it - row.c.begin();
                row.c.insert(row.c.begin() + p, col);
                row.v.insert(row.v.begin() + p, v);
            };
            if (ha) put(b, va);
            if (hb) put(a, vb);
        }
    };

    int64_t k = 0;
    while (k < n) {
        double lambda = 0.0;
        int32_t r = -1;
        for (size_t q = 0; q < S[k].c.size(); ++q)
            if (S[k].c[q] > k && std::fabs(S[k].v[q]) > lambda) {
                lambda = std::fabs(S[k].v[q]);
                r = S[k].c[q];
            }
        bool two = false;
        const double akk = row_get(S[k], (int32_t)k);
        if (lambda > 0.0 && std::fabs(akk) < kAlphaBK * lambda) {
            double sigma = 0.0;
            for (size_t q = 0; q < S[r].c.size(); ++q)
                if (S[r].c[q] >= k && S[r].c[q] != r && std::fabs(S[r].v[q]) > sigma)
                    sigma = std::fabs(S[r].v[q]);
            if (std::fabs(akk) * sigma >= kAlphaBK * lambda * lambda) {
                // 1x1 at k
            } else if (std::fabs(row_get(S[r], r)) >= kAlphaBK * sigma) {
                swap_idx(r, (int32_t)k);
            } else {
                swap_idx(r, (int32_t)(k + 1));
                two = true;
            }
        }
        idx.clear();
        if (!two) {
            const double d = row_get(S[k], (int32_t)k);
            if (d == 0.0) return ECNT_ENOTHPD;
            F.dd[k] = d;
            double nrm = 0.0;
            for (size_t q = 0; q < S[k].c.size(); ++q) {
                const int32_t i = S[k].c[q];
                if (i <= k) continue;
                l1[i] = S[k].v[q] / d;
                nrm += std::fabs(l1[i]);
            }
            const double thr = t * nrm;
            for (size_t q = 0; q < S[k].c.size(); ++q) {
                const int32_t i = S[k].c[q];
                if (i <= k) continue;
                if (std::fabs(l1[i]) < thr) l1[i] = 0.0;
                if (l1[i] != 0.0) idx.push_back(i);
            }
            // every active row that held column k loses it
            for (size_t q = 0; q < S[k].c.size(); ++q)
                if (S[k].c[q] > k) row_erase(S[S[k].c[q]], (int32_t)k);
            cols.assign(idx.begin(), idx.end());
            delta.resize(idx.size());
            for (int32_t i : idx) {
                for (size_t q = 0; q < idx.size(); ++q) {
                    const int32_t j = idx[q];
                    const int32_t hi = std::max(i, j), lo = std::min(i, j);
                    delta[q] = (l1[hi] * d) * l1[lo];
                }
                row_sub(S[i], cols, delta, tc, tv);
            }
            for (int32_t i : idx) Lrows[i].emplace_back((int32_t)k, l1[i]);
            for (size_t q = 0; q < S[k].c.size(); ++q)
                if (S[k].c[q] > k) l1[S[k].c[q]] = 0.0;
            S[k] = Row();
            k += 1;
        } else {
            const double a = row_get(S[k], (int32_t)k), b = row_get(S[k + 1], (int32_t)k),
                         c = row_get(S[k + 1], (int32_t)(k + 1));
            const double det = a * c - b * b;
            if (det == 0.0) return ECNT_ENOTHPD;
            F.dd[k] = a;
            F.dd[k + 1] = c;
            F.doff[k] = b;
            ++F.n2x2;
            // rows beyond the pivot that touch column k or k+1, in order
            touched.clear();
            for (int32_t cc : S[k].c)
                if (cc > k + 1) touched.push_back(cc);
            for (int32_t cc : S[k + 1].c)
                if (cc > k + 1) touched.push_back(cc);
            std::sort(touched.begin(), touched.end());
            touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
            double n1 = 0.0, n2 = 0.0;
            for (int32_t i : touched) {
                const double s1 = row_get(S[k], i), s2 = row_get(S[k + 1], i);
                l1[i] = (s1 * c - s2 * b) / det;
                l2[i] = (s2 * a - s1 * b) / det;
                n1 += std::fabs(l1[i]);
                n2 += std::fabs(l2[i]);
            }
            const double t1 = t * n1, t2 = t * n2;
            for (int32_t i : touched) {
                if (std::fabs(l1[i]) < t1) l1[i] = 0.0;
                if (std::fabs(l2[i]) < t2) l2[i] = 0.0;
                if (l1[i] != 0.0 || l2[i] != 0.0) idx.push_back(i);
            }
            for (int32_t i : touched) {
                row_erase(S[i], (int32_t)k);
                row_erase(S[i], (int32_t)(k + 1));
            }
            cols.assign(idx.begin(), idx.end());
            delta.resize(idx.size());
            for (int32_t i : idx) {
                for (size_t q = 0; q < idx.size(); ++q) {
                    const int32_t j = idx[q];
                    const int32_t hi = std::max(i, j), lo = std::min(i, j);
                    const double w1 = l1[hi] * a + l2[hi] * b;
                    const double w2 = l1[hi] * b + l2[hi] * c;
                    delta[q] = w1 * l1[lo] + w2 * l2[lo];
                }
                row_sub(S[i], cols, delta, tc, tv);
            }
            for (int32_t i : idx) {
                if (l1[i] != 0.0) Lrows[i].emplace_back((int32_t)k, l1[i]);
                if (l2[i] != 0.0) Lrows[i].emplace_back((int32_t)(k + 1), l2[i]);
            }
            for (int32_t i : touched) l1[i] = l2[i] = 0.0;
            S[k] = Row();
            S[k + 1] = Row();
            k += 2;
        }
    }
    // L by rows, inertia of D, bandwidth
    F.lrp.assign(n + 1, 0);
    size_t nnz = 0;
    for (int64_t i = 0; i < n; ++i) nnz += Lrows[i].size();
    if (nnz >= (size_t)INT32_MAX) return ECNT_EUNSUPPORTED;
    F.lci.resize(nnz);
    F.lval.resize(nnz);
    size_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (const auto &pr : Lrows[i]) {
            F.lci[e] = pr.first;
            F.lval[e] = pr.second;
            F.bandwidth = std::max<int32_t>(F.bandwidth, (int32_t)(i - pr.first));
            ++e;
        }
        F.lrp[i + 1] = (int32_t)e;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (i + 1 < n && F.doff[i] != 0.0) {
            // a 2x2 block with b != 0 and det < 0 has one negative eigenvalue;
            // det > 0 two of the sign of its trace
            const double a = F.dd[i], b = F.doff[i], c = F.dd[i + 1];
            const double det = a * c - b * b;
            F.nneg += det < 0.0 ? 1 : ((a + c) < 0.0 ? 2 : 0);
            ++i;
        } else {
            F.nneg += F.dd[i] < 0.0 ? 1 : 0;
        }
    }
    return ECNT_OK;
}

}  // namespace

extern "C" {

ECNT_API ecnt_status ecnt_ildl_factor(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                      const double *val, double tau, double droptol,
                                      ecnt_ildl *out)
{
    if (!out) return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: out is NULL");
    *out = nullptr;
    if (n < 1 || n >= INT32_MAX || !row_ptr || !col_idx || !val)
        return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: bad matrix");
    if (!std::isfinite(tau) || !(droptol >= 0.0) || !std::isfinite(droptol))
        return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: tau and droptol must be finite, droptol >= 0");
    if (row_ptr[0] != 0) return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: row_ptr[0] != 0");
    for (int64_t r = 0; r < n; ++r) {
        if (row_ptr[r + 1] < row_ptr[r])
            return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: row_ptr not monotone");
        for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
            if (col_idx[p] < 0 || col_idx[p] >= n)
                return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: column index out of range");
    }
    ecnt_ildl_s *F = new (std::nothrow) ecnt_ildl_s();
    if (!F) return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: out of host memory");
    ecnt_status st;
    try {
        st = factor(*F, n, row_ptr, col_idx, val, tau, droptol);
    } catch (const std::bad_alloc &) {
        delete F;
        return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: out of host memory");
    } catch (...) {   // no C++ exception crosses the ABI
        delete F;
        return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_factor: internal error");
    }
    if (st != ECNT_OK) {
        delete F;
        if (st == ECNT_ENOTHPD)
            return ecnt::set_error(st, "ecnt_ildl_factor: zero pivot (A - tau I singular in the factorization)");
        return ecnt::set_error(st, "ecnt_ildl_factor: factor exceeds int32 indexing");
    }
    *out = F;
    return ECNT_OK;
}

ECNT_API ecnt_status ecnt_ildl_sizes(const ecnt_ildl f, int64_t *nnz, int32_t *bandwidth,
                                     int32_t *n2x2, int32_t *nneg)
{
    if (!f) return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_sizes: NULL factor");
    if (nnz) *nnz = (int64_t)f->lci.size();
    if (bandwidth) *bandwidth = f->bandwidth;
    if (n2x2) *n2x2 = f->n2x2;
    if (nneg) *nneg = f->nneg;
    return ECNT_OK;
}

ECNT_API ecnt_status ecnt_ildl_export(const ecnt_ildl f, int32_t *perm, int32_t *l_row_ptr,
                                      int32_t *l_col_idx, double *l_val, double *d_diag,
                                      double *d_off)
{
    if (!f) return ecnt::set_error(ECNT_EINVAL, "ecnt_ildl_export: NULL factor");
    const int64_t n = f->n;
    const size_t nnz = f->lci.size();
    if (perm) std::memcpy(perm, f->perm.data(), sizeof(int32_t) * n);
    if (l_row_ptr) std::memcpy(l_row_ptr, f->lrp.data(), sizeof(int32_t) * (n + 1));
    if (l_col_idx && nnz) std::memcpy(l_col_idx, f->lci.data(), sizeof(int32_t) * nnz);
    if (l_val && nnz) std::memcpy(l_val, f->lval.data(), sizeof(double) * nnz);
    if (d_diag) std::memcpy(d_diag, f->dd.data(), sizeof(double) * n);
    if (d_off) std::memcpy(d_off, f->doff.data(), sizeof(double) * n);
    return ECNT_OK;
}

ECNT_API void ecnt_ildl_free(ecnt_ildl f) { delete f; }

}  // extern "C"
