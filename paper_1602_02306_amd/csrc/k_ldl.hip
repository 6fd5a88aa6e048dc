// Factored absolute-value preconditioner of Section 6 on a block of columns:
//   M x   = |D|^{-1/2} L^{-1} P x      (k_ldl_solve<FWD> with the gather, then k_ldl_eapply)
//   M^* x = P^T L^{-T} |D|^{-1/2} x    (k_ldl_eapply, then k_ldl_solve<BWD> with the scatter)
// with P (A - tau I) P^T ~ L D L^T the factor of the columns' shift.
//
// The substitutions are sequential in the rows; the columns (probes) are the
// parallel dimension: one wavefront owns 64 columns and walks all n rows,
// keeping the last kRing solved rows of its columns in LDS (a ring indexed by
// row mod kRing), so every x_j a row needs comes from LDS when the factor's
// bandwidth is at most kRing.  The row's entries (index, value) are the same
// for every lane: they are staged in LDS two rows ahead and read back as
// broadcasts.  Four partial sums break the dependence chain of a long row.
#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

namespace {
constexpr int kRing = 256;   // rows kept per column: 256 x 64 x 8 B = 128 KiB of LDS
}

// |D|^{-1/2} block by block, for one shift.  A 2 x 2 block [[a, b], [b, c]]
// (b != 0) has eigenvalues mu_{1,2} = (a + c)/2 +- r, r = hypot((a - c)/2, b),
// and f(D) = (f(mu_1) (D - mu_2 I) - f(mu_2) (D - mu_1 I)) / (mu_1 - mu_2) for
// f(mu) = |mu|^{-1/2} (Sylvester's formula).  With x = (a - c)/2,
// a - mu_2 = r + x = p, c - mu_2 = r - x = q (p, q >= 0, p q = b^2), so
//   f(D)_11 = (f1 p + f2 q) / 2r,  f(D)_22 = (f1 q + f2 p) / 2r,
//   f(D)_12 = (f1 - f2) b / 2r,
// the smaller of p, q taken as b^2 / the larger (no cancellation).
__global__ void k_ldl_eblocks(int64_t n, const double *__restrict__ dd,
                              const double *__restrict__ doff, double *__restrict__ ed,
                              double *__restrict__ eo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i > 0 && doff[i - 1] != 0.0) return;   // second row of a block: done by row i-1
    if (i + 1 < n && doff[i] != 0.0) {
        const double a = dd[i], b = doff[i], c = dd[i + 1];
        const double x = 0.5 * (a - c), r = hypot(x, b);
        const double big = r + fabs(x), small = (b * b) / big;
        const double p = x >= 0.0 ? big : small, q = x >= 0.0 ? small : big;
        const double mid = 0.5 * (a + c);
        const double f1 = 1.0 / sqrt(fabs(mid + r)), f2 = 1.0 / sqrt(fabs(mid - r));
        const double inv = 1.0 / (2.0 * r);
        ed[i] = (f1 * p + f2 * q) * inv;
        ed[i + 1] = (f1 * q + f2 * p) * inv;
        eo[i] = (f1 - f2) * b * inv;
        eo[i + 1] = 0.0;
    } else {
        ed[i] = 1.0 / sqrt(fabs(dd[i]));
        eo[i] = 0.0;
    }
}

// Y = |D|^{-1/2} (xs .* X) on columns [c_lo, c_hi): one thread per (row, column).
template <typename T>
__global__ __launch_bounds__(256) void k_ldl_eapply(int64_t n, int C, int c_lo, int c_hi,
                                                    const double *__restrict__ doff,
                                                    const double *__restrict__ ed,
                                                    const double *__restrict__ eo,
                                                    const T *__restrict__ X,
                                                    const double *__restrict__ xs,
                                                    T *__restrict__ Y)
{
    const int w = c_hi - c_lo;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n * w) return;
    const int64_t r = g / w;
    const int c = c_lo + (int)(g - r * w);
    const double sc = xs ? xs[c] : 1.0;
    auto x = [&](int64_t i) { return static_cast<double>(X[(size_t)i * C + c]) * sc; };
    double y;
    if (r + 1 < n && doff[r] != 0.0) y = ed[r] * x(r) + eo[r] * x(r + 1);
    else if (r > 0 && doff[r - 1] != 0.0) y = eo[r - 1] * x(r - 1) + ed[r] * x(r);
    else y = ed[r] * x(r);
    Y[(size_t)r * C + c] = static_cast<T>(y);
}

// Substitution with the unit triangular factor on columns [c_lo, c_hi):
//   FWD: y_r = (xs .* X)[perm[r]] - sum_{j<r} l_rj y_j, rows r = 0..n-1, Y[r] = y_r
//   BWD: w_r = X[r] - sum_{j>r} l_jr w_j (rows of L^T), r = n-1..0, Y[perm[r]] = w_r
// One wavefront, one column per lane.  Row t of the walk (t = 0..n-1) uses:
//   - its entries, staged in LDS (value, ring offset) at the end of row t-1,
//     loaded from HBM at the end of row t-2 (two register sets by row parity);
//   - its input value, loaded at the end of row t-2;
//   - its entry range and permutation index, loaded 64 rows ahead (lane l of a
//     chunk register holds row 64k + l) and read with readlane.
// Entries past the row's count are staged as (0, offset 0); the ring starts at 0.
template <typename T, bool FWD>
__global__ __launch_bounds__(64) void k_ldl_solve(int64_t n, int C, int c_lo, int c_hi,
                                                  int64_t nnz, const int32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ lv,
                                                  const T *__restrict__ X,
                                                  const double *__restrict__ xs,
                                                  T *__restrict__ Y)
{
    constexpr int kQ = kRing / 64;   // staging chunks of 64 entries
    __shared__ double ring[kRing * 64];
    __shared__ double sv[2][kRing];
    __shared__ int32_t so[2][kRing];
    const int lane = threadIdx.x;
    const int craw = c_lo + blockIdx.x * 64 + lane;
    const bool ok = craw < c_hi;
    const int c = ok ? craw : c_lo;
    const double sc = (FWD && xs) ? xs[c] : 1.0;
    for (int q = 0; q < kRing; ++q) ring[q * 64 + lane] = 0.0;

    auto row_of = [&](int64_t t) -> int64_t { return FWD ? t : n - 1 - t; };
    // chunk registers: entry start, entry count, permutation of rows 64k + lane
    int32_t mA0 = 0, mAc = 0, mAp = 0, mB0 = 0, mBc = 0, mBp = 0;
    auto load_chunk = [&](int64_t k, int32_t &m0, int32_t &mc, int32_t &mp) {
        const int64_t t = k * 64 + lane;
        if (t < n) {
            const int64_t r = row_of(t);
            int32_t a = rp[r], b = rp[r + 1];
            a = a < 0 ? 0 : (a > nnz ? (int32_t)nnz : a);
            b = b < a ? a : (b > nnz ? (int32_t)nnz : b);
            int32_t pr = perm[r];
            pr = pr < 0 ? 0 : (pr >= n ? (int32_t)(n - 1) : pr);
            m0 = a;
            mc = (b - a) > kRing ? kRing : (b - a);
            mp = pr;
        } else {
            m0 = 0;
            mc = 0;
            mp = 0;
        }
    };
    int64_t chunkA = 0;   // chunk held in mA*; mB* holds chunkA + 1
    load_chunk(0, mA0, mAc, mAp);
    load_chunk(1, mB0, mBc, mBp);
    struct Meta {
        int32_t p0, cnt, pr;
    };
    auto meta = [&](int64_t t) -> Meta {
        const int l = (int)(t & 63);
        if ((t >> 6) == chunkA)
            return {__builtin_amdgcn_readlane(mA0, l), __builtin_amdgcn_readlane(mAc, l),
                    __builtin_amdgcn_readlane(mAp, l)};
        return {__builtin_amdgcn_readlane(mB0, l), __builtin_amdgcn_readlane(mBc, l),
                __builtin_amdgcn_readlane(mBp, l)};
    };
    struct Set {
        double v[kQ];
        int32_t o[kQ];
        double b;
        int32_t cnt;
    };
    auto fetch = [&](int64_t t, Set &S) {
        const Meta m = meta(t);
        S.cnt = m.cnt;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int e = q * 64 + lane;
            const bool in = e < m.cnt;
            S.v[q] = in ? lv[m.p0 + e] : 0.0;
            S.o[q] = in ? (ci[m.p0 + e] & (kRing - 1)) * 64 : 0;
        }
        const int64_t src = FWD ? (int64_t)m.pr : row_of(t);
        S.b = static_cast<double>(X[(size_t)src * C + c]) * sc;
    };
    auto commit = [&](const Set &S, int buf) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            sv[buf][q * 64 + lane] = S.v[q];
            so[buf][q * 64 + lane] = S.o[q];
        }
    };
    // row t: entries in staging buffer t & 1, input b
    auto solve_row = [&](int64_t t, int buf, int32_t cnt, double b) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        const double *v = sv[buf];
        const int32_t *o = so[buf];
        for (int e = 0; e < cnt; e += 4) {
            a0 += v[e] * ring[o[e] + lane];
            a1 += v[e + 1] * ring[o[e + 1] + lane];
            a2 += v[e + 2] * ring[o[e + 2] + lane];
            a3 += v[e + 3] * ring[o[e + 3] + lane];
        }
        const double y = b - ((a0 + a1) + (a2 + a3));
        const int64_t r = row_of(t);
        ring[(int)(r & (kRing - 1)) * 64 + lane] = y;
        const int64_t dst = FWD ? r : (int64_t)meta(t).pr;
        if (ok) Y[(size_t)dst * C + c] = static_cast<T>(y);
    };

    Set S0, S1;   // rows of even / odd walk index
    fetch(0, S0);
    commit(S0, 0);
    int32_t cnt_cur = S0.cnt;
    double b_cur = S0.b;
    if (n > 1) fetch(1, S1);
    if (n > 2) fetch(2, S0);
    for (int64_t t = 0; t < n; t += 2) {
        // even row t (staging 0), then odd row t+1 (staging 1)
        if ((t >> 6) != chunkA) {   // entering a new chunk: shift and load the next one
            chunkA = t >> 6;
            mA0 = mB0;
            mAc = mBc;
            mAp = mBp;
            load_chunk(chunkA + 1, mB0, mBc, mBp);
        }
        solve_row(t, 0, cnt_cur, b_cur);
        if (t + 1 >= n) break;
        commit(S1, 1);
        cnt_cur = S1.cnt;
        b_cur = S1.b;
        if (t + 3 < n) fetch(t + 3, S1);
        solve_row(t + 1, 1, cnt_cur, b_cur);
        if (t + 2 >= n) break;
        commit(S0, 0);
        cnt_cur = S0.cnt;
        b_cur = S0.b;
        if (t + 4 < n) fetch(t + 4, S0);
    }
}

int ldl_ring_rows() { return kRing; }

void launch_ldl_eblocks(const Plan &p, hipStream_t st)
{
    for (int s = 0; s < p.S; ++s) {
        double *ed = p.e_blk + (size_t)s * 2 * p.n, *eo = ed + p.n;
        k_ldl_eblocks<<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(p.n, p.ldl[s].dd, p.ldl[s].doff,
                                                                     ed, eo);
    }
}

// columns of the wave that belong to shift s: [lo, hi)
static inline bool shift_cols(const Plan &p, int s, int &lo, int &hi)
{
    const int g0 = s * p.m, g1 = (s + 1) * p.m;
    lo = (g0 > p.c_off ? g0 : p.c_off) - p.c_off;
    hi = (g1 < p.c_off + p.C ? g1 : p.c_off + p.C) - p.c_off;
    return hi > lo;
}

template <typename T>
static void ldl_t(const Plan &p, int what, const void *X, const double *xs, void *Y, hipStream_t st)
{
    for (int s = 0; s < p.S; ++s) {
        int lo, hi;
        if (!shift_cols(p, s, lo, hi)) continue;
        const LdlDev &f = p.ldl[s];
        const double *ed = p.e_blk + (size_t)s * 2 * p.n, *eo = ed + p.n;
        if (what == 0) {
            const int64_t total = p.n * (hi - lo);
            k_ldl_eapply<T><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(
                p.n, p.C, lo, hi, f.doff, ed, eo, (const T *)X, xs, (T *)Y);
            continue;
        }
        const unsigned grid = (unsigned)((hi - lo + 63) / 64);
        if (what == 1)
            k_ldl_solve<T, true><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, f.nnz, f.perm, f.lrp, f.lci,
                                                      f.lval, (const T *)X, xs, (T *)Y);
        else
            k_ldl_solve<T, false><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, f.nnz, f.perm, f.ltrp,
                                                       f.ltci, f.ltval, (const T *)X, xs, (T *)Y);
    }
}

// what: 0 = |D|^{-1/2} blocks, 1 = forward substitution with the gather by P,
// 2 = back substitution with L^T and the scatter by P^T
void launch_ldl(const Plan &p, int what, const void *X, const double *xs, void *Y, hipStream_t st)
{
    if (p.vec_f32) ldl_t<float>(p, what, X, xs, Y, st);
    else ldl_t<double>(p, what, X, xs, Y, st);
}

}  // namespace ecnt
