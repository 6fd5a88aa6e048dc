// Factored absolute-value preconditioner of Section 6 on a block of columns:
//   M x   = |D|^{-1/2} L^{-1} P x      (gather, k_ldl_solve<FWD>, k_ldl_eapply)
//   M^* x = P^T L^{-T} |D|^{-1/2} x    (k_ldl_eapply, k_ldl_solve<BWD>, scatter)
// with P (A - tau I) P^T ~ L D L^T the factor of the columns' shift.
//
// The substitutions are sequential in the rows; the columns (probes) are the
// parallel dimension: one wavefront owns 2, 4 or 8 columns and walks all n rows,
// keeping the last kRing solved rows of its columns in LDS (a ring indexed by
// row mod kRing), so every x_j a row needs comes from LDS when the factor's
// bandwidth is at most kRing.  The factor is used in band form (each row as
// 256 values by distance from the diagonal, built once per call), so a row
// needs no column indices; 32, 16 or 8 lanes share a column and split its row.
#include <type_traits>
#include <utility>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

namespace {
constexpr int kRing = 256;   // rows kept per column (the largest bandwidth served)
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

// Band form of one factor, built once per call: row i of L as 256 values
// bf[i][256 - d] = l_{i, i-d}, and row i of L^T as bb[i][256 - d] = l_{i+d, i}
// (d = 1..256; zeros where L has no entry).
__global__ void k_ldl_band_zero(int64_t n, double *__restrict__ bf, double *__restrict__ bb)
{
    const int64_t total = n * kRing;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        bf[g] = 0.0;
        bb[g] = 0.0;
    }
}

__global__ void k_ldl_band_fill(int64_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                const int32_t *__restrict__ ci, const double *__restrict__ lv,
                                double *__restrict__ bf, double *__restrict__ bb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t p0 = rp[i], p1 = rp[i + 1];
    p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
    p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
    for (int64_t p = p0; p < p1; ++p) {
        const int64_t j = ci[p], d = i - j;
        if (j < 0 || j >= n || d < 1 || d > kRing) continue;   // outside the declared bandwidth
        bf[(size_t)i * kRing + kRing - d] = lv[p];
        bb[(size_t)j * kRing + kRing - d] = lv[p];
    }
}

// Sum over NS (8, 16 or 32) consecutive lanes (the entry slices of one
// column), by DPP: swap neighbours, swap pairs, mirror the two quads of each
// 8 lanes, (16) mirror the two halves of each 16 lanes, (32) swap the two
// halves of each 32 lanes.
template <int NS>
__device__ __forceinline__ double sum_slices(double x)
{
    auto dpp = [](double v, auto ctrl_tag) -> double {
        constexpr int ctrl = decltype(ctrl_tag)::value;
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xf, 0xf, false);
        return __hiloint2double(hi, lo);
    };
    x += dpp(x, std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
    x += dpp(x, std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
    x += dpp(x, std::integral_constant<int, 0x141>{});  // row_half_mirror
    if constexpr (NS >= 16) x += dpp(x, std::integral_constant<int, 0x140>{});   // row_mirror
    if constexpr (NS == 32) {   // lane ^ 16 within 32 lanes (ds_swizzle bit mode)
        const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), 0x401F);
        const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), 0x401F);
        x += __hiloint2double(hi, lo);
    }
    return x;
}

// Y[r] = X[perm[r]] (gather) or Y[perm[r]] = X[r] (scatter) on columns [c_lo, c_hi).
template <typename T, bool GATHER>
__global__ __launch_bounds__(256) void k_ldl_permute(int64_t n, int C, int c_lo, int c_hi,
                                                     const int32_t *__restrict__ perm,
                                                     const T *__restrict__ X, T *__restrict__ Y)
{
    const int w = c_hi - c_lo;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n * w) return;
    const int64_t r = g / w;
    const int c = c_lo + (int)(g - r * w);
    int64_t pr = perm[r];
    pr = pr < 0 ? 0 : (pr >= n ? n - 1 : pr);
    if (GATHER) Y[(size_t)r * C + c] = X[(size_t)pr * C + c];
    else Y[(size_t)pr * C + c] = X[(size_t)r * C + c];
}

// Substitution with the unit triangular factor on columns [c_lo, c_hi):
//   FWD: y_r = X[r] - sum_{j<r} l_rj y_j, rows r = 0..n-1
//   BWD: w_r = X[r] - sum_{j>r} l_jr w_j, rows r = n-1..0
// (Y[r] = y_r / w_r).  NS lanes share a column (a wavefront owns 64 / NS
// columns); lane = NS * column + slice, and slice q takes the band entries
// k = q + NS rr (rr = 0 .. 256/NS - 1) of every row, so the slices of a
// column read NS consecutive ring rows.  The ring keeps each solved row twice
// (rows j mod 256 and j mod 256 + 256), so all reads of one row use immediate
// offsets from a single base.  Rows are fetched in batches of kBatch (band
// rows and inputs into registers) one batch ahead and staged into LDS at the
// batch boundary: one wait on HBM per batch.
template <typename T, bool FWD, int NS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_ldl_solve(
    int64_t n, int C, int c_lo, int c_hi, const double *__restrict__ band,
    const T *__restrict__ X, T *__restrict__ Y)
{
    constexpr int kBatch = 16;
    constexpr int NC = 64 / NS;        // columns per wavefront
    constexpr int NR = kRing / NS;     // rounds per row
    __shared__ double ring[2 * kRing * NC];
    __shared__ double stg[kBatch][kRing];
    const int lane = threadIdx.x;
    const int cl = lane / NS, q = lane % NS;
    const int craw = c_lo + blockIdx.x * NC + cl;
    const bool ok = craw < c_hi;
    const int c = ok ? craw : c_lo;
    for (int e = lane; e < 2 * kRing * NC; e += 64) ring[e] = 0.0;

    auto row_of = [&](int64_t t) -> int64_t {
        const int64_t tt = t < n ? t : n - 1;   // past the end: repeat the last row (unused)
        return FWD ? tt : n - 1 - tt;
    };
    double nv[kBatch][4];   // next batch: band values 2 lane, 2 lane + 1, 128 + 2 lane, 129 + 2 lane
    T nx[kBatch];           // next batch: inputs
    T cx[kBatch];           // current batch: inputs
    auto load_batch = [&](int64_t t0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t r = row_of(t0 + u);
            const double2 *row = reinterpret_cast<const double2 *>(band + (size_t)r * kRing);
            const double2 a = row[lane], b = row[64 + lane];
            nv[u][0] = a.x;
            nv[u][1] = a.y;
            nv[u][2] = b.x;
            nv[u][3] = b.y;
            nx[u] = X[(size_t)r * C + c];
        }
    };
    auto stage_batch = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            double2 a, b;
            a.x = nv[u][0];
            a.y = nv[u][1];
            b.x = nv[u][2];
            b.y = nv[u][3];
            reinterpret_cast<double2 *>(stg[u])[lane] = a;
            reinterpret_cast<double2 *>(stg[u])[64 + lane] = b;
            cx[u] = nx[u];
        }
    };
    auto solve_row = [&](int64_t t, int u, double b) __attribute__((always_inline)) {
        const int64_t r = row_of(t);
        // ring row of round rr: FWD (r + q + NS rr) mod 256, BWD (r - q - NS rr) mod 256;
        // every round is read (entries outside the row's span are zeros)
        const int x = (int)((FWD ? r + q : r - q) & (kRing - 1));
        const double *rb = FWD ? ring + (x * NC + cl) : ring + ((x + NS) * NC + cl);
        const double *vb = stg[u] + q;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int rr = 0; rr < NR; rr += 4) {
            a0 += vb[NS * rr] * rb[NS * NC * (FWD ? rr : NR - 1 - rr)];
            a1 += vb[NS * (rr + 1)] * rb[NS * NC * (FWD ? rr + 1 : NR - 2 - rr)];
            a2 += vb[NS * (rr + 2)] * rb[NS * NC * (FWD ? rr + 2 : NR - 3 - rr)];
            a3 += vb[NS * (rr + 3)] * rb[NS * NC * (FWD ? rr + 3 : NR - 4 - rr)];
        }
        const double y = b - sum_slices<NS>((a0 + a1) + (a2 + a3));
        const int w = (int)(r & (kRing - 1));
        if (q == 0) {
            ring[w * NC + cl] = y;
            ring[(w + kRing) * NC + cl] = y;
            if (ok) Y[(size_t)r * C + c] = static_cast<T>(y);
        }
    };

    load_batch(0);
    stage_batch();
    load_batch(kBatch);
    for (int64_t t0 = 0; t0 < n; t0 += kBatch) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (t0 + u < n) solve_row(t0 + u, u, static_cast<double>(cx[u]));
        if (t0 + kBatch < n) {
            stage_batch();                  // the batch loaded one batch ago
            load_batch(t0 + 2 * kBatch);
        }
    }
}

int ldl_ring_rows() { return kRing; }

void launch_ldl_eblocks(const Plan &p, hipStream_t st)
{
    for (int s = 0; s < p.S; ++s) {
        double *ed = p.e_blk + (size_t)s * 2 * p.n, *eo = ed + p.n;
        k_ldl_eblocks<<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(p.n, p.ldl[s].dd, p.ldl[s].doff,
                                                                     ed, eo);
        double *bf = p.band + (size_t)s * 2 * p.n * kRing, *bb = bf + (size_t)p.n * kRing;
        k_ldl_band_zero<<<1024, 256, 0, st>>>(p.n, bf, bb);
        k_ldl_band_fill<<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(
            p.n, p.ldl[s].nnz, p.ldl[s].lrp, p.ldl[s].lci, p.ldl[s].lval, bf, bb);
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
        const int64_t total = p.n * (hi - lo);
        const unsigned egrid = (unsigned)((total + 255) / 256);
        switch (what) {
        case 0:
            k_ldl_eapply<T><<<egrid, 256, 0, st>>>(p.n, p.C, lo, hi, f.doff, ed, eo, (const T *)X,
                                                   xs, (T *)Y);
            break;
        case 3:
            k_ldl_permute<T, true><<<egrid, 256, 0, st>>>(p.n, p.C, lo, hi, f.perm, (const T *)X,
                                                          (T *)Y);
            break;
        case 4:
            k_ldl_permute<T, false><<<egrid, 256, 0, st>>>(p.n, p.C, lo, hi, f.perm, (const T *)X,
                                                           (T *)Y);
            break;
        default: {
            const double *bf = p.band + (size_t)s * 2 * p.n * kRing, *bb = bf + (size_t)p.n * kRing;
            // more lanes per column (fewer rounds per row) while the columns
            // fill at most 256 wavefronts; 8 lanes (least LDS traffic per
            // column) beyond that
            if (hi - lo <= 2 * 256) {
                const unsigned grid = (unsigned)((hi - lo + 1) / 2);
                if (what == 1)
                    k_ldl_solve<T, true, 32><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, bf, (const T *)X, (T *)Y);
                else
                    k_ldl_solve<T, false, 32><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, bb, (const T *)X, (T *)Y);
            } else if (hi - lo <= 4 * 256) {
                const unsigned grid = (unsigned)((hi - lo + 3) / 4);
                if (what == 1)
                    k_ldl_solve<T, true, 16><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, bf, (const T *)X, (T *)Y);
                else
                    k_ldl_solve<T, false, 16><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, bb, (const T *)X, (T *)Y);
            } else {
                const unsigned grid = (unsigned)((hi - lo + 7) / 8);
                if (what == 1)
                    k_ldl_solve<T, true, 8><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, bf, (const T *)X, (T *)Y);
                else
                    k_ldl_solve<T, false, 8><<<grid, 64, 0, st>>>(p.n, p.C, lo, hi, bb, (const T *)X, (T *)Y);
            }
        }
        }
    }
}

// what: 0 = |D|^{-1/2} blocks (with the column scales xs), 1 = forward
// substitution with L, 2 = back substitution with L^T, 3 = gather by P,
// 4 = scatter by P^T
void launch_ldl(const Plan &p, int what, const void *X, const double *xs, void *Y, hipStream_t st)
{
    if (p.vec_f32) ldl_t<float>(p, what, X, xs, Y, st);
    else ldl_t<double>(p, what, X, xs, Y, st);
}

}  // namespace ecnt
