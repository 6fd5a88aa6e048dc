// Factored absolute-value preconditioner of Section 6 on a block of columns:
//   M x   = |D|^{-1/2} L^{-1} P x      (gather, k_ldl_solve<FWD>, k_ldl_eapply)
//   M^* x = P^T L^{-T} |D|^{-1/2} x    (k_ldl_eapply, k_ldl_solve<BWD>, scatter)
// with P (A - tau I) P^T ~ L D L^T the factor of the columns' shift.
//
// The substitutions are sequential in the rows; the columns (probes) are the
// parallel dimension: one wavefront owns a column and walks all n rows in
// column form, keeping the pending sums of the next kRing rows in registers,
// which serves any factor of bandwidth at most kRing.  The factor is used in
// band form (each row as 256 values by distance from the diagonal, built once
// per call), so no column indices are read.
#include <type_traits>
#include <utility>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

namespace {
constexpr int kRing = 256;   // band width (the largest bandwidth served)
// rows of padding before and after each band: a batch of rows staged past
// either end of the walk reads them (never used), so no row index is clamped
constexpr int kPad = 32;
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
// (d = 1..256; zeros where L has no entry), each with kPad zero rows before
// and after (bf and bb point at row 0).
__global__ void k_ldl_band_zero(int64_t n, double *__restrict__ bf, double *__restrict__ bb)
{
    const int64_t total = (n + 2 * kPad) * kRing;
    bf -= (size_t)kPad * kRing;
    bb -= (size_t)kPad * kRing;
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
    // a wavefront per row, its lanes over the row's entries (each entry has
    // its own slot in either band)
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    int64_t p0 = rp[i], p1 = rp[i + 1];
    p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
    p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
    for (int64_t p = p0 + lane; p < p1; p += 64) {
        const int64_t j = ci[p], d = i - j;
        if (j < 0 || j >= n || d < 1 || d > kRing) continue;   // outside the declared bandwidth
        bf[(size_t)i * kRing + kRing - d] = lv[p];
        bb[(size_t)j * kRing + kRing - d] = lv[p];
    }
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

// Substitution with the unit triangular factor on columns [c_lo, c_hi), in
// column (right-looking) form:
//   FWD: y_r = X[r] - sum_{j<r} l_rj y_j, rows r = 0..n-1
//   BWD: w_r = X[r] - sum_{j>r} l_jr w_j, rows r = n-1..0
// (Y[r] = y_r / w_r).  In walk order t (FWD r = t, BWD r = n-1-t) the value of
// step t enters steps t+1 .. t+256 with the coefficients of one band row:
// band[r][256 - d] links step t to step t + d (FWD: column r of L, i.e. the
// band of L^T; BWD: row r of L).  A wavefront owns one column: lane q keeps
// the pending sums of steps T0 + q + 64 s (s = 0..4) of the current group of
// 64 steps in registers (5 slots: from step T0 + 63 the values reach
// T0 + 319).  Step t = T0 + Q0: lane Q0 forms y = X - pending, v_readlane
// broadcasts it through scalar registers, and every lane adds coefficient * y
// to its 5 pending sums; at the end of a group the sums shift by one slot.
// The chain from one row to the next is a subtraction, the broadcast and one
// FMA; the next step's 5 coefficients are read from LDS before the current
// step's broadcast (two register sets alternate by step parity).  Band rows
// are loaded 16 steps ahead into registers and staged into LDS per 16 steps
// between 64 zeros on each side (read for distances outside 1..256).  All
// shifts of the wave in one launch (each solve is a latency-bound chain, so
// the shifts' chains run side by side): blocks [blk0[s], blk0[s+1]) serve
// shift s, its columns [lo[s], hi[s]) and its factor's band.
struct LdlSolveSet {
    int nsh;
    int blk0[kMaxShifts + 1];
    int lo[kMaxShifts], hi[kMaxShifts];
    const double *band[kMaxShifts];
};

template <typename T, bool FWD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_ldl_solve(
    int64_t n, int C, const LdlSolveSet set, const T *__restrict__ X, T *__restrict__ Y)
{
    int sh = 0;
    while (sh + 1 < set.nsh && (int)blockIdx.x >= set.blk0[sh + 1]) ++sh;
    const int c_lo = set.lo[sh], c_hi = set.hi[sh];
    const double *__restrict__ band = set.band[sh];
    const int blk = (int)blockIdx.x - set.blk0[sh];
    constexpr int NS = 64;             // lanes per column, steps per group
    constexpr int NR = kRing / NS;     // the pending sums per lane are NR + 1
    constexpr int kBatch = 16;         // band rows staged at a time
    constexpr int kRow = NS + kRing + NS;   // staged row: zeros, band, zeros
    __shared__ double stg[kBatch][kRow];
    const int q = threadIdx.x;
    const int craw = c_lo + blk;
    const bool ok = craw < c_hi;
    const int c = ok ? craw : c_lo;
    for (int u = 0; u < kBatch; ++u) {
        stg[u][q] = 0.0;
        stg[u][NS + kRing + q] = 0.0;
    }

    auto row_of = [&](int64_t t) -> int64_t {
        const int64_t tt = t < n ? t : n - 1;   // past the end: repeat the last row (unused)
        return FWD ? tt : n - 1 - tt;
    };
    double nv[kBatch][4];   // next batch: band values 2 q, 2 q + 1, 128 + 2 q, 129 + 2 q
    // rows of steps t0 .. t0 + 15: consecutive band rows (up in FWD, down in
    // BWD) from one row pointer; t0 < n + 16, so the rows stay within the
    // kPad rows of padding past either end
    auto load_batch = [&](int64_t t0) __attribute__((always_inline)) {
        const double2 *row0 =
            reinterpret_cast<const double2 *>(band + (FWD ? t0 : n - 1 - t0) * (int64_t)kRing);
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const double2 *row = row0 + (FWD ? u : -u) * (kRing / 2);
            const double2 a = row[q], b = row[64 + q];
            nv[u][0] = a.x;
            nv[u][1] = a.y;
            nv[u][2] = b.x;
            nv[u][3] = b.y;
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
            reinterpret_cast<double2 *>(stg[u] + NS)[q] = a;
            reinterpret_cast<double2 *>(stg[u] + NS)[64 + q] = b;
        }
    };
    auto load_b = [&](int64_t T0) -> T { return X[(size_t)row_of(T0 + q) * C + c]; };

    double slot[NR + 1];
#pragma unroll
    for (int s2 = 0; s2 <= NR; ++s2) slot[s2] = 0.0;
    T b_own = load_b(0), b_next = load_b(NS);

    // coefficients of a step (position Q0 in the group, staging row u) for
    // slot s: distance d = q - Q0 + 64 s, staged index 64 + 256 - d (zero
    // unless 1 <= d <= 256).  Lane q's slot 0 takes only zeros from step
    // T0 + q on, so its y is b - slot[0] at the end of the group.
    double ca[NR + 1], cb[NR + 1];
    auto coefs = [&](int Q0, int u, double (&c_)[NR + 1]) __attribute__((always_inline)) {
        const double *sr = stg[u] + (NS - q + Q0);
#pragma unroll
        for (int s2 = 0; s2 <= NR; ++s2) c_[s2] = sr[NS * (NR - s2)];
    };
    // one step: Q0 = position in the group (compile-time), U = staging row
    auto step = [&]<int Q0>(std::integral_constant<int, Q0>, int u) __attribute__((always_inline)) {
        double(&cur)[NR + 1] = (Q0 & 1) ? cb : ca;
        double(&nxt)[NR + 1] = (Q0 & 1) ? ca : cb;
        if (u + 1 < kBatch) coefs(Q0 + 1, u + 1, nxt);
        const double y = static_cast<double>(b_own) - slot[0];   // meaningful in lane Q0
        const int lo = __builtin_amdgcn_readlane(__double2loint(y), Q0);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(y), Q0);
        const double yb = __hiloint2double(hi, lo);
#pragma unroll
        for (int s2 = 0; s2 <= NR; ++s2) slot[s2] += cur[s2] * yb;
        // every pending sum is complete after its step (the compiler would
        // otherwise defer the FMAs of slots 1.. to the end of the group and
        // hold every step's coefficients and y until then)
#pragma unroll
        for (int s2 = 1; s2 <= NR; ++s2) asm volatile("" : "+v"(slot[s2]));
    };
    // batch B of the group (steps 16 B .. 16 B + 15), staged in stg; FULL: the
    // whole group lies before step n (no test per step)
    auto batch = [&]<int B, bool FULL>(int64_t T0, std::integral_constant<int, B>,
                                       std::bool_constant<FULL>) __attribute__((always_inline)) {
        if constexpr ((B * kBatch) & 1) coefs(B * kBatch, 0, cb);
        else coefs(B * kBatch, 0, ca);
        [&]<int... U>(std::integer_sequence<int, U...>) __attribute__((always_inline)) {
            ((FULL || T0 + B * kBatch + U < n ? step(std::integral_constant<int, B * kBatch + U>{}, U)
                                              : void()),
             ...);
        }(std::make_integer_sequence<int, kBatch>{});
    };
    // after a batch: stage the next one (loaded one batch ago), load the one after it
    auto advance = [&](int64_t t_next) __attribute__((always_inline)) {
        if (t_next < n) {
            stage_batch();
            load_batch(t_next + kBatch);
        }
    };
    auto group = [&]<bool FULL>(int64_t T0, std::bool_constant<FULL> f) __attribute__((always_inline)) {
        batch(T0, std::integral_constant<int, 0>{}, f);
        advance(T0 + kBatch);
        batch(T0, std::integral_constant<int, 1>{}, f);
        advance(T0 + 2 * kBatch);
        batch(T0, std::integral_constant<int, 2>{}, f);
        advance(T0 + 3 * kBatch);
        batch(T0, std::integral_constant<int, 3>{}, f);
    };

    load_batch(0);
    stage_batch();
    load_batch(kBatch);
    // after a group: store its y, shift the pending sums by one slot
    auto finish_group = [&](int64_t T0) __attribute__((always_inline)) {
        if (ok && T0 + q < n)
            Y[(size_t)row_of(T0 + q) * C + c] = static_cast<T>(static_cast<double>(b_own) - slot[0]);
#pragma unroll
        for (int s2 = 0; s2 < NR; ++s2) slot[s2] = slot[s2 + 1];
        slot[NR] = 0.0;
        b_own = b_next;
        b_next = load_b(T0 + 2 * NS);
        advance(T0 + NS);
    };
    // the groups that end before step n, then the partial last group
    int64_t T0 = 0;
    for (; T0 + NS <= n; T0 += NS) {
        group(T0, std::true_type{});
        finish_group(T0);
    }
    if (T0 < n) {
        group(T0, std::false_type{});
        finish_group(T0);
    }
}

int ldl_ring_rows() { return kRing; }

size_t ldl_band_bytes(int64_t n, int S) { return sizeof(double) * 2 * (size_t)S * (n + 2 * kPad) * kRing; }

// row 0 of the band of shift s: which = 0 rows of L, 1 rows of L^T
static double *band_of(const Plan &p, int s, int which)
{
    return p.band + ((size_t)(2 * s + which) * (p.n + 2 * kPad) + kPad) * kRing;
}

void launch_ldl_eblocks(const Plan &p, hipStream_t st)
{
    for (int s = 0; s < p.S; ++s) {
        double *ed = p.e_blk + (size_t)s * 2 * p.n, *eo = ed + p.n;
        k_ldl_eblocks<<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(p.n, p.ldl[s].dd, p.ldl[s].doff,
                                                                     ed, eo);
        double *bf = band_of(p, s, 0), *bb = band_of(p, s, 1);
        k_ldl_band_zero<<<1024, 256, 0, st>>>(p.n, bf, bb);
        k_ldl_band_fill<<<(unsigned)((p.n + 3) / 4), 256, 0, st>>>(
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
    if (what == 1 || what == 2) {
        // forward substitution walks the columns of L (the band of L^T),
        // back substitution the rows of L
        LdlSolveSet set;
        set.nsh = 0;
        set.blk0[0] = 0;
        for (int s = 0; s < p.S; ++s) {
            int lo, hi;
            if (!shift_cols(p, s, lo, hi)) continue;
            const double *bf = band_of(p, s, 0), *bb = band_of(p, s, 1);
            const int k = set.nsh++;
            set.lo[k] = lo;
            set.hi[k] = hi;
            set.band[k] = what == 1 ? bb : bf;
            set.blk0[k + 1] = set.blk0[k] + (hi - lo);   // one wavefront per column
        }
        if (set.nsh == 0) return;
        const unsigned grid = (unsigned)set.blk0[set.nsh];
        if (what == 1)
            k_ldl_solve<T, true><<<grid, 64, 0, st>>>(p.n, p.C, set, (const T *)X, (T *)Y);
        else
            k_ldl_solve<T, false><<<grid, 64, 0, st>>>(p.n, p.C, set, (const T *)X, (T *)Y);
        return;
    }
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
        default:
            break;
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
