// Lanczos recurrence with full reorthogonalization for small problems in one
// launch (Algorithm 1; the probe loop of Algorithm 2 run data-parallel over
// columns): one workgroup per probe column runs all k steps, with its basis in
// a column-contiguous region of the workspace and the current q_i and w in
// LDS.  It computes what the column-wave kernels of k_lanczos.hip compute:
//   w      = C q_i - beta_i q_{i-1}
//   g_l    = q_l^T w,  p_l = q_l^T q_i,  l = 1..i
//   alpha_i = g_i;  c_l = g_l - alpha_i (p_l - [l = i])
//   w     <- w - sum_l c_l q_l
//   beta_{i+1} = |w|,  q_{i+1} = w / beta_{i+1}
// with C = M (A - tau I) M, M = I or the Jacobi scaling |diag(A) - tau I|^{-1/2}
// (Section 5, the diagonal preconditioner), and the same breakdown rule
// (beta_{i+1} <= 1e3 eps max(|alpha_l|, beta_l)).  A small count is latency
// bound: the column-wave form spends about five launches per step, this form
// one per count.  The workgroup first copies its column's operator into LDS
// (the segment's rows of A with both scalings folded into the values, column
// indices local, and tau d_r^2 per row), so every product reads LDS only.
// Sums are in a fixed order (a wavefront sums all rows of one basis vector,
// lanes then DPP row rotations and row swaps), so results are reproducible.
#include <float.h>

#include "device_common.h"
#include "ecount.h"
#include "ecount_internal.h"

namespace ecnt {

namespace {
constexpr int kSmallThreads = 512;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kLPer = (kFusedMaxK + kSmallWaves - 1) / kSmallWaves;   // basis vectors per wavefront
static_assert(kLPer % 2 == 0, "the dots reduce two basis vectors at a time");
}

// sum over the workgroup, wavefronts in order; every thread gets the value
__device__ __forceinline__ double group_sum(double x, double *red)
{
    x = wave_sum_dpp(x);
    const int wv = threadIdx.x >> 6;
    __syncthreads();   // red is free (its last readers are past this point)
    if ((threadIdx.x & 63) == 0) red[wv] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSmallWaves; ++w) s += red[w];
    return s;
}

// One workgroup per virtual column vc = seg*C + c of the wave (global column
// c_off + c: shift s = (c_off + c) / m, probe j = (c_off + c) % m).  The rows
// of its segment are r0 .. r0 + ns - 1; slot l of its basis (q_{l+1},
// normalized) is basis + (k+1) (C r0 + c ns) + l ns.  Outputs as the
// column-wave form: alpha[(i-1) NC + vc], beta[i NC + vc] (beta_1 = 0),
// nu[vc] = |v|^2, kused[seg ku_ld + ku_off + c].  Dynamic LDS (fused_lds_bytes):
// q, w and tau d_r^2 (nmax doubles each, nmax >= every segment's rows), the
// scaled values (nzmax doubles, nzmax >= every segment's nonzeros), their
// local columns (nzmax ints) and row starts (nmax + 1 ints).
template <typename VT, bool JAC>
__global__ __launch_bounds__(kSmallThreads) void k_lanczos_fused(
    int C, int nseg, int m, int c_off, int k, int S, int64_t n, int nmax, int64_t nzmax,
    const int64_t *__restrict__ seg_row, const double *__restrict__ seg_taus,
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const VT *__restrict__ val,
    const double *__restrict__ jac, const double *__restrict__ V, double *__restrict__ basis,
    double *__restrict__ alpha, double *__restrict__ beta, double *__restrict__ nu,
    int32_t *__restrict__ kused, int ku_ld, int ku_off, double eps)
{
    extern __shared__ double lds[];
    __shared__ double gp[2][kFusedMaxK];   // g_l, p_l
    __shared__ double cf[kFusedMaxK];      // c_l
    __shared__ double red[kSmallWaves];
    double *qs = lds, *ws = lds + nmax, *dt = lds + 2 * (size_t)nmax, *lv = lds + 3 * (size_t)nmax;
    int32_t *lc = reinterpret_cast<int32_t *>(lv + nzmax), *lr = lc + nzmax;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int vc = blockIdx.x;
    const int seg = vc / C, c = vc - seg * C;
    const int cg = c_off + c, s = cg / m, j = cg - s * m;
    const int64_t r0 = seg_row[seg];
    const int ns = (int)(seg_row[seg + 1] - r0);
    const double tau = seg_taus[(size_t)seg * S + s];
    const double *d = JAC ? jac + (size_t)s * n : nullptr;
    double *Q = basis + (size_t)(k + 1) * ((size_t)C * r0 + (size_t)c * ns);
    const size_t NC = (size_t)nseg * C;

    // the column's operator: values d_r a_rj d_j (d = 1 without preconditioner),
    // local columns (an index outside the segment, which a block-diagonal A
    // does not have, gets value 0), row starts, and tau d_r^2
    const int p0 = rp[r0], nz = rp[r0 + ns] - p0;
    for (int e = t; e <= ns; e += kSmallThreads) lr[e] = rp[r0 + e] - p0;
    for (int rl = t; rl < ns; rl += kSmallThreads) {
        const double dr = JAC ? d[r0 + rl] : 1.0;
        dt[rl] = tau * dr * dr;
    }
    __syncthreads();
    for (int rl = t; rl < ns; rl += kSmallThreads) {
        const double dr = JAC ? d[r0 + rl] : 1.0;
        for (int e = lr[rl]; e < lr[rl + 1]; ++e) {
            const int cj = ci[p0 + e];
            const int lj = (int)(cj - r0);
            const bool in = (unsigned)lj < (unsigned)ns;
            lc[e] = in ? lj : 0;
            lv[e] = in ? dr * static_cast<double>(val[p0 + e]) * (JAC ? d[cj] : 1.0) : 0.0;
        }
    }
    (void)nz;
    // q_1 = v / |v|
    double acc = 0.0;
    for (int rl = t; rl < ns; rl += kSmallThreads) {
        const double v = V[(size_t)(r0 + rl) * m + j];
        ws[rl] = v;
        acc += v * v;
    }
    const double vv = group_sum(acc, red);
    if (t == 0) {
        nu[vc] = vv;
        beta[vc] = 0.0;   // beta_1 = 0
    }
    int ku = vv > 0.0 ? k : 0;
    if (ku > 0) {
        const double iv = 1.0 / sqrt(vv);
        for (int rl = t; rl < ns; rl += kSmallThreads) {
            const double q = ws[rl] * iv;
            qs[rl] = q;
            Q[rl] = q;
        }
        __syncthreads();
        double rm = 0.0, bprev = 0.0;
        for (int i = 1; i <= k; ++i) {
            // w = C q_i - beta_i q_{i-1}
            const double *Qi1 = i >= 2 ? Q + (size_t)(i - 2) * ns : Q;
            for (int rl = t; rl < ns; rl += kSmallThreads) {
                double sum = 0.0;
                for (int e = lr[rl]; e < lr[rl + 1]; ++e) sum += lv[e] * qs[lc[e]];
                double y = sum - dt[rl] * qs[rl];
                if (i >= 2) y -= bprev * Qi1[rl];
                ws[rl] = y;
            }
            __syncthreads();
            // g_l and p_l: wavefront wv takes l = wv + j kSmallWaves, each over
            // all rows, and reduces its partial sums two vectors at a time
            // (four independent chains)
            double g[kLPer], pq[kLPer];
#pragma unroll
            for (int j = 0; j < kLPer; ++j) {
                g[j] = 0.0;
                pq[j] = 0.0;
                const int l = wv + j * kSmallWaves;
                if (l < i) {
                    const double *Ql = Q + (size_t)l * ns;
#pragma unroll 4
                    for (int rl = lane; rl < ns; rl += 64) {
                        const double q = Ql[rl];
                        g[j] += q * ws[rl];
                        pq[j] += q * qs[rl];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kLPer; j += 2) {
                const int l = wv + j * kSmallWaves;
                if (l < i) {
                    const double g0 = wave_sum_dpp(g[j]), p0 = wave_sum_dpp(pq[j]);
                    const double g1 = wave_sum_dpp(g[j + 1]), p1 = wave_sum_dpp(pq[j + 1]);
                    if (lane == 0) {
                        gp[0][l] = g0;
                        gp[1][l] = p0;
                        if (l + kSmallWaves < i) {
                            gp[0][l + kSmallWaves] = g1;
                            gp[1][l + kSmallWaves] = p1;
                        }
                    }
                }
            }
            __syncthreads();
            const double al = gp[0][i - 1];
            if (t < i) cf[t] = gp[0][t] - al * (gp[1][t] - (t == i - 1 ? 1.0 : 0.0));
            if (t == 0) alpha[(size_t)(i - 1) * NC + vc] = al;
            __syncthreads();
            // w <- w - sum_l c_l q_l, |w|^2
            double ss = 0.0;
            for (int rl = t; rl < ns; rl += kSmallThreads) {
                double w = ws[rl];
#pragma unroll 4
                for (int l = 0; l < i; ++l) w -= cf[l] * Q[(size_t)l * ns + rl];
                ws[rl] = w;
                ss += w * w;
            }
            const double b = sqrt(group_sum(ss, red));
            if (t == 0) beta[(size_t)i * NC + vc] = b;
            rm = fmax(rm, fabs(al));
            if (i > 1) rm = fmax(rm, bprev);
            if (b <= 1e3 * eps * rm) {   // breakdown: the column stops at k_used = i
                ku = i;
                break;
            }
            if (i == k) break;
            const double ib = 1.0 / b;
            for (int rl = t; rl < ns; rl += kSmallThreads) {
                const double q = ws[rl] * ib;
                qs[rl] = q;
                Q[(size_t)i * ns + rl] = q;
            }
            bprev = b;
            __syncthreads();
        }
    }
    // the steps after the last carry zeros, as in the column-wave form
    for (int i = ku + 1 + t; i <= k; i += kSmallThreads) {
        alpha[(size_t)(i - 1) * NC + vc] = 0.0;
        beta[(size_t)i * NC + vc] = 0.0;
    }
    if (t == 0) kused[(size_t)seg * ku_ld + ku_off + c] = ku;
}

static size_t fused_lds_bytes(int64_t nmax, int64_t nzmax)
{
    return sizeof(double) * 3 * nmax + (sizeof(double) + sizeof(int32_t)) * nzmax +
           sizeof(int32_t) * (nmax + 1);
}

bool fused_applies(const Plan &p, int64_t nnz)
{
    // nnz bounds every segment's nonzeros
    return p.req_fused == 0 && !p.vec_f32 && !p.grad && !p.arnoldi && !p.block &&
           (p.prec_kind == ECNT_PREC_NONE || p.prec_kind == ECNT_PREC_JACOBI) &&
           p.max_rows <= kFusedMaxRows && p.k <= kFusedMaxK &&
           fused_lds_bytes(p.max_rows, nnz) <= kFusedLdsBytes;
}

void launch_lanczos_fused(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                          int64_t nnz, const void *probes, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    const int nmax = (int)p.max_rows;
    const size_t lds = fused_lds_bytes(nmax, nnz);
    const double eps = DBL_EPSILON;
    const bool jac = p.prec_kind == ECNT_PREC_JACOBI;
    auto go = [&](auto vt, auto jc) {
        using VT = decltype(vt);
        constexpr bool J = decltype(jc)::value;
        // more than the default 64 KiB of dynamic LDS (not a stream operation)
        (void)hipFuncSetAttribute((const void *)k_lanczos_fused<VT, J>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes);
        k_lanczos_fused<VT, J><<<NC, kSmallThreads, lds, st>>>(
            p.C, p.nseg, p.m, p.c_off, p.k, p.S, p.n, nmax, nnz, p.seg_row, p.seg_taus, row_ptr, col_idx,
            (const VT *)val, p.jac, (const double *)probes, (double *)p.basis, p.alpha, p.beta, p.nu,
            p.kused, p.Ct, p.c_off, eps);
    };
    if (p.val_f32) {
        if (jac) go(float{}, std::true_type{});
        else go(float{}, std::false_type{});
    } else {
        if (jac) go(double{}, std::true_type{});
        else go(double{}, std::false_type{});
    }
}

}  // namespace ecnt
