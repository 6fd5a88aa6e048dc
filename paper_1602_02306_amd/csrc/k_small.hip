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
// one per count.  Sums are in a fixed order (a wavefront sums all rows of one
// basis vector, lanes then the butterfly), so results are reproducible.
#include <float.h>

#include "device_common.h"
#include "ecount.h"
#include "ecount_internal.h"

namespace ecnt {

namespace {
constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / 64;
}

// sum over the wavefront; every lane gets the same value (each butterfly
// stage adds two equal partial sums in either order)
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// sum over the workgroup, wavefronts in order; every thread gets the value
__device__ __forceinline__ double group_sum(double x, double *red)
{
    x = wave_sum(x);
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
// nu[vc] = |v|^2, kused[seg ku_ld + ku_off + c].  Dynamic LDS: q and w,
// 2 * nmax doubles (nmax >= every segment's rows).
template <typename VT, bool JAC>
__global__ __launch_bounds__(kSmallThreads) void k_lanczos_fused(
    int C, int nseg, int m, int c_off, int k, int S, int64_t n, int nmax,
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
    double *qs = lds, *ws = lds + nmax;
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
            // w = C q_i - beta_i q_{i-1} (a column index outside the segment,
            // which a block-diagonal A does not have, contributes 0)
            const double *Qi1 = i >= 2 ? Q + (size_t)(i - 2) * ns : Q;
            for (int rl = t; rl < ns; rl += kSmallThreads) {
                const int64_t r = r0 + rl;
                double sum = 0.0;
                for (int p = rp[r]; p < rp[r + 1]; ++p) {
                    const int cj = ci[p];
                    const int lj = (int)(cj - r0);
                    const bool in = (unsigned)lj < (unsigned)ns;
                    const double x = qs[in ? lj : 0];
                    sum += in ? static_cast<double>(val[p]) * (JAC ? d[cj] : 1.0) * x : 0.0;
                }
                const double dr = JAC ? d[r] : 1.0;
                double y = dr * (sum - tau * dr * qs[rl]);
                if (i >= 2) y -= bprev * Qi1[rl];
                ws[rl] = y;
            }
            __syncthreads();
            // g_l and p_l: wavefront wv takes l = wv + 4u, all rows, in one pass
            // (a lane keeps the sums of all its l, so their loads overlap)
            {
                constexpr int U = kFusedMaxK / kSmallWaves;
                const int nu_ = (i - wv + kSmallWaves - 1) / kSmallWaves;   // l's of this wavefront
                double g[U], pq[U];
#pragma unroll
                for (int u = 0; u < U; ++u) g[u] = pq[u] = 0.0;
                for (int rl = lane; rl < ns; rl += 64) {
                    const double wr = ws[rl], qr = qs[rl];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (u < nu_) {
                            const double q = Q[(size_t)(wv + kSmallWaves * u) * ns + rl];
                            g[u] += q * wr;
                            pq[u] += q * qr;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (u < nu_) {
                        const double gs = wave_sum(g[u]), ps = wave_sum(pq[u]);
                        if (lane == 0) {
                            gp[0][wv + kSmallWaves * u] = gs;
                            gp[1][wv + kSmallWaves * u] = ps;
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

bool fused_applies(const Plan &p)
{
    return p.req_fused == 0 && !p.vec_f32 && !p.grad && !p.arnoldi && !p.block &&
           (p.prec_kind == ECNT_PREC_NONE || p.prec_kind == ECNT_PREC_JACOBI) &&
           p.max_rows <= kFusedMaxRows && p.k <= kFusedMaxK;
}

void launch_lanczos_fused(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                          const void *probes, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    const int nmax = (int)p.max_rows;
    const size_t lds = sizeof(double) * 2 * (size_t)nmax;
    const double eps = DBL_EPSILON;
    const bool jac = p.prec_kind == ECNT_PREC_JACOBI;
    auto go = [&](auto vt, auto jc) {
        using VT = decltype(vt);
        constexpr bool J = decltype(jc)::value;
        k_lanczos_fused<VT, J><<<NC, kSmallThreads, lds, st>>>(
            p.C, p.nseg, p.m, p.c_off, p.k, p.S, p.n, nmax, p.seg_row, p.seg_taus, row_ptr, col_idx,
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
