// Reverse-mode derivative of the erf-smoothed estimator.
//
// Forward, per column (probe j at shift tau), as computed by the forward
// kernels (q_l = sig_{l-1} * slot_{l-1}; Algorithm 1 with alpha_i taken first
// and one classical Gram-Schmidt pass, fused into one update):
//   y_i = C q_i,  w_i = y_i - beta_i q_{i-1},  g = Q_i^T w_i,  alpha_i = g[i],
//   p = Q_i^T q_i,  c = g - alpha_i (p - e_i),  r_i = w_i - Q_i c,
//   beta_{i+1} = |r_i|,  q_{i+1} = r_i / beta_{i+1},
//   s = nu * e_1^T S_w(J_k) e_1,  S_w(x) = erfc(x / w) / 2,
//   C = M (A - tau I) M,  A = L + diag(V),  M independent of V and tau.
// Reverse, for i = k..1 (bars are adjoints; all sums over l run to i):
//   rbar    = qbar_{i+1} / beta_{i+1} + betabar_{i+1} q_{i+1}
//             (betabar_{i+1} first decreased by qbar_{i+1}^T q_{i+1} / beta_{i+1})
//   cbar_l  = -q_l^T rbar,   alphabar = alphabar_J - (p - e_i)^T cbar
//   gbar    = cbar + alphabar e_i,   u = Q_i cbar
//   wbar    = rbar + Q_i gbar
//   qbar_l += gbar_l w_i - c_l rbar - alpha_i cbar_l q_i
//   qbar_i += alphabar w_i - alpha_i u          (through p = Q^T Q e_i and alpha_i = q_i^T w_i)
//   qbar_{i-1} -= beta_i wbar,  betabar_i -= wbar^T q_{i-1},  ybar = wbar,
//   qbar_i += C ybar,  Vbar += (M ybar) .* (M q_i),  taubar -= (M ybar)^T (M q_i)
// with alphabar_J, betabar of the tridiagonal step from Daleckii-Krein:
//   Jbar = sbar * nu * Z (S[1] o z z^T) Z^T,  z = first row of Z.
// M q_i is kept from the forward (one block vector per step); c and p - e_i
// of every step too (k x k per column each).
#include <float.h>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

__device__ __forceinline__ double smooth_step(double th, double w) { return 0.5 * erfc(th / w); }
__device__ __forceinline__ double smooth_step_d(double th, double w)
{
    return -exp(-(th / w) * (th / w)) / (w * 1.7724538509055160273);   // sqrt(pi)
}

// ---- tridiagonal adjoint: full eigendecomposition of J_ku, then alphabar, betabar ----
// Z (k x k per column) lives in global scratch at Z[(a*k + b)*C + c].
__global__ __launch_bounds__(64) void k_tridiag_bwd(int C, int k, int m, double smooth_w,
                                                    double g_out,
                                                    const double *__restrict__ alpha,
                                                    const double *__restrict__ beta,
                                                    const int32_t *__restrict__ kused,
                                                    const double *__restrict__ nu,
                                                    double *__restrict__ Zg, double *__restrict__ th,
                                                    double *__restrict__ sv,
                                                    double *__restrict__ abar,
                                                    double *__restrict__ bbar,
                                                    int32_t *__restrict__ flags)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
#define Z_(a, b) Zg[((size_t)(a) * k + (b)) * C + c]
#define A_(i) th[(size_t)(i) * C + c]
    // offdiagonal kept in bbar during the iteration, overwritten at the end
#define B_(i) bbar[(size_t)(i) * C + c]
    const int N = kused[c];
    for (int i = 0; i <= k; ++i) B_(i) = 0.0;
    for (int i = 0; i < k; ++i) abar[(size_t)i * C + c] = 0.0;
    if (N < 1) return;
    for (int i = 0; i < N; ++i) {
        A_(i) = alpha[(size_t)i * C + c];
        if (i + 1 < N) B_(i) = beta[(size_t)(i + 1) * C + c];
        for (int j = 0; j < N; ++j) Z_(i, j) = i == j ? 1.0 : 0.0;
    }
    int hi = N - 1, iter = 0;
    bool failed = false;
    while (hi > 0) {
        if (fabs(B_(hi - 1)) <= DBL_EPSILON * (fabs(A_(hi - 1)) + fabs(A_(hi))) ||
            fabs(B_(hi - 1)) < DBL_MIN) {
            B_(hi - 1) = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0) {
            const double bl = fabs(B_(lo - 1));
            if (bl <= DBL_EPSILON * (fabs(A_(lo - 1)) + fabs(A_(lo))) || bl < DBL_MIN) {
                B_(lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (++iter > 60 * N) {
            failed = true;
            break;
        }
        const double bb = B_(hi - 1);
        const double d = 0.5 * (A_(hi - 1) - A_(hi));
        const double den = d + copysign(hypot(d, bb), d);
        const double mu = A_(hi) - (den != 0.0 ? bb * bb / den : 0.0);
        double x = A_(lo) - mu, y = B_(lo);
        for (int kk = lo; kk < hi; ++kk) {
            const double r = hypot(x, y);
            double cs = 1.0, sn = 0.0;
            if (r > 0.0) {
                cs = x / r;
                sn = y / r;
            }
            if (kk > lo) B_(kk - 1) = r;
            const double ak = A_(kk), ak1 = A_(kk + 1), bk = B_(kk);
            A_(kk) = cs * cs * ak + 2.0 * cs * sn * bk + sn * sn * ak1;
            A_(kk + 1) = sn * sn * ak - 2.0 * cs * sn * bk + cs * cs * ak1;
            const double nbk = cs * sn * (ak1 - ak) + (cs * cs - sn * sn) * bk;
            B_(kk) = nbk;
            if (kk + 1 < hi) {
                const double bk1 = B_(kk + 1);
                y = sn * bk1;
                B_(kk + 1) = cs * bk1;
                x = nbk;
            }
            for (int rr = 0; rr < N; ++rr) {
                const double z0 = Z_(rr, kk), z1 = Z_(rr, kk + 1);
                Z_(rr, kk) = cs * z0 + sn * z1;
                Z_(rr, kk + 1) = -sn * z0 + cs * z1;
            }
        }
    }
    if (failed) atomicOr(&flags[1], 1);
    // seed: d estimate / d s_c = +-1/m (eta columns +, xi columns -)
    const double sbar = g_out * ((c >= m) ? 1.0 : -1.0) / (double)m;
    const double scale = sbar * nu[c];
    for (int a = 0; a < N; ++a) sv[(size_t)a * C + c] = smooth_step(A_(a), smooth_w);
    // u^(l)_a = sum_b F_ab Z[l][b],  F_ab = S[1](th_a, th_b) z_a z_b;  then
    // abar_l = scale * Z[l] . u^(l),  bbar_{l+1} = 2 * scale * Z[l] . u^(l+1)
    for (int i = 0; i <= k; ++i) B_(i) = 0.0;
    for (int l = N - 1; l >= 0; --l) {
        double diag = 0.0, off = 0.0;
        for (int a = 0; a < N; ++a) {
            const double ta = A_(a), za = Z_(0, a);
            double ua = 0.0, uan = 0.0;
            for (int b = 0; b < N; ++b) {
                const double tb = A_(b);
                double D;
                if (fabs(ta - tb) < 1e-8 * (1.0 + fabs(ta)))
                    D = smooth_step_d(0.5 * (ta + tb), smooth_w);
                else
                    D = (sv[(size_t)a * C + c] - sv[(size_t)b * C + c]) / (ta - tb);
                const double F = D * za * Z_(0, b);
                ua += F * Z_(l, b);
                if (l + 1 < N) uan += F * Z_(l + 1, b);
            }
            diag += Z_(l, a) * ua;
            off += Z_(l, a) * uan;
        }
        abar[(size_t)l * C + c] = scale * diag;
        if (l + 1 < N) B_(l + 1) = 2.0 * scale * off;   // betabar_{l+2} (array index l+1)
    }
#undef Z_
#undef A_
#undef B_
}

// ---- backward dots: raw[s] = slot_s . qbar_{i+1} (s = 0..i), raw[i+1+s] = slot_s . slot_i (s < i)
template <int NS>
__global__ __launch_bounds__(64) void k_bdots(int64_t n, int C, int nct, int64_t rpc,
                                              const double *__restrict__ basis,
                                              const double *__restrict__ qbar, size_t ss, int i,
                                              double *__restrict__ part)
{
    // NS = i + 1 slots (0..i)
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int c = ct * 64 + (int)threadIdx.x;
    if (c >= C) return;
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    double accD[NS], accE[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) accD[s] = accE[s] = 0.0;
    const double *QB = qbar + (size_t)i * ss;   // qbar_{i+1}
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c;
        double q[NS];
        const double qb = QB[e];
#pragma unroll
        for (int s = 0; s < NS; ++s) q[s] = basis[(size_t)s * ss + e];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            accD[s] += q[s] * qb;
            accE[s] += q[s] * q[NS - 1];
        }
    }
    double *P = part + (size_t)chunk * 64 * C + c;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        P[(size_t)s * C] = accD[s];
        if (s + 1 < NS) P[(size_t)(NS + s) * C] = accE[s];
    }
}

// sums[row][c] = sum over chunks of part[chunk][row][c], one thread per (row, c)
__global__ void k_rowsum(int C, int nchunk, int nrows, const double *__restrict__ part,
                         double *__restrict__ sums)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows * C) return;
    const int row = idx / C, c = idx % C;
    double t = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) t += part[((size_t)ch * 64 + row) * C + c];
    sums[idx] = t;
}

// Per column: finish betabar_{i+1}, form the coefficients of rbar and gbar.
// coef layout (each [32][C]): cA = gbar*sig (wbar), cW = c*sig (w), cG = gbar, cR = c;
// scal[0][c] = a (qbar_{i+1} weight in rbar), scal[1][c] = b*sig_i (slot_i weight),
// scal[2][c] = -alpha_i sig_{i-1} (lambda: slot_{i-1} weight folded into w),
// scal[3][c] = alphabar sig_{i-1} (mu: slot_{i-1} weight of the alphabar term of wbar),
// scal[4][c] = -alpha_i.
__global__ void k_bdots_fin(int C, int k, int nchunk, int i, int have_dots,
                            const double *__restrict__ part, const double *__restrict__ sig,
                            const double *__restrict__ beta, const double *__restrict__ alpha,
                            const double *__restrict__ gall, const double *__restrict__ pall,
                            const double *__restrict__ abar, double *__restrict__ bbar,
                            const int32_t *__restrict__ kused, double *__restrict__ cA,
                            double *__restrict__ cW, double *__restrict__ cG,
                            double *__restrict__ cR, double *__restrict__ scal)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int ku = kused[c];
    double a = 0.0, b = 0.0;
    const double sgi = sig[(size_t)i * C + c];
    // part holds the chunk-summed dots here (k_rowsum)
    auto raw = [&](int row) { return part[(size_t)row * C + c]; };
    (void)nchunk;
    if (have_dots && i < ku) {
        const double bi1 = beta[(size_t)i * C + c];                  // beta_{i+1}
        const double cc = sgi * raw(i);                              // qbar_{i+1}^T q_{i+1}
        double bb = bbar[(size_t)i * C + c] - cc / bi1;              // betabar_{i+1}
        bbar[(size_t)i * C + c] = bb;
        a = 1.0 / bi1;
        b = bb;
    }
    auto cbar = [&](int s) {   // -q_s^T rbar
        if (a == 0.0 && b == 0.0) return 0.0;
        const double sg = sig[(size_t)s * C + c];
        return -(a * sg * raw(s) + b * sg * sgi * raw(i + 1 + s));
    };
    double ab = i <= ku ? abar[(size_t)(i - 1) * C + c] : 0.0;
    for (int s = 0; s < i; ++s) ab -= pall[((size_t)(i - 1) * k + s) * C + c] * cbar(s);
    for (int s = 0; s < i; ++s) {
        const double sg = sig[(size_t)s * C + c];
        double gb = cbar(s);
        if (s == i - 1) gb += ab;
        const double cl = gall[((size_t)(i - 1) * k + s) * C + c];
        cA[(size_t)s * C + c] = gb * sg;
        cW[(size_t)s * C + c] = cl * sg;
        cG[(size_t)s * C + c] = gb;
        cR[(size_t)s * C + c] = cl;
    }
    const double al = alpha[(size_t)(i - 1) * C + c];
    const double sgq = sig[(size_t)(i - 1) * C + c];
    scal[c] = a;
    scal[(size_t)C + c] = b * sgi;
    scal[(size_t)2 * C + c] = -al * sgq;
    scal[(size_t)3 * C + c] = ab * sgq;
    scal[(size_t)4 * C + c] = -al;
}

// One sweep per row: rbar, wbar (= ybar) and w of step i, the partial
// wbar . slot_{i-2}, then qbar_s += cG_s (w - alpha_i q_i) - cR_s rbar (s < i),
// qbar_i += -alpha_i (u - alphabar q_i) (u = wbar - rbar - alphabar q_i) and
// qbar_{i-1} -= beta_i wbar.  rbar and w never leave registers.  A workgroup
// is four wavefronts on four row chunks of one column tile; they share the
// 4*NB coefficients of their columns through LDS.
template <int NB, bool HASQ, bool FIRST>
__global__ __launch_bounds__(256) void k_bupdate(int64_t n, int C, int nct, int64_t rpc,
                                                 int64_t nchunk, const double *__restrict__ basis,
                                                 double *__restrict__ qbar, size_t ss, int i,
                                                 const double *__restrict__ coef,
                                                 const double *__restrict__ scal,
                                                 const double *__restrict__ beta,
                                                 double *__restrict__ ybar,
                                                 double *__restrict__ part)
{
    // NB = i (slots 0..i-1), plus slot i.  coef: cA, cW, cG, cR, each [32][C]
    __shared__ double cf[4][NB][64];
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t grp = L / nct;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = ct * 64 + lane;
    const bool colok = c < C;
    for (int idx = wv; idx < 4 * NB; idx += 4) {
        const int kind = idx / NB, s = idx - kind * NB;
        cf[kind][s][lane] = colok ? coef[((size_t)kind * 32 + s) * C + c] : 0.0;
    }
    __syncthreads();
    const int64_t chunk = grp * 4 + wv;
    if (!colok || chunk >= nchunk) return;
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    const double a = scal[c], bq = scal[(size_t)C + c];
    const double lam = scal[(size_t)2 * C + c], mu = scal[(size_t)3 * C + c];
    const double nal = scal[(size_t)4 * C + c];
    const double bi = i >= 2 ? beta[(size_t)(i - 1) * C + c] : 0.0;   // beta_i
    const double *QB = qbar + (size_t)i * ss;
    const double *SI = basis + (size_t)i * ss;
    const int sm = i >= 2 ? i - 2 : 0;
    double dotm = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c;
        double q[NB];
        const double si = SI[e];
        const double qb = HASQ ? QB[e] : 0.0;
#pragma unroll
        for (int s = 0; s < NB; ++s) q[s] = __builtin_nontemporal_load(basis + (size_t)s * ss + e);
        __builtin_amdgcn_sched_barrier(0);
        const double rb = a * qb + bq * si;
        double wb = rb, w = si;
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            wb += cf[0][s][lane] * q[s];
            w += cf[1][s][lane] * q[s];
        }
        ybar[e] = wb;
        double qsm = 0.0;   // q[sm] by selects: a runtime index would move q to scratch
#pragma unroll
        for (int s = 0; s < NB; ++s) qsm = s == sm ? q[s] : qsm;
        dotm += wb * qsm;
        const double qi = q[NB - 1];                          // slot i-1 (q_i unnormalized)
        const double wq = w + lam * qi;                       // w - alpha_i q_i
        const double xq = nal * (wb - rb - 2.0 * mu * qi);    // -alpha_i (u - alphabar q_i)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < NB; ++s) q[s] = FIRST ? 0.0 : qbar[(size_t)s * ss + e];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            double v = q[s] + cf[2][s][lane] * wq - cf[3][s][lane] * rb;
            if (s == i - 2) v -= bi * wb;
            if (s == NB - 1) v += xq;
            qbar[(size_t)s * ss + e] = v;
        }
    }
    part[(size_t)chunk * 64 * C + c] = dotm;
}

// betabar_i -= sig_{i-2} * sum_chunks (wbar . slot_{i-2})
__global__ void k_bnorm_fin(int C, int nchunk, int i, const double *__restrict__ part,
                            const double *__restrict__ sig, double *__restrict__ bbar)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C || i < 2) return;
    double t = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) t += part[(size_t)ch * 64 * C + c];
    bbar[(size_t)(i - 1) * C + c] -= sig[(size_t)(i - 2) * C + c] * t;
}

// Vbar and taubar contributions of step i: tb = M ybar_i, tq = M q_i.
// vpart[ct][r] (+)= sum over the tile's columns of tb*tq (fixed-order lane
// reduction); part[chunk][0][c] = sum over the chunk's rows of tb*tq.
__global__ __launch_bounds__(64) void k_vgrad(int64_t n, int C, int nct, int64_t rpc,
                                              const double *__restrict__ tb,
                                              const double *__restrict__ tq, int first,
                                              double *__restrict__ vpart,
                                              double *__restrict__ part)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int lane = threadIdx.x;
    const int c = ct * 64 + lane;
    const bool ok = c < C;
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    double tacc = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c;
        double p = ok ? tb[e] * tq[e] : 0.0;
        tacc += p;
        // fixed-order butterfly over the 64 lanes
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, 64);
        if (lane == 0) {
            double *dst = vpart + (size_t)ct * n + r;
            *dst = first ? p : *dst + p;
        }
    }
    if (ok) part[(size_t)chunk * 64 * C + c] = tacc;
}

__global__ void k_vgrad_fin(int C, int nchunk, const double *__restrict__ part,
                            double *__restrict__ taubar, int first)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double t = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) t += part[(size_t)ch * 64 * C + c];
    taubar[c] = (first ? 0.0 : taubar[c]) - t;
}

// dV[r] = sum_ct vpart[ct][r]
__global__ void k_grad_v(int64_t n, int nct, const double *__restrict__ vpart, double *__restrict__ dV)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double t = 0.0;
    for (int ct = 0; ct < nct; ++ct) t += vpart[(size_t)ct * n + r];
    dV[r] = t;
}

// out[0] = sum of taubar over the xi columns, out[1] over the eta columns.
__global__ __launch_bounds__(256) void k_grad_tau(int m, const double *__restrict__ taubar,
                                                  double *__restrict__ out)
{
    __shared__ double sh[256];
    for (int s = 0; s < 2; ++s) {
        double acc = 0.0;
        for (int j = threadIdx.x; j < m; j += 256) acc += taubar[(size_t)s * m + j];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[s] = sh[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers

static inline unsigned red_blocks(const Plan &p)
{
    const int nct = (p.C + 63) / 64;
    return (unsigned)((int64_t)p.nchunk * nct);
}

void launch_tridiag_bwd(const Plan &p, double g_out, hipStream_t st)
{
    k_tridiag_bwd<<<(p.C + 63) / 64, 64, 0, st>>>(p.C, p.k, p.m, p.smooth_w, g_out, p.alpha, p.beta,
                                                   p.kused, p.nu, p.g_Z, p.g_theta, p.g_sval, p.g_abar,
                                                   p.g_bbar, p.flags);
}

#define ECNT_NS_CASES(F)                                                                        \
    F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16)   \
    F(17) F(18) F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30)     \
    F(31) F(32)

void launch_bdots(const Plan &p, int i, hipStream_t st)
{
    const int nct = (p.C + 63) / 64;
    const size_t ss = slot_elems(p);
    switch (i + 1) {
#define ECNT_CASE(N)                                                                             \
    case N:                                                                                      \
        k_bdots<N><<<red_blocks(p), 64, 0, st>>>(p.n, p.C, nct, p.rpc, (const double *)p.basis, \
                                                 p.g_qbar, ss, i, p.part);                       \
        break;
        ECNT_NS_CASES(ECNT_CASE)
#undef ECNT_CASE
    default:
        break;
    }
}

void launch_bdots_fin(const Plan &p, int i, bool have_dots, hipStream_t st)
{
    const size_t C = p.C;
    if (have_dots) {
        const int rows = 2 * i + 1;
        k_rowsum<<<(rows * p.C + 255) / 256, 256, 0, st>>>(p.C, p.nchunk, rows, p.part, p.g_sums);
    }
    k_bdots_fin<<<(p.C + 255) / 256, 256, 0, st>>>(p.C, p.k, p.nchunk, i, have_dots ? 1 : 0,
                                                   p.g_sums, p.sig, p.beta, p.alpha, p.g_gall,
                                                   p.g_pall, p.g_abar,
                                                   p.g_bbar, p.kused, p.g_coef, p.g_coef + 32 * C,
                                                   p.g_coef + 64 * C, p.g_coef + 96 * C, p.g_scal);
}

void launch_bupdate(const Plan &p, int i, bool first, hipStream_t st)
{
    const int nct = (p.C + 63) / 64;
    const size_t ss = slot_elems(p);
    const size_t C = p.C;
    const bool hasq = i < p.k;
    (void)C;
    const dim3 grid((unsigned)(((int64_t)p.nchunk + 3) / 4 * nct));
    switch (i) {
#define ECNT_LAUNCH(N, HQ, FI)                                                                    \
    k_bupdate<N, HQ, FI><<<grid, 256, 0, st>>>(p.n, p.C, nct, p.rpc, (int64_t)p.nchunk,           \
                                               (const double *)p.basis, p.g_qbar, ss, i, p.g_coef, \
                                               p.g_scal, p.beta, p.g_ybar, p.part)
#define ECNT_CASE(N)                                                                              \
    case N:                                                                                       \
        if (hasq) {                                                                               \
            if (first) ECNT_LAUNCH(N, true, true);                                                \
            else ECNT_LAUNCH(N, true, false);                                                     \
        } else {                                                                                  \
            if (first) ECNT_LAUNCH(N, false, true);                                               \
            else ECNT_LAUNCH(N, false, false);                                                    \
        }                                                                                         \
        break;
        ECNT_NS_CASES(ECNT_CASE)
#undef ECNT_CASE
#undef ECNT_LAUNCH
    default:
        break;
    }
}

void launch_bnorm_fin(const Plan &p, int i, hipStream_t st)
{
    k_bnorm_fin<<<(p.C + 255) / 256, 256, 0, st>>>(p.C, p.nchunk, i, p.part, p.sig, p.g_bbar);
}

void launch_vgrad(const Plan &p, const double *tq, bool first, hipStream_t st)
{
    const int nct = (p.C + 63) / 64;
    k_vgrad<<<red_blocks(p), 64, 0, st>>>(p.n, p.C, nct, p.rpc, p.g_tbar, tq, first ? 1 : 0,
                                          p.g_vpart, p.part);
    k_vgrad_fin<<<(p.C + 255) / 256, 256, 0, st>>>(p.C, p.nchunk, p.part, p.g_taubar, first ? 1 : 0);
}

void launch_grad_out(const Plan &p, double *dV, hipStream_t st)
{
    const int nct = (p.C + 63) / 64;
    k_grad_v<<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(p.n, nct, p.g_vpart, dV);
    k_grad_tau<<<1, 256, 0, st>>>(p.m, p.g_taubar, p.result + 4 * kMaxShifts);
}

}  // namespace ecnt
