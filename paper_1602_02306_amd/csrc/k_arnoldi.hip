// Arnoldi estimator for an unfactored HPD preconditioner T (Section 4,
// Algorithms 3 and 4) on C = T (A - tau I).
//
// The basis, the operator and the row sweeps are those of the Lanczos path
// (unnormalized slots with per-column scales).  Each Arnoldi step
// orthogonalizes w = C q_j against q_1..q_j by two classical Gram-Schmidt
// passes (h = Q^T w, w -= Q h, twice, h summed): in exact arithmetic the
// coefficients of Algorithm 3's modified Gram-Schmidt loop, and orthogonal
// to working precision where one classical pass is not.  The Hessenberg
// column j holds h_{1..j, j} and h_{j+1, j} = |w|.
//
// Quadrature (eq. arnoldi_quad): |v|^2 e_1^T h(H_k) e_1 with h = 1 on the
// open left half-plane, i.e. the spectral projector of H_k on its
// eigenvalues with negative real part, (I - sign(H_k)) / 2.  It is computed
// per column by the Newton iteration for the matrix sign function
// (X <- (mu X + (mu X)^{-1}) / 2, determinant scaling mu = |det X|^{-1/N}
// until the steps are small, then unscaled), which needs no complex
// arithmetic: sign(H_k) is real for real H_k.
#include <float.h>
#include <math.h>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

// h_{l0+l+1, j} (+)= g_l = sig_l * sum_chunks part; cf_l = g_l * sig_l.
__global__ void k_arn_fin(int C, int nseg, int step, int l0, int nb, int k, int pass,
                          const int64_t *__restrict__ seg_chunk, const double *__restrict__ part,
                          const double *__restrict__ sig, const int32_t *__restrict__ active,
                          double *__restrict__ cf, double *__restrict__ H)
{
    const int NC = nseg * C;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * NC) return;
    const int l = idx / NC, vc = idx - l * NC;
    const int seg = vc / C, c = vc - seg * C;
    double s = 0.0;
    for (int64_t ch = seg_chunk[seg]; ch < seg_chunk[seg + 1]; ++ch)
        s += part[((size_t)ch * kPartRows + l) * C + c];
    const double sg = sig[(size_t)(l0 + l) * NC + vc];
    const double g = active[vc] ? s * sg : 0.0;
    cf[(size_t)(l0 + l) * NC + vc] = g * sg;
    double *h = H + ((size_t)(step - 1) * (k + 1) + l0 + l) * NC + vc;
    *h = pass == 1 ? g : *h + g;
}

// h_{j+1,j} = |w|, breakdown test against the largest |h| so far, next scale.
__global__ void k_arn_norm_fin(int C, int nseg, int step, int k, double eps_vec,
                               const int64_t *__restrict__ seg_chunk,
                               const double *__restrict__ part, double *__restrict__ H,
                               double *__restrict__ sig, double *__restrict__ runmax,
                               int32_t *__restrict__ active, int32_t *__restrict__ kused,
                               int ku_ld, int ku_off)
{
    const int vc = blockIdx.x * blockDim.x + threadIdx.x;
    const int NC = nseg * C;
    if (vc >= NC) return;
    const int seg = vc / C, cc = vc - seg * C;
    const int j = step;
    double ss = 0.0;
    for (int64_t ch = seg_chunk[seg]; ch < seg_chunk[seg + 1]; ++ch)
        ss += part[(size_t)ch * kPartRows * C + cc];
    const double b = sqrt(ss);
    double rm = runmax[vc];
    for (int i = 0; i < j; ++i) rm = fmax(rm, fabs(H[((size_t)(j - 1) * (k + 1) + i) * NC + vc]));
    double *hsub = H + ((size_t)(j - 1) * (k + 1) + j) * NC + vc;
    if (active[vc]) {
        if (b <= 1e3 * eps_vec * rm) {   // invariant Krylov space: stop with H_j
            active[vc] = 0;
            kused[(size_t)seg * ku_ld + ku_off + cc] = j;
            sig[(size_t)j * NC + vc] = 0.0;
            *hsub = b;
        } else {
            sig[(size_t)j * NC + vc] = 1.0 / b;
            *hsub = b;
            rm = fmax(rm, b);
        }
    } else {
        sig[(size_t)j * NC + vc] = 0.0;
        *hsub = 0.0;
    }
    runmax[vc] = rm;
}

// One lane per column: s_c = nu_c (1 - sign(H_N)_{11}) / 2, N = k_used.
// Scratch: three N x N matrices per column at sgn[(m*k*k + a*k + b)*NC + vc].
__global__ __launch_bounds__(64) void k_arn_quad(int NC, int C, int ld, int off, int k,
                                                 const double *__restrict__ H,
                                                 const int32_t *__restrict__ kused_all,
                                                 const double *__restrict__ nu,
                                                 double *__restrict__ sgn,
                                                 double *__restrict__ s_all,
                                                 double *__restrict__ minabs_all,
                                                 int32_t *__restrict__ flags)
{
    const int vc = blockIdx.x * blockDim.x + threadIdx.x;
    if (vc >= NC) return;
    const int seg = vc / C;
    const size_t gidx = (size_t)seg * ld + off + (vc - seg * C);
    const int N = kused_all[gidx];
    minabs_all[gidx] = INFINITY;   // eigenvalues are not formed
    if (N < 1) {
        s_all[gidx] = 0.0;
        return;
    }
    const size_t kk = (size_t)k * k;
#define X_(a, b) sgn[((size_t)(a) * k + (b)) * NC + vc]
#define W_(a, b) sgn[(kk + (size_t)(a) * k + (b)) * NC + vc]
#define Y_(a, b) sgn[(2 * kk + (size_t)(a) * k + (b)) * NC + vc]
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            X_(a, b) = (a <= b + 1) ? H[((size_t)b * (k + 1) + a) * NC + vc] : 0.0;
    bool scaled = true, done = false, failed = false;
    for (int it = 0; it < 100 && !done; ++it) {
        // Y = X^{-1} by Gauss-Jordan elimination with partial pivoting on W
        double logdet = 0.0;
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) {
                W_(a, b) = X_(a, b);
                Y_(a, b) = a == b ? 1.0 : 0.0;
            }
        for (int col = 0; col < N && !failed; ++col) {
            int piv = col;
            double pv = fabs(W_(col, col));
            for (int r = col + 1; r < N; ++r)
                if (fabs(W_(r, col)) > pv) {
                    pv = fabs(W_(r, col));
                    piv = r;
                }
            if (!(pv > 0.0) || !isfinite(pv)) {
                failed = true;
                break;
            }
            if (piv != col)
                for (int b = 0; b < N; ++b) {
                    double t = W_(col, b);
                    W_(col, b) = W_(piv, b);
                    W_(piv, b) = t;
                    t = Y_(col, b);
                    Y_(col, b) = Y_(piv, b);
                    Y_(piv, b) = t;
                }
            const double d = W_(col, col);
            logdet += log(fabs(d));
            const double inv = 1.0 / d;
            for (int b = 0; b < N; ++b) {
                W_(col, b) *= inv;
                Y_(col, b) *= inv;
            }
            for (int r = 0; r < N; ++r) {
                if (r == col) continue;
                const double f = W_(r, col);
                if (f == 0.0) continue;
                for (int b = 0; b < N; ++b) {
                    W_(r, b) -= f * W_(col, b);
                    Y_(r, b) -= f * Y_(col, b);
                }
            }
        }
        if (failed) break;
        const double mu = scaled ? exp(-logdet / N) : 1.0;
        double num = 0.0, den = 0.0;
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) {
                const double xn = 0.5 * (mu * X_(a, b) + Y_(a, b) / mu);
                const double dd = xn - X_(a, b);
                num += dd * dd;
                den += xn * xn;
                X_(a, b) = xn;
            }
        const double rel = sqrt(num / den);
        if (rel < 1e-2) scaled = false;
        if (!scaled && rel < 1e-13) done = true;
    }
    if (!done || failed) {
        atomicOr(&flags[1], 1);
        s_all[gidx] = NAN;
        return;
    }
    s_all[gidx] = nu[vc] * 0.5 * (1.0 - X_(0, 0));
#undef X_
#undef W_
#undef Y_
}

void launch_arn_fin(const Plan &p, int step, int l0, int nb, int pass, hipStream_t st)
{
    const int tot = nb * p.nseg * p.C;
    k_arn_fin<<<(tot + 255) / 256, 256, 0, st>>>(p.C, p.nseg, step, l0, nb, p.k, pass, p.seg_chunk,
                                                 p.part, p.sig, p.active, p.cf, p.H);
}

void launch_arn_norm_fin(const Plan &p, int step, hipStream_t st)
{
    const double eps = p.vec_f32 ? (double)FLT_EPSILON : DBL_EPSILON;
    const int NC = p.nseg * p.C;
    k_arn_norm_fin<<<(NC + 255) / 256, 256, 0, st>>>(p.C, p.nseg, step, p.k, eps, p.seg_chunk,
                                                     p.part, p.H, p.sig, p.runmax, p.active,
                                                     p.kused, p.Ct, p.c_off);
}

void launch_arn_quad(const Plan &p, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    k_arn_quad<<<(NC + 63) / 64, 64, 0, st>>>(NC, p.C, p.Ct, p.c_off, p.k, p.H, p.kused, p.nu,
                                              p.sgn, p.s_out, p.minabs, p.flags);
}

}  // namespace ecnt
