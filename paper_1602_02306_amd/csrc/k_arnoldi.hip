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
// arithmetic: sign(H_k) is real for real H_k.  One wavefront per column, the
// matrices in LDS.
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
    const int l = blockIdx.y;
    const int vc = blockIdx.x * 64 + (threadIdx.x & 63);
    const bool valid = vc < NC;
    const int seg = valid ? vc / C : 0, c = valid ? vc - seg * C : 0;
    const double s = block_chunk_sum(part, kPartRows, C, l, c, seg_chunk[seg], seg_chunk[seg + 1], valid);
    if (!valid || threadIdx.x >= 64) return;
    (void)nb;
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
    const int vc = blockIdx.x * 64 + (threadIdx.x & 63);
    const int NC = nseg * C;
    const bool valid = vc < NC;
    const int seg = valid ? vc / C : 0, cc = valid ? vc - seg * C : 0;
    const int j = step;
    const double ss = block_chunk_sum(part, kPartRows, C, 0, cc, seg_chunk[seg], seg_chunk[seg + 1], valid);
    if (!valid || threadIdx.x >= 64) return;
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

// One wavefront per column: s_c = nu_c (1 - sign(H_N)_{11}) / 2, N = k_used.
// X, W (work copy) and Y = X^{-1} live in LDS, lane a holding row a; each
// Gauss-Jordan pivot is found by a fixed-order wave reduction (ties to the
// lower row), row swaps and scalings go column-parallel, eliminations
// row-parallel.
template <int KMAX>
__global__ __launch_bounds__(64) void k_arn_quad(int C, int ld, int off, int k,
                                                 const double *__restrict__ H,
                                                 const int32_t *__restrict__ kused_all,
                                                 const double *__restrict__ nu,
                                                 double *__restrict__ s_all,
                                                 double *__restrict__ minabs_all,
                                                 int32_t *__restrict__ flags)
{
    constexpr int LDK = KMAX + 1;
    __shared__ double X[KMAX * LDK], W[KMAX * LDK], Y[KMAX * LDK];
    const int NC = gridDim.x;
    const int vc = blockIdx.x;
    const int lane = threadIdx.x;
    const int seg = vc / C;
    const size_t gidx = (size_t)seg * ld + off + (vc - seg * C);
    const int N = kused_all[gidx];
    if (N < 1) {   // uniform over the block
        if (lane == 0) {
            s_all[gidx] = 0.0;
            minabs_all[gidx] = INFINITY;
        }
        return;
    }
    for (int e = lane; e < N * N; e += 64) {
        const int a = e / N, b = e % N;
        X[a * LDK + b] = (a <= b + 1) ? H[((size_t)b * (k + 1) + a) * NC + vc] : 0.0;
    }
    __syncthreads();
    bool scaled = true, done = false, failed = false;
    for (int it = 0; it < 100 && !done && !failed; ++it) {
        for (int e = lane; e < N * N; e += 64) {
            const int a = e / N, b = e % N;
            W[a * LDK + b] = X[a * LDK + b];
            Y[a * LDK + b] = a == b ? 1.0 : 0.0;
        }
        __syncthreads();
        double logdet = 0.0;
        for (int col = 0; col < N; ++col) {
            // pivot: largest |W[a][col]|, a >= col, lowest row on ties
            double pv = (lane >= col && lane < N) ? fabs(W[lane * LDK + col]) : -1.0;
            int pr = lane;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double qv = __shfl_xor(pv, o, 64);
                const int qr = __shfl_xor(pr, o, 64);
                if (qv > pv || (qv == pv && qr < pr)) {
                    pv = qv;
                    pr = qr;
                }
            }
            if (!(pv > 0.0) || !isfinite(pv)) {   // uniform: every lane holds the same pair
                failed = true;
                break;
            }
            if (pr != col && lane < N) {   // column-parallel row swap
                double t = W[col * LDK + lane];
                W[col * LDK + lane] = W[pr * LDK + lane];
                W[pr * LDK + lane] = t;
                t = Y[col * LDK + lane];
                Y[col * LDK + lane] = Y[pr * LDK + lane];
                Y[pr * LDK + lane] = t;
            }
            __syncthreads();
            const double d = W[col * LDK + col];
            logdet += log(fabs(d));
            __syncthreads();
            if (lane < N) {
                const double inv = 1.0 / d;
                W[col * LDK + lane] *= inv;
                Y[col * LDK + lane] *= inv;
            }
            __syncthreads();
            if (lane < N && lane != col) {   // row-parallel elimination
                const double f = W[lane * LDK + col];
                if (f != 0.0)
                    for (int b = 0; b < N; ++b) {
                        W[lane * LDK + b] -= f * W[col * LDK + b];
                        Y[lane * LDK + b] -= f * Y[col * LDK + b];
                    }
            }
            __syncthreads();
        }
        if (failed) break;
        const double mu = scaled ? exp(-logdet / N) : 1.0;
        double num = 0.0, den = 0.0;
        if (lane < N)
            for (int b = 0; b < N; ++b) {
                const double xo = X[lane * LDK + b];
                const double xn = 0.5 * (mu * xo + Y[lane * LDK + b] / mu);
                num += (xn - xo) * (xn - xo);
                den += xn * xn;
                X[lane * LDK + b] = xn;
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            num += __shfl_xor(num, o, 64);
            den += __shfl_xor(den, o, 64);
        }
        // the lanes' sums may differ in the last bit: take lane 0's, so that
        // every lane takes the same branch below
        num = __shfl(num, 0, 64);
        den = __shfl(den, 0, 64);
        __syncthreads();
        const double rel = sqrt(num / den);
        if (rel < 1e-2) scaled = false;
        if (!scaled && rel < 1e-13) done = true;
    }
    if (lane == 0) {
        minabs_all[gidx] = INFINITY;   // the eigenvalues of H_N are not formed
        if (!done || failed) {
            atomicOr(&flags[1], 1);
            s_all[gidx] = NAN;
        } else {
            s_all[gidx] = nu[vc] * 0.5 * (1.0 - X[0]);
        }
    }
}

void launch_arn_fin(const Plan &p, int step, int l0, int nb, int pass, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    k_arn_fin<<<dim3((NC + 63) / 64, nb), 64 * kFinWaves, 0, st>>>(p.C, p.nseg, step, l0, nb, p.k, pass, p.seg_chunk,
                                                 p.part, p.sig, p.active, p.cf, p.H);
}

void launch_arn_norm_fin(const Plan &p, int step, hipStream_t st)
{
    const double eps = p.vec_f32 ? (double)FLT_EPSILON : DBL_EPSILON;
    const int NC = p.nseg * p.C;
    k_arn_norm_fin<<<(NC + 63) / 64, 64 * kFinWaves, 0, st>>>(p.C, p.nseg, step, p.k, eps, p.seg_chunk,
                                                     p.part, p.H, p.sig, p.runmax, p.active,
                                                     p.kused, p.Ct, p.c_off);
}

void launch_arn_quad(const Plan &p, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    if (p.k <= 32)
        k_arn_quad<32><<<NC, 64, 0, st>>>(p.C, p.Ct, p.c_off, p.k, p.H, p.kused, p.nu, p.s_out,
                                          p.minabs, p.flags);
    else
        k_arn_quad<64><<<NC, 64, 0, st>>>(p.C, p.Ct, p.c_off, p.k, p.H, p.kused, p.nu, p.s_out,
                                          p.minabs, p.flags);
}

}  // namespace ecnt
