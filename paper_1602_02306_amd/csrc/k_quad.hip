// Quadrature kernels: batched symmetric tridiagonal eigensolve and the probe
// average.
//
// Per column c (one lane each): the Lanczos matrix J_k (Section 3.1, eq. Tk),
// or the generalized averaged matrix of Section 3.4 (eq. GA_Tk), is
// diagonalized by implicit QR sweeps with Wilkinson shifts, accumulating only
// the first row of the eigenvector matrix (its entries are the z_i(1) of
// eq. gauss_quad).  Then
//   s_c = |v|^2 * sum_i z_i(1)^2 h(theta_i)         (eq. gauss_quad, Algorithm 2)
// and, over probes, the mean and sample variance of the per-probe values
// (eq. rand_prec_quad; the interval count is the difference of two shifts).
#include <float.h>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

constexpr int kQuadLdsBytes = 48 * 1024;

template <int KMAX>
struct QuadGeom {
    static constexpr int lanes = (kQuadLdsBytes / (24 * KMAX)) < 64 ? (kQuadLdsBytes / (24 * KMAX)) : 64;
};

__device__ __forceinline__ double step_fn(double th, double w)
{
    if (w > 0.0) return 0.5 * erfc(th / w);
    return th < 0.0 ? 1.0 : 0.0;
}

// One lane per virtual column vc = seg*C + c (alpha, beta, nu indexed [row][NC]);
// kused, s_out and minabs are global: [seg*ld + off + c].  A workgroup is
// blockDim.x lanes (at most QuadGeom<KMAX>::lanes): the columns' QR
// iterations diverge, so a wavefront runs as long as the union of its lanes'
// paths, and few columns go one to a wavefront (the launcher's choice).  The
// matrices live in dynamic LDS, 3 * KMAX doubles per lane.
template <int KMAX>
__global__ __launch_bounds__(64) void k_tridiag(int NC, int C, int ld, int off, int k, int rule,
                                                double smooth_w,
                                                const double *__restrict__ alpha,
                                                const double *__restrict__ beta,
                                                const int32_t *__restrict__ kused_all,
                                                const double *__restrict__ nu,
                                                double *__restrict__ s_all,
                                                double *__restrict__ minabs_all,
                                                int32_t *__restrict__ flags)
{
    extern __shared__ double lds[];
    const int LN = blockDim.x;
    const int lane = threadIdx.x;
    const int vc = blockIdx.x * LN + lane;
    if (vc >= NC) return;
    const int seg = vc / C;
    const size_t gidx = (size_t)seg * ld + off + (vc - seg * C);
    const int c = vc;
    C = NC;   // alpha, beta, nu below are indexed [row][NC] by the virtual column
    double *a = lds + lane;
    double *b = lds + KMAX * LN + lane;
    double *z = lds + 2 * KMAX * LN + lane;
#define A_(i) a[(i) * LN]
#define B_(i) b[(i) * LN]
#define Z_(i) z[(i) * LN]
    const int ku = kused_all[gidx];
    if (ku < 1) {
        s_all[gidx] = 0.0;
        minabs_all[gidx] = INFINITY;
        return;
    }
    int N;
    if (rule == 1 && ku == k && k >= 2) {
        // eq. GA_Tk: diag (a_1..a_k, a_{k-1}..a_1), off (b_2..b_k, b_{k+1}, b_{k-1}..b_2)
        N = 2 * k - 1;
        for (int i = 0; i < k; ++i) A_(i) = alpha[(size_t)i * C + c];
        for (int i = k; i < N; ++i) A_(i) = alpha[(size_t)(2 * k - 2 - i) * C + c];
        for (int i = 0; i < k; ++i) B_(i) = beta[(size_t)(i + 1) * C + c];
        for (int i = k; i < N - 1; ++i) B_(i) = beta[(size_t)(2 * k - 2 - i) * C + c];
    } else {
        N = ku;
        for (int i = 0; i < N; ++i) A_(i) = alpha[(size_t)i * C + c];
        for (int i = 0; i < N - 1; ++i) B_(i) = beta[(size_t)(i + 1) * C + c];
    }
    for (int i = 0; i < N; ++i) Z_(i) = i == 0 ? 1.0 : 0.0;
    B_(N - 1) = 0.0;   // past the last row: what a sweep's last rotation reads

    int hi = N - 1;
    int iter = 0;
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
        // Wilkinson shift from the trailing 2x2 block of the active window
        const double bb = B_(hi - 1);
        const double d = 0.5 * (A_(hi - 1) - A_(hi));
        const double den = d + copysign(hypot(d, bb), d);
        const double mu = A_(hi) - (den != 0.0 ? bb * bb / den : 0.0);
        double x = A_(lo) - mu, y = B_(lo);
        // The values a rotation changes and the next one reads (A(kk), B(kk),
        // Z(kk)) are carried in registers; the ones it reads ahead (A(kk+1),
        // B(kk+1), Z(kk+1), not yet written in this sweep) come from three
        // register sets by position mod 3, each reloaded three indices ahead
        // once its rotation has used it (the first (hi - lo) mod 3 rotations
        // read theirs directly).  Indices are clamped to hi, with no
        // condition on a load: B(hi) is 0 (set when hi moved down, or past
        // the last row), which is what a sweep's last rotation takes.
        double ak = A_(lo), bk = B_(lo), zk = Z_(lo), nbk = bk;
        auto rot = [&](int kk, double ak1, double bk1, double z1) __attribute__((always_inline)) {
            // |x|, |y| far from the under/overflow range: J_k holds O(|C|) entries
            const double q2 = x * x + y * y;
            const bool nz = q2 > 0.0;
            const double ir = rsqrt_pos(nz ? q2 : 1.0);
            const double r = nz ? q2 * ir : 0.0;
            const double cs = nz ? x * ir : 1.0;
            const double sn = nz ? y * ir : 0.0;
            if (kk > lo) B_(kk - 1) = r;
            A_(kk) = cs * cs * ak + 2.0 * cs * sn * bk + sn * sn * ak1;
            const double na1 = sn * sn * ak - 2.0 * cs * sn * bk + cs * cs * ak1;
            nbk = cs * sn * (ak1 - ak) + (cs * cs - sn * sn) * bk;
            Z_(kk) = cs * zk + sn * z1;
            zk = -sn * zk + cs * z1;
            ak = na1;
            bk = cs * bk1;
            x = nbk;
            y = sn * bk1;
        };
        int kk = lo;
        for (const int k0 = lo + (hi - lo) % 3; kk < k0; ++kk) rot(kk, A_(kk + 1), B_(kk + 1), Z_(kk + 1));
        if (kk < hi) {
            int i0 = kk + 1, i1 = min(kk + 2, hi), i2 = min(kk + 3, hi);
            double a0 = A_(i0), b0 = B_(i0), z0 = Z_(i0);
            double a1 = A_(i1), b1 = B_(i1), z1 = Z_(i1);
            double a2 = A_(i2), b2 = B_(i2), z2 = Z_(i2);
            for (; kk < hi; kk += 3) {
                rot(kk, a0, b0, z0);
                i0 = min(kk + 4, hi);
                a0 = A_(i0);
                b0 = B_(i0);
                z0 = Z_(i0);
                rot(kk + 1, a1, b1, z1);
                i1 = min(kk + 5, hi);
                a1 = A_(i1);
                b1 = B_(i1);
                z1 = Z_(i1);
                rot(kk + 2, a2, b2, z2);
                i2 = min(kk + 6, hi);
                a2 = A_(i2);
                b2 = B_(i2);
                z2 = Z_(i2);
            }
        }
        A_(hi) = ak;
        B_(hi - 1) = nbk;
        Z_(hi) = zk;
    }
    double s = 0.0, mn = INFINITY;
    for (int i = 0; i < N; ++i) {
        const double th = A_(i);
        const double zz = Z_(i);
        s += zz * zz * step_fn(th, smooth_w);
        mn = fmin(mn, fabs(th));
    }
    s_all[gidx] = nu[c] * s;
    minabs_all[gidx] = mn;
    if (failed) atomicOr(&flags[1], 1);
#undef A_
#undef B_
#undef Z_
}

// Probe average.  res[s] = mean_j s_out[s*m + j]; for t < S-1:
// res[S + t] = mean_j d_j, res[2S - 1 + t] = sum_j (d_j - mean)^2 / ((m-1) m),
// d_j = s_out[(t+1)*m + j] - s_out[t*m + j]; res[3S - 2] = min over columns of minabs.
// One 256-thread workgroup; fixed reduction order.
__device__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One workgroup per segment (problem): s_out, minabs at seg*S*m, results at seg*kResStride.
__global__ __launch_bounds__(256) void k_reduce(int S, int m, const double *__restrict__ s_all,
                                                const double *__restrict__ minabs_all,
                                                double *__restrict__ res_all)
{
    __shared__ double sh[256];
    const double *s_out = s_all + (size_t)blockIdx.x * S * m;
    const double *minabs = minabs_all + (size_t)blockIdx.x * S * m;
    double *res = res_all + (size_t)blockIdx.x * kResStride;
    for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int j = threadIdx.x; j < m; j += 256) acc += s_out[(size_t)s * m + j];
        const double tot = block_sum(acc, sh);
        if (threadIdx.x == 0) res[s] = tot / m;
    }
    for (int t = 0; t + 1 < S; ++t) {
        double acc = 0.0;
        for (int j = threadIdx.x; j < m; j += 256)
            acc += s_out[(size_t)(t + 1) * m + j] - s_out[(size_t)t * m + j];
        const double mean = block_sum(acc, sh) / m;
        double v = 0.0;
        for (int j = threadIdx.x; j < m; j += 256) {
            const double d = s_out[(size_t)(t + 1) * m + j] - s_out[(size_t)t * m + j] - mean;
            v += d * d;
        }
        const double vs = block_sum(v, sh);
        if (threadIdx.x == 0) {
            res[S + t] = mean;
            res[2 * S - 1 + t] = m > 1 ? vs / ((double)(m - 1) * m) : NAN;
        }
    }
    double mn = INFINITY;
    for (int c = threadIdx.x; c < S * m; c += 256) mn = fmin(mn, minabs[c]);
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) res[3 * S - 2] = sh[0];
}

// The same eigensolve with one wavefront per column (few columns): every lane
// runs the rotation chain on the same values, the search for the unreduced
// block takes 64 candidates at a time (a ballot), and each sweep carries its
// changing values in registers with the values ahead loaded three rotations
// early, as the lane form does.  A rotation's writes come from every lane (the
// same values to the same slots); lane 0 makes the others.
template <int KMAX>
__global__ __launch_bounds__(64) void k_tridiag_wave(int NC, int C, int ld, int off, int k, int rule,
                                                     double smooth_w,
                                                     const double *__restrict__ alpha,
                                                     const double *__restrict__ beta,
                                                     const int32_t *__restrict__ kused_all,
                                                     const double *__restrict__ nu,
                                                     double *__restrict__ s_all,
                                                     double *__restrict__ minabs_all,
                                                     int32_t *__restrict__ flags)
{
    __shared__ double A_[KMAX + 1], B_[KMAX + 1], Z_[KMAX + 1];
    const int lane = threadIdx.x;
    const int vc = blockIdx.x;
    const int seg = vc / C;
    const size_t gidx = (size_t)seg * ld + off + (vc - seg * C);
    const int c = vc;
    C = NC;   // alpha, beta, nu below are indexed [row][NC] by the virtual column
    const int ku = kused_all[gidx];
    if (ku < 1) {
        if (lane == 0) {
            s_all[gidx] = 0.0;
            minabs_all[gidx] = INFINITY;
        }
        return;
    }
    int N;
    if (rule == 1 && ku == k && k >= 2) {
        // eq. GA_Tk: diag (a_1..a_k, a_{k-1}..a_1), off (b_2..b_k, b_{k+1}, b_{k-1}..b_2)
        N = 2 * k - 1;
        for (int i = lane; i < N; i += 64) {
            A_[i] = alpha[(size_t)(i < k ? i : 2 * k - 2 - i) * C + c];
            if (i < N - 1) B_[i] = beta[(size_t)(i < k ? i + 1 : 2 * k - 2 - i) * C + c];
        }
    } else {
        N = ku;
        for (int i = lane; i < N; i += 64) {
            A_[i] = alpha[(size_t)i * C + c];
            if (i < N - 1) B_[i] = beta[(size_t)(i + 1) * C + c];
        }
    }
    for (int i = lane; i < N; i += 64) Z_[i] = i == 0 ? 1.0 : 0.0;
    if (lane == 0) B_[N - 1] = 0.0;   // past the last row: what a sweep's last rotation reads
    __syncthreads();

    int hi = N - 1, iter = 0;
    bool failed = false;
    while (hi > 0) {
        if (fabs(B_[hi - 1]) <= DBL_EPSILON * (fabs(A_[hi - 1]) + fabs(A_[hi])) ||
            fabs(B_[hi - 1]) < DBL_MIN) {
            __syncthreads();
            if (lane == 0) B_[hi - 1] = 0.0;
            __syncthreads();
            --hi;
            continue;
        }
        // the largest lo < hi with B[lo-1] negligible (or 0), 64 candidates at a time
        int lo = 0;
        for (int base = hi - 1; base > 0; base -= 64) {
            const int i = base - lane;
            bool neg = false;
            if (i >= 1) {
                const double bl = fabs(B_[i - 1]);
                neg = bl <= DBL_EPSILON * (fabs(A_[i - 1]) + fabs(A_[i])) || bl < DBL_MIN;
            }
            const unsigned long long msk = __ballot(neg);
            if (msk) {
                lo = base - (__ffsll((long long)msk) - 1);
                break;
            }
        }
        if (++iter > 60 * N) {
            failed = true;
            break;
        }
        // Wilkinson shift from the trailing 2x2 block of the active window
        const double bb = B_[hi - 1];
        const double d = 0.5 * (A_[hi - 1] - A_[hi]);
        const double den = d + copysign(hypot(d, bb), d);
        const double mu = A_[hi] - (den != 0.0 ? bb * bb / den : 0.0);
        if (lo > 0 && lane == 0) B_[lo - 1] = 0.0;   // the split found above (not read by the sweep)
        double x = A_[lo] - mu, y = B_[lo];
        double ak = A_[lo], bk = B_[lo], zk = Z_[lo], nbk = bk;
        auto rot = [&](int q, double ak1, double bk1, double z1) __attribute__((always_inline)) {
            // |x|, |y| far from the under/overflow range: J_k holds O(|C|) entries
            // (q2 = 0 only when x = y = 0: then r = sn = 0 as they stand)
            const double q2 = x * x + y * y;
            const bool nz = q2 > 0.0;
            const double ir = rsqrt_pos(nz ? q2 : 1.0);
            const double r = q2 * ir;
            const double cs = nz ? x * ir : 1.0;
            const double sn = y * ir;
            const double na = cs * cs * ak + 2.0 * cs * sn * bk + sn * sn * ak1;
            const double nz1 = cs * zk + sn * z1;
            // every lane holds the same values and writes them to the same
            // slots; the first rotation of a sweep has no B to write (slot
            // KMAX is never read)
            B_[q > lo ? q - 1 : KMAX] = r;
            A_[q] = na;
            Z_[q] = nz1;
            const double na1 = sn * sn * ak - 2.0 * cs * sn * bk + cs * cs * ak1;
            nbk = cs * sn * (ak1 - ak) + (cs * cs - sn * sn) * bk;
            zk = -sn * zk + cs * z1;
            ak = na1;
            bk = cs * bk1;
            x = nbk;
            y = sn * bk1;
        };
        int q = lo;
        for (const int q0 = lo + (hi - lo) % 3; q < q0; ++q) rot(q, A_[q + 1], B_[q + 1], Z_[q + 1]);
        if (q < hi) {
            int i0 = q + 1, i1 = min(q + 2, hi), i2 = min(q + 3, hi);
            double a0 = A_[i0], b0 = B_[i0], z0 = Z_[i0];
            double a1 = A_[i1], b1 = B_[i1], z1 = Z_[i1];
            double a2 = A_[i2], b2 = B_[i2], z2 = Z_[i2];
            for (; q < hi; q += 3) {
                rot(q, a0, b0, z0);
                i0 = min(q + 4, hi);
                a0 = A_[i0];
                b0 = B_[i0];
                z0 = Z_[i0];
                rot(q + 1, a1, b1, z1);
                i1 = min(q + 5, hi);
                a1 = A_[i1];
                b1 = B_[i1];
                z1 = Z_[i1];
                rot(q + 2, a2, b2, z2);
                i2 = min(q + 6, hi);
                a2 = A_[i2];
                b2 = B_[i2];
                z2 = Z_[i2];
            }
        }
        if (lane == 0) {
            A_[hi] = ak;
            B_[hi - 1] = nbk;
            Z_[hi] = zk;
        }
        __syncthreads();
    }
    __syncthreads();
    // s = |v|^2 sum_i z_i(1)^2 h(theta_i): lanes take i = lane, lane + 64, ...,
    // then the butterfly (the same sum in every lane)
    double s = 0.0, mn = INFINITY;
    for (int i = lane; i < N; i += 64) {
        const double th = A_[i], zz = Z_[i];
        s += zz * zz * step_fn(th, smooth_w);
        mn = fmin(mn, fabs(th));
    }
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        mn = fmin(mn, __shfl_xor(mn, o, 64));
    }
    if (lane == 0) {
        s_all[gidx] = nu[c] * s;
        minabs_all[gidx] = mn;
        if (failed) atomicOr(&flags[1], 1);
    }
}

template <int KMAX>
static void tridiag_t(const Plan &p, hipStream_t st)
{
    // up to 2048 columns (about two wavefronts per CU): a wavefront per column;
    // beyond, lanes per workgroup doubling to keep about 2048 workgroups
    const int NC = p.nseg * p.C;
    if (NC <= 2048) {
        k_tridiag_wave<KMAX><<<NC, 64, 0, st>>>(NC, p.C, p.Ct, p.c_off, p.k, p.rule, p.smooth_w,
                                                p.alpha, p.beta, p.kused, p.nu, p.s_out, p.minabs,
                                                p.flags);
        return;
    }
    int LN = 1;
    while (LN < QuadGeom<KMAX>::lanes && NC > 2048 * LN) LN *= 2;
    const int blocks = (NC + LN - 1) / LN;
    const size_t lds = sizeof(double) * 3 * KMAX * LN;
    k_tridiag<KMAX><<<blocks, LN, lds, st>>>(NC, p.C, p.Ct, p.c_off, p.k, p.rule, p.smooth_w, p.alpha,
                                             p.beta, p.kused, p.nu, p.s_out, p.minabs, p.flags);
}

void launch_tridiag(const Plan &p, hipStream_t st)
{
    const int N = (p.rule == 1) ? 2 * p.k - 1 : p.k;
    if (N <= 32) tridiag_t<32>(p, st);
    else if (N <= 64) tridiag_t<64>(p, st);
    else if (N <= 128) tridiag_t<128>(p, st);
    else if (N <= 256) tridiag_t<256>(p, st);
    else tridiag_t<512>(p, st);
}

void launch_reduce(const Plan &p, hipStream_t st)
{
    k_reduce<<<p.nseg, 256, 0, st>>>(p.S, p.m, p.s_out, p.minabs, p.result);
}

}  // namespace ecnt
