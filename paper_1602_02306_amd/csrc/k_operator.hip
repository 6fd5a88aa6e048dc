// Operator kernels: w = M (A - tau_c I) M^* x on a probe block
// (Algorithm 1, step "w <- M(A - tau I)M^* q_i"; Section 2, eq. negi_T).
//
// Every column c of the block carries its own shift tau_{c / m}.  Rows are
// processed by wavefronts (one lane per column, 64 columns per wave), so the
// CSR row structure and the grid coordinates of a row are wave-uniform
// (scalar loads), and every vector access is a contiguous 64-column segment.
#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

constexpr int kRowsPerWave = 4;
constexpr int kRowsPerBlock = 4 * kRowsPerWave;   // 4 waves per 256-thread block

// |a_rr - tau_s|^(-1/2) for the Jacobi preconditioner, per shift.
template <typename VT>
__global__ __launch_bounds__(256) void k_jacobi_diag(int64_t n, int S, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const VT *__restrict__ val,
                                                     const double *__restrict__ taus,
                                                     double *__restrict__ jac, int32_t *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double arr = 0.0;
    for (int p = rp[r]; p < rp[r + 1]; ++p)
        if (ci[p] == r) arr = static_cast<double>(val[p]);
    for (int s = 0; s < S; ++s) {
        const double d = fabs(arr - taus[s]);
        if (d == 0.0) atomicOr(&flags[0], 1);
        jac[(size_t)s * n + r] = 1.0 / sqrt(d);
    }
}

// y(r, c) = xs_c * d_s(r) * ( sum_p a_{r,j_p} d_s(j_p) x(j_p, c) - tau_s d_s(r) x(r, c) )
// with d_s the Jacobi scaling of shift s (or 1 without preconditioner).
template <typename T, typename VT, bool JAC>
__global__ __launch_bounds__(256) void k_csr_op(int64_t n, int C, int m, int nct,
                                                const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const VT *__restrict__ val, const T *__restrict__ x,
                                                const double *__restrict__ xs,
                                                const double *__restrict__ jac,
                                                const double *__restrict__ taus, T *__restrict__ y)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t rg = L / nct;
    const int lane = threadIdx.x & 63;
    const int wv = uniform(threadIdx.x >> 6);
    const int c = ct * kColTile + lane;
    if (c >= C) return;
    const int s = c / m;
    const double tau = taus[s];
    const double xsc = xs ? xs[c] : 1.0;
    const double *js = JAC ? jac + (size_t)s * n : nullptr;
    for (int t = 0; t < kRowsPerWave; ++t) {
        const int64_t r = rg * kRowsPerBlock + wv * kRowsPerWave + t;
        if (r >= n) break;
        const int p0 = rp[r], p1 = rp[r + 1];
        double acc = 0.0;
        for (int p = p0; p < p1; ++p) {
            const int64_t j = ci[p];
            double xv = ld(x, (size_t)j * C + c);
            if (JAC) xv *= js[j];
            acc += static_cast<double>(val[p]) * xv;
        }
        double xr = ld(x, (size_t)r * C + c);
        if (JAC) xr *= js[r];
        double out = acc - tau * xr;
        if (JAC) out *= js[r];
        y[(size_t)r * C + c] = static_cast<T>(out * xsc);
    }
}

// One Clenshaw sweep for M = sum_j c_j T_j(B), B = (2(L + sI) - (lo+hi)I)/(hi-lo):
//   out = cx*xs_c*X + cb*B(u) - cz*Z,   u = (in_is_x ? xs_c : 1) * IN
// with B u (r) = bd*u(r) - bo*sum_{grid neighbours} u.
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_sweep(int64_t n, int C, int nct, int d0, int d1, int d2,
                                                    const T *__restrict__ X,
                                                    const double *__restrict__ xs, double cx,
                                                    const T *__restrict__ IN, int in_is_x,
                                                    double cbd, double cbo,
                                                    const T *__restrict__ Z, double cz,
                                                    T *__restrict__ out)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t rg = L / nct;
    const int lane = threadIdx.x & 63;
    const int wv = uniform(threadIdx.x >> 6);
    const int c = ct * kColTile + lane;
    if (c >= C) return;
    const double xsc = xs ? xs[c] : 1.0;
    const double isc = in_is_x ? xsc : 1.0;
    const int64_t s1 = d2, s0 = (int64_t)d1 * d2;
    for (int t = 0; t < kRowsPerWave; ++t) {
        const int64_t r = rg * kRowsPerBlock + wv * kRowsPerWave + t;
        if (r >= n) break;
        const int64_t i2 = r % d2, q = r / d2;
        const int64_t i1 = q % d1, i0 = q / d1;
        const size_t e = (size_t)r * C + c;
        double acc = 0.0;
        double val = cx * xsc * ld(X, e);
        if (IN) {
            double nb = 0.0;
            if (i2 > 0) nb += ld(IN, e - C);
            if (i2 + 1 < d2) nb += ld(IN, e + C);
            if (i1 > 0) nb += ld(IN, e - s1 * C);
            if (i1 + 1 < d1) nb += ld(IN, e + s1 * C);
            if (i0 > 0) nb += ld(IN, e - s0 * C);
            if (i0 + 1 < d0) nb += ld(IN, e + s0 * C);
            acc = isc * (cbd * ld(IN, e) - cbo * nb);
        }
        val += acc;
        if (Z) val -= cz * ld(Z, e);
        out[e] = static_cast<T>(val);
    }
}

static inline int64_t row_blocks(const Plan &p)
{
    return (p.n + kRowsPerBlock - 1) / kRowsPerBlock * p.nct;
}

void launch_jacobi_diag(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx,
                        const void *val, hipStream_t st)
{
    dim3 grid((unsigned)((p.n + 255) / 256));
    if (p.val_f32)
        k_jacobi_diag<float><<<grid, 256, 0, st>>>(p.n, p.S, row_ptr, col_idx, (const float *)val,
                                                   p.taus, p.jac, p.flags);
    else
        k_jacobi_diag<double><<<grid, 256, 0, st>>>(p.n, p.S, row_ptr, col_idx, (const double *)val,
                                                    p.taus, p.jac, p.flags);
}

template <typename T, typename VT>
static void csr_op_t(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                     const void *x, const double *xs, const double *jac, void *y, hipStream_t st)
{
    dim3 grid((unsigned)row_blocks(p));
    if (jac)
        k_csr_op<T, VT, true><<<grid, 256, 0, st>>>(p.n, p.C, p.m, p.nct, rp, ci, (const VT *)val,
                                                    (const T *)x, xs, jac, p.taus, (T *)y);
    else
        k_csr_op<T, VT, false><<<grid, 256, 0, st>>>(p.n, p.C, p.m, p.nct, rp, ci, (const VT *)val,
                                                     (const T *)x, xs, nullptr, p.taus, (T *)y);
}

void launch_csr_op(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                   const void *x, const double *xs, const double *jac, void *y, hipStream_t st)
{
    if (p.vec_f32) {
        if (p.val_f32) csr_op_t<float, float>(p, rp, ci, val, x, xs, jac, y, st);
        else csr_op_t<float, double>(p, rp, ci, val, x, xs, jac, y, st);
    } else {
        if (p.val_f32) csr_op_t<double, float>(p, rp, ci, val, x, xs, jac, y, st);
        else csr_op_t<double, double>(p, rp, ci, val, x, xs, jac, y, st);
    }
}

void launch_cheb_sweep(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                       bool in_is_x, double cb, const void *Z, double cz, void *out, hipStream_t st)
{
    // B u = ((2*(2*ndim + s) - (lo + hi)) u - 2 * sum_nb u) / (hi - lo)
    const double w = p.hi - p.lo;
    const double bd = (2.0 * (2.0 * p.ndim + p.s) - (p.lo + p.hi)) / w;
    const double bo = 2.0 / w;
    dim3 grid((unsigned)row_blocks(p));
    if (p.vec_f32)
        k_cheb_sweep<float><<<grid, 256, 0, st>>>(p.n, p.C, p.nct, p.dims[0], p.dims[1], p.dims[2],
                                                  (const float *)X, xs, cx, (const float *)IN,
                                                  in_is_x ? 1 : 0, cb * bd, cb * bo,
                                                  (const float *)Z, cz, (float *)out);
    else
        k_cheb_sweep<double><<<grid, 256, 0, st>>>(p.n, p.C, p.nct, p.dims[0], p.dims[1], p.dims[2],
                                                   (const double *)X, xs, cx, (const double *)IN,
                                                   in_is_x ? 1 : 0, cb * bd, cb * bo,
                                                   (const double *)Z, cz, (double *)out);
}

}  // namespace ecnt
