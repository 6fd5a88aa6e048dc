// Operator kernels: w = M (A - tau_c I) M^* x on a probe block
// (Algorithm 1, step "w <- M(A - tau I)M^* q_i"; Section 2, eq. negi_T).
//
// Every column c of the block carries its own shift tau_{c / m}.  Each lane
// owns VW consecutive columns (one 8- or 16-byte vector access per row), a
// wavefront covers 64*VW columns of one row, so all vector accesses are
// contiguous row segments.  Boundary handling is branch-free (clamped
// addresses with zero weights) so that every load of a row is in flight at
// once.
#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

// |a_rr - tau_s|^(-1/2) for the Jacobi preconditioner, per shift.
template <typename VT>
__global__ __launch_bounds__(256) void k_jacobi_diag(int64_t n, int S, int nseg,
                                                     const int64_t *__restrict__ seg_row,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const VT *__restrict__ val,
                                                     const double *__restrict__ seg_taus,
                                                     double *__restrict__ jac, int32_t *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double *taus = seg_taus + (size_t)find_seg(seg_row, nseg, r) * S;
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
// with d_s the Jacobi scaling of shift s = c / m (or 1 without preconditioner).
// One wavefront per row; the row's nonzeros are taken four at a time with
// clamped indices so that four row segments are loaded together.
template <typename T, typename VT, bool JAC, int VW>
__global__ __launch_bounds__(256) void k_csr_op(int64_t n, int C, int m, int c_off, int ncg, int S,
                                                int nseg, const int64_t *__restrict__ seg_row,
                                                const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const VT *__restrict__ val, const T *__restrict__ x,
                                                const double *__restrict__ xs,
                                                const double *__restrict__ jac,
                                                const double *__restrict__ seg_taus, T *__restrict__ y)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int cg = (int)(L % ncg);
    const int64_t r = (L / ncg) * 4 + uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int c0 = (cg * 64 + lane) * VW;
    if (r >= n || c0 >= C) return;
    const int seg = find_seg(seg_row, nseg, r);
    const double *taus = seg_taus + (size_t)seg * S;
    double tau[VW], xsc[VW];
    const double *js[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        const int s = (c_off + c0 + v) / m;
        tau[v] = taus[s];
        xsc[v] = xs ? xs[(size_t)seg * C + c0 + v] : 1.0;
        js[v] = JAC ? jac + (size_t)s * n : nullptr;
    }
    const int p0 = rp[r], p1 = rp[r + 1];
    double acc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = 0.0;
    for (int p = p0; p < p1; p += 4) {
        int j[4];
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int pp = min(p + q, p1 - 1);
            j[q] = ci[pp];
            a[q] = (p + q < p1) ? static_cast<double>(val[pp]) : 0.0;
        }
        double xv[4][VW];
#pragma unroll
        for (int q = 0; q < 4; ++q) vload<T, VW>(x, (size_t)j[q] * C + c0, xv[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                double xq = xv[q][v];
                if (JAC) xq *= js[v][j[q]];
                acc[v] += a[q] * xq;
            }
    }
    double xr[VW], out[VW];
    vload<T, VW>(x, (size_t)r * C + c0, xr);
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        double xv = xr[v];
        if (JAC) xv *= js[v][r];
        double o = acc[v] - tau[v] * xv;
        if (JAC) o *= js[v][r];
        out[v] = o * xsc[v];
    }
    vstore<T, VW>(y, (size_t)r * C + c0, out);
}

// One stencil sweep on the grid Laplacian L (diagonal 2*ndim, neighbours -1):
//   out = cx*xs_c*X + B(u) - cz*Z,   B u(r) = cbd*u(r) - cbo*sum_{grid neighbours} u,
//   u = (in_is_x ? xs_c : 1) * IN
// (cbd, cbo carry the scaling of B = (2(L + sI) - (lo+hi)I)/(hi-lo) and any
// factor applied to it).
//
// Register tiling: one wavefront owns a TX x TY block of z-lines (grid
// points (x, y, 0..d2-1)) for 64*VW columns and walks z, keeping the z-1, z
// and z+1 values of all its lines in registers.  The lateral neighbours
// inside the block come from registers as well; only the block's boundary
// lines and the next z value of each line are loaded: (TX*TY + 2*TX + 2*TY)
// row loads per TX*TY outputs instead of 5 per output.  Lines outside the
// grid (ragged blocks, Dirichlet boundary) are loaded from a clamped address
// with weight 0, so every load of a z step is issued together.
template <typename T, int VW, int TX, int TY, bool HASIN, bool XSEP, bool HASZ>
__global__ __launch_bounds__(256) void k_stencil(int C, int ncg, int nseg,
                                                 const int64_t *__restrict__ seg_row,
                                                 const int64_t *__restrict__ seg_tile,
                                                 const int32_t *__restrict__ seg_dims,
                                                 int64_t ntiles, const T *__restrict__ X,
                                                 const double *__restrict__ xs_all, double cx,
                                                 const T *__restrict__ IN, int in_is_x, double cbd,
                                                 double cbo, const T *__restrict__ Z, double cz,
                                                 T *__restrict__ out)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t gw = L * 4 + uniform(threadIdx.x >> 6);
    const int cg = (int)(gw % ncg);
    const int64_t tile = gw / ncg;
    const int lane = threadIdx.x & 63;
    const int c0 = (cg * 64 + lane) * VW;
    if (tile >= ntiles || c0 >= C) return;
    // the line block's segment (problem) and its grid
    const int seg = find_seg(seg_tile, nseg, tile);
    const int d0 = seg_dims[3 * seg], d1 = seg_dims[3 * seg + 1], d2 = seg_dims[3 * seg + 2];
    const int nty = (d1 + TY - 1) / TY;
    const int lt = (int)(tile - seg_tile[seg]);
    const int x0 = (lt / nty) * TX, y0 = (lt % nty) * TY;
    const double *xs = xs_all ? xs_all + (size_t)seg * C : nullptr;
    const size_t zs = (size_t)C;                       // element stride of z
    const size_t ys = (size_t)d2 * C;                  // of y
    const size_t xs_ = (size_t)d1 * d2 * C;            // of x
    const size_t base = (size_t)seg_row[seg] * C + (size_t)x0 * xs_ + (size_t)y0 * ys + c0;
    // tile lines and boundary lines: offset from `base` (clamped) and weight
    size_t off[TX][TY];
    double wt[TX][TY];
    size_t offym[TX], offyp[TX], offxm[TY], offxp[TY];
    double wym[TX], wyp[TX], wxm[TY], wxp[TY];
#pragma unroll
    for (int a = 0; a < TX; ++a)
#pragma unroll
        for (int b = 0; b < TY; ++b) {
            const bool ok = x0 + a < d0 && y0 + b < d1;
            off[a][b] = ok ? (size_t)a * xs_ + (size_t)b * ys : 0;
            wt[a][b] = ok ? 1.0 : 0.0;
        }
#pragma unroll
    for (int a = 0; a < TX; ++a) {
        const bool okx = x0 + a < d0;
        const bool okm = okx && y0 > 0, okp = okx && y0 + TY < d1;
        offym[a] = okm ? (size_t)a * xs_ - ys : 0;
        offyp[a] = okp ? (size_t)a * xs_ + (size_t)TY * ys : 0;
        wym[a] = okm ? 1.0 : 0.0;
        wyp[a] = okp ? 1.0 : 0.0;
    }
#pragma unroll
    for (int b = 0; b < TY; ++b) {
        const bool oky = y0 + b < d1;
        const bool okm = oky && x0 > 0, okp = oky && x0 + TX < d0;
        offxm[b] = okm ? (size_t)b * ys - xs_ : 0;
        offxp[b] = okp ? (size_t)b * ys + (size_t)TX * xs_ : 0;
        wxm[b] = okm ? 1.0 : 0.0;
        wxp[b] = okp ? 1.0 : 0.0;
    }
    double xsc[VW], isc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        xsc[v] = xs ? xs[c0 + v] : 1.0;
        isc[v] = in_is_x ? xsc[v] : 1.0;
    }
    double prev[TX][TY][VW], cur[TX][TY][VW];
#pragma unroll
    for (int a = 0; a < TX; ++a)
#pragma unroll
        for (int b = 0; b < TY; ++b) {
            double t[VW];
            if (HASIN) vload<T, VW>(IN, base + off[a][b], t);
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                prev[a][b][v] = 0.0;
                cur[a][b][v] = HASIN ? wt[a][b] * t[v] : 0.0;
            }
        }
    size_t ez = base;
    for (int z = 0; z < d2; ++z, ez += zs) {
        const bool hasn = z + 1 < d2;
        const size_t en = hasn ? ez + zs : ez;
        double nxt[TX][TY][VW], ym[TX][VW], yp[TX][VW], xm[TY][VW], xp[TY][VW];
        double xv[TX][TY][VW], zv[TX][TY][VW];
        if (HASIN) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b) vload<T, VW>(IN, en + off[a][b], nxt[a][b]);
#pragma unroll
            for (int a = 0; a < TX; ++a) {
                vload<T, VW>(IN, ez + offym[a], ym[a]);
                vload<T, VW>(IN, ez + offyp[a], yp[a]);
            }
#pragma unroll
            for (int b = 0; b < TY; ++b) {
                vload<T, VW>(IN, ez + offxm[b], xm[b]);
                vload<T, VW>(IN, ez + offxp[b], xp[b]);
            }
        }
        if (XSEP) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b) vload<T, VW>(X, ez + off[a][b], xv[a][b]);
        }
        if (HASZ) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b) vload<T, VW>(Z, ez + off[a][b], zv[a][b]);
        }
        __builtin_amdgcn_sched_barrier(0);
        const double zn = hasn ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < TX; ++a)
#pragma unroll
            for (int b = 0; b < TY; ++b) {
                double o[VW];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    double val = cx * xsc[v] * (XSEP ? xv[a][b][v] : cur[a][b][v]);
                    if (HASIN) {
                        const double nym = b > 0 ? cur[a][b - 1][v] : wym[a] * ym[a][v];
                        const double nyp = b + 1 < TY ? cur[a][b + 1][v] : wyp[a] * yp[a][v];
                        const double nxm = a > 0 ? cur[a - 1][b][v] : wxm[b] * xm[b][v];
                        const double nxp = a + 1 < TX ? cur[a + 1][b][v] : wxp[b] * xp[b][v];
                        const double nb = prev[a][b][v] + zn * nxt[a][b][v] + nym + nyp + nxm + nxp;
                        val += isc[v] * (cbd * cur[a][b][v] - cbo * nb);
                    }
                    if (HASZ) val -= cz * zv[a][b][v];
                    o[v] = val;
                }
                if (wt[a][b] != 0.0) vstore<T, VW>(out, ez + off[a][b], o);
            }
        if (HASIN) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b)
#pragma unroll
                    for (int v = 0; v < VW; ++v) {
                        prev[a][b][v] = cur[a][b][v];
                        cur[a][b][v] = wt[a][b] * nxt[a][b][v];
                    }
        }
    }
}

void launch_jacobi_diag(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx,
                        const void *val, hipStream_t st)
{
    dim3 grid((unsigned)((p.n + 255) / 256));
    if (p.val_f32)
        k_jacobi_diag<float><<<grid, 256, 0, st>>>(p.n, p.S, p.nseg, p.seg_row, row_ptr, col_idx,
                                                   (const float *)val, p.seg_taus, p.jac, p.flags);
    else
        k_jacobi_diag<double><<<grid, 256, 0, st>>>(p.n, p.S, p.nseg, p.seg_row, row_ptr, col_idx,
                                                    (const double *)val, p.seg_taus, p.jac, p.flags);
}

template <typename T, typename VT, int VW>
static void csr_op_t(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                     const void *x, const double *xs, const double *jac, void *y, hipStream_t st)
{
    const int ncg = (p.C + 64 * VW - 1) / (64 * VW);
    dim3 grid((unsigned)(((p.n + 3) / 4) * ncg));
    if (jac)
        k_csr_op<T, VT, true, VW><<<grid, 256, 0, st>>>(p.n, p.C, p.m, p.c_off, ncg, p.S, p.nseg,
                                                        p.seg_row, rp, ci, (const VT *)val,
                                                        (const T *)x, xs, jac, p.seg_taus, (T *)y);
    else
        k_csr_op<T, VT, false, VW><<<grid, 256, 0, st>>>(p.n, p.C, p.m, p.c_off, ncg, p.S, p.nseg,
                                                         p.seg_row, rp, ci, (const VT *)val,
                                                         (const T *)x, xs, nullptr, p.seg_taus, (T *)y);
}

template <typename T, typename VT>
static void csr_op_vw(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                      const void *x, const double *xs, const double *jac, void *y, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        if (p.vw == 4) {
            csr_op_t<T, VT, 4>(p, rp, ci, val, x, xs, jac, y, st);
            return;
        }
    }
    if (p.vw == 2) csr_op_t<T, VT, 2>(p, rp, ci, val, x, xs, jac, y, st);
    else csr_op_t<T, VT, 1>(p, rp, ci, val, x, xs, jac, y, st);
}

void launch_csr_op(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                   const void *x, const double *xs, const double *jac, void *y, hipStream_t st)
{
    if (p.vec_f32) {
        if (p.val_f32) csr_op_vw<float, float>(p, rp, ci, val, x, xs, jac, y, st);
        else csr_op_vw<float, double>(p, rp, ci, val, x, xs, jac, y, st);
    } else {
        if (p.val_f32) csr_op_vw<double, float>(p, rp, ci, val, x, xs, jac, y, st);
        else csr_op_vw<double, double>(p, rp, ci, val, x, xs, jac, y, st);
    }
}

template <typename T, int VW, int TX, int TY, bool HASIN, bool XSEP, bool HASZ>
static void stencil_t(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                      bool in_is_x, double cbd, double cbo, const void *Z, double cz, void *out,
                      hipStream_t st)
{
    const int ncg = (p.C + 64 * VW - 1) / (64 * VW);
    const int64_t waves = p.ntiles * ncg;
    dim3 grid((unsigned)((waves + 3) / 4));
    k_stencil<T, VW, TX, TY, HASIN, XSEP, HASZ><<<grid, 256, 0, st>>>(
        p.C, ncg, p.nseg, p.seg_row, p.seg_tile, p.seg_dims, p.ntiles, (const T *)X, xs, cx,
        (const T *)IN, in_is_x ? 1 : 0, cbd, cbo, (const T *)Z, cz, (T *)out);
}

template <typename T, int VW, int TX, int TY>
static void stencil_flags(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                          bool in_is_x, double cbd, double cbo, const void *Z, double cz, void *out,
                          hipStream_t st)
{
    if (!IN) {
        stencil_t<T, VW, TX, TY, false, true, false>(p, X, xs, cx, IN, false, 0, 0, nullptr, 0, out, st);
    } else if (IN == X && !Z) {
        stencil_t<T, VW, TX, TY, true, false, false>(p, X, xs, cx, IN, in_is_x, cbd, cbo, nullptr, 0, out, st);
    } else if (!Z) {
        stencil_t<T, VW, TX, TY, true, true, false>(p, X, xs, cx, IN, in_is_x, cbd, cbo, nullptr, 0, out, st);
    } else {
        stencil_t<T, VW, TX, TY, true, true, true>(p, X, xs, cx, IN, in_is_x, cbd, cbo, Z, cz, out, st);
    }
}

// line-block shape (x lines by y lines): 4 x 4, 2 x 4 or 1 x 8
template <typename T, int VW>
static void stencil_shape(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                          bool in_is_x, double cbd, double cbo, const void *Z, double cz, void *out,
                          hipStream_t st)
{
    if (p.tx == 4) stencil_flags<T, VW, 4, 4>(p, X, xs, cx, IN, in_is_x, cbd, cbo, Z, cz, out, st);
    else if (p.tx == 2) stencil_flags<T, VW, 2, 4>(p, X, xs, cx, IN, in_is_x, cbd, cbo, Z, cz, out, st);
    else stencil_flags<T, VW, 1, 8>(p, X, xs, cx, IN, in_is_x, cbd, cbo, Z, cz, out, st);
}

void launch_stencil(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                    bool in_is_x, double cb, const void *Z, double cz, void *out, hipStream_t st)
{
    // B u = ((2*(2*ndim + s) - (lo + hi)) u - 2 * sum_nb u) / (hi - lo), scaled by cb
    const double w = p.hi - p.lo;
    const double bd = cb * (2.0 * (2.0 * p.ndim + p.s) - (p.lo + p.hi)) / w;
    const double bo = cb * 2.0 / w;
    // one column per lane (FP64) / two (FP32, when the width is even): the
    // register tile holds 3 z-values of TX*TY lines per column
    if (p.vec_f32 && p.C % 2 == 0)
        stencil_shape<float, 2>(p, X, xs, cx, IN, in_is_x, bd, bo, Z, cz, out, st);
    else if (p.vec_f32)
        stencil_shape<float, 1>(p, X, xs, cx, IN, in_is_x, bd, bo, Z, cz, out, st);
    else
        stencil_shape<double, 1>(p, X, xs, cx, IN, in_is_x, bd, bo, Z, cz, out, st);
}

}  // namespace ecnt
