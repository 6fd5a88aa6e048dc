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
// One wavefront per group of RPW consecutive rows; the nonzeros of all the
// group's rows are taken NZ per row at a time with clamped indices, so that
// NZ*RPW row segments are loaded together (with NZ = 8 a 7-point stencil row
// in one pass).  Each row sums its nonzeros in CSR order.  Block order:
// column groups fastest; `remap` spreads contiguous row ranges over the XCDs
// (each XCD's L2 then sees its own rows' neighbours), otherwise all XCDs walk
// the rows together and rows a grid plane apart meet in the shared cache.
template <typename T, typename VT, bool JAC, int VW, int RPW, int NZ>
__global__ __launch_bounds__(256) void k_csr_op(int64_t n, int C, int m, int c_off, int ncg, int S,
                                                int nseg, const int64_t *__restrict__ seg_row,
                                                const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const VT *__restrict__ val, const T *__restrict__ x,
                                                const double *__restrict__ xs,
                                                const double *__restrict__ jac,
                                                const double *__restrict__ seg_taus, T *__restrict__ y,
                                                int remap, const int32_t *__restrict__ gate)
{
    // gate (the status flags): the stencil form applied A already unless flags[2] is set
    if (gate && gate[2] == 0) return;
    const int64_t L = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int cg = (int)(L % ncg);
    const int64_t r0 = ((L / ncg) * 4 + uniform(threadIdx.x >> 6)) * RPW;
    const int lane = threadIdx.x & 63;
    const int c0 = (cg * 64 + lane) * VW;
    if (r0 >= n || c0 >= C) return;
    int64_t row[RPW];
    int p0[RPW], len[RPW], maxlen = 0;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        row[i] = min(r0 + i, n - 1);   // rows past the end repeat the last one (not stored)
        p0[i] = rp[row[i]];
        len[i] = rp[row[i] + 1] - p0[i];
        maxlen = max(maxlen, len[i]);
    }
    // an index inside the longest row: where the loads of shorter rows are clamped
    int safe = p0[0];
#pragma unroll
    for (int i = RPW - 1; i >= 0; --i)
        if (len[i] == maxlen) safe = p0[i];
    double acc[RPW][VW];
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[i][v] = 0.0;
    const double *js[VW];
    int sh[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        sh[v] = (c_off + c0 + v) / m;
        js[v] = JAC ? jac + (size_t)sh[v] * n : nullptr;
    }
    for (int p = 0; p < maxlen; p += NZ) {
        int j[RPW][NZ];
        double a[RPW][NZ];
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
            for (int q = 0; q < NZ; ++q) {
                const bool ok = p + q < len[i];
                const int pp = ok ? p0[i] + p + q : safe;
                j[i][q] = ci[pp];
                a[i][q] = ok ? static_cast<double>(val[pp]) : 0.0;
            }
        double xv[RPW][NZ][VW];
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
            for (int q = 0; q < NZ; ++q) vload<T, VW>(x, (size_t)j[i][q] * C + c0, xv[i][q]);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
            for (int q = 0; q < NZ; ++q)
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    double xq = xv[i][q][v];
                    if (JAC) xq *= js[v][j[i][q]];
                    acc[i][v] += a[i][q] * xq;
                }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int64_t r = row[i];
        const int seg = find_seg(seg_row, nseg, r);
        const double *taus = seg_taus + (size_t)seg * S;
        double xr[VW], out[VW];
        vload<T, VW>(x, (size_t)r * C + c0, xr);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            double xv = xr[v];
            if (JAC) xv *= js[v][r];
            double o = acc[i][v] - taus[sh[v]] * xv;
            if (JAC) o *= js[v][r];
            const double xsc = xs ? xs[(size_t)seg * C + c0 + v] : 1.0;
            out[v] = o * xsc;
        }
        if (r0 + i < n) vstore_nt<T, VW>(y, (size_t)r * C + c0, out);
    }
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
    // column-group-major: the waves of a workgroup and consecutive workgroups
    // take neighbouring line blocks of one column group, so that boundary
    // lines loaded by one block are still in cache for its neighbours
    const int64_t gw = L * 4 + uniform(threadIdx.x >> 6);
    const int cg = (int)(gw / ntiles);
    const int64_t tile = gw % ntiles;
    if (cg >= ncg) return;
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
    // Loads of one z step: the next z value of the block's lines, this z
    // value of the boundary lines, and X, Z at this z.
    struct StepLoads {
        double nxt[TX][TY][VW], ym[TX][VW], yp[TX][VW], xm[TY][VW], xp[TY][VW];
        double xv[TX][TY][VW], zv[TX][TY][VW];
    };
    auto issue = [&](StepLoads &L, int z) {
        const size_t ez = base + (size_t)z * zs;
        const size_t en = z + 1 < d2 ? ez + zs : ez;
        if (HASIN) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b) vload<T, VW>(IN, en + off[a][b], L.nxt[a][b]);
#pragma unroll
            for (int a = 0; a < TX; ++a) {
                vload<T, VW>(IN, ez + offym[a], L.ym[a]);
                vload<T, VW>(IN, ez + offyp[a], L.yp[a]);
            }
#pragma unroll
            for (int b = 0; b < TY; ++b) {
                vload<T, VW>(IN, ez + offxm[b], L.xm[b]);
                vload<T, VW>(IN, ez + offxp[b], L.xp[b]);
            }
        }
        if (XSEP) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b) vload<T, VW>(X, ez + off[a][b], L.xv[a][b]);
        }
        if (HASZ) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TY; ++b) vload<T, VW>(Z, ez + off[a][b], L.zv[a][b]);
        }
    };
    auto compute = [&](const StepLoads &L, int z) {
        const size_t ez = base + (size_t)z * zs;
        const double zn = z + 1 < d2 ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < TX; ++a)
#pragma unroll
            for (int b = 0; b < TY; ++b) {
                double o[VW];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    double val = cx * xsc[v] * (XSEP ? L.xv[a][b][v] : cur[a][b][v]);
                    if (HASIN) {
                        const double nym = b > 0 ? cur[a][b - 1][v] : wym[a] * L.ym[a][v];
                        const double nyp = b + 1 < TY ? cur[a][b + 1][v] : wyp[a] * L.yp[a][v];
                        const double nxm = a > 0 ? cur[a - 1][b][v] : wxm[b] * L.xm[b][v];
                        const double nxp = a + 1 < TX ? cur[a + 1][b][v] : wxp[b] * L.xp[b][v];
                        const double nb = prev[a][b][v] + zn * L.nxt[a][b][v] + nym + nyp + nxm + nxp;
                        val += isc[v] * (cbd * cur[a][b][v] - cbo * nb);
                    }
                    if (HASZ) val -= cz * L.zv[a][b][v];
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
                        cur[a][b][v] = wt[a][b] * L.nxt[a][b][v];
                    }
        }
    };
    // all loads of a step issued together, then the step computed
    for (int z = 0; z < d2; ++z) {
        StepLoads L;
        issue(L, z);
        __builtin_amdgcn_sched_barrier(0);
        compute(L, z);
    }
}

// ---- one quadratic factor of the preconditioner in a single sweep ----
//   t = c1*u + cb*B(u),  out = B(t) + c2*u - cz*Z,   u = xs_c * X
// i.e. the factor cb*(B^2 - 2a B + b) of the product form (c1 = -2a*cb,
// c2 = b*cb) computed as the two plain sweeps compute it, with t never
// written to memory: 1 read and 1 write of a block vector instead of 3 reads
// and 2 writes.  t is rounded to the storage type as the
// two-sweep form stores it, and every value is summed in the same order.
//
// A workgroup owns a 4 x 4 block of z-lines (the line blocks of the plain
// sweep with the 4 x 4 shape) for 64*VW columns; each of its four wavefronts
// owns a 2 x 2 quadrant and walks z.  It needs t on its lines and on the ring
// of lines at distance 1 (for the lateral neighbours of B t), hence u on the
// lines at distance <= 2.  Line table: 0..3 the quadrant, 4..11 distance 1,
// 12..23 distance 2; (i, j) steps along the first and second grid axes.
namespace quad {
constexpr int LI[24] = {0, 0, 1, 1, -1, -1, 2, 2, 0, 1, 0, 1, -2, -2, 3, 3, 0, 1, 0, 1, -1, -1, 2, 2};
constexpr int LJ[24] = {0, 1, 0, 1, 0, 1, 0, 1, -1, -1, 2, 2, 0, 1, 0, 1, -2, -2, 3, 3, -1, 2, -1, 2};
// lateral neighbours of lines 0..11: (i, j-1), (i, j+1), (i-1, j), (i+1, j)
constexpr int NYM[12] = {8, 0, 9, 2, 20, 4, 22, 6, 16, 17, 1, 3};
constexpr int NYP[12] = {1, 10, 3, 11, 5, 21, 7, 23, 0, 2, 18, 19};
constexpr int NXM[12] = {4, 5, 0, 1, 12, 13, 2, 3, 20, 8, 21, 10};
constexpr int NXP[12] = {2, 3, 6, 7, 0, 1, 14, 15, 9, 22, 11, 23};
}  // namespace quad

template <typename T, int VW, bool HASZ>
__global__ __launch_bounds__(256) void k_quad_sweep(int C, int ncg, int nseg,
                                                    const int64_t *__restrict__ seg_row,
                                                    const int64_t *__restrict__ seg_tile,
                                                    const int32_t *__restrict__ seg_dims,
                                                    int64_t ntiles, const T *__restrict__ X,
                                                    const double *__restrict__ xs_all, double c1,
                                                    double bd1, double bo1, double c2, double bd2,
                                                    double bo2, const T *__restrict__ Z, double cz,
                                                    T *__restrict__ out)
{
    using namespace quad;
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int cg = (int)(L / ntiles);   // column-group-major, as in the plain sweep
    const int64_t tile = L % ntiles;
    const int wv = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int c0 = (cg * 64 + lane) * VW;
    if (tile >= ntiles || c0 >= C) return;
    const int seg = find_seg(seg_tile, nseg, tile);
    const int d0 = seg_dims[3 * seg], d1 = seg_dims[3 * seg + 1], d2 = seg_dims[3 * seg + 2];
    const int nty = (d1 + 3) / 4;
    const int lt = (int)(tile - seg_tile[seg]);
    const int tx0 = (lt / nty) * 4, ty0 = (lt % nty) * 4;       // the 4 x 4 block
    const int bx = tx0 + 2 * (wv >> 1), by = ty0 + 2 * (wv & 1);  // this quadrant
    const double *xs = xs_all ? xs_all + (size_t)seg * C : nullptr;
    const int64_t zs = C, ys = (int64_t)d2 * C, xst = (int64_t)d1 * d2 * C;
    // the block's first line is always inside the grid: clamp targets
    const int64_t base = (int64_t)seg_row[seg] * C + (int64_t)tx0 * xst + (int64_t)ty0 * ys + c0;
    int64_t off[24];
    double w[24];
#pragma unroll
    for (int q = 0; q < 24; ++q) {
        const int gi = bx + LI[q], gj = by + LJ[q];
        const bool ok = gi >= 0 && gi < d0 && gj >= 0 && gj < d1;
        off[q] = ok ? (int64_t)(gi - tx0) * xst + (int64_t)(gj - ty0) * ys : 0;
        w[q] = ok ? 1.0 : 0.0;
    }
    double xsc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) xsc[v] = xs ? xs[c0 + v] : 1.0;
    // values are kept in the storage type (u as loaded, t as the two-sweep
    // form stores it) and widened to double for the arithmetic
    auto ldT = [&](const T *P, int64_t e, T (&o)[VW]) {
        using V = typename VecT<T, VW>::type;
        const V x = *reinterpret_cast<const V *>(P + e);
        if constexpr (VW == 1) {
            o[0] = x;
        } else {
            o[0] = x.x;
            o[1] = x.y;
        }
    };
    const T zero = T(0);
    // u (weighted by the line's inside-grid flag) on lines 0..11 at z-1, z,
    // z+1 and on lines 12..23 at z; t on lines 0..3 at z-2, z-1 and on lines
    // 4..11 at z-1
    T um[12][VW], u0[12][VW], tm2[4][VW], tm1[4][VW], r1[8][VW];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        T a[VW];
        ldT(X, base + off[q], a);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            um[q][v] = zero;
            u0[q][v] = w[q] != 0.0 ? a[v] : zero;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) tm2[q][v] = tm1[q][v] = zero;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) r1[q][v] = zero;
    // loads of iteration z: u at z+1 on lines 0..11, u at z on lines 12..23,
    // Z at z-1 on lines 0..3 (addresses clamped past the ends)
    struct StepLoads {
        T un[12][VW], u2[12][VW], zv[4][VW];
    };
    auto issue = [&](StepLoads &S, int z) {
        const int64_t ez = base + (int64_t)z * zs;
        const int64_t en = z + 1 < d2 ? ez + zs : base;
        const int64_t ec = z < d2 ? ez : base;
        const int64_t ep = z >= 1 ? ez - zs : base;
#pragma unroll
        for (int q = 0; q < 12; ++q) ldT(X, en + off[q], S.un[q]);
#pragma unroll
        for (int q = 0; q < 12; ++q) ldT(X, ec + off[12 + q], S.u2[q]);
        if (HASZ) {
#pragma unroll
            for (int q = 0; q < 4; ++q) ldT(Z, ep + off[q], S.zv[q]);
        }
    };
    auto compute = [&](const StepLoads &S, int z) {
        const int64_t ep = z >= 1 ? base + (int64_t)(z - 1) * zs : base;
        const bool has_t = z < d2;                 // t at plane z exists
        const double zn = z + 1 < d2 ? 1.0 : 0.0;  // u at plane z+1 exists
        // t at plane z on lines 0..11 (zero outside the grid and past the last plane)
        T tn[12][VW];
#pragma unroll
        for (int q = 0; q < 12; ++q)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                auto uat = [&](int r) -> double {
                    return r < 12 ? (double)u0[r][v] : w[r] * (double)S.u2[r - 12][v];
                };
                const double cu = u0[q][v];
                const double nb = (double)um[q][v] + zn * (double)S.un[q][v] + uat(NYM[q]) +
                                  uat(NYP[q]) + uat(NXM[q]) + uat(NXP[q]);
                double t = c1 * xsc[v] * cu;
                t += xsc[v] * (bd1 * cu - bo1 * nb);
                tn[q][v] = (has_t && w[q] != 0.0) ? static_cast<T>(t) : zero;
            }
        // out at plane z-1 on lines 0..3
        if (z >= 1) {
            const double znt = has_t ? 1.0 : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double o[VW];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    auto tat = [&](int r) -> double {
                        return r < 4 ? (double)tm1[r][v] : (double)r1[r - 4][v];
                    };
                    const double nb = (double)tm2[q][v] + znt * (double)tn[q][v] + tat(NYM[q]) +
                                      tat(NYP[q]) + tat(NXM[q]) + tat(NXP[q]);
                    double val = c2 * xsc[v] * (double)um[q][v];
                    val += 1.0 * (bd2 * (double)tm1[q][v] - bo2 * nb);
                    if (HASZ) val -= cz * (double)S.zv[q][v];
                    o[v] = val;
                }
                if (w[q] != 0.0) vstore<T, VW>(out, ep + off[q], o);
            }
        }
        // advance one plane
#pragma unroll
        for (int v = 0; v < VW; ++v) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                tm2[q][v] = tm1[q][v];
                tm1[q][v] = tn[q][v];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) r1[q][v] = tn[4 + q][v];
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                um[q][v] = u0[q][v];
                u0[q][v] = w[q] != 0.0 ? S.un[q][v] : zero;
            }
        }
    };
    for (int z = 0; z <= d2; ++z) {
        StepLoads S;
        issue(S, z);
        __builtin_amdgcn_sched_barrier(0);
        compute(S, z);
    }
}

// ---- the same quadratic factor, workgroup-cooperative ----
// Sixteen wavefronts share one 8 x 8 block of z-lines for 64*VW columns: each
// owns a 2 x 2 quadrant of output lines and two of the 32 lines of the
// distance-1 ring around the block (where t is needed too).  Per z value the
// block's u on every line within distance 2 (132 lines) and its t on the block
// and ring (96 lines) pass through LDS, so every u line is loaded from memory
// once per workgroup instead of once per neighbouring quadrant.  The u values
// of a wavefront's own lines are loaded two z values ahead.  Two barriers per
// z value; every wavefront runs the same number of iterations and reaches
// every barrier.
namespace quadwg {
// the 32 lines at distance 1 and the 36 at distance 2 from the 8 x 8 block
constexpr int R1I[32] = {-1, -1, -1, -1, -1, -1, -1, -1, 8, 8, 8, 8, 8, 8, 8, 8,
                         0,  1,  2,  3,  4,  5,  6,  7, 0, 1, 2, 3, 4, 5, 6, 7};
constexpr int R1J[32] = {0,  1,  2,  3,  4,  5,  6,  7,  0, 1, 2, 3, 4, 5, 6, 7,
                         -1, -1, -1, -1, -1, -1, -1, -1, 8, 8, 8, 8, 8, 8, 8, 8};
constexpr int R2I[36] = {-2, -2, -2, -2, -2, -2, -2, -2, 9, 9, 9, 9, 9, 9, 9, 9, 0, 1,
                         2,  3,  4,  5,  6,  7,  0,  1, 2, 3, 4, 5, 6, 7, -1, -1, 8, 8};
constexpr int R2J[36] = {0, 1, 2, 3, 4,  5,  6,  7,  0,  1,  2,  3,  4, 5, 6, 7, -2, -2,
                         -2, -2, -2, -2, -2, -2, 9, 9, 9, 9, 9, 9, 9, 9, -1, 8, -1, 8};
constexpr int UW = 12;   // u plane: (i, j) in [-2, 10)^2 at (i + 2) * UW + (j + 2)
constexpr int TW = 10;   // t plane: (i, j) in [-1, 9)^2 at (i + 1) * TW + (j + 1)
}  // namespace quadwg

template <typename T, int VW, bool HASZ>
__global__ __launch_bounds__(1024) void k_quad_sweep_wg(int C, int ncg, int nseg,
                                                        const int64_t *__restrict__ seg_row,
                                                        const int64_t *__restrict__ seg_tile,
                                                        const int32_t *__restrict__ seg_dims,
                                                        int64_t ntiles, const T *__restrict__ X,
                                                        const double *__restrict__ xs_all,
                                                        double c1, double bd1, double bo1, double c2,
                                                        double bd2, double bo2,
                                                        const T *__restrict__ Z, double cz,
                                                        T *__restrict__ out)
{
    using namespace quadwg;
    using V = typename VecT<T, VW>::type;
    // arithmetic in the storage type: FP32 storage already bounds the FP32
    // form's accuracy, and FP64 temporaries for two columns per lane would
    // not fit the 128 registers that sixteen wavefronts per CU leave
    using R = T;
    const R rc1 = (R)c1, rbd1 = (R)bd1, rbo1 = (R)bo1, rc2 = (R)c2, rbd2 = (R)bd2, rbo2 = (R)bo2,
            rcz = (R)cz;
    constexpr int NT = 6;   // lines of a wavefront: 4 of its quadrant, 2 of the ring
    __shared__ V su[UW * UW * 64];
    __shared__ V stp[TW * TW * 64];
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int cg = (int)(L / ntiles);   // column-group-major
    const int64_t tile = L % ntiles;
    const int wv = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
    // lanes past the last column load column 0 and store nothing, and take
    // part in every barrier
    const int craw = (cg * 64 + lane) * VW;
    const bool colok = craw < C;
    const int c0 = colok ? craw : 0;
    const int seg = find_seg(seg_tile, nseg, tile);
    const int d0 = seg_dims[3 * seg], d1 = seg_dims[3 * seg + 1], d2 = seg_dims[3 * seg + 2];
    const int nty = (d1 + 7) / 8;
    const int lt = (int)(tile - seg_tile[seg]);
    const int bx = (lt / nty) * 8, by = (lt % nty) * 8;   // block origin (inside the grid)
    const double *xs = xs_all ? xs_all + (size_t)seg * C : nullptr;
    const int64_t zs = C, ys = (int64_t)d2 * C, xst = (int64_t)d1 * d2 * C;
    const int64_t base = (int64_t)seg_row[seg] * C + (int64_t)bx * xst + (int64_t)by * ys + c0;
    auto inside = [&](int i, int j) { return bx + i < d0 && by + j < d1 && bx + i >= 0 && by + j >= 0; };
    auto offset = [&](int i, int j) -> int64_t {
        return inside(i, j) ? (int64_t)i * xst + (int64_t)j * ys : 0;
    };
    auto ldT = [&](int64_t e, T (&o)[VW]) {
        const V x = *reinterpret_cast<const V *>(X + e);
        if constexpr (VW == 1) {
            o[0] = x;
        } else {
            o[0] = x.x;
            o[1] = x.y;
        }
    };
    auto toV = [](const T (&a)[VW]) {
        V v;
        if constexpr (VW == 1) {
            v = a[0];
        } else {
            v.x = a[0];
            v.y = a[1];
        }
        return v;
    };
    auto fromV = [](const V &v, int e) -> R {
        if constexpr (VW == 1) {
            (void)e;
            return (R)v;
        } else {
            return (R)(e == 0 ? v.x : v.y);
        }
    };
    const T zero = T(0);
    const int qx = wv >> 2, qy = wv & 3;
    int LI[NT], LJ[NT];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        LI[q] = 2 * qx + (q >> 1);
        LJ[q] = 2 * qy + (q & 1);
    }
#pragma unroll
    for (int q = 4; q < NT; ++q) {
        LI[q] = R1I[2 * wv + q - 4];
        LJ[q] = R1J[2 * wv + q - 4];
    }
    int64_t off[NT];
    double w[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        off[q] = offset(LI[q], LJ[q]);
        w[q] = inside(LI[q], LJ[q]) ? 1.0 : 0.0;
    }
    // ring-2 share
    int64_t off2[3];
    double w2[3];
    int slot2[3];
    bool has2[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int r = wv + 16 * s;
        has2[s] = r < 36;
        const int i = has2[s] ? R2I[r] : 0, j = has2[s] ? R2J[r] : 0;
        off2[s] = has2[s] ? offset(i, j) : 0;
        w2[s] = has2[s] && inside(i, j) ? 1.0 : 0.0;
        slot2[s] = (i + 2) * UW + (j + 2);
    }
    R xsc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) xsc[v] = xs ? (R)xs[c0 + v] : R(1);
    // u of the own lines at z-1, z, z+1 (um, u0, un); ring-2 u at z (r2)
    T um[NT][VW], u0[NT][VW], un[NT][VW], r2[3][VW], tm2[4][VW], tm1[4][VW];
    const int64_t e1 = d2 > 1 ? zs : 0;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        T a[VW], b[VW];
        ldT(base + off[q], a);
        ldT(base + e1 + off[q], b);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            um[q][v] = zero;
            u0[q][v] = w[q] != 0.0 ? a[v] : zero;
            un[q][v] = (w[q] != 0.0 && d2 > 1) ? b[v] : zero;
        }
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        T a[VW];
        ldT(base + off2[s], a);
#pragma unroll
        for (int v = 0; v < VW; ++v) r2[s][v] = w2[s] != 0.0 ? a[v] : zero;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) tm2[q][v] = tm1[q][v] = zero;
    for (int z = 0; z <= d2; ++z) {
        const bool has_t = z < d2, has_n = z + 1 < d2, has_nn = z + 2 < d2;
        const int64_t enn = has_nn ? (int64_t)(z + 2) * zs : 0;
        const int64_t en = has_n ? (int64_t)(z + 1) * zs : 0;
        const int64_t ep = z >= 1 ? (int64_t)(z - 1) * zs : 0;
        // loads in flight during this z value: own lines at z+2, ring 2 at z+1, Z at z-1
        T unn[NT][VW], r2n[3][VW], zv[4][VW];
#pragma unroll
        for (int q = 0; q < NT; ++q) ldT(base + enn + off[q], unn[q]);
#pragma unroll
        for (int s = 0; s < 3; ++s) ldT(base + en + off2[s], r2n[s]);
        if (HASZ) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const V zz = *reinterpret_cast<const V *>(Z + base + ep + off[q]);
                if constexpr (VW == 1) {
                    zv[q][0] = zz;
                } else {
                    zv[q][0] = zz.x;
                    zv[q][1] = zz.y;
                }
            }
        }
        // u at z into the shared plane
        if (has_t) {
#pragma unroll
            for (int q = 0; q < NT; ++q)
                su[((LI[q] + 2) * UW + (LJ[q] + 2)) * 64 + lane] = toV(u0[q]);
#pragma unroll
            for (int s = 0; s < 3; ++s)
                if (has2[s]) su[slot2[s] * 64 + lane] = toV(r2[s]);
        }
        __syncthreads();
        // t at z on this wavefront's lines
        const R zn = has_n ? R(1) : R(0);
        T tn[NT][VW];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            if (!has_t) {
#pragma unroll
                for (int v = 0; v < VW; ++v) tn[q][v] = zero;
                continue;
            }
            const int i = LI[q], j = LJ[q];
            // lateral neighbours: inside the wavefront's own quadrant from
            // registers (the same values it wrote to the plane), else from LDS
            const bool qd = q < 4;
            const bool in_ym = qd && (q & 1), in_yp = qd && !(q & 1);
            const bool in_xm = qd && (q >> 1), in_xp = qd && !(q >> 1);
            V vym, vyp, vxm, vxp;
            if (!in_ym) vym = su[((i + 2) * UW + (j + 1)) * 64 + lane];
            if (!in_yp) vyp = su[((i + 2) * UW + (j + 3)) * 64 + lane];
            if (!in_xm) vxm = su[((i + 1) * UW + (j + 2)) * 64 + lane];
            if (!in_xp) vxp = su[((i + 3) * UW + (j + 2)) * 64 + lane];
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const R cu = u0[q][v];
                const R uym = in_ym ? (R)u0[q - 1][v] : fromV(vym, v);
                const R uyp = in_yp ? (R)u0[q + 1][v] : fromV(vyp, v);
                const R uxm = in_xm ? (R)u0[q - 2][v] : fromV(vxm, v);
                const R uxp = in_xp ? (R)u0[q + 2][v] : fromV(vxp, v);
                const R nb = (R)um[q][v] + zn * (R)un[q][v] + uym + uyp + uxm + uxp;
                R t = rc1 * xsc[v] * cu;
                t += xsc[v] * (rbd1 * cu - rbo1 * nb);
                tn[q][v] = w[q] != 0.0 ? static_cast<T>(t) : zero;
            }
        }
        // out at z-1 on the quadrant (t at z-1 of the neighbours outside it from LDS)
        if (z >= 1) {
            const R znt = has_t ? R(1) : R(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = LI[q], j = LJ[q];
                const bool in_ym = q & 1, in_xm = q >> 1;   // the other two are in the quadrant too
                V tym, typ, txm, txp;
                if (!in_ym) tym = stp[((i + 1) * TW + j) * 64 + lane];
                if (in_ym) typ = stp[((i + 1) * TW + (j + 2)) * 64 + lane];
                if (!in_xm) txm = stp[(i * TW + (j + 1)) * 64 + lane];
                if (in_xm) txp = stp[((i + 2) * TW + (j + 1)) * 64 + lane];
                double o[VW];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const R tyn = in_ym ? (R)tm1[q - 1][v] : fromV(tym, v);
                    const R typn = in_ym ? fromV(typ, v) : (R)tm1[q + 1][v];
                    const R txn = in_xm ? (R)tm1[q - 2][v] : fromV(txm, v);
                    const R txpn = in_xm ? fromV(txp, v) : (R)tm1[q + 2][v];
                    const R nb = (R)tm2[q][v] + znt * (R)tn[q][v] + tyn + typn + txn + txpn;
                    R val = rc2 * xsc[v] * (R)um[q][v];
                    val += R(1) * (rbd2 * (R)tm1[q][v] - rbo2 * nb);
                    if (HASZ) val -= rcz * (R)zv[q][v];
                    o[v] = (double)val;
                }
                if (w[q] != 0.0 && colok) vstore_nt<T, VW>(out, base + ep + off[q], o);
            }
        }
        __syncthreads();
        // t at z into the shared plane
        if (has_t) {
#pragma unroll
            for (int q = 0; q < NT; ++q)
                stp[((LI[q] + 1) * TW + (LJ[q] + 1)) * 64 + lane] = toV(tn[q]);
        }
        // advance one z value
#pragma unroll
        for (int v = 0; v < VW; ++v) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                tm2[q][v] = tm1[q][v];
                tm1[q][v] = tn[q][v];
            }
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                um[q][v] = u0[q][v];
                u0[q][v] = un[q][v];
                un[q][v] = (w[q] != 0.0 && has_nn) ? unn[q][v] : zero;
            }
#pragma unroll
            for (int s = 0; s < 3; ++s) r2[s][v] = (w2[s] != 0.0 && has_n) ? r2n[s][v] : zero;
        }
    }
}

// ---- A as a grid stencil ----
// A of the form L_off + diag(d) on each problem's grid (the (2*ndim+1)-point
// pattern, every off-diagonal entry equal to one value a_off, any diagonal:
// a kinetic stencil plus a local potential) is applied by a z-march like
// k_stencil instead of row by row: the x rows of neighbouring grid planes
// then come from registers and from the L2 copies of neighbouring line
// blocks rather than from HBM again.
//
// k_stencil_check verifies, per row, that its CSR entries are exactly the
// in-grid neighbours and the diagonal in ascending column order and that the
// off-diagonal values equal a_off (the first off-diagonal of row ref_row, the
// first row of the first problem with more than one row); it copies the
// diagonal to `diag` and a_off to coff[0].  Any mismatch sets flags[2]:
// the CSR sweep then applies A instead (both kernels read the flag).
template <typename VT>
__global__ __launch_bounds__(256) void k_stencil_check(int64_t n, int nseg,
                                                       const int64_t *__restrict__ seg_row,
                                                       const int32_t *__restrict__ seg_dims,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const VT *__restrict__ val, int64_t ref_row,
                                                       double *__restrict__ diag,
                                                       double *__restrict__ coff,
                                                       int32_t *__restrict__ flags)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    // the reference row has its diagonal and at least one neighbour when A is of the form
    const bool refok = ref_row < 0 || rp[ref_row + 1] - rp[ref_row] >= 2;
    const double ref = (ref_row >= 0 && refok) ? static_cast<double>(val[rp[ref_row] + 1]) : 0.0;
    if (r == 0) coff[0] = ref;
    if (!refok) atomicOr(&flags[2], 1);
    const int seg = find_seg(seg_row, nseg, r);
    const int64_t d0 = seg_dims[3 * seg], d1 = seg_dims[3 * seg + 1], d2 = seg_dims[3 * seg + 2];
    const int64_t rl = r - seg_row[seg];
    const int64_t x = rl / (d1 * d2), y = (rl / d2) % d1, z = rl % d2;
    // expected columns in ascending order; slot 3 is the diagonal
    int64_t col[7];
    bool has[7];
    has[0] = x > 0;      col[0] = r - d1 * d2;
    has[1] = y > 0;      col[1] = r - d2;
    has[2] = z > 0;      col[2] = r - 1;
    has[3] = true;       col[3] = r;
    has[4] = z < d2 - 1; col[4] = r + 1;
    has[5] = y < d1 - 1; col[5] = r + d2;
    has[6] = x < d0 - 1; col[6] = r + d1 * d2;
    int cnt = 0;
    for (int k = 0; k < 7; ++k) cnt += has[k] ? 1 : 0;
    const int32_t p0 = rp[r], len = rp[r + 1] - p0;
    bool ok = len == cnt;
    double dg = 0.0;
    if (ok) {
        int p = p0;
        for (int k = 0; k < 7; ++k) {
            if (!has[k]) continue;
            const double v = static_cast<double>(val[p]);
            ok = ok && ci[p] == col[k];
            if (k == 3) dg = v;
            else ok = ok && v == ref;
            ++p;
        }
    }
    diag[r] = dg;
    if (!ok) atomicOr(&flags[2], 1);
}

// y = xs_c * ((A - tau_c I) x) with A = a_off * (grid neighbours) + diag(d),
// summed in the order the CSR sweep sums a row (ascending columns, then the
// shift), so both forms give the same values.  Line blocks as in k_stencil;
// a tile of QX*TX by QY*TY lines is split into QX*QY wavefronts, and the z
// range into nzc chunks (a wavefront per chunk, starting from its own z-1
// plane): more wavefronts in flight for the same loads.  Wavefront order:
// column group, z chunk, tile, quadrant (fastest), so that neighbouring line
// blocks at the same z run together and share their boundary lines in L2.
// Runs only when k_stencil_check found the stencil form (flags[2] == 0).
template <typename T, int VW, int TX, int TY, int QX, int QY>
__global__ __launch_bounds__(256) void k_stencil_a(int C, int m, int c_off, int ncg, int nzc, int S,
                                                   int nseg,
                                                   const int64_t *__restrict__ seg_row,
                                                   const int64_t *__restrict__ seg_tile,
                                                   const int32_t *__restrict__ seg_dims,
                                                   int64_t ntiles, const T *__restrict__ IN,
                                                   const double *__restrict__ xs_all,
                                                   const double *__restrict__ diag,
                                                   const double *__restrict__ coff,
                                                   const double *__restrict__ seg_taus,
                                                   const int32_t *__restrict__ flags,
                                                   T *__restrict__ out)
{
    if (flags[2] != 0) return;
    constexpr int Q = QX * QY;
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t gw = L * 4 + uniform(threadIdx.x >> 6);
    const int64_t per_zc = ntiles * Q;
    const int64_t czc = gw / per_zc;   // cg * nzc + zc
    const int cg = (int)(czc / nzc), zc = (int)(czc % nzc);
    if (cg >= ncg) return;
    const int64_t rem = gw % per_zc;
    const int64_t tile = rem / Q;
    const int q = (int)(rem % Q);
    const int lane = threadIdx.x & 63;
    const int c0 = (cg * 64 + lane) * VW;
    if (c0 >= C) return;
    const int seg = find_seg(seg_tile, nseg, tile);
    const int d0 = seg_dims[3 * seg], d1 = seg_dims[3 * seg + 1], d2 = seg_dims[3 * seg + 2];
    const int zlen = (d2 + nzc - 1) / nzc;
    const int za = zc * zlen, zb = min(d2, za + zlen);
    if (za >= zb) return;
    const int nty = (d1 + QY * TY - 1) / (QY * TY);
    const int lt = (int)(tile - seg_tile[seg]);
    const int x0 = (lt / nty) * (QX * TX) + (q % QX) * TX;
    const int y0 = (lt % nty) * (QY * TY) + (q / QX) * TY;
    if (x0 >= d0 || y0 >= d1) return;
    const double *xs = xs_all ? xs_all + (size_t)seg * C : nullptr;
    const double aoff = coff[0];
    const size_t zs = (size_t)C, ys = (size_t)d2 * C, xs_ = (size_t)d1 * d2 * C;
    const int64_t row0 = seg_row[seg] + (int64_t)x0 * d1 * d2 + (int64_t)y0 * d2;
    const size_t base = (size_t)row0 * C + c0;
    size_t off[TX][TY];
    int64_t roff[TX][TY];
    double wt[TX][TY];
    size_t offym[TX], offyp[TX], offxm[TY], offxp[TY];
    double wym[TX], wyp[TX], wxm[TY], wxp[TY];
#pragma unroll
    for (int a = 0; a < TX; ++a)
#pragma unroll
        for (int b = 0; b < TY; ++b) {
            const bool ok = x0 + a < d0 && y0 + b < d1;
            off[a][b] = ok ? (size_t)a * xs_ + (size_t)b * ys : 0;
            roff[a][b] = ok ? (int64_t)a * d1 * d2 + (int64_t)b * d2 : 0;
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
    double xsc[VW], tau[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        xsc[v] = xs ? xs[c0 + v] : 1.0;
        tau[v] = seg_taus[(size_t)seg * S + (c_off + c0 + v) / m];
    }
    double prev[TX][TY][VW], cur[TX][TY][VW];
    const double wpv = za > 0 ? 1.0 : 0.0;
    const size_t epv = za > 0 ? (size_t)(za - 1) * zs : 0;
#pragma unroll
    for (int a = 0; a < TX; ++a)
#pragma unroll
        for (int b = 0; b < TY; ++b) {
            double t[VW], tp[VW];
            vload<T, VW>(IN, base + (size_t)za * zs + off[a][b], t);
            vload<T, VW>(IN, base + epv + off[a][b], tp);
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                prev[a][b][v] = wpv * wt[a][b] * tp[v];
                cur[a][b][v] = wt[a][b] * t[v];
            }
        }
    struct StepLoads {
        double nxt[TX][TY][VW], ym[TX][VW], yp[TX][VW], xm[TY][VW], xp[TY][VW], dg[TX][TY];
    };
    auto issue = [&](StepLoads &Ld, int z) {
        const size_t ez = base + (size_t)z * zs;
        const size_t en = z + 1 < d2 ? ez + zs : ez;
#pragma unroll
        for (int a = 0; a < TX; ++a)
#pragma unroll
            for (int b = 0; b < TY; ++b) vload<T, VW>(IN, en + off[a][b], Ld.nxt[a][b]);
#pragma unroll
        for (int a = 0; a < TX; ++a) {
            vload<T, VW>(IN, ez + offym[a], Ld.ym[a]);
            vload<T, VW>(IN, ez + offyp[a], Ld.yp[a]);
        }
#pragma unroll
        for (int b = 0; b < TY; ++b) {
            vload<T, VW>(IN, ez + offxm[b], Ld.xm[b]);
            vload<T, VW>(IN, ez + offxp[b], Ld.xp[b]);
        }
#pragma unroll
        for (int a = 0; a < TX; ++a)
#pragma unroll
            for (int b = 0; b < TY; ++b) Ld.dg[a][b] = diag[row0 + roff[a][b] + z];
    };
    auto compute = [&](const StepLoads &Ld, int z) {
        const size_t ez = base + (size_t)z * zs;
        const double zn = z + 1 < d2 ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < TX; ++a)
#pragma unroll
            for (int b = 0; b < TY; ++b) {
                double o[VW];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const double nxm = a > 0 ? cur[a - 1][b][v] : wxm[b] * Ld.xm[b][v];
                    const double nym = b > 0 ? cur[a][b - 1][v] : wym[a] * Ld.ym[a][v];
                    const double nyp = b + 1 < TY ? cur[a][b + 1][v] : wyp[a] * Ld.yp[a][v];
                    const double nxp = a + 1 < TX ? cur[a + 1][b][v] : wxp[b] * Ld.xp[b][v];
                    double acc = 0.0;
                    acc += aoff * nxm;
                    acc += aoff * nym;
                    acc += aoff * prev[a][b][v];
                    acc += Ld.dg[a][b] * cur[a][b][v];
                    acc += aoff * (zn * Ld.nxt[a][b][v]);
                    acc += aoff * nyp;
                    acc += aoff * nxp;
                    const double r = acc - tau[v] * cur[a][b][v];
                    o[v] = r * xsc[v];
                }
                if (wt[a][b] != 0.0) vstore_nt<T, VW>(out, ez + off[a][b], o);
            }
#pragma unroll
        for (int a = 0; a < TX; ++a)
#pragma unroll
            for (int b = 0; b < TY; ++b)
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    prev[a][b][v] = cur[a][b][v];
                    cur[a][b][v] = wt[a][b] * Ld.nxt[a][b][v];
                }
    };
    for (int z = za; z < zb; ++z) {
        StepLoads Ld;
        issue(Ld, z);
        __builtin_amdgcn_sched_barrier(0);
        compute(Ld, z);
    }
}

// z chunks of the stencil sweeps: enough wavefronts to keep about 32 per CU
// busy, at least 8 planes per chunk
static int z_chunks(const Plan &p, int64_t waves)
{
    const int64_t want = (8192 + waves - 1) / (waves > 0 ? waves : 1);
    int nzc = (int)(want < 64 ? want : 64);
    const int maxc = p.max_d2 / 8 > 0 ? p.max_d2 / 8 : 1;
    if (nzc > maxc) nzc = maxc;
    return nzc < 1 ? 1 : nzc;
}

void launch_stencil_check(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx,
                          const void *val, hipStream_t st)
{
    dim3 grid((unsigned)((p.n + 255) / 256));
    if (p.val_f32)
        k_stencil_check<float><<<grid, 256, 0, st>>>(p.n, p.nseg, p.seg_row, p.seg_dims, row_ptr,
                                                     col_idx, (const float *)val, p.st_ref_row,
                                                     p.st_diag, p.st_coff, p.flags);
    else
        k_stencil_check<double><<<grid, 256, 0, st>>>(p.n, p.nseg, p.seg_row, p.seg_dims, row_ptr,
                                                      col_idx, (const double *)val, p.st_ref_row,
                                                      p.st_diag, p.st_coff, p.flags);
}

template <typename T, int VW, int TX, int TY, int QX, int QY>
static void stencil_a_t(const Plan &p, const void *x, const double *xs, void *y, hipStream_t st)
{
    const int ncg = (p.C + 64 * VW - 1) / (64 * VW);
    const int64_t waves1 = p.ntiles * QX * QY * ncg;
    const int nzc = z_chunks(p, waves1);
    const int64_t waves = waves1 * nzc;
    k_stencil_a<T, VW, TX, TY, QX, QY><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(
        p.C, p.m, p.c_off, ncg, nzc, p.S, p.nseg, p.seg_row, p.seg_tile, p.seg_dims, p.ntiles,
        (const T *)x, xs, p.st_diag, p.st_coff, p.seg_taus, p.flags, (T *)y);
}

template <typename T, int VW>
static void stencil_a_shape(const Plan &p, const void *x, const double *xs, void *y, hipStream_t st)
{
    if (p.tx == 8) stencil_a_t<T, VW, 2, 4, 4, 2>(p, x, xs, y, st);   // 8 x 8 tiles: eight 2 x 4 blocks
    else if (p.tx == 4) stencil_a_t<T, VW, 4, 4, 1, 1>(p, x, xs, y, st);
    else if (p.tx == 2) stencil_a_t<T, VW, 2, 4, 1, 1>(p, x, xs, y, st);
    else stencil_a_t<T, VW, 1, 8, 1, 1>(p, x, xs, y, st);
}

void launch_stencil_a(const Plan &p, const void *x, const double *xs, void *y, hipStream_t st)
{
    // one column per lane (FP64) / two (FP32, when the width is even), as the plain sweep
    if (p.vec_f32 && p.C % 2 == 0) stencil_a_shape<float, 2>(p, x, xs, y, st);
    else if (p.vec_f32) stencil_a_shape<float, 1>(p, x, xs, y, st);
    else stencil_a_shape<double, 1>(p, x, xs, y, st);
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

// Measured shapes: 8-byte columns two per lane, two rows per wave, 8-nonzero
// chunks, linear block order; 4-byte columns four per lane, one row per wave,
// 4-nonzero chunks, XCD-remapped order.
template <typename T, typename VT, int VW, int RPW = (VW == 4 ? 1 : 2), int NZ = (VW == 4 ? 4 : 8)>
static void csr_op_t(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                     const void *x, const double *xs, const double *jac, void *y, hipStream_t st,
                     const int32_t *gate, int remap = (VW == 4 ? 1 : 0))
{
    const int ncg = (p.C + 64 * VW - 1) / (64 * VW);
    dim3 grid((unsigned)(((p.n + 4 * RPW - 1) / (4 * RPW)) * ncg));
    if (jac)
        k_csr_op<T, VT, true, VW, RPW, NZ><<<grid, 256, 0, st>>>(
            p.n, p.C, p.m, p.c_off, ncg, p.S, p.nseg, p.seg_row, rp, ci, (const VT *)val,
            (const T *)x, xs, jac, p.seg_taus, (T *)y, remap, gate);
    else
        k_csr_op<T, VT, false, VW, RPW, NZ><<<grid, 256, 0, st>>>(
            p.n, p.C, p.m, p.c_off, ncg, p.S, p.nseg, p.seg_row, rp, ci, (const VT *)val,
            (const T *)x, xs, nullptr, p.seg_taus, (T *)y, remap, gate);
}

template <typename T, typename VT>
static void csr_op_vw(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                      const void *x, const double *xs, const double *jac, void *y, hipStream_t st,
                      const int32_t *gate)
{
    if constexpr (sizeof(T) == 4) {
        if (p.vw == 4) {
            csr_op_t<T, VT, 4>(p, rp, ci, val, x, xs, jac, y, st, gate);
            return;
        }
    }
    if (p.vw == 2) csr_op_t<T, VT, 2>(p, rp, ci, val, x, xs, jac, y, st, gate);
    else csr_op_t<T, VT, 1>(p, rp, ci, val, x, xs, jac, y, st, gate);
}

void launch_csr_op(const Plan &p, const int32_t *rp, const int32_t *ci, const void *val,
                   const void *x, const double *xs, const double *jac, void *y, hipStream_t st,
                   const int32_t *gate)
{
    if (p.vec_f32) {
        if (p.val_f32) csr_op_vw<float, float>(p, rp, ci, val, x, xs, jac, y, st, gate);
        else csr_op_vw<float, double>(p, rp, ci, val, x, xs, jac, y, st, gate);
    } else {
        if (p.val_f32) csr_op_vw<double, float>(p, rp, ci, val, x, xs, jac, y, st, gate);
        else csr_op_vw<double, double>(p, rp, ci, val, x, xs, jac, y, st, gate);
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

namespace ecnt {

template <typename T, int VW, bool HASZ>
static void quad_sweep_t(const Plan &p, const void *X, const double *xs, double c1, double bd1,
                   double bo1, double c2, double bd2, double bo2, const void *Z, double cz,
                   void *out, hipStream_t st)
{
    const int ncg = (p.C + 64 * VW - 1) / (64 * VW);
    dim3 grid((unsigned)(p.ntiles * ncg));
    k_quad_sweep<T, VW, HASZ><<<grid, 256, 0, st>>>(p.C, ncg, p.nseg, p.seg_row, p.seg_tile,
                                                    p.seg_dims, p.ntiles, (const T *)X, xs, c1,
                                                    bd1, bo1, c2, bd2, bo2, (const T *)Z, cz,
                                                    (T *)out);
}

template <typename T, int VW, bool HASZ>
static void quad_sweep_wg_t(const Plan &p, const void *X, const double *xs, double c1, double bd1,
                            double bo1, double c2, double bd2, double bo2, const void *Z, double cz,
                            void *out, hipStream_t st)
{
    const int ncg = (p.C + 64 * VW - 1) / (64 * VW);
    dim3 grid((unsigned)(p.ntiles * ncg));
    k_quad_sweep_wg<T, VW, HASZ><<<grid, 1024, 0, st>>>(p.C, ncg, p.nseg, p.seg_row, p.seg_tile,
                                                        p.seg_dims, p.ntiles, (const T *)X, xs, c1,
                                                        bd1, bo1, c2, bd2, bo2, (const T *)Z, cz,
                                                        (T *)out);
}

bool quad_sweep_supported(const Plan &p)
{
    return ((p.tx == 4 && p.ty == 4) || (p.tx == 8 && p.ty == 8)) && !p.no_fuse;
}

void launch_quad_sweep(const Plan &p, const void *X, const double *xs, double c1, double cb,
                       double c2, const void *Z, double cz, void *out, hipStream_t st)
{
    const double w = p.hi - p.lo;
    const double bd = (2.0 * (2.0 * p.ndim + p.s) - (p.lo + p.hi)) / w;
    const double bo = 2.0 / w;
    const double bd1 = cb * bd, bo1 = cb * 2.0 / w;
    if (p.tx == 8) {   // workgroup-cooperative form on 8 x 8 line blocks, one column per lane
        // (two in FP32 when the width is even: the planes then take what FP64's do)
        if (p.vec_f32 && p.C % 2 == 0) {
            if (Z) quad_sweep_wg_t<float, 2, true>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
            else quad_sweep_wg_t<float, 2, false>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
        } else if (p.vec_f32) {
            if (Z) quad_sweep_wg_t<float, 1, true>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
            else quad_sweep_wg_t<float, 1, false>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
        } else {
            if (Z) quad_sweep_wg_t<double, 1, true>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
            else quad_sweep_wg_t<double, 1, false>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
        }
        return;
    }
    if (p.vec_f32 && p.C % 2 == 0) {
        if (Z) quad_sweep_t<float, 2, true>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
        else quad_sweep_t<float, 2, false>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
    } else if (p.vec_f32) {
        if (Z) quad_sweep_t<float, 1, true>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
        else quad_sweep_t<float, 1, false>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
    } else {
        if (Z) quad_sweep_t<double, 1, true>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
        else quad_sweep_t<double, 1, false>(p, X, xs, c1, bd1, bo1, c2, bd, bo, Z, cz, out, st);
    }
}

}  // namespace ecnt
