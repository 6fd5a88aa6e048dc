// Lanczos recurrence with full reorthogonalization on a block of independent
// probe columns (Algorithm 1; Section 3.2, the probe loop of Algorithm 2 run
// data-parallel over columns).
//
// Step i of Algorithm 1, per column c (q_l = sig_{l-1} * slot_{l-1}):
//   y      = C q_i                                (operator kernels, into slot i)
//   w      = y - beta_i q_{i-1}
//   g_l    = q_l^T w,  l = 1..i;  alpha_i = g_i   (k_dots + k_dots_fin)
//   w     <- w - sum_l g_l q_l                    (k_update, in place in slot i)
//   beta_{i+1} = |w|; sig_i = 1/beta_{i+1}        (k_norm_fin)
// The single Gram-Schmidt pass against q_1..q_i (including q_i) also removes
// the alpha_i q_i component: the result differs from "alpha first, then
// reorthogonalize" only by rounding, since q_l^T q_i = delta_li + O(eps).
//
// Column reductions are two-phase and deterministic: each workgroup writes
// the partial sums of its row chunk, a finalize kernel adds them in chunk
// order.  No floating-point atomics.
#include <float.h>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

// ---- probe setup: slot 0 = v (for every shift), partial |v|^2 ----
template <typename T>
__global__ __launch_bounds__(256) void k_setup(int64_t n, int C, int m, int c_off, int nct,
                                               int64_t rpc, const T *__restrict__ V,
                                               T *__restrict__ slot0, double *__restrict__ part)
{
    __shared__ double red[4][kColTile];
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = ct * kColTile + lane;
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    double acc = 0.0;
    if (c < C) {
        const int j = (c_off + c) % m;
        for (int64_t r = r0 + wv; r < r1; r += 4) {
            const T v = V[(size_t)r * m + j];
            slot0[(size_t)r * C + c] = v;
            const double dv = static_cast<double>(v);
            acc += dv * dv;
        }
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && c < C)
        part[(size_t)chunk * kPartRows * C + c] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

__global__ void k_setup_fin(int C, int k, int nchunk, const double *__restrict__ part,
                            double *__restrict__ nu, double *__restrict__ sig,
                            double *__restrict__ kappa, double *__restrict__ runmax,
                            double *__restrict__ beta, int32_t *__restrict__ active,
                            int32_t *__restrict__ kused)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[(size_t)ch * kPartRows * C + c];
    nu[c] = s;
    const bool ok = s > 0.0;
    sig[c] = ok ? 1.0 / sqrt(s) : 0.0;
    kappa[c] = 0.0;
    runmax[c] = 0.0;
    beta[c] = 0.0;   // beta_1 = 0 (Algorithm 1, first step)
    active[c] = ok ? 1 : 0;
    kused[c] = ok ? k : 0;
}

// ---- reorthogonalization dots: part[chunk][l][c] = sum_rows slot_{l0+l} * w ----
// One wavefront per (row chunk, column tile); NB is the exact number of basis
// vectors of the launch, so all NB + 2 row loads are issued back to back.
template <typename T, int NB, int VW>
__global__ __launch_bounds__(64) void k_dots(int64_t n, int C, int nct, int64_t rpc,
                                             const T *__restrict__ basis, size_t ss, int slot_y,
                                             int l0, int slot_m, const double *__restrict__ kappa,
                                             double *__restrict__ part)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int c0 = (ct * 64 + (int)threadIdx.x) * VW;
    if (c0 >= C) return;
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    double acc[NB][VW];
#pragma unroll
    for (int l = 0; l < NB; ++l)
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[l][v] = 0.0;
    double kap[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) kap[v] = slot_m >= 0 ? kappa[c0 + v] : 0.0;
    const T *Y = basis + (size_t)slot_y * ss;
    const T *Qm = basis + (size_t)(slot_m >= 0 ? slot_m : 0) * ss;
    const T *Q0 = basis + (size_t)l0 * ss;
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c0;
        double y[VW], qm[VW], q[NB][VW];
        vload<T, VW>(Y, e, y);
        vload<T, VW>(Qm, e, qm);
#pragma unroll
        for (int l = 0; l < NB; ++l) vload<T, VW>(Q0 + (size_t)l * ss, e, q[l]);
        // keep all NB + 2 loads of the row in flight before the first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const double w = y[v] - kap[v] * qm[v];
#pragma unroll
            for (int l = 0; l < NB; ++l) acc[l][v] += q[l][v] * w;
        }
    }
#pragma unroll
    for (int l = 0; l < NB; ++l)
#pragma unroll
        for (int v = 0; v < VW; ++v)
            part[((size_t)chunk * kPartRows + l) * C + c0 + v] = acc[l][v];
}

// g_l = sig_l * sum_chunks part; cf_l = g_l * sig_l; alpha_i = g_i.
__global__ void k_dots_fin(int C, int nchunk, int step, int l0, int nb, int k,
                           const double *__restrict__ part, const double *__restrict__ sig,
                           const int32_t *__restrict__ active, double *__restrict__ cf,
                           double *__restrict__ alpha, double *__restrict__ gall)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * C) return;
    const int l = idx / C, c = idx % C;
    double s = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[((size_t)ch * kPartRows + l) * C + c];
    const double sg = sig[(size_t)(l0 + l) * C + c];
    const double g = s * sg;
    cf[(size_t)(l0 + l) * C + c] = g * sg;
    if (l0 + l == step - 1) alpha[(size_t)(step - 1) * C + c] = active[c] ? g : 0.0;
    if (gall) gall[((size_t)(step - 1) * k + l0 + l) * C + c] = g;   // kept for the backward
}

// w <- w - sum_l cf_l slot_{l0+l} (first chunk: w = y - kappa*slot_m), in place in
// slot_w; the last chunk also writes partial |w|^2 into part[chunk][0][c]
// (of the value as stored, i.e. after rounding to T).
template <typename T, int NB, int VW>
__global__ __launch_bounds__(64) void k_update(int64_t n, int C, int nct, int64_t rpc,
                                               T *__restrict__ basis, size_t ss, int slot_w, int l0,
                                               int slot_m, const double *__restrict__ kappa,
                                               const double *__restrict__ cf, int last,
                                               double *__restrict__ part)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int c0 = (ct * 64 + (int)threadIdx.x) * VW;
    if (c0 >= C) return;
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    double co[NB][VW], kap[VW], nrm[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        kap[v] = slot_m >= 0 ? kappa[c0 + v] : 0.0;
        nrm[v] = 0.0;
#pragma unroll
        for (int l = 0; l < NB; ++l) co[l][v] = cf[(size_t)(l0 + l) * C + c0 + v];
    }
    T *W = basis + (size_t)slot_w * ss;
    const T *Qm = basis + (size_t)(slot_m >= 0 ? slot_m : 0) * ss;
    const T *Q0 = basis + (size_t)l0 * ss;
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c0;
        double w[VW], qm[VW], q[NB][VW];
        vload<T, VW>(W, e, w);
        vload<T, VW>(Qm, e, qm);
#pragma unroll
        for (int l = 0; l < NB; ++l) vload<T, VW>(Q0 + (size_t)l * ss, e, q[l]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            double x = w[v] - kap[v] * qm[v];
#pragma unroll
            for (int l = 0; l < NB; ++l) x -= co[l][v] * q[l][v];
            w[v] = x;
            const double xr = rounded<T>(x);
            nrm[v] += xr * xr;
        }
        vstore<T, VW>(W, e, w);
    }
    if (last) {
#pragma unroll
        for (int v = 0; v < VW; ++v) part[(size_t)chunk * kPartRows * C + c0 + v] = nrm[v];
    }
}

// beta_{i+1} = |w|, breakdown test, next scales.
__global__ void k_norm_fin(int C, int nchunk, int step, double eps_vec,
                           const double *__restrict__ part, const double *__restrict__ alpha,
                           double *__restrict__ beta, double *__restrict__ sig,
                           double *__restrict__ kappa, double *__restrict__ runmax,
                           int32_t *__restrict__ active, int32_t *__restrict__ kused)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int i = step;
    double ss = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) ss += part[(size_t)ch * kPartRows * C + c];
    const double b = sqrt(ss);
    double rm = fmax(runmax[c], fabs(alpha[(size_t)(i - 1) * C + c]));
    if (i > 1) rm = fmax(rm, beta[(size_t)(i - 1) * C + c]);
    runmax[c] = rm;
    if (active[c]) {
        beta[(size_t)i * C + c] = b;
        if (b <= 1e3 * eps_vec * rm) {
            active[c] = 0;
            kused[c] = i;
            sig[(size_t)i * C + c] = 0.0;
            kappa[c] = 0.0;
        } else {
            sig[(size_t)i * C + c] = 1.0 / b;
            kappa[c] = b * sig[(size_t)(i - 1) * C + c];
        }
    } else {
        beta[(size_t)i * C + c] = 0.0;
        sig[(size_t)i * C + c] = 0.0;
        kappa[c] = 0.0;
    }
}

// ------------------------------------------------------------------ launchers

static inline dim3 red_grid(const Plan &p) { return dim3((unsigned)((int64_t)p.nchunk * p.nct)); }
static inline size_t slot_elems(const Plan &p) { return (size_t)p.n * p.C; }

void launch_setup(const Plan &p, const void *probes, hipStream_t st)
{
    if (p.vec_f32)
        k_setup<float><<<red_grid(p), 256, 0, st>>>(p.n, p.C, p.m, p.c_off, p.nct, p.rpc,
                                                    (const float *)probes, (float *)p.basis, p.part);
    else
        k_setup<double><<<red_grid(p), 256, 0, st>>>(p.n, p.C, p.m, p.c_off, p.nct, p.rpc,
                                                     (const double *)probes, (double *)p.basis,
                                                     p.part);
}

void launch_setup_fin(const Plan &p, hipStream_t st)
{
    k_setup_fin<<<(p.C + 255) / 256, 256, 0, st>>>(p.C, p.k, p.nchunk, p.part, p.nu, p.sig,
                                                   p.kappa, p.runmax, p.beta, p.active, p.kused);
}

template <typename T, int NB, int VW>
static void dots_t(const Plan &p, int step, int l0, hipStream_t st)
{
    const int nct = (p.C + 64 * VW - 1) / (64 * VW);
    k_dots<T, NB, VW><<<(unsigned)((int64_t)p.nchunk * nct), 64, 0, st>>>(
        p.n, p.C, nct, p.rpc, (const T *)p.basis, slot_elems(p), step, l0,
        step >= 2 ? step - 2 : -1, p.kappa, p.part);
}

template <typename T, int NB, int VW>
static void update_t(const Plan &p, int step, int l0, bool first, bool last, hipStream_t st)
{
    const int nct = (p.C + 64 * VW - 1) / (64 * VW);
    k_update<T, NB, VW><<<(unsigned)((int64_t)p.nchunk * nct), 64, 0, st>>>(
        p.n, p.C, nct, p.rpc, (T *)p.basis, slot_elems(p), step, l0,
        (first && step >= 2) ? step - 2 : -1, p.kappa, p.cf, last ? 1 : 0, p.part);
}

// exact-NB dispatch (1..kBasisChunk)
#define ECNT_NB_CASES(F)                                                                        \
    F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16)   \
    F(17) F(18) F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30)     \
    F(31) F(32)

template <typename T, int VW>
static void dots_nb(const Plan &p, int step, int l0, int nb, hipStream_t st)
{
    switch (nb) {
#define ECNT_CASE(N) \
    case N:          \
        dots_t<T, N, VW>(p, step, l0, st); \
        break;
        ECNT_NB_CASES(ECNT_CASE)
#undef ECNT_CASE
    default:
        break;
    }
}

template <typename T, int VW>
static void update_nb(const Plan &p, int step, int l0, int nb, bool first, bool last, hipStream_t st)
{
    switch (nb) {
#define ECNT_CASE(N) \
    case N:          \
        update_t<T, N, VW>(p, step, l0, first, last, st); \
        break;
        ECNT_NB_CASES(ECNT_CASE)
#undef ECNT_CASE
    default:
        break;
    }
}

// Columns per lane of the reduction kernels: FP32 pairs (8-byte loads) when the
// wave width is even; FP64 one column per lane (the NB accumulators per column
// already fill the register budget).  Must match the geometry of the plan.
static inline int red_vw(const Plan &p) { return (p.vec_f32 && p.C % 2 == 0) ? 2 : 1; }

void launch_dots(const Plan &p, int step, int l0, int nb, hipStream_t st)
{
    if (p.vec_f32) {
        if (red_vw(p) == 2) dots_nb<float, 2>(p, step, l0, nb, st);
        else dots_nb<float, 1>(p, step, l0, nb, st);
    } else {
        dots_nb<double, 1>(p, step, l0, nb, st);
    }
}

void launch_dots_fin(const Plan &p, int step, int l0, int nb, hipStream_t st)
{
    const int tot = nb * p.C;
    k_dots_fin<<<(tot + 255) / 256, 256, 0, st>>>(p.C, p.nchunk, step, l0, nb, p.k, p.part, p.sig,
                                                  p.active, p.cf, p.alpha, p.g_gall);
}

void launch_update(const Plan &p, int step, int l0, int nb, bool first, bool last, hipStream_t st)
{
    if (p.vec_f32) {
        if (red_vw(p) == 2) update_nb<float, 2>(p, step, l0, nb, first, last, st);
        else update_nb<float, 1>(p, step, l0, nb, first, last, st);
    } else {
        update_nb<double, 1>(p, step, l0, nb, first, last, st);
    }
}

void launch_norm_fin(const Plan &p, int step, hipStream_t st)
{
    const double eps = p.vec_f32 ? (double)FLT_EPSILON : DBL_EPSILON;
    k_norm_fin<<<(p.C + 255) / 256, 256, 0, st>>>(p.C, p.nchunk, step, eps, p.part, p.alpha,
                                                  p.beta, p.sig, p.kappa, p.runmax, p.active,
                                                  p.kused);
}

}  // namespace ecnt
