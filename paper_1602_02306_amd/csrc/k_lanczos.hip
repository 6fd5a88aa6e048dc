// Lanczos recurrence with full reorthogonalization on a block of independent
// probe columns (Algorithm 1; Section 3.2, the probe loop of Algorithm 2 run
// data-parallel over columns).
//
// Step i of Algorithm 1, per column c (q_l = sig_{l-1} * slot_{l-1}):
//   y      = C q_i                                (operator kernels, into slot i)
//   w      = y - beta_i q_{i-1}
//   g_l    = q_l^T w,  p_l = q_l^T q_i,  l = 1..i (k_dots, one read of the basis)
//   alpha_i = g_i;  c_l = g_l - alpha_i (p_l - [l = i])          (k_dots_fin)
//   w     <- w - sum_l c_l q_l                    (k_update, in place in slot i)
//   beta_{i+1} = |w|; sig_i = 1/beta_{i+1}        (k_norm_fin)
// Since Q^T (w - alpha_i q_i) = g - alpha_i p, the single update equals
// Algorithm 1's order (alpha_i first, then one classical Gram-Schmidt pass
// against q_1..q_i) up to rounding.  Taking p = e_i instead (all coefficients
// from w) is not such a change: the orthogonality error of q_i would re-enter
// every step multiplied by about |alpha_i| / beta_{i+1}.
//
// Column reductions are two-phase and deterministic: each workgroup writes
// the partial sums of its row chunk, a finalize kernel adds them in chunk
// order.  No floating-point atomics.
#include <float.h>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

// ---- probe setup: slot 0 = v (for every shift), partial |v|^2 ----
// Rows of chunk `chunk`: chunks are numbered segment by segment and never
// straddle a segment.
__device__ __forceinline__ void chunk_rows(const int64_t *__restrict__ seg_row,
                                           const int64_t *__restrict__ seg_chunk, int nseg,
                                           int64_t rpc, int64_t chunk, int &seg, int64_t &r0,
                                           int64_t &r1)
{
    seg = find_seg(seg_chunk, nseg, chunk);
    r0 = seg_row[seg] + (chunk - seg_chunk[seg]) * rpc;
    r1 = min(seg_row[seg + 1], r0 + rpc);
}

template <typename T>
__global__ __launch_bounds__(256) void k_setup(int C, int m, int c_off, int nct, int64_t rpc,
                                               int nseg, const int64_t *__restrict__ seg_row,
                                               const int64_t *__restrict__ seg_chunk,
                                               const T *__restrict__ V, T *__restrict__ slot0,
                                               double *__restrict__ part)
{
    __shared__ double red[4][kColTile];
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = ct * kColTile + lane;
    int seg;
    int64_t r0, r1;
    chunk_rows(seg_row, seg_chunk, nseg, rpc, chunk, seg, r0, r1);
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

// Per virtual column vc = seg*C + c.  kused is global: kused[seg*ku_ld + ku_off + c].
__global__ void k_setup_fin(int C, int nseg, int k, const int64_t *__restrict__ seg_chunk,
                            const double *__restrict__ part, double *__restrict__ nu,
                            double *__restrict__ sig, double *__restrict__ kappa,
                            double *__restrict__ runmax, double *__restrict__ beta,
                            int32_t *__restrict__ active, int32_t *__restrict__ kused, int ku_ld,
                            int ku_off)
{
    // block: kFinWaves wavefronts over the chunks of 64 virtual columns
    const int vc = blockIdx.x * 64 + (threadIdx.x & 63);
    const bool valid = vc < nseg * C;
    const int seg = valid ? vc / C : 0, c = valid ? vc - seg * C : 0;
    const double s = block_chunk_sum(part, kPartRows, C, 0, c, seg_chunk[seg], seg_chunk[seg + 1], valid);
    if (!valid || threadIdx.x >= 64) return;
    nu[vc] = s;
    const bool ok = s > 0.0;
    sig[vc] = ok ? 1.0 / sqrt(s) : 0.0;
    kappa[vc] = 0.0;
    runmax[vc] = 0.0;
    beta[vc] = 0.0;   // beta_1 = 0 (Algorithm 1, first step)
    active[vc] = ok ? 1 : 0;
    kused[(size_t)seg * ku_ld + ku_off + c] = ok ? k : 0;
}

// ---- reorthogonalization dots: part[chunk][l][c] = sum_rows slot_{l0+l} * w ----
// One wavefront per (row chunk, column tile); NB is the exact number of basis
// vectors of the launch, so all NB + 2 row loads are issued back to back.
// GRAM > 0: also part[chunk][NB + l][c] = sum_rows slot_{l0+l} * slot_i (the
// column of the basis' Gram matrix at q_i, from the same row loads).  GRAM = 1:
// slot_i is the launch's last basis vector (always so in the launch holding
// q_i); GRAM = 2: slot_i is read as one more row.
// Rows r0..r1 of the dots sweep; HASM: w = y - kappa q_{i-1} (otherwise w = y,
// and q_{i-1} is not read).
template <typename T, int NB, int VW, int GRAM, bool HASM>
__device__ __forceinline__ void dots_rows(int C, int c0, int64_t r0, int64_t r1, const T *__restrict__ Y,
                                          const T *__restrict__ Qm, const T *__restrict__ Qi,
                                          const T *__restrict__ Q0, size_t ss, const double (&kap)[VW],
                                          double (&acc)[NB][VW], double (&gr)[GRAM > 0 ? NB : 1][VW])
{
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c0;
        double y[VW], qm[VW], qi[VW], q[NB][VW];
        vload<T, VW>(Y, e, y);
        if (HASM) vload<T, VW>(Qm, e, qm);
        if (GRAM == 2) vload<T, VW>(Qi, e, qi);
#pragma unroll
        for (int l = 0; l < NB; ++l) vload_nt<T, VW>(Q0 + (size_t)l * ss, e, q[l]);
        // keep all the row's loads in flight before the first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const double w = HASM ? y[v] - kap[v] * qm[v] : y[v];
#pragma unroll
            for (int l = 0; l < NB; ++l) acc[l][v] += q[l][v] * w;
            if (GRAM > 0) {
                const double qv = GRAM == 1 ? (double)q[NB - 1][v] : qi[v];
#pragma unroll
                for (int l = 0; l < NB; ++l) gr[l][v] += q[l][v] * qv;
            }
        }
    }
}

template <typename T, int NB, int VW, int GRAM>
__global__ __launch_bounds__(64) void k_dots(int C, int nct, int64_t rpc, int nseg,
                                             const int64_t *__restrict__ seg_row,
                                             const int64_t *__restrict__ seg_chunk,
                                             const T *__restrict__ basis, size_t ss, int slot_y,
                                             int l0, int slot_m, const double *__restrict__ kappa_all,
                                             int slot_i, double *__restrict__ part)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int c0 = (ct * 64 + (int)threadIdx.x) * VW;
    if (c0 >= C) return;
    int seg;
    int64_t r0, r1;
    chunk_rows(seg_row, seg_chunk, nseg, rpc, chunk, seg, r0, r1);
    const double *kappa = kappa_all + (size_t)seg * C;
    double acc[NB][VW], gr[GRAM > 0 ? NB : 1][VW];
#pragma unroll
    for (int l = 0; l < NB; ++l)
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[l][v] = 0.0;
#pragma unroll
    for (int l = 0; l < (GRAM > 0 ? NB : 1); ++l)
#pragma unroll
        for (int v = 0; v < VW; ++v) gr[l][v] = 0.0;
    double kap[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) kap[v] = slot_m >= 0 ? kappa[c0 + v] : 0.0;
    const T *Y = basis + (size_t)slot_y * ss;
    const T *Qm = basis + (size_t)(slot_m >= 0 ? slot_m : 0) * ss;
    const T *Qi = basis + (size_t)(GRAM == 2 ? slot_i : 0) * ss;
    const T *Q0 = basis + (size_t)l0 * ss;
    if (slot_m >= 0)
        dots_rows<T, NB, VW, GRAM, true>(C, c0, r0, r1, Y, Qm, Qi, Q0, ss, kap, acc, gr);
    else
        dots_rows<T, NB, VW, GRAM, false>(C, c0, r0, r1, Y, Qm, Qi, Q0, ss, kap, acc, gr);
#pragma unroll
    for (int l = 0; l < NB; ++l)
#pragma unroll
        for (int v = 0; v < VW; ++v)
            part[((size_t)chunk * kPartRows + l) * C + c0 + v] = acc[l][v];
    if (GRAM > 0) {
#pragma unroll
        for (int l = 0; l < NB; ++l)
#pragma unroll
            for (int v = 0; v < VW; ++v)
                part[((size_t)chunk * kPartRows + NB + l) * C + c0 + v] = gr[l][v];
    }
}

// g_l = sig_l * sum_chunks part; cf_l = g_l * sig_l; alpha_i = g_i.
// With the Gram column (gram != 0), p_l = q_l^T q_i = sig_l sig_i * sum_chunks
// part[.][nb + l] and the coefficients are those of Algorithm 1's order (alpha
// first, then the pass over q_1..q_i): with w1 = w - alpha_i q_i,
// Q^T w1 = g - alpha_i p, so the update w - alpha_i q_i - Q (Q^T w1) subtracts
// slot l with cf_l = sig_l (g_l - alpha_i p_l) + [l = i] alpha_i sig_i.  (Taking
// p = e_i instead lets the orthogonality error of q_i re-enter every step
// multiplied by about |alpha_i| / beta_{i+1}.)  Every block of the launch that
// holds q_i sums alpha_i itself; the others read it, that launch running first.
// Arrays indexed [row][nseg*C].
__global__ void k_dots_fin(int C, int nseg, int step, int l0, int nb, int k,
                           const int64_t *__restrict__ seg_chunk, const double *__restrict__ part,
                           const double *__restrict__ sig, const int32_t *__restrict__ active,
                           double *__restrict__ cf, double *__restrict__ alpha,
                           double *__restrict__ gall, double *__restrict__ pall, int gram)
{
    // block (x: 64 virtual columns, y: basis vector l), kFinWaves wavefronts over the chunks
    const int NC = nseg * C;
    const int l = blockIdx.y;
    const int vc = blockIdx.x * 64 + (threadIdx.x & 63);
    const bool valid = vc < NC;
    const int seg = valid ? vc / C : 0, c = valid ? vc - seg * C : 0;
    const int64_t ch0 = seg_chunk[seg], ch1 = seg_chunk[seg + 1];
    const int arow = step - 1 - l0;   // row of q_i in this launch, if it holds q_i
    const double s = block_chunk_sum(part, kPartRows, C, l, c, ch0, ch1, valid);
    double sp = 0.0, sa = 0.0;
    if (gram) {
        sp = block_chunk_sum(part, kPartRows, C, nb + l, c, ch0, ch1, valid);
        if (arow < nb) sa = block_chunk_sum(part, kPartRows, C, arow, c, ch0, ch1, valid);
    }
    if (!valid || threadIdx.x >= 64) return;
    const double sg = sig[(size_t)(l0 + l) * NC + vc];
    const double g = s * sg;
    double c_l = g, pe = 0.0;   // coefficient of q_l in the update; p_l - [l = i]
    if (gram) {
        const double si = sig[(size_t)(step - 1) * NC + vc];
        const double a = arow < nb ? (active[vc] ? sa * si : 0.0) : alpha[(size_t)(step - 1) * NC + vc];
        pe = sp * sg * si - (l0 + l == step - 1 ? 1.0 : 0.0);
        c_l = g - a * pe;
    }
    cf[(size_t)(l0 + l) * NC + vc] = c_l * sg;
    if (l0 + l == step - 1) alpha[(size_t)(step - 1) * NC + vc] = active[vc] ? g : 0.0;
    if (gall) {   // kept for the backward
        gall[((size_t)(step - 1) * k + l0 + l) * NC + vc] = c_l;
        pall[((size_t)(step - 1) * k + l0 + l) * NC + vc] = pe;
    }
}

// Rows r0..r1 of the update sweep; HASM: the first chunk's -kappa q_{i-1} term
// (otherwise q_{i-1} is not read).
template <typename T, int NB, int VW, bool HASM>
__device__ __forceinline__ void update_rows(int C, int c0, int64_t r0, int64_t r1, T *__restrict__ W,
                                            const T *__restrict__ Qm, const T *__restrict__ Q0,
                                            size_t ss, const double (&kap)[VW],
                                            const double (&co)[NB][VW], double (&nrm)[VW])
{
    for (int64_t r = r0; r < r1; ++r) {
        const size_t e = (size_t)r * C + c0;
        double w[VW], qm[VW];
        T q[NB][VW];   // in the storage type until used (half the registers for FP32)
        vload<T, VW>(W, e, w);
        if (HASM) vload<T, VW>(Qm, e, qm);
#pragma unroll
        for (int l = 0; l < NB; ++l) vload_nt_raw<T, VW>(Q0 + (size_t)l * ss, e, q[l]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            double x = HASM ? w[v] - kap[v] * qm[v] : w[v];
#pragma unroll
            for (int l = 0; l < NB; ++l) x -= co[l][v] * static_cast<double>(q[l][v]);
            w[v] = x;
            const double xr = rounded<T>(x);
            nrm[v] += xr * xr;
        }
        vstore<T, VW>(W, e, w);
    }
}

// w <- w - sum_l cf_l slot_{l0+l} (first chunk: w = y - kappa*slot_m), in place in
// slot_w; the last chunk also writes partial |w|^2 into part[chunk][0][c]
// (of the value as stored, i.e. after rounding to T).
template <typename T, int NB, int VW>
__global__ __launch_bounds__(64) void k_update(int C, int nct, int64_t rpc, int nseg,
                                               const int64_t *__restrict__ seg_row,
                                               const int64_t *__restrict__ seg_chunk,
                                               T *__restrict__ basis, size_t ss, int slot_w, int l0,
                                               int slot_m, const double *__restrict__ kappa_all,
                                               const double *__restrict__ cf, int last,
                                               double *__restrict__ part)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = (int)(L % nct);
    const int64_t chunk = L / nct;
    const int c0 = (ct * 64 + (int)threadIdx.x) * VW;
    if (c0 >= C) return;
    int seg;
    int64_t r0, r1;
    chunk_rows(seg_row, seg_chunk, nseg, rpc, chunk, seg, r0, r1);
    const size_t NC = (size_t)nseg * C, vc0 = (size_t)seg * C + c0;
    double co[NB][VW], kap[VW], nrm[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        kap[v] = slot_m >= 0 ? kappa_all[vc0 + v] : 0.0;
        nrm[v] = 0.0;
#pragma unroll
        for (int l = 0; l < NB; ++l) co[l][v] = cf[(size_t)(l0 + l) * NC + vc0 + v];
    }
    T *W = basis + (size_t)slot_w * ss;
    const T *Qm = basis + (size_t)(slot_m >= 0 ? slot_m : 0) * ss;
    const T *Q0 = basis + (size_t)l0 * ss;
    if (slot_m >= 0)
        update_rows<T, NB, VW, true>(C, c0, r0, r1, W, Qm, Q0, ss, kap, co, nrm);
    else
        update_rows<T, NB, VW, false>(C, c0, r0, r1, W, Qm, Q0, ss, kap, co, nrm);
    if (last) {
#pragma unroll
        for (int v = 0; v < VW; ++v) part[(size_t)chunk * kPartRows * C + c0 + v] = nrm[v];
    }
}

// beta_{i+1} = |w|, breakdown test, next scales.
__global__ void k_norm_fin(int C, int nseg, int step, double eps_vec,
                           const int64_t *__restrict__ seg_chunk, const double *__restrict__ part,
                           const double *__restrict__ alpha, double *__restrict__ beta,
                           double *__restrict__ sig, double *__restrict__ kappa,
                           double *__restrict__ runmax, int32_t *__restrict__ active,
                           int32_t *__restrict__ kused, int ku_ld, int ku_off)
{
    const int vc = blockIdx.x * 64 + (threadIdx.x & 63);
    const int NC = nseg * C;
    const bool valid = vc < NC;
    const int seg = valid ? vc / C : 0, cc = valid ? vc - seg * C : 0;
    const int i = step;
    const double ss = block_chunk_sum(part, kPartRows, C, 0, cc, seg_chunk[seg], seg_chunk[seg + 1], valid);
    if (!valid || threadIdx.x >= 64) return;
    const int c = vc;   // per-virtual-column arrays below
    const size_t C_ = NC;
    const double b = sqrt(ss);
    double rm = fmax(runmax[c], fabs(alpha[(size_t)(i - 1) * C_ + c]));
    if (i > 1) rm = fmax(rm, beta[(size_t)(i - 1) * C_ + c]);
    runmax[c] = rm;
    if (active[c]) {
        beta[(size_t)i * C_ + c] = b;
        if (b <= 1e3 * eps_vec * rm) {
            active[c] = 0;
            kused[(size_t)seg * ku_ld + ku_off + cc] = i;
            sig[(size_t)i * C_ + c] = 0.0;
            kappa[c] = 0.0;
        } else {
            sig[(size_t)i * C_ + c] = 1.0 / b;
            kappa[c] = b * sig[(size_t)(i - 1) * C_ + c];
        }
    } else {
        beta[(size_t)i * C_ + c] = 0.0;
        sig[(size_t)i * C_ + c] = 0.0;
        kappa[c] = 0.0;
    }
}

// ------------------------------------------------------------------ launchers

static inline dim3 red_grid(const Plan &p) { return dim3((unsigned)((int64_t)p.nchunk * p.nct)); }

void launch_setup(const Plan &p, const void *probes, hipStream_t st)
{
    if (p.vec_f32)
        k_setup<float><<<red_grid(p), 256, 0, st>>>(p.C, p.m, p.c_off, p.nct, p.rpc, p.nseg,
                                                    p.seg_row, p.seg_chunk, (const float *)probes,
                                                    (float *)p.basis, p.part);
    else
        k_setup<double><<<red_grid(p), 256, 0, st>>>(p.C, p.m, p.c_off, p.nct, p.rpc, p.nseg,
                                                     p.seg_row, p.seg_chunk, (const double *)probes,
                                                     (double *)p.basis, p.part);
}

void launch_setup_fin(const Plan &p, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    k_setup_fin<<<(NC + 63) / 64, 64 * kFinWaves, 0, st>>>(p.C, p.nseg, p.k, p.seg_chunk, p.part, p.nu, p.sig,
                                                  p.kappa, p.runmax, p.beta, p.active, p.kused,
                                                  p.Ct, p.c_off);
}

template <typename T, int NB, int VW>
static void dots_t(const Plan &p, int step, int l0, bool gram, hipStream_t st)
{
    const int nct = (p.C + 64 * VW - 1) / (64 * VW);
    const dim3 grid((unsigned)((int64_t)p.nchunk * nct));
    const int sm = (step >= 2 && !p.arnoldi) ? step - 2 : -1;
    if (gram && step - 1 == l0 + NB - 1)
        k_dots<T, NB, VW, 1><<<grid, 64, 0, st>>>(p.C, nct, p.rpc, p.nseg, p.seg_row, p.seg_chunk,
                                                  (const T *)p.basis, slot_elems(p), step, l0, sm,
                                                  p.kappa, step - 1, p.part);
    else if (gram)
        k_dots<T, NB, VW, 2><<<grid, 64, 0, st>>>(p.C, nct, p.rpc, p.nseg, p.seg_row, p.seg_chunk,
                                                  (const T *)p.basis, slot_elems(p), step, l0, sm,
                                                  p.kappa, step - 1, p.part);
    else
        k_dots<T, NB, VW, 0><<<grid, 64, 0, st>>>(p.C, nct, p.rpc, p.nseg, p.seg_row, p.seg_chunk,
                                                  (const T *)p.basis, slot_elems(p), step, l0, sm,
                                                  p.kappa, -1, p.part);
}

template <typename T, int NB, int VW>
static void update_t(const Plan &p, int step, int l0, bool first, bool last, hipStream_t st)
{
    const int nct = (p.C + 64 * VW - 1) / (64 * VW);
    k_update<T, NB, VW><<<(unsigned)((int64_t)p.nchunk * nct), 64, 0, st>>>(
        p.C, nct, p.rpc, p.nseg, p.seg_row, p.seg_chunk, (T *)p.basis, slot_elems(p), step, l0,
        (first && step >= 2) ? step - 2 : -1, p.kappa, p.cf, last ? 1 : 0, p.part);
}

// exact-NB dispatch (1..kBasisChunk)
#define ECNT_NB_CASES(F)                                                                        \
    F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16)   \
    F(17) F(18) F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30)     \
    F(31) F(32)

template <typename T, int VW>
static void dots_nb(const Plan &p, int step, int l0, int nb, bool gram, hipStream_t st)
{
    switch (nb) {
#define ECNT_CASE(N) \
    case N:          \
        dots_t<T, N, VW>(p, step, l0, gram, st); \
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

// Columns per lane of the FP32 dots: pairs (8-byte loads) when the wave width
// is even; FP64 takes one column per lane (the NB accumulators per column
// already fill the register budget).  Each launch derives its column tiles
// from its own width; the partial sums are indexed by column.
static inline int red_vw(const Plan &p) { return (p.vec_f32 && p.C % 2 == 0) ? 2 : 1; }

void launch_dots(const Plan &p, int step, int l0, int nb, bool gram, hipStream_t st)
{
    if (p.vec_f32) {
        // column pairs with the Gram column would spill beyond 24 basis vectors
        if (red_vw(p) == 2 && !(gram && nb > 24)) dots_nb<float, 2>(p, step, l0, nb, gram, st);
        else dots_nb<float, 1>(p, step, l0, nb, gram, st);
    } else {
        dots_nb<double, 1>(p, step, l0, nb, gram, st);
    }
}

void launch_dots_fin(const Plan &p, int step, int l0, int nb, bool gram, hipStream_t st)
{
    const int NC = p.nseg * p.C;
    k_dots_fin<<<dim3((NC + 63) / 64, nb), 64 * kFinWaves, 0, st>>>(
        p.C, p.nseg, step, l0, nb, p.k, p.seg_chunk, p.part, p.sig, p.active, p.cf, p.alpha,
        p.g_gall, p.g_pall, gram ? 1 : 0);
}

void launch_update(const Plan &p, int step, int l0, int nb, bool first, bool last, hipStream_t st)
{
    if (p.vec_f32) {
        // one column per lane: column pairs would hold 2 x nb FP64 coefficients
        // per lane, and the fewer wavefronts resident cost more than the
        // 4-byte loads (measured at every basis size)
        update_nb<float, 1>(p, step, l0, nb, first, last, st);
    } else {
        update_nb<double, 1>(p, step, l0, nb, first, last, st);
    }
}

void launch_norm_fin(const Plan &p, int step, hipStream_t st)
{
    const double eps = p.vec_f32 ? (double)FLT_EPSILON : DBL_EPSILON;
    const int NC = p.nseg * p.C;
    k_norm_fin<<<(NC + 63) / 64, 64 * kFinWaves, 0, st>>>(p.C, p.nseg, step, eps, p.seg_chunk, p.part, p.alpha,
                                                 p.beta, p.sig, p.kappa, p.runmax, p.active, p.kused,
                                                 p.Ct, p.c_off);
}

}  // namespace ecnt
