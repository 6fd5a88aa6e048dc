// Block-Lanczos form of the estimator: the probes taken 16 at a time, one
// block Lanczos process (Golub and Underwood) per block of 16 columns, and the
// block Gauss rule
//     V_b^T h(C) V_b ~ R_0^T E_1^T h(T_k) E_1 R_0
// whose diagonal holds the per-probe values s_j of Section 3.2 (eq.
// rand_prec_quad; with one column per block it is eq. gauss_quad itself).
//
// Storage: slot l of the basis holds X_{l+1} with Q_{l+1} = X_{l+1} S_{l+1},
// S = R2^{-1} close to the identity (Cholesky QR applied twice).  Step i:
//   Y   = C X_i                                      (operator kernels, slot i)
//   G_l = X_l^T Y                                    (k_blk_dots, MFMA)
//   H_l = S_l^T G_l S_i,  A_i = sym(H_i),  K_l = S_l S_l^T G_l   (k_blk_dots_fin)
//   Y  <- Y - sum_l X_l K_l,  Gram Y^T Y             (k_blk_update, MFMA)
//        [then W = Y S_i = C Q_i - sum_l Q_l H_l: one Gram-Schmidt pass]
//   W^T W = R1^T R1,  T = S_i R1^{-1}                (k_blk_norm_fin, mode 0)
//   X_{i+1} = Y T,  Gram X^T X = R2^T R2             (k_blk_normalize, MFMA)
//   S_{i+1} = R2^{-1},  B_{i+1} = R2 R1              (k_blk_norm_fin, mode 1)
// The 16 x 16 contractions run on v_mfma_f64_16x16x4f64: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; accumulator register v of lane l holds
// D[4v + l/16][l%16].
//
// Quadrature (k_blk_quad): T_k (order 16 k_used, half-bandwidth 16) is reduced
// to tridiagonal form by Givens rotations with bulge chasing (Schwarz), then
// diagonalized by implicit QR sweeps with Wilkinson shifts; every rotation is
// also applied to the first 16 rows of the accumulated eigenvector matrix,
// all in LDS.
#include <float.h>

#include "device_common.h"
#include "ecount_internal.h"

namespace ecnt {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

// h (eq. h), or its erf-smoothed form erfc(theta / w) / 2 when w > 0
__device__ __forceinline__ double blk_step(double th, double w)
{
    if (w > 0.0) return 0.5 * erfc(th / w);
    return th < 0.0 ? 1.0 : 0.0;
}

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---- G_l = X_l^T Y for slots l0..l0+nb-1 (nb <= kBlkChunk) against slot ys ----
// One workgroup of kBlkWaves wavefronts per (row chunk, column block).
// Wavefront w accumulates the basis blocks l0 + w, l0 + w + 4, ... (at most 8);
// all four stream the same rows of Y, whose repeated reads hit the caches.
// MFMA v of a 16-row tile takes rows t0 + 4(lane/16) + v: A = X_l (row,
// column lane%16), B = Y (row, column lane%16).
constexpr int kBlkWaves = 4;
constexpr int kBlkPerWave = kBlkChunk / kBlkWaves;

__global__ __launch_bounds__(64 * kBlkWaves) void k_blk_dots(int64_t n, int C, int nblk, int64_t rpc,
                                                             const double *__restrict__ basis,
                                                             size_t ss, int l0, int nb, int ys,
                                                             double *__restrict__ part)
{
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = (int)(L % nblk);
    const int64_t chunk = L / nblk;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int nw = (nb - wv + kBlkWaves - 1) / kBlkWaves;   // basis blocks of this wavefront
    if (nw <= 0) return;                                    // (no barrier in this kernel)
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    const int col = blk * kBlk + li;
    const double *Y = basis + (size_t)ys * ss;
    const double *X0 = basis + (size_t)(l0 + wv) * ss;
    const size_t xs = (size_t)kBlkWaves * ss;
    d4_t acc[kBlkPerWave];
#pragma unroll
    for (int j = 0; j < kBlkPerWave; ++j) acc[j] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int64_t t0 = r0; t0 < r1; t0 += 16) {
        double y[4], x[kBlkPerWave][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = t0 + 4 * lk + v;
            const bool ok = row < r1;
            const size_t e = (size_t)(ok ? row : r0) * C + col;
            y[v] = ok ? Y[e] : 0.0;
#pragma unroll
            for (int j = 0; j < kBlkPerWave; ++j)
                x[j][v] = (ok && j < nw) ? __builtin_nontemporal_load(X0 + j * xs + e) : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int j = 0; j < kBlkPerWave; ++j)
                if (j < nw) acc[j] = mfma16(x[j][v], y[v], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < kBlkPerWave; ++j) {
        if (j >= nw) break;
        const int l = wv + kBlkWaves * j;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            part[(((size_t)chunk * nb + l) * nblk + blk) * 256 + (4 * v + lk) * 16 + li] = acc[j][v];
    }
}

// ---- Y <- Y - sum_l X_l K_l in place for l = l0..l0+nb-1 (ZI: Y <- X T with
// X the slot itself), and the Gram matrix of the result per row chunk when
// `last` ----
// One workgroup of kBlkWaves wavefronts per (row chunk, column block); the
// coefficients (-K_l or T, in B-operand order: for MFMA q, lane l holds
// K[4(l/16)+q][l%16] at [l*4 + q]) are staged in LDS and the wavefronts take
// the row chunk's 16-row tiles in turn.  The A operand of MFMA q is
// X_l[t0 + l%16][4(l/16) + q], so each lane loads 4 consecutive columns.
template <bool ZI>
__global__ __launch_bounds__(64 * kBlkWaves) void k_blk_update(int64_t n, int C, int nblk, int64_t rpc,
                                                               double *__restrict__ basis, size_t ss,
                                                               int l0, int nb, int ws,
                                                               const double *__restrict__ Kop, int last,
                                                               double *__restrict__ part)
{
    extern __shared__ double kl[];   // nb * 256 coefficients
    __shared__ double gred[kBlkWaves - 1][256];
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = (int)(L % nblk);
    const int64_t chunk = L / nblk;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    for (int e = threadIdx.x; e < nb * 256; e += 64 * kBlkWaves)
        kl[e] = Kop[((size_t)(l0 + (e >> 8)) * nblk + blk) * 256 + (e & 255)];
    __syncthreads();
    const int64_t r0 = chunk * rpc, r1 = min(n, r0 + rpc);
    const int col = blk * kBlk + li;
    double *W = basis + (size_t)ws * ss;
    const double *X0 = ZI ? W : basis + (size_t)l0 * ss;
    d4_t gram = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t0 = r0 + 16 * wv; t0 < r1; t0 += 16 * kBlkWaves) {
        d4_t d = {0.0, 0.0, 0.0, 0.0};
        if (!ZI) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = t0 + 4 * v + lk;
                d[v] = row < r1 ? W[(size_t)row * C + col] : 0.0;
            }
        }
        const int64_t ra = t0 + li;
        const bool oka = ra < r1;
        const size_t ea = (size_t)(oka ? ra : r0) * C + blk * kBlk + 4 * lk;
        // groups of 8 basis blocks; the next group's loads are issued before
        // the current group's MFMAs
        double xa[2][8][4];
        auto load_group = [&](int lg, double (&dst)[8][4]) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                d2_t a = {0.0, 0.0}, b = {0.0, 0.0};
                if (lg + u < nb) {
                    const d2_t *src = reinterpret_cast<const d2_t *>(X0 + (size_t)(lg + u) * ss + ea);
                    a = ZI ? src[0] : __builtin_nontemporal_load(src);
                    b = ZI ? src[1] : __builtin_nontemporal_load(src + 1);
                }
                dst[u][0] = oka ? a[0] : 0.0;
                dst[u][1] = oka ? a[1] : 0.0;
                dst[u][2] = oka ? b[0] : 0.0;
                dst[u][3] = oka ? b[1] : 0.0;
            }
        };
        load_group(0, xa[0]);
        for (int lg = 0; lg < nb; lg += 16) {
            if (lg + 8 < nb) load_group(lg + 8, xa[1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (lg + u >= nb) break;
                const d4_t kv = *reinterpret_cast<const d4_t *>(kl + (lg + u) * 256 + lane * 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) d = mfma16(xa[0][u][q], kv[q], d);
            }
            if (lg + 8 >= nb) break;
            if (lg + 16 < nb) load_group(lg + 16, xa[0]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (lg + 8 + u >= nb) break;
                const d4_t kv = *reinterpret_cast<const d4_t *>(kl + (lg + 8 + u) * 256 + lane * 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) d = mfma16(xa[1][u][q], kv[q], d);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = t0 + 4 * v + lk;
            if (row < r1) W[(size_t)row * C + col] = d[v];
        }
        if (last) {
#pragma unroll
            for (int v = 0; v < 4; ++v) gram = mfma16(d[v], d[v], gram);
        }
    }
    if (last) {
        // the wavefronts' Gram matrices added in wavefront order
        if (wv > 0)
#pragma unroll
            for (int v = 0; v < 4; ++v) gred[wv - 1][(4 * v + lk) * 16 + li] = gram[v];
        __syncthreads();
        if (wv == 0)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int idx = (4 * v + lk) * 16 + li;
                double g = gram[v];
#pragma unroll
                for (int w = 0; w < kBlkWaves - 1; ++w) g += gred[w][idx];
                part[((size_t)chunk * nblk + blk) * 256 + idx] = g;
            }
    }
}

// ---- small 16 x 16 algebra of one block, one workgroup of 256 threads ----
// (thread t = element (t/16, t%16)).  Matrices row-major in LDS.

// Sum over the row chunks of a 16 x 16 partial: eight running sums over the
// chunks ch = 8q + u (u = 0..7), added in u order, so the result does not
// depend on the launch and the loads are not one dependent chain.
__device__ __forceinline__ double chunk_sum16(const double *__restrict__ part, int nchunk, int NB,
                                              int l, int nblk, int blk, int t)
{
    const size_t stride = (size_t)NB * nblk * 256;
    const double *p = part + ((size_t)l * nblk + blk) * 256 + t;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int ch = 0;
    for (; ch + 8 <= nchunk; ch += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += p[(size_t)(ch + u) * stride];
    for (int u = 0; ch + u < nchunk; ++u) s[u] += p[(size_t)(ch + u) * stride];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// out = op(a) * b with op(a) = a or a^T; every thread computes its element.
__device__ __forceinline__ double mm16(const double *a, bool ta, const double *b, int t)
{
    const int r = t >> 4, c = t & 15;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += (ta ? a[k * 16 + r] : a[r * 16 + k]) * b[k * 16 + c];
    return s;
}

// Upper Cholesky factor R (G = R^T R) and its inverse, by one thread.
// Returns false if a pivot is not positive and finite.
__device__ bool chol_inv16(const double *G, double *R, double *Ri)
{
    for (int i = 0; i < 256; ++i) {
        R[i] = 0.0;
        Ri[i] = 0.0;
    }
    for (int j = 0; j < 16; ++j) {
        double s = G[j * 16 + j];
        for (int k = 0; k < j; ++k) s -= R[k * 16 + j] * R[k * 16 + j];
        if (!(s > 0.0) || !isfinite(s)) return false;
        const double rjj = sqrt(s);
        R[j * 16 + j] = rjj;
        for (int c = j + 1; c < 16; ++c) {
            double u = G[j * 16 + c];
            for (int k = 0; k < j; ++k) u -= R[k * 16 + j] * R[k * 16 + c];
            R[j * 16 + c] = u / rjj;
        }
    }
    for (int j = 0; j < 16; ++j) {
        Ri[j * 16 + j] = 1.0 / R[j * 16 + j];
        for (int r = j - 1; r >= 0; --r) {
            double u = 0.0;
            for (int k = r + 1; k <= j; ++k) u += R[r * 16 + k] * Ri[k * 16 + j];
            Ri[r * 16 + j] = -u / R[r * 16 + r];
        }
    }
    return true;
}

// element (r, c) of a 16 x 16 matrix -> its slot in B-operand order
__device__ __forceinline__ int op_index(int r, int c) { return ((r >> 2) * 16 + c) * 4 + (r & 3); }

// Coefficients after the dots: K_l = S_l S_l^T G_l (stored negated, operand
// order) and, for the current block (slot icur), A_i = sym(S^T G S).
__global__ __launch_bounds__(256) void k_blk_dots_fin(int nblk, int nchunk, int NB, int l0, int icur,
                                                      const double *__restrict__ part,
                                                      const double *__restrict__ Sm,
                                                      double *__restrict__ Kop,
                                                      double *__restrict__ Aout)
{
    __shared__ double G[256], Sl[256], U[256], H[256];
    const int blk = blockIdx.x, l = blockIdx.y, t = threadIdx.x;
    const int r = t >> 4, c = t & 15;
    const int slot = l0 + l;
    G[t] = chunk_sum16(part, nchunk, NB, l, nblk, blk, t);
    Sl[t] = Sm[((size_t)slot * nblk + blk) * 256 + t];
    __syncthreads();
    U[t] = mm16(Sl, true, G, t);                       // S^T G
    __syncthreads();
    const double K = mm16(Sl, false, U, t);            // S S^T G
    Kop[((size_t)slot * nblk + blk) * 256 + op_index(r, c)] = -K;
    if (slot == icur) {
        H[t] = mm16(U, false, Sl, t);                  // S^T G S
        __syncthreads();
        Aout[(size_t)blk * 256 + t] = 0.5 * (H[t] + H[c * 16 + r]);
    }
}

// Normalization of one block (one workgroup of 256 threads per block).
//   mode 2: Gram of the probe block, R1 = chol, T = R1^{-1}
//   mode 3: Gram after X = V T: R2 = chol, S_1 = R2^{-1}, R_0 = R2 R1,
//           k_used = k for the columns of the block
//   mode 0: step i, Gram of Y: G_W = S_i^T G S_i = R1^T R1, T = S_i R1^{-1}
//   mode 1: step i, Gram after X = Y T: R2, S_{i+1} = R2^{-1}, B_{i+1} = R2 R1;
//           breakdown when min diag(B_{i+1}) <= 1e3 eps rm, rm the largest
//           |entry| of A_1..A_i and B_2..B_i.
// A breakdown (or a failed factorization) ends the block: k_used = i and its
// transforms are zeroed, so the later sweeps carry zeros.
__global__ __launch_bounds__(256) void k_blk_norm_fin(int mode, int step, int k, int nblk, int nchunk,
                                                      int c_off, const double *__restrict__ part,
                                                      double *__restrict__ Sm,
                                                      const double *__restrict__ Ab,
                                                      double *__restrict__ Bb,
                                                      double *__restrict__ R0,
                                                      double *__restrict__ R1,
                                                      double *__restrict__ Top,
                                                      double *__restrict__ rm,
                                                      int32_t *__restrict__ act,
                                                      int32_t *__restrict__ kused)
{
    __shared__ double G[256], Sl[256], U[256], R[256], Ri[256];
    __shared__ int ok_s;
    const int blk = blockIdx.x, t = threadIdx.x;
    const int i = step;
    const bool alive = mode >= 2 || act[blk] != 0;
    G[t] = chunk_sum16(part, nchunk, 1, 0, nblk, blk, t);
    if (mode == 0) Sl[t] = Sm[((size_t)(i - 1) * nblk + blk) * 256 + t];
    __syncthreads();
    if (mode == 0) {
        U[t] = mm16(Sl, true, G, t);
        __syncthreads();
        const double g = mm16(U, false, Sl, t);
        __syncthreads();
        G[t] = g;
        __syncthreads();
    }
    if (t == 0) {
        bool ok = alive && chol_inv16(G, R, Ri);
        if (ok && mode == 1) {
            // B_{i+1} = R2 R1 (diagonal = products of the diagonals)
            double r = rm[blk];
            for (int e = 0; e < 256; ++e) r = fmax(r, fabs(Ab[(size_t)blk * 256 + e]));
            if (i > 1)
                for (int e = 0; e < 256; ++e)
                    r = fmax(r, fabs(Bb[((size_t)(i - 1) * nblk + blk) * 256 + e]));
            rm[blk] = r;
            double mn = INFINITY;
            for (int j = 0; j < 16; ++j)
                mn = fmin(mn, R[j * 16 + j] * R1[(size_t)blk * 256 + j * 16 + j]);
            if (mn <= 1e3 * DBL_EPSILON * r) ok = false;
        }
        if (mode == 2) rm[blk] = 0.0;
        ok_s = ok ? 1 : 0;
        if (alive && !ok) {
            act[blk] = 0;
            for (int j = 0; j < 16; ++j) kused[c_off + blk * kBlk + j] = mode >= 2 ? 0 : i;
        }
        if (mode >= 2 && ok) act[blk] = 1;
    }
    __syncthreads();
    const bool ok = ok_s != 0;
    const int r = t >> 4, c = t & 15;
    if (mode == 2 || mode == 0) {
        // T = S_i R1^{-1} (mode 0) or R1^{-1}; keep R1
        double tv = 0.0;
        if (ok) tv = mode == 0 ? mm16(Sl, false, Ri, t) : Ri[t];
        Top[(size_t)blk * 256 + op_index(r, c)] = tv;
        R1[(size_t)blk * 256 + t] = ok ? R[t] : 0.0;
    } else {
        Sm[((size_t)(mode == 3 ? 0 : i) * nblk + blk) * 256 + t] = ok ? Ri[t] : 0.0;
        // R2 R1: upper triangular product
        double b = 0.0;
        if (ok)
            for (int q = 0; q < 16; ++q) b += R[r * 16 + q] * R1[(size_t)blk * 256 + q * 16 + c];
        if (mode == 3) {
            R0[(size_t)blk * 256 + t] = b;
            if (t < 16) kused[c_off + blk * kBlk + t] = ok ? k : 0;
        } else {
            Bb[((size_t)i * nblk + blk) * 256 + t] = b;
        }
    }
}

// ---- quadrature: one workgroup (one wavefront) per block ----
constexpr int kQMax = kBlk * kBlkMaxK;   // largest order of T_k
// LDS row stride: one double more than the order, so that lanes walking a row
// of the band (one diagonal to the next) or the 16 rows of Z hit distinct banks
constexpr int kQN = kQMax + 1;
constexpr int kBand = kBlk + 2;         // diagonals kept: 0..16 and the bulge

__device__ __forceinline__ int bidx(int r, int c)
{
    // symmetric band storage: (r, c) with |r - c| <= 17 -> diagonal |r-c| at column min(r, c)
    return r >= c ? (r - c) * kQN + c : (c - r) * kQN + r;
}

__global__ __launch_bounds__(64) void k_blk_quad(int nblk, int c_off, double smooth_w,
                                                 const double *__restrict__ Ab,
                                                 const double *__restrict__ Bb,
                                                 const double *__restrict__ R0,
                                                 const int32_t *__restrict__ kused,
                                                 double *__restrict__ s_out,
                                                 double *__restrict__ minabs,
                                                 int32_t *__restrict__ flags)
{
    __shared__ double Lb[kBand * kQN];
    __shared__ double Z[kBlk * kQN];
    __shared__ double F[256];
    const int blk = blockIdx.x, lane = threadIdx.x;
    const int col0 = c_off + blk * kBlk;
    const int ku = kused[col0];
    if (ku < 1) {
        if (lane < kBlk) {
            s_out[col0 + lane] = 0.0;
            minabs[col0 + lane] = INFINITY;
        }
        return;
    }
    const int N = ku * kBlk;
    // T_k into band storage: A_i on the diagonal blocks, B_{i+1} (upper
    // triangular) in block (i, i-1); the bulge diagonal starts at zero
    for (int e = lane; e < kBand * N; e += 64) {
        const int d = e / N, c = e - d * N, r = c + d;
        double v = 0.0;
        if (d <= kBlk && r < N) {
            const int bi = r / kBlk, bj = c / kBlk, rr = r % kBlk, cc = c % kBlk;
            if (bi == bj) v = Ab[((size_t)bi * nblk + blk) * 256 + rr * 16 + cc];
            else if (bi == bj + 1) v = Bb[((size_t)bi * nblk + blk) * 256 + rr * 16 + cc];
        }
        Lb[d * kQN + c] = v;
    }
    for (int e = lane; e < kBlk * N; e += 64) {
        const int r = e / N, c = e - r * N;
        Z[r * kQN + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();

    // one Givens rotation in the plane (p, p+1) that zeroes T[p+1][t]
    auto rotate = [&](int p, int t) {
        const int q = p + 1;
        const double x = Lb[bidx(p, t)], y = Lb[bidx(q, t)];
        // |x|, |y| far from the under/overflow range: T_k holds O(|C|) entries
        const double q2 = x * x + y * y;
        if (q2 == 0.0) return;
        const double ir = rsqrt(q2);
        const double rr = q2 * ir;
        const double c = x * ir, s = y * ir;
        const int hi = min(N - 1, q + kBlk);
        // reads
        const int xx = t + lane;
        const bool el = lane < 2 * kBlk + 2 && xx <= hi && xx != p && xx != q;
        double u = 0.0, w = 0.0;
        if (el) {
            u = Lb[bidx(p, xx)];
            w = Lb[bidx(q, xx)];
        }
        const double a = Lb[bidx(p, p)], bb = Lb[bidx(q, p)], dd = Lb[bidx(q, q)];
        const int zr = lane - 48;
        double zp = 0.0, zq = 0.0;
        if (zr >= 0) {
            zp = Z[zr * kQN + p];
            zq = Z[zr * kQN + q];
        }
        // one wavefront: every lane's reads above are issued before any write below
        if (el) {
            Lb[bidx(p, xx)] = c * u + s * w;
            Lb[bidx(q, xx)] = -s * u + c * w;
        }
        if (lane == 0) {
            Lb[bidx(p, t)] = rr;
            Lb[bidx(q, t)] = 0.0;
            Lb[bidx(p, p)] = c * c * a + 2.0 * c * s * bb + s * s * dd;
            Lb[bidx(q, q)] = s * s * a - 2.0 * c * s * bb + c * c * dd;
            Lb[bidx(q, p)] = c * s * (dd - a) + (c * c - s * s) * bb;
        }
        if (zr >= 0) {
            Z[zr * kQN + p] = c * zp + s * zq;
            Z[zr * kQN + q] = -s * zp + c * zq;
        }
        __syncthreads();
    };
    // band -> tridiagonal: zero column j below the first subdiagonal from the
    // bottom of the band up, chasing each bulge off the end
    for (int j = 0; j + 2 < N; ++j) {
        for (int d = min(kBlk, N - 1 - j); d >= 2; --d) {
            const int p = j + d - 1;
            rotate(p, j);
            int pc = p, r = p + 1 + kBlk;
            while (r < N) {
                rotate(r - 1, pc);
                pc = r - 1;
                r += kBlk;
            }
        }
    }
    // implicit QR sweeps with Wilkinson shifts on (diagonal 0, diagonal 1);
    // every lane runs the scalar chain, lanes 0..15 rotate their row of Z
    double *A_ = Lb;
    double *B_ = Lb + kQN;
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
        int lo = hi - 1;
        while (lo > 0) {
            const double bl = fabs(B_[lo - 1]);
            if (bl <= DBL_EPSILON * (fabs(A_[lo - 1]) + fabs(A_[lo])) || bl < DBL_MIN) break;
            --lo;
        }
        if (++iter > 60 * N) {
            failed = true;
            break;
        }
        const double bb0 = B_[hi - 1];
        const double dh = 0.5 * (A_[hi - 1] - A_[hi]);
        const double den = dh + copysign(hypot(dh, bb0), dh);
        const double mu = A_[hi] - (den != 0.0 ? bb0 * bb0 / den : 0.0);
        double x = A_[lo] - mu, y = B_[lo];
        if (lo > 0 && lane == 0) B_[lo - 1] = 0.0;   // the split found above (not read by the sweep)
        // the values a rotation changes and the next one reads (A[kk], B[kk],
        // row `lane` of Z at kk) are carried in registers; what it reads ahead
        // (A[kk+1], B[kk+1], Z at kk+1) is not yet written in this sweep
        double ak = A_[lo], bk = B_[lo];
        double zk = lane < kBlk ? Z[lane * kQN + lo] : 0.0;
        double nbk = bk;
        double ak1 = A_[lo + 1];
        double bk1 = lo + 1 < hi ? B_[lo + 1] : 0.0;
        double z1 = lane < kBlk ? Z[lane * kQN + lo + 1] : 0.0;
        for (int kk = lo; kk < hi; ++kk) {
            // next iteration's operands, loaded before this iteration's writes
            const double ak2 = kk + 2 <= hi ? A_[kk + 2] : 0.0;
            const double bk2 = kk + 2 < hi ? B_[kk + 2] : 0.0;
            const double z2 = (lane < kBlk && kk + 2 <= hi) ? Z[lane * kQN + kk + 2] : 0.0;
            const double q2 = x * x + y * y;
            double cs = 1.0, sn = 0.0, r = 0.0;
            if (q2 > 0.0) {
                const double ir = rsqrt(q2);
                r = q2 * ir;
                cs = x * ir;
                sn = y * ir;
            }
            const double na = cs * cs * ak + 2.0 * cs * sn * bk + sn * sn * ak1;
            const double na1 = sn * sn * ak - 2.0 * cs * sn * bk + cs * cs * ak1;
            nbk = cs * sn * (ak1 - ak) + (cs * cs - sn * sn) * bk;
            if (lane == 0) {
                if (kk > lo) B_[kk - 1] = r;
                A_[kk] = na;
            }
            if (lane < kBlk) Z[lane * kQN + kk] = cs * zk + sn * z1;
            zk = -sn * zk + cs * z1;
            ak = na1;
            bk = cs * bk1;
            x = nbk;
            y = sn * bk1;
            ak1 = ak2;
            bk1 = bk2;
            z1 = z2;
        }
        if (lane == 0) {
            A_[hi] = ak;
            B_[hi - 1] = nbk;
        }
        if (lane < kBlk) Z[lane * kQN + hi] = zk;
        __syncthreads();
    }
    __syncthreads();
    // F = Z h(Theta) Z^T, then S = R0^T F R0 (diagonal only)
    for (int e = lane; e < 256; e += 64) {
        const int a = e >> 4, b = e & 15;
        double s = 0.0;
        for (int q = 0; q < N; ++q) s += Z[a * kQN + q] * Z[b * kQN + q] * blk_step(A_[q], smooth_w);
        F[e] = s;
    }
    __syncthreads();
    if (lane < kBlk) {
        const double *R = R0 + (size_t)blk * 256;
        double s = 0.0;
        for (int a = 0; a <= lane; ++a)
            for (int b = 0; b <= lane; ++b) s += R[a * 16 + lane] * F[a * 16 + b] * R[b * 16 + lane];
        double mn = INFINITY;
        for (int q = 0; q < N; ++q) mn = fmin(mn, fabs(A_[q]));
        s_out[col0 + lane] = s;
        minabs[col0 + lane] = mn;
    }
    if (failed && lane == 0) atomicOr(&flags[1], 1);
}

// ------------------------------------------------------------------ launchers

static inline unsigned blk_grid(const Plan &p) { return (unsigned)((int64_t)p.bk_nchunk * p.nblk); }

void launch_blk_dots(const Plan &p, int l0, int nb, int ys, hipStream_t st)
{
    k_blk_dots<<<blk_grid(p), 64 * kBlkWaves, 0, st>>>(p.n, p.C, p.nblk, p.bk_rpc,
                                                       (const double *)p.basis, slot_elems(p),
                                                       l0, nb, ys, p.bk_part);
}

void launch_blk_dots_fin(const Plan &p, int l0, int nb, int icur, hipStream_t st)
{
    k_blk_dots_fin<<<dim3((unsigned)p.nblk, (unsigned)nb), 256, 0, st>>>(
        p.nblk, p.bk_nchunk, nb, l0, icur, p.bk_part, p.bk_S, p.bk_K,
        p.bk_A + (size_t)(icur >= 0 ? icur : 0) * p.nblk * 256);
}

void launch_blk_update(const Plan &p, int l0, int nb, int ws, bool last, hipStream_t st)
{
    k_blk_update<false><<<blk_grid(p), 64 * kBlkWaves, sizeof(double) * 256 * nb, st>>>(
        p.n, p.C, p.nblk, p.bk_rpc, (double *)p.basis, slot_elems(p), l0, nb, ws, p.bk_K,
        last ? 1 : 0, p.bk_part);
}

void launch_blk_normalize(const Plan &p, int ws, hipStream_t st)
{
    k_blk_update<true><<<blk_grid(p), 64 * kBlkWaves, sizeof(double) * 256, st>>>(
        p.n, p.C, p.nblk, p.bk_rpc, (double *)p.basis, slot_elems(p), 0, 1, ws, p.bk_T, 1,
        p.bk_part);
}

void launch_blk_norm_fin(const Plan &p, int mode, int step, hipStream_t st)
{
    k_blk_norm_fin<<<(unsigned)p.nblk, 256, 0, st>>>(
        mode, step, p.k, p.nblk, p.bk_nchunk, p.c_off, p.bk_part, p.bk_S,
        p.bk_A + (size_t)(step >= 1 ? step - 1 : 0) * p.nblk * 256, p.bk_B, p.bk_R0, p.bk_R1,
        p.bk_T, p.bk_rm, p.bk_act, p.kused);
}

void launch_blk_quad(const Plan &p, hipStream_t st)
{
    k_blk_quad<<<(unsigned)p.nblk, 64, 0, st>>>(p.nblk, p.c_off, p.smooth_w, p.bk_A, p.bk_B, p.bk_R0,
                                                p.kused, p.s_out, p.minabs, p.flags);
}

}  // namespace ecnt
