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
// to tridiagonal form by Householder bulge chasing, then diagonalized by
// implicit QR sweeps with Wilkinson shifts; the first 16 rows of the
// accumulated eigenvector matrix follow every transform, all in LDS.
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
// LDS row stride (one row per diagonal).  Lanes that walk the columns of a
// block touch (r - c) kQN + c, a stride of kQN - 1 doubles, and the rows of
// Z (below) are kQN - 1 apart too: kQN - 1 odd keeps both free of bank
// conflicts.  The 18 columns past the largest order hold the start of Z's
// rows 1..15 for its first columns.
constexpr int kQN = kQMax + 18;
// diagonals held: the half-bandwidth kBlk plus the fill that the chase leaves
// behind (distance at most 2 kBlk - 2 from the diagonal)
constexpr int kDiag = 2 * kBlk - 1;

__device__ __forceinline__ int bidx(int r, int c)
{
    // symmetric band storage: (r, c) -> diagonal |r - c| at column min(r, c)
    return r >= c ? (r - c) * kQN + c : (c - r) * kQN + r;
}

// Z[r][c] (r < 16) after the chase: diagonal 2 + r at column c - r, a slot
// whose band column is finished once Z's column c is (columns c - r <= c;
// for c < r the address falls in diagonal 1 + r's columns past the order)
__device__ __forceinline__ int zidx(int r, int c)
{
    return (2 + r) * kQN + c - r;
}

// Quadrature of one block.  T_k (order N = 16 k_used, half-bandwidth 16) is
// brought to tridiagonal form by Householder bulge chasing: sweep j takes
// column j with one reflector on rows j+1..j+16, and the fill that the
// reflector's right side leaves in the 16 x 16 block below is removed one
// column at a time, each step's reflector acting on the next 16 rows (the
// rest of that fill is removed by the following sweeps, so it never reaches
// beyond distance 30 from the diagonal).  A step is done by the whole
// wavefront on 16 x 16 blocks, lane (kk, g) holding rows 4g..4g+3 of column kk:
//   (a) H on the rows of the window, columns left of it (the column that gave
//       the reflector becomes (beta, 0, ..., 0)),
//   (b) H D H on the diagonal block,
//   (c) the rows below times H; their first column gives the next reflector.
// Z = E_1^T Q (the first 16 rows of the accumulated transform) starts as
// [I 0]; only the first reflector of each sweep meets its nonzero columns
// (they grow by one column per sweep), so it is kept as a sliding 16 x 16
// window in registers, and each finished column is stored in the band slots
// of its T column, which the chase no longer uses.  Then implicit QR sweeps
// with Wilkinson shifts diagonalize the tridiagonal form, every rotation also
// applied to Z, all in LDS.
__global__ __launch_bounds__(64) void k_blk_quad(int nblk, int c_off, double smooth_w,
                                                 const double *__restrict__ Ab,
                                                 const double *__restrict__ Bb,
                                                 const double *__restrict__ R0,
                                                 const int32_t *__restrict__ kused,
                                                 double *__restrict__ s_out,
                                                 double *__restrict__ minabs,
                                                 int32_t *__restrict__ flags)
{
    __shared__ double Lb[kDiag * kQN];
    __shared__ double F[256];
    __shared__ double xbuf[kBlk];     // the column that gives the next reflector
    __shared__ double dump[64];       // per-lane target of the writes a lane does not make
    __shared__ double zslot[1];       // 0.0: the source of the reads a lane does not make
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
    // triangular) in block (i, i-1); the fill diagonals start at zero
    for (int e = lane; e < kDiag * N; e += 64) {
        const int d = e / N, c = e - d * N, r = c + d;
        double v = 0.0;
        if (d <= kBlk && r < N) {
            const int bi = r / kBlk, bj = c / kBlk, rr = r % kBlk, cc = c % kBlk;
            if (bi == bj) v = Ab[((size_t)bi * nblk + blk) * 256 + rr * 16 + cc];
            else if (bi == bj + 1) v = Bb[((size_t)bi * nblk + blk) * 256 + rr * 16 + cc];
        }
        Lb[d * kQN + c] = v;
    }
    if (lane == 0) zslot[0] = 0.0;
    __syncthreads();

    const int kk = lane & 15, g = lane >> 4;
    double *const mydump = dump + lane;
    // Lane (kk, g) holds rows i = 4g + t (t = 0..3) of column kk of a 16 x 16
    // block.  Its element offsets are fixed: in the diagonal block at w0,
    // (w0 + i, w0 + kk) sits at w0 + offD[t]; in a block of the 16 rows below a
    // full window (and in the window's rows left of it, 16 columns back),
    // (w0 + 16 + i, w0 + kk) sits at w0 + offE[t] (distance 16 + i - kk,
    // held when at most kDiag - 1: all but (15, 0)).
    int offD[4], offE[4];
    bool lowD[4], heldE[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int i = 4 * g + t;
        offD[t] = i >= kk ? (i - kk) * kQN + kk : (kk - i) * kQN + i;
        lowD[t] = i >= kk;
        offE[t] = (kBlk + i - kk) * kQN + kk;
        heldE[t] = kBlk + i - kk < kDiag;
    }
    const int offX = (1 + kk) * kQN;           // column j, row j + 1 + kk
    int offXr[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) offXr[t] = (1 + 4 * g + t) * kQN;
    const int offA1 = (1 + lane) * kQN, offA16 = (kBlk + lane) * kQN;   // column writes of (a)

    // ---- band -> tridiagonal ----
    double zw[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) zw[t] = (1 + 4 * g + t == kk) ? 1.0 : 0.0;   // Z columns 1..16
    double zst = kk == 0 ? 1.0 : 0.0;                                        // Z column 0
    for (int j = 0; j + 2 < N; ++j) {
        int w0 = j + 1, c = j;
        int w1 = min(w0 + kBlk - 1, N - 1), L = w1 - w0 + 1;
        int Ln = min(kBlk, N - 1 - w1);
        // the first step's blocks: D (rows and columns w0..w1), E (the rows
        // below; a block below exists only under a full window); later steps
        // get them loaded one step ahead, and P (the window's rows left of
        // it) is the previous step's E, kept in registers
        double D[4], E[4], P[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            D[t] = *(4 * g + t < L && kk < L ? &Lb[w0 + offD[t]] : zslot);
            E[t] = *(4 * g + t < Ln && heldE[t] ? &Lb[w0 + offE[t]] : zslot);
            P[t] = 0.0;
        }
        for (int s = 0;; ++s) {
            const bool more = w1 + 1 <= N - 2;   // a next window of at least 2 rows
            // the reflector: x = column c on the window's rows (band column j
            // in the first step, else the column kept in xbuf by step (c))
            const double x0 = s == 0 ? Lb[kQN + j] : xbuf[0];
            const double xk = *(kk < L ? (s == 0 ? &Lb[offX + j] : &xbuf[kk]) : zslot);
            double xr[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                xr[t] = *(4 * g + t < L ? (s == 0 ? &Lb[offXr[t] + j] : &xbuf[4 * g + t]) : zslot);
            // the next step's D and E (regions this step does not write)
            const int w0n = w1 + 1, w1n = min(w0n + kBlk - 1, N - 1);
            const int Lnn = min(kBlk, N - 1 - w1n);
            double Dn[4], En[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                Dn[t] = *(more && 4 * g + t < Ln && kk < Ln ? &Lb[w0n + offD[t]] : zslot);
                En[t] = *(more && 4 * g + t < Lnn && heldE[t] ? &Lb[w0n + offE[t]] : zslot);
            }
            const double sig2 = row_sum16(kk >= 1 ? xk * xk : 0.0);
            const bool refl = sig2 > 0.0;
            const double mu = sqrt(x0 * x0 + sig2);
            const double bc = x0 >= 0.0 ? -mu : mu;
            const double inv = refl ? 1.0 / (x0 - bc) : 0.0;
            const double tau = refl ? (bc - x0) / bc : 0.0;
            const double beta = refl ? bc : x0;
            const double vk = kk == 0 ? 1.0 : xk * inv;
            double vr[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) vr[t] = 4 * g + t == 0 ? 1.0 : xr[t] * inv;
            // (c) the 16 rows below, columns of the window: E <- E H (only under
            // a full window, so Ln >= 1 means L = 16).  Column 0 gives the next
            // step's reflector (xbuf); the other columns are the next step's P.
            // With no next step all of E goes back into the band.
            if (Ln >= 1) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    // (15, 0) is not held (distance 31) and reads 0, but E H
                    // fills it: it goes to xbuf like the rest of column 0 (with no
                    // next step there is one row below at most, all held)
                    const int i = 4 * g + t;
                    const bool ok = i < Ln;
                    const double z = tau * row_sum16(E[t] * vk);
                    E[t] -= z * vk;
                    double *dst = ok && !more ? &Lb[w0 + offE[t]] : (kk == 0 ? &xbuf[i] : mydump);
                    *dst = ok ? E[t] : 0.0;
                }
            }
            if (s == 0) {
                // Z <- Z H on the sweep's first window (lane (kk, g): row kk)
                double y = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) y += zw[t] * vr[t];
                y = group_sum4(y);
#pragma unroll
                for (int t = 0; t < 4; ++t) zw[t] -= tau * y * vr[t];
            }
            // (a) rows w0.., columns c..w0-1: column c becomes (beta, 0, ..., 0)
            // (distance 1 + lane in the first step, 16 + lane after)
            {
                const bool ok = lane < L && (s == 0 || kBlk + lane < kDiag);
                double *dst = ok ? &Lb[(s == 0 ? offA1 : offA16) + c] : mydump;
                *dst = lane == 0 ? beta : 0.0;
            }
            if (s > 0) {
                double y = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) y += vr[t] * P[t];
                y = tau * group_sum4(y);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool ok = kk >= 1 && 4 * g + t < L;
                    double *dst = ok ? &Lb[c + offE[t]] : mydump;
                    *dst = P[t] - y * vr[t];
                }
            }
            // (b) D <- H D H = D - v w^T - w v^T, w = p - (tau/2)(v^T p) v, p = tau D v
            {
                double p = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) p += vr[t] * D[t];
                p = tau * group_sum4(p);
                const double K = 0.5 * tau * row_sum16(vk * p);
                const double wk = p - K * vk;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double wi = __shfl(wk, 4 * g + t, 64);
                    const bool ok = 4 * g + t < L && kk < L && lowD[t];
                    double *dst = ok ? &Lb[w0 + offD[t]] : mydump;
                    *dst = D[t] - (vr[t] * wk + wi * vk);
                }
            }
            if (!more) break;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                P[t] = E[t];
                D[t] = Dn[t];
                E[t] = En[t];
            }
            c = w0;
            w0 = w0n;
            w1 = w1n;
            L = Ln;
            Ln = Lnn;
        }
        // column j is finished (so are the band columns Z's column j goes to);
        // column j+1 leaves the window, which moves down by one
        if (g == 0) Lb[zidx(kk, j)] = zst;
        zst = zw[0];
        const double nxt = __shfl_down(zw[0], 16, 64);
        zw[0] = zw[1];
        zw[1] = zw[2];
        zw[2] = zw[3];
        zw[3] = g < 3 ? nxt : 0.0;
    }
    {
        const int jl = N - 2;   // the last two columns (N >= 16)
        if (g == 0) {
            Lb[zidx(kk, jl)] = zst;
            Lb[zidx(kk, jl + 1)] = zw[0];
        }
    }
    __syncthreads();

    // ---- implicit QR sweeps with Wilkinson shifts on (diagonal 0, diagonal 1) ----
    // every lane runs the scalar chain and rotates row lane mod 16 of Z
    double *A_ = Lb;
    double *B_ = Lb + kQN;
    const int zrow = lane & 15;
    double *Zr = Lb + zidx(zrow, 0);   // row zrow of Z (lanes 16.. repeat rows 0..15)
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
        // the largest lo < hi with B_[lo-1] negligible (or 0), 64 candidates at a time
        int lo = 0;
        for (int base = hi - 1; base > 0; base -= 64) {
            const int i = base - lane;
            bool neg = false;
            if (i >= 1) {
                const double bl = fabs(B_[i - 1]);
                neg = bl <= DBL_EPSILON * (fabs(A_[i - 1]) + fabs(A_[i])) || bl < DBL_MIN;
            }
            const unsigned long long m = __ballot(neg);
            if (m) {
                lo = base - (__ffsll((long long)m) - 1);
                break;
            }
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
        // the values a rotation changes and the next one reads (A[q], B[q],
        // row `zrow` of Z at q) are carried in registers; the ones it reads
        // ahead (A[q+1], B[q+1], Z at q+1, not yet written in this sweep) come
        // from three register sets by position mod 3, each reloaded three
        // indices ahead once its rotation has used it.  The main loop runs
        // three rotations with no condition inside (the first (hi - lo) mod 3
        // rotations read their operands directly), so every load lands in the
        // register that carries it and stays in flight for two rotations.
        // Indices are clamped to hi: B[hi] is 0 (set when hi last moved down,
        // or beyond the matrix), which is what a sweep's last rotation takes
        // for B[q+1].
        double ak = A_[lo], bk = B_[lo];
        double zk = Zr[lo];
        double nbk = bk;
        auto rot = [&](int q, double ak1, double bk1, double z1) __attribute__((always_inline)) {
            // (q2 = 0 only when x = y = 0: then r = sn = 0 as they stand)
            const double q2 = x * x + y * y;
            const bool nz = q2 > 0.0;
            const double ir = rsqrt_pos(nz ? q2 : 1.0);
            const double r = q2 * ir;
            const double cs = nz ? x * ir : 1.0;
            const double sn = y * ir;
            const double na = cs * cs * ak + 2.0 * cs * sn * bk + sn * sn * ak1;
            const double na1 = sn * sn * ak - 2.0 * cs * sn * bk + cs * cs * ak1;
            nbk = cs * sn * (ak1 - ak) + (cs * cs - sn * sn) * bk;
            // every lane writes: the scalar values are the same in all lanes,
            // and lanes 16.. repeat the Z rows of lanes 0..15 with the same
            // values; the first rotation of a sweep has no B to write (slot
            // kQN - 1, past every B the sweeps read and before Z's first row)
            B_[q > lo ? q - 1 : kQN - 1] = r;
            A_[q] = na;
            Zr[q] = cs * zk + sn * z1;
            zk = -sn * zk + cs * z1;
            ak = na1;
            bk = cs * bk1;
            x = nbk;
            y = sn * bk1;
        };
        int q = lo;
        for (const int q0 = lo + (hi - lo) % 3; q < q0; ++q) {
            const int i = q + 1;
            rot(q, A_[i], B_[i], Zr[i]);
        }
        if (q < hi) {
            int i0 = q + 1, i1 = min(q + 2, hi), i2 = min(q + 3, hi);
            double a0 = A_[i0], b0 = B_[i0], z0 = Zr[i0];
            double a1 = A_[i1], b1 = B_[i1], z1 = Zr[i1];
            double a2 = A_[i2], b2 = B_[i2], z2 = Zr[i2];
            for (; q < hi; q += 3) {
                rot(q, a0, b0, z0);
                i0 = min(q + 4, hi);
                a0 = A_[i0];
                b0 = B_[i0];
                z0 = Zr[i0];
                rot(q + 1, a1, b1, z1);
                i1 = min(q + 5, hi);
                a1 = A_[i1];
                b1 = B_[i1];
                z1 = Zr[i1];
                rot(q + 2, a2, b2, z2);
                i2 = min(q + 6, hi);
                a2 = A_[i2];
                b2 = B_[i2];
                z2 = Zr[i2];
            }
        }
        if (lane == 0) {
            A_[hi] = ak;
            B_[hi - 1] = nbk;
        }
        Zr[hi] = zk;
        __syncthreads();
    }
    __syncthreads();
    // F = Z h(Theta) Z^T, then S = R0^T F R0 (diagonal only)
    for (int e = lane; e < 256; e += 64) {
        const int a = e >> 4, b = e & 15;
        double s = 0.0;
        for (int q = 0; q < N; ++q) s += Lb[zidx(a, q)] * Lb[zidx(b, q)] * blk_step(A_[q], smooth_w);
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
