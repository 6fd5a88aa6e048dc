// Internal interfaces of the eigenvalue-count library (not part of the ABI).
//
// Device data layout (all block vectors "probe-minor"):
//   a block vector of the run is n rows x C columns, element (r, c) at r*C + c,
//   with C = nshift * m columns: column c = s*m + j is probe j at shift s.
//   basis: (k+1) slots of one block vector each.  Slot l holds the Lanczos
//   vector q_{l+1} *unnormalized*; its per-column scale sig[l][c] (1/|v| for
//   l = 0, 1/beta_{l+1} afterwards, 0 once the column has stopped) turns it
//   into q_{l+1}.  Slot i first receives C q_i (operator output) and is then
//   overwritten in place by the reorthogonalized residual.
//
// Segments: a batch of independent problems is stored block-diagonally, the
// rows of problem b (a "segment") at [seg_row[b], seg_row[b+1]).  Every
// column-wise scalar (nu, alpha, beta, sig, kappa, ...) is kept per
// (segment, column), "virtual column" vc = b*C + c, and every reduction runs
// over the rows of one segment only (row chunks never straddle segments), so
// the batch is exactly nseg independent runs.  A single problem is nseg = 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace ecnt {

constexpr int kColTile = 64;       // columns per wavefront (one lane per column)
constexpr int kBasisChunk = 32;    // basis vectors per reorthogonalization launch
constexpr int kMaxShifts = 64;
constexpr int kMaxK = 512;
constexpr int kBlk = 16;           // probe columns per block of the block-Lanczos form
constexpr int kBlkMaxK = 32;       // block-Lanczos steps (T_k of order <= 512)
constexpr int kBlkChunk = 32;      // basis blocks per block reorthogonalization launch

// One shift's factor of the LDL preconditioner (device pointers).
struct LdlDev {
    const int32_t *perm = nullptr, *lrp = nullptr, *lci = nullptr;
    const double *lval = nullptr;
    const double *dd = nullptr, *doff = nullptr;
    int64_t nnz = 0;
    int bw = 0;
};

struct Plan {
    int64_t n = 0;
    int m = 0, S = 0, k = 0;
    int Ct = 0;           // all Lanczos columns, m * S
    int C = 0;            // columns of the current wave (block vector width)
    int wave_cols = 0;    // columns per wave (== Ct unless bounded by opts.max_cols)
    int c_off = 0;        // global index of the wave's first column
    int vec_f32 = 0;      // 0: FP64 vectors, 1: FP32 vectors
    int val_f32 = 0;      // A values FP32
    int prec_kind = 0;
    int ndim = 0, dims[3] = {1, 1, 1};
    int max_d2 = 1;            // largest z extent of the segments' grids
    int64_t max_rows = 0;      // largest segment (rows)
    int degree = 0;
    double coef[17] = {0};
    double s = 0, lo = 0, hi = 0;
    int rule = 0;
    double smooth_w = 0;
    // M = lead * prod_f factor_f(B): linear (B - a) or quadratic (B^2 - 2aB + b),
    // from the roots of the Chebyshev series (used when they reproduce it).
    int product = 0;
    int nfac = 0;
    int fac_quad[16] = {0};
    double fac_a[16] = {0}, fac_b[16] = {0};
    double lead = 1.0;
    // geometry
    int vw = 1;           // columns per lane in the CSR sweep
    int req_tile = 0, req_red_waves = 0, req_vw = 0;   // launch-shape requests (0: default)
    int req_fused = 0;    // opts.fused: 0 the one-launch form when it applies, 1 never
    int nct = 0;          // column tiles of 64 (setup kernel)
    int nchunk = 0;       // row chunks of the two-phase column reductions (all segments)
    int64_t rpc = 0;      // rows per chunk
    // segments
    int nseg = 1;
    int tx = 4, ty = 4;   // stencil line-block shape (4x4, 2x4 or 1x8)
    int no_fuse = 0;      // 1: quadratic factors as two plain sweeps
    int64_t ntiles = 0;   // stencil line blocks over all segments
    int64_t *seg_row = nullptr;    // device, nseg+1
    int64_t *seg_chunk = nullptr;  // device, nseg+1
    int64_t *seg_tile = nullptr;   // device, nseg+1
    int32_t *seg_dims = nullptr;   // device, 3*nseg (d0, d1, d2; d2 contiguous)
    double *seg_taus = nullptr;    // device, nseg*S
    // workspace carve (device pointers)
    void *basis = nullptr;     // (k+1) slots of n * C elements, slot_elems() apart
    size_t slot_pad = 0;       // elements between consecutive slots beyond n * C
    void *tmp[3] = {nullptr, nullptr, nullptr};
    double *part = nullptr;    // nchunk * kPartRows * C
    double *sig = nullptr;     // (k+1) * C
    double *alpha = nullptr;   // k * C
    double *beta = nullptr;    // (k+1) * C
    double *cf = nullptr;      // (k+1) * NC   (update coefficients of the basis slots)
    double *kappa = nullptr;   // C                 (beta_i * sig_{i-2})
    double *runmax = nullptr;  // C
    double *nu = nullptr;      // C

    double *s_out = nullptr;   // Ct  per-column quadrature s_c (wave views are offset)
    double *minabs = nullptr;  // Ct
    double *jac = nullptr;     // S * n (Jacobi scaling)
    double *result = nullptr;  // 4*S + 8 small results
    int32_t *active = nullptr; // C
    int32_t *kused = nullptr;  // Ct
    int32_t *flags = nullptr;  // 4 status flags: Jacobi singular, tridiagonal diverged,
                               // A not of the stencil form
    // ---- A applied as a grid stencil (Laplacian-polynomial preconditioner) ----
    int stencil_a = 0;         // A may be a stencil on the preconditioner's grid
    int a_mode = 0;            // 0: decided on the device (both forms launched, each gated
                               // on flags[2]); 1: the stencil form; 2: the CSR form
    int64_t st_ref_row = -1;   // row whose first off-diagonal value is a_off
    double *st_diag = nullptr; // n: diagonal of A
    double *st_coff = nullptr; // 1: a_off
    // ---- LDL preconditioner: one factor per shift, |D|^{-1/2} blocks ----
    LdlDev ldl[kMaxShifts];
    double *e_blk = nullptr;   // S * 2n: e_diag then e_off of every shift
    double *band = nullptr;    // S * 2 * n * 256: rows of L and of L^T by distance
    // ---- Arnoldi estimator for an unfactored T (one problem) ----
    int arnoldi = 0;
    double *H = nullptr;       // k x (k+1) x NC: H[(l*(k+1) + i)*NC + vc] = h_{i+1,l+1}
    // ---- block-Lanczos form: blocks of kBlk columns, FP64, one problem ----
    int block = 0;
    int nblk = 0;              // column blocks of a wave (wave_cols / kBlk)
    int bk_nchunk = 0;         // row chunks of the block reductions
    int64_t bk_rpc = 0;        // rows per chunk, a multiple of 16
    double *bk_part = nullptr; // bk_nchunk * kBlkChunk * nblk * 256 partial 16 x 16 sums
    double *bk_S = nullptr;    // (k+1) * nblk * 256: S_l (Q_l = X_l S_l)
    double *bk_K = nullptr;    // k * nblk * 256: -K_l in MFMA operand order
    double *bk_A = nullptr;    // k * nblk * 256: A_1..A_k
    double *bk_B = nullptr;    // (k+1) * nblk * 256: B[i] = B_{i+1}
    double *bk_R0 = nullptr;   // nblk * 256
    double *bk_R1 = nullptr;   // nblk * 256: first Cholesky factor of the current step
    double *bk_T = nullptr;    // nblk * 256: normalizing transform, operand order
    double *bk_rm = nullptr;   // nblk: largest |entry| of the A_i, B_i so far
    int32_t *bk_act = nullptr; // nblk
    // ---- differentiated form (smoothed count), single wave, FP64 ----
    int grad = 0;
    void *g_tslots = nullptr;  // k blocks: M q_i of every forward step
    double *g_qbar = nullptr;  // k blocks: adjoints of q_1..q_k (slot-indexed)
    double *g_ybar = nullptr;  // block: adjoint of C q_i
    double *g_tbar = nullptr;  // block: M ybar
    double *g_gall = nullptr;  // k*k*C: update coefficients c_i[l] of every step
    double *g_pall = nullptr;  // k*k*C: Gram column q_l^T q_i - [l = i] of every step
    double *g_Z = nullptr;     // k*k*C: eigenvectors of J
    double *g_theta = nullptr; // k*C
    double *g_sval = nullptr;  // k*C
    double *g_abar = nullptr;  // k*C
    double *g_bbar = nullptr;  // (k+1)*C
    double *g_coef = nullptr;  // 4*32*C
    double *g_scal = nullptr;  // 2*C
    double *g_vpart = nullptr; // ceil(C/64)*n
    double *g_taubar = nullptr;// C
    double *g_sums = nullptr;  // 64*C: chunk-summed backward dots
    size_t bytes = 0;
};

constexpr int kPartRows = 64;      // rows per chunk of the partial-sum buffer

// When a block vector is an exact power of two in size, consecutive basis
// slots (and the per-step slots of the differentiated form) are this many
// bytes further apart: slots 2^k bytes apart send the ~30 streams of a
// reorthogonalization sweep to the same HBM channels and banks row after row
// (measured at 64^3 x 512 columns: +6% for the dots sweep, +4% for the update
// sweep).  Other sizes keep contiguous slots (at 96^3 x 256 columns the pad
// cost the backward update sweep 8%).  A multiple of 256.
constexpr size_t kSlotPadBytes = 4352;
inline size_t slot_elems(const Plan &p) { return (size_t)p.n * p.C + p.slot_pad; }
inline size_t slot_bytes(const Plan &p) { return slot_elems(p) * (p.vec_f32 ? 4 : 8); }
constexpr int kResStride = 4 * kMaxShifts + 8;   // result doubles per segment

// Host copy of the segment tables.
struct SegHost {
    std::vector<int64_t> row, chunk, tile;
    std::vector<int32_t> dims;
    std::vector<double> taus;
};

size_t plan_layout(Plan &p, char *base);   // base == nullptr: size only

// ---- launchers (all enqueue on `st`) ----
void launch_jacobi_diag(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx,
                        const void *val, hipStream_t st);
void launch_setup(const Plan &p, const void *probes, hipStream_t st);
void launch_setup_fin(const Plan &p, hipStream_t st);
// y = M (A - tau_c I) M x  for the Jacobi / no-preconditioner path (one fused sweep)
// (gate: the status flags; the launch does nothing when flags[2] == 0, i.e.
// when the stencil form applies A)
void launch_csr_op(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                   const void *x, const double *xscale, const double *pre_post, void *y,
                   hipStream_t st, const int32_t *gate = nullptr);
// A as a grid stencil: the pattern / value check (sets flags[2] if A is not of
// that form, fills st_diag, st_coff) and y = xs .* ((A - tau_c I) x) by a
// stencil sweep that runs only when the check passed
void launch_stencil_check(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx,
                          const void *val, hipStream_t st);
void launch_stencil_a(const Plan &p, const void *x, const double *xs, void *y, hipStream_t st);
// out = cx*xs*X + cb*B(ins*IN) - cz*Z  (one stencil sweep on the grid Laplacian)
void launch_stencil(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                    bool in_is_x, double cb, const void *Z, double cz, void *out, hipStream_t st);
// One quadratic factor in one sweep: t = c1*u + cb*B(u), out = B(t) + c2*u - cz*Z,
// u = xs .* X (Z may be null).  Needs the 4 x 4 line-block geometry.
bool quad_sweep_supported(const Plan &p);
void launch_quad_sweep(const Plan &p, const void *X, const double *xs, double c1, double cb,
                       double c2, const void *Z, double cz, void *out, hipStream_t st);
void launch_dots(const Plan &p, int step, int l0, int nb, bool gram, hipStream_t st);
void launch_dots_fin(const Plan &p, int step, int l0, int nb, bool gram, hipStream_t st);
void launch_update(const Plan &p, int step, int l0, int nb, bool first, bool last, hipStream_t st);
void launch_norm_fin(const Plan &p, int step, hipStream_t st);
void launch_tridiag(const Plan &p, hipStream_t st);
// the one-launch Lanczos form of small problems (k_small.hip)
constexpr int kFusedMaxRows = 3072;   // rows of the largest segment
constexpr int kFusedMaxK = 64;
constexpr size_t kFusedLdsBytes = 150 * 1024;   // the column's operator, q and w in LDS
bool fused_applies(const Plan &p, int64_t nnz);
void launch_lanczos_fused(const Plan &p, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                          int64_t nnz, const void *probes, hipStream_t st);
void launch_reduce(const Plan &p, hipStream_t st);
// Arnoldi estimator
void launch_arn_fin(const Plan &p, int step, int l0, int nb, int pass, hipStream_t st);
void launch_arn_norm_fin(const Plan &p, int step, hipStream_t st);
void launch_arn_quad(const Plan &p, hipStream_t st);
// backward of the smoothed count
void launch_tridiag_bwd(const Plan &p, double g_out, hipStream_t st);
void launch_bdots(const Plan &p, int i, hipStream_t st);
void launch_bdots_fin(const Plan &p, int i, bool have_dots, hipStream_t st);
void launch_bupdate(const Plan &p, int i, bool first, hipStream_t st);
void launch_bnorm_fin(const Plan &p, int i, hipStream_t st);
void launch_vgrad(const Plan &p, const double *tq, bool first, hipStream_t st);
void launch_grad_out(const Plan &p, double *dV, hipStream_t st);

// block-Lanczos form (k_block.hip); slots are basis slot indices
void launch_blk_dots(const Plan &p, int l0, int nb, int ys, hipStream_t st);
void launch_blk_dots_fin(const Plan &p, int l0, int nb, int icur, hipStream_t st);
void launch_blk_update(const Plan &p, int l0, int nb, int ws, bool last, hipStream_t st);
void launch_blk_normalize(const Plan &p, int ws, hipStream_t st);
void launch_blk_norm_fin(const Plan &p, int mode, int step, hipStream_t st);
void launch_blk_quad(const Plan &p, hipStream_t st);

// LDL preconditioner: |D|^{-1/2} blocks and band form of every shift's
// factor; on the columns of the current wave (X and Y distinct):
// what = 0: Y = |D|^{-1/2}(xs.*X), 1: Y = L^{-1} X, 2: Y = L^{-T} X,
// 3: Y = P X, 4: Y = P^T X
void launch_ldl_eblocks(const Plan &p, hipStream_t st);
void launch_ldl(const Plan &p, int what, const void *X, const double *xs, void *Y, hipStream_t st);
int ldl_ring_rows();
size_t ldl_band_bytes(int64_t n, int S);   // the band forms of S factors, with their padding

// bandwidth probes (k_probe.hip): 0 copy, 1 read, 2 update mix; 0 ok, -1 HIP error
int run_probe(int kind, void *buf, size_t bytes, int reps, hipStream_t st, double *gbs);

// the message ecnt_last_error() returns; gives back st
int32_t set_error(int32_t st, const char *msg);

}  // namespace ecnt
