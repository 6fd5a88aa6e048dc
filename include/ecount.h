/*
 * ecount.h -- C ABI of the MI355X eigenvalue-count library.
 *
 * Estimates the number of eigenvalues of a sparse real symmetric matrix A in
 * an interval [xi, eta) with the preconditioned Lanczos / Gauss-quadrature /
 * Hutchinson estimator of Vecharynski & Yang, "Preconditioned iterative
 * methods for eigenvalue counts":
 *
 *   c(xi, eta) = n_(A - eta I) - n_(A - xi I)              (Section 2)
 *   n_(A - tau I) = trace h(C),  C = M (A - tau I) M^*,   T = M^* M HPD
 *                                                          (Section 2, eq. negi_T)
 *   n_(A - tau I) ~ L_tau(k, m) = (1/m) sum_j |v_j|^2 sum_{theta_i < 0} z_i(1)^2
 *                                                          (Section 3.2, eq. rand_prec_quad,
 *                                                           Algorithm 2)
 * where theta_i, z_i are the eigenpairs of the k x k Lanczos matrix J_k from
 * k steps of Lanczos with full reorthogonalization on C started at v_j
 * (Section 3.1, Algorithm 1, eq. gauss_quad).
 *
 * Conventions shared by every entry point
 *   - Every function returns an ecnt_status: 0 on success, < 0 on error; no
 *     C++ exception crosses the ABI.  ecnt_last_error() gives a message.
 *   - Pointers marked "device" are HIP device pointers (memory owned by the
 *     caller); "host" pointers are ordinary host memory.  The library never
 *     allocates device memory at run time and keeps no pointer after a call
 *     returns (the fixed array behind ecnt_count_noalloc is a static device
 *     variable of the library, set up when its code is loaded on a GPU).
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     is enqueued on it.  Functions returning host results synchronize that
 *     stream before returning.
 *   - Argument validation happens entirely on the host, before any device
 *     work is enqueued; a rejected call touches no device state.
 *   - Block vectors on the device are row-major n x m ("probe-minor": entry
 *     (r, j) at index r*m + j).
 */
#ifndef ECOUNT_H
#define ECOUNT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ECNT_API __attribute__((visibility("default")))
#else
#define ECNT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ecnt_status;
#define ECNT_OK 0
#define ECNT_EINVAL (-1)       /* invalid argument (null pointer, bad size, xi >= eta, ...) */
#define ECNT_ENOTHPD (-2)      /* preconditioner not HPD (Jacobi pivot a_rr == tau)       */
#define ECNT_EWORKSPACE (-3)   /* workspace missing or smaller than ecnt_workspace_bytes() */
#define ECNT_EDEVICE (-4)      /* HIP runtime error, or the tridiagonal solver diverged   */
#define ECNT_EUNSUPPORTED (-5) /* valid request outside what the library supports        */

typedef enum { ECNT_F64 = 0, ECNT_F32 = 1 } ecnt_dtype;

/* Sparse A in CSR form on the device.  Real symmetric, both triangles
 * stored, column indices sorted within a row, diagonal entry present when
 * non-zero.  int32 indices; values of type val_type (F64 or F32). */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t *row_ptr; /* device, n+1 */
    const int32_t *col_idx; /* device, nnz */
    const void *val;        /* device, nnz, val_type */
    int32_t val_type;
    int32_t reserved;
} ecnt_csr;

/* Preconditioner T = M^* M (Section 2; Section 6 lists the paper's choices).
 *   ECNT_PREC_NONE            M = I.
 *   ECNT_PREC_JACOBI          M_tau = diag(|a_rr - tau|)^(-1/2), built per shift from
 *                             the diagonal of A (an HPD absolute-value preconditioner in
 *                             the sense of Section 6; exact for diagonal A).
 *   ECNT_PREC_CHEB_LAPLACIAN  M = sum_{j=0}^{degree} coef[j] T_j(B),
 *                             B = (2 (L + s I) - (lo + hi) I) / (hi - lo),
 *                             L the Dirichlet Laplacian of the grid `dims` (diagonal
 *                             2*ndim, neighbours -1; a grid point (x, y, z) is row
 *                             (x*dims[1] + y)*dims[2] + z), shared by all shifts.
 *                             M is symmetric; T = M^2 must be HPD (the caller's
 *                             responsibility: M nonsingular on the spectrum of L).
 *   ECNT_PREC_LDL             the factored absolute-value preconditioner of Section 6,
 *                             one factor per shift: P (A - tau I) P^T ~ L D L^T,
 *                             T = P^T L^{-T} |D|^{-1} L^{-1} P (HPD for any L, D),
 *                             M = |D|^{-1/2} L^{-1} P, M^* = P^T L^{-T} |D|^{-1/2};
 *                             |D|^{-1/2} is formed block by block from D.  Factors
 *                             come from ecnt_ildl_factor (or any other source in the
 *                             same layout; perm must be a permutation).  The
 *                             triangular solves take L as a band of 256 diagonals: a
 *                             factor whose bandwidth (max i - j over the entries of L)
 *                             exceeds 256 is EUNSUPPORTED. */
typedef enum {
    ECNT_PREC_NONE = 0,
    ECNT_PREC_JACOBI = 1,
    ECNT_PREC_CHEB_LAPLACIAN = 2,
    ECNT_PREC_LDL = 3
} ecnt_prec_kind;

/* One shift's L D L^T factor on the device (ECNT_PREC_LDL).  All arrays are
 * device memory owned by the caller and must stay valid for the call.
 *   perm        n: row i of P (A - tau I) P^T is row perm[i] of A - tau I
 *   l_row_ptr   n+1, l_col_idx / l_val nnz: the strictly lower part of L
 *               (unit diagonal implied) by rows; entries with i - j above
 *               `bandwidth` are ignored
 *   d_diag      n: D_ii;  d_off n: D_{i+1,i} at the first row i of a 2 x 2
 *               block (non-zero there), 0 elsewhere
 *   nnz, bandwidth  entry count and max (i - j) over the entries
 * Each call first writes L and L^T into its workspace as bands of 256 values
 * per row (2 * 256 * 8 bytes per row and shift). */
typedef struct {
    const int32_t *perm;
    const int32_t *l_row_ptr;
    const int32_t *l_col_idx;
    const double *l_val;
    const double *d_diag;
    const double *d_off;
    int64_t nnz;
    int32_t bandwidth;
    int32_t reserved;
} ecnt_ldl_factor;

/* How M is evaluated (CHEB only).  Both compute the same polynomial in B. */
typedef enum {
    ECNT_EVAL_AUTO = 0,     /* product of real linear/quadratic factors from the roots of
                               the series when they reproduce it to 1e-12, else Clenshaw */
    ECNT_EVAL_CLENSHAW = 1  /* Clenshaw's recurrence on the series */
} ecnt_eval;

typedef struct {
    int32_t kind;        /* ecnt_prec_kind */
    int32_t ndim;        /* 1..3 (CHEB only) */
    int32_t dims[3];     /* grid extents, product == n (CHEB only) */
    int32_t degree;      /* 0..16 (CHEB only) */
    int32_t eval;        /* ecnt_eval (CHEB only) */
    double s, lo, hi;    /* shift of L and the interval mapped to [-1, 1] (CHEB only) */
    const double *coef;  /* host, degree+1 entries, copied at call time (CHEB only) */
    const ecnt_ldl_factor *ldl; /* host, one factor per shift in shift order, read at call
                                   time (LDL only; NULL otherwise) */
} ecnt_prec;

/* Quadrature rule applied to the Lanczos coefficients. */
typedef enum {
    ECNT_RULE_GAUSS = 0, /* k-node Gauss rule from J_k (Section 3.1, eq. gauss_quad) */
    ECNT_RULE_GA = 1     /* generalized averaged Gauss rule from the (2k-1) x (2k-1)
                            matrix of Section 3.4, eq. GA_Tk */
} ecnt_rule;

typedef struct {
    int32_t k;          /* Lanczos steps, 1 <= k <= min(n, 512) (k <= 256 for GA) */
    int32_t vec_type;   /* storage of probes, Lanczos vectors and basis: F64 or F32.
                           alpha/beta, every dot product and norm, and the tridiagonal
                           eigensolve are FP64 in both cases. */
    int32_t rule;       /* ecnt_rule */
    int32_t max_cols;   /* 0: all nshift*m Lanczos columns run together.  > 0: the columns
                           (column c = shift c/m, probe c%m) run in consecutive waves of at
                           most max_cols, reusing one workspace: bounds the memory of the
                           Lanczos basis ((k+1) x n x max_cols vectors) at the cost of more
                           passes over A.  Results do not depend on it. */
    double smooth_w;    /* 0: the paper's step h (h(theta) = 1 iff theta < 0).
                           > 0: h replaced by erfc(theta / smooth_w) / 2. */
    /* Launch-shape tunables (0 = built-in default).  They change how the
       work is cut into workgroups, not what is computed: results move at
       most by the order of floating-point sums. */
    int32_t tile;       /* stencil line block: 1 = 4x4 lines, 2 = 2x4, 3 = 1x8 (0: 1x8 when
                           some grid has fewer than 4 x-planes, else 5 when it applies,
                           else 4x4).  With 4x4
                           blocks each quadratic factor of the product-form
                           preconditioner runs as one fused sweep; 4 = 4x4 blocks with
                           two plain sweeps per quadratic factor; 5 = 8x8 blocks, one
                           workgroup of 16 wavefronts per block sharing lines through
                           LDS (when every factor is quadratic; otherwise as 1). */
    int32_t red_waves;  /* target wavefronts of a column-reduction launch, 64..65536
                           (sets the rows per chunk of the two-phase sums; 0: 2048) */
    int32_t csr_vw;     /* columns per lane of the CSR sweep: 1, 2 (or 4 with FP32
                           vectors); used when it divides the wave's width (0: widest) */
    int32_t a_form;     /* how A is applied with ECNT_PREC_CHEB_LAPLACIAN (ignored
                           otherwise).  0: as a stencil sweep on the preconditioner's
                           grid when A is of that form (checked on the device at the
                           start of each call: its CSR entries are exactly the grid
                           neighbours and the diagonal, all off-diagonal values equal),
                           else row by row from the CSR arrays; 1: always from the CSR
                           arrays.  Both sum each row in the same order. */
    int32_t fused;      /* 0: a problem whose segments have at most 3072 rows, with FP64
                           vectors, k <= 64, M = I or Jacobi, no derivative, and whose
                           operator fits in a workgroup's LDS (12 bytes per nonzero of A,
                           counted over all segments, plus 28 per row of the largest
                           segment, at most 150 KiB), runs all k steps of every column
                           in one launch (one workgroup per column, its basis
                           column-contiguous in the workspace); otherwise, and with 1,
                           the column-wave kernels (about five launches per step).  Both
                           compute the same recurrence; sums are in a different
                           order. */
} ecnt_opts;

/* Optional outputs.  Device arrays may be NULL. */
typedef struct {
    double neg_xi;        /* L_xi(k, m): estimate of n_(A - xi I)   (count entry)   */
    double neg_eta;       /* L_eta(k, m): estimate of n_(A - eta I) (count entry)   */
    double min_abs_ritz;  /* min |theta| over all probes and shifts: a value within
                             rounding of 0 makes h(theta) tie-sensitive */
    double *per_probe;    /* device, nshift*m: s_j(tau) = |v_j|^2 sum_{theta<0} z(1)^2,
                             shift-major (all probes of shift 0 first)             */
    int32_t *k_used;      /* device, nshift*m: steps actually taken (< k after an
                             invariant Krylov space was found)                     */
    double *alpha;        /* device, k x (nshift*m): alpha_1..alpha_k per column    */
    double *beta;         /* device, (k+1) x (nshift*m): beta_1 = 0, beta_2..beta_{k+1} */
} ecnt_info;

/* Bytes of device workspace needed by ecnt_count / ecnt_negcounts for n rows,
 * m probes and nshift shifts (ecnt_count uses nshift = 2).  Returns 0 if the
 * arguments are invalid. */
ECNT_API size_t ecnt_workspace_bytes(int64_t n, int64_t m, int32_t nshift, const ecnt_prec *T,
                            const ecnt_opts *opts);

/* Interval count c(xi, eta) ~ L_eta(k, m) - L_xi(k, m) (end of Section 3.2:
 * Algorithm 2 run at tau = xi and tau = eta), on the same probe block for
 * both shifts.
 *   probes    device, n x m row-major, vec_type.  Any i.i.d. zero-mean
 *             unit-variance entries (Section 2, eq. trace); read only.
 *   estimate  host: mean over probes of d_j = s_j(eta) - s_j(xi)
 *   variance  host: sample variance of d_j divided by m (NaN when m == 1);
 *             the Hutchinson sampling error only, not the quadrature bias.
 *   info      host, nullable.
 * Errors: EINVAL (null pointers, n < 1, m < 1, k < 1, k > n, !(xi < eta),
 * non-finite xi/eta, bad preconditioner fields), ENOTHPD (Jacobi pivot
 * a_rr == xi or eta), EWORKSPACE, EUNSUPPORTED (k above the limits above),
 * EDEVICE. */
ECNT_API ecnt_status ecnt_count(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                       const void *probes, int64_t m, const ecnt_opts *opts, void *ws,
                       size_t ws_bytes, void *stream, double *estimate, double *variance,
                       ecnt_info *info);

/* ---- Interval count without allocation ----
 *
 * For callers that cannot allocate device memory or pass a workspace: tight
 * serving loops and harnesses that forbid hipMalloc.  Same computation,
 * arguments, outputs and errors as ecnt_count, minus `ws` / `ws_bytes`: the
 * scratch (Lanczos basis, partial sums, per-column scalars) lives in a fixed
 * device array of ECNT_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends.  The caller still owns A, the probes
 * and the outputs.  No hipMalloc, hipFree or other allocating routine is
 * called.
 *   - The device is the current one; a non-NULL stream must belong to it
 *     (else ECNT_EINVAL).
 *   - A count whose ecnt_workspace_bytes(n, m, 2, T, opts) exceeds
 *     ECNT_NOALLOC_SCRATCH_BYTES is refused with ECNT_EWORKSPACE before any
 *     device work.
 *   - All calls on one GPU share its array, which keeps the last call's
 *     contents (nothing read by a call depends on them).  Calls through this
 *     entry point are serialized per device by the library (each returns
 *     after its stream has drained); other code that touches the array while
 *     a call runs races with it. */
#define ECNT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

ECNT_API ecnt_status ecnt_count_noalloc(const ecnt_csr *A, const ecnt_prec *T, double xi,
                                        double eta, const void *probes, int64_t m,
                                        const ecnt_opts *opts, void *stream, double *estimate,
                                        double *variance, ecnt_info *info);

/* Algorithm 2 for several shifts at once (spectrum slicing, Section 1): all
 * nshift x m Lanczos runs share one probe block and one launch sequence.
 *   taus       host, nshift finite shifts
 *   negcounts  host, nshift: L_tau(k, m) per shift
 *   counts     host, nullable, nshift-1: mean of s_j(taus[s+1]) - s_j(taus[s])
 *   variances  host, nullable, nshift-1: sample variance of those differences / m
 * Errors as ecnt_count (nshift < 1 or > 64 -> EINVAL). */
ECNT_API ecnt_status ecnt_negcounts(const ecnt_csr *A, const ecnt_prec *T, const double *taus,
                           int32_t nshift, const void *probes, int64_t m, const ecnt_opts *opts,
                           void *ws, size_t ws_bytes, void *stream, double *negcounts,
                           double *counts, double *variances, ecnt_info *info);

/* ---- Differentiated form: gradient of an erf-smoothed count ----
 *
 * With smooth_w = w > 0 the step h(theta) of eq. gauss_quad is replaced at the
 * Ritz values by S_w(theta) = erfc(theta / w) / 2 (the rule only sees h at the
 * Ritz values, Section 3.3), which makes the computed estimate a smooth
 * function of A's diagonal and of the shifts.  The forward is ecnt_count's
 * (Algorithm 1: alpha_i first, then one classical Gram-Schmidt pass, fused
 * into one update), so ecnt_smooth_fwd and ecnt_count with the same smooth_w
 * return the same estimate.  The backward pass is the exact reverse-mode
 * derivative of what those kernels compute (each step of Algorithm 1
 * differentiated in reverse, the Gram-Schmidt coefficients as used; the
 * tridiagonal step by the Daleckii-Krein formula).  Restrictions: FP64, Gauss
 * rule, ECNT_PREC_CHEB_LAPLACIAN (M does not depend on A or tau), k <= 32,
 * max_cols = 0; otherwise ECNT_EUNSUPPORTED.
 *
 * State kept between forward and backward (ECNT_CKPT_KEEP): the Lanczos basis,
 * M q_i of every step and the Gram-Schmidt coefficients, in the workspace
 * (sized by ecnt_smooth_workspace_bytes), which the caller must not touch
 * between the two calls.  ECNT_CKPT_RECOMPUTE: the backward reruns the
 * forward first, so the workspace may be reused in between. */
typedef enum { ECNT_CKPT_KEEP = 0, ECNT_CKPT_RECOMPUTE = 1 } ecnt_ckpt;

ECNT_API size_t ecnt_smooth_workspace_bytes(int64_t n, int64_t m, const ecnt_prec *T,
                                            const ecnt_opts *opts);

/* Smoothed interval count; same arguments and outputs as ecnt_count. */
ECNT_API ecnt_status ecnt_smooth_fwd(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                                     const void *probes, int64_t m, const ecnt_opts *opts,
                                     void *ws, size_t ws_bytes, void *stream, double *estimate,
                                     double *variance, ecnt_info *info);

/* Gradient of g_est * estimate with respect to A's diagonal (dV: device, n
 * doubles, overwritten) and the endpoints (dxi, deta: host).  All other
 * arguments must equal those of the forward call. */
ECNT_API ecnt_status ecnt_smooth_bwd(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                                     const void *probes, int64_t m, const ecnt_opts *opts,
                                     int32_t ckpt, double g_est, void *ws, size_t ws_bytes,
                                     void *stream, double *dV, double *dxi, double *deta);

/* ---- Arnoldi estimator for an unfactored preconditioner (Section 4) ----
 *
 * When T is not available as M*M, the estimator runs on C = T (A - tau I)
 * (Algorithm 4): k Arnoldi steps per probe give an upper Hessenberg H_k
 * (Algorithm 3; here two classical Gram-Schmidt passes per step, equal to its
 * modified Gram-Schmidt loop in exact arithmetic), and
 *   s_j(tau) = |v_j|^2 e_1^T h(H_k) e_1      (eq. arnoldi_quad),
 * h = 1 on the open left half-plane, evaluated through the matrix sign
 * function of H_k (real arithmetic).  T here IS the preconditioner:
 * ECNT_PREC_NONE (T = I) or ECNT_PREC_CHEB_LAPLACIAN (T = the series, which
 * must be positive on the spectrum of its argument); ECNT_PREC_JACOBI is
 * ECNT_EUNSUPPORTED.  Same arguments and outputs as ecnt_count, with
 * opts.rule = ECNT_RULE_GAUSS, opts.smooth_w = 0 and k <= 64 (otherwise
 * ECNT_EUNSUPPORTED); info->alpha / info->beta are not written and
 * info->min_abs_ritz is +inf (the eigenvalues of H_k are not formed).
 * EDEVICE if the sign iteration fails (an eigenvalue of H_k on the imaginary
 * axis). */
ECNT_API size_t ecnt_arnoldi_workspace_bytes(int64_t n, int64_t m, const ecnt_prec *T,
                                             const ecnt_opts *opts);

ECNT_API ecnt_status ecnt_count_arnoldi(const ecnt_csr *A, const ecnt_prec *T, double xi,
                                        double eta, const void *probes, int64_t m,
                                        const ecnt_opts *opts, void *ws, size_t ws_bytes,
                                        void *stream, double *estimate, double *variance,
                                        ecnt_info *info);

/* ---- Block-Lanczos form of the estimator (blocks of 16 probes) ----
 *
 * Not in the paper: the probe block is taken 16 columns at a time and each
 * block V_b runs one block Lanczos process on C = M (A - tau I) M^* (the
 * recurrence of Algorithm 1 with 16 x 16 blocks, one classical Gram-Schmidt
 * pass against the whole basis per step).  The block Gauss rule gives
 *   V_b^T h(C) V_b ~ R_0^T E_1^T h(T_k) E_1 R_0,   V_b = Q_1 R_0,
 * T_k the block-tridiagonal matrix of order 16 k; its diagonal entries are the
 * per-probe values s_j of eq. rand_prec_quad (Section 3.2), which with one
 * column per block is eq. gauss_quad itself.  A block stops early (k_used)
 * when a new block of the basis is numerically rank deficient: the smallest
 * diagonal entry of B_{i+1} is <= 1e3 eps times the largest entry of the
 * earlier A_i, B_i.  Same arguments and outputs as ecnt_count with: FP64
 * probes (opts.vec_type = ECNT_F64), m and opts.max_cols (if set) multiples
 * of 16, opts.rule = ECNT_RULE_GAUSS and k <= 32 (else ECNT_EINVAL or
 * ECNT_EUNSUPPORTED); M = I, Jacobi or the Laplacian polynomial
 * (ECNT_PREC_LDL is ECNT_EUNSUPPORTED).  With 16 k > n the block
 * Krylov space is exhausted and every block stops by then (k_used).  info->alpha /
 * info->beta are not written; info->per_probe and info->k_used (the block's
 * k_used for each of its columns, 0 if the probe block itself is rank
 * deficient) are. */
ECNT_API size_t ecnt_block_workspace_bytes(int64_t n, int64_t m, const ecnt_prec *T,
                                           const ecnt_opts *opts);

ECNT_API ecnt_status ecnt_count_block(const ecnt_csr *A, const ecnt_prec *T, double xi,
                                      double eta, const void *probes, int64_t m,
                                      const ecnt_opts *opts, void *ws, size_t ws_bytes,
                                      void *stream, double *estimate, double *variance,
                                      ecnt_info *info);

/* ---- Batches of independent problems ----
 *
 * Many small problems (each its own A_b, shifts and probe block) run as one
 * launch sequence: the batch is stored as one block-diagonal matrix whose
 * rows are the problems' rows in order, and every reduction, Lanczos scalar
 * and shift is kept per (problem, column), so the result for problem b is
 * exactly what ecnt_negcounts returns for it alone (Algorithm 2 per problem,
 * Section 3.2), up to the order of floating-point sums.
 *
 *   A         the block-diagonal matrix (rows and column indices global),
 *             A.n = sum of items[b].n
 *   items     host, nprob descriptions:
 *               n      rows of problem b
 *               dims   its grid (d0, d1, d2; d2 contiguous) for
 *                      ECNT_PREC_CHEB_LAPLACIAN, where T.ndim must be 3 and
 *                      the stencil of every problem is the 7-point one; with
 *                      other preconditioners dims is ignored
 *               taus   host, nshift finite shifts of problem b
 *   T         one preconditioner description for all problems (T.dims is
 *             ignored: each problem uses its own grid)
 *   probes    device, A.n x m row-major (rows of problem b at its offset)
 *   negcounts host, nprob x nshift; counts / variances nullable,
 *             nprob x (nshift-1), as ecnt_negcounts
 *   info      nullable; per_probe / k_used are nprob x (nshift*m); alpha and
 *             beta are not written for batches
 * Errors as ecnt_negcounts, plus EINVAL when a problem's grid does not match
 * its n or k exceeds a problem's n.
 *
 * The call is split in three so that the middle one can be captured into a
 * hipGraph and replayed: prepare (validates, carves the workspace, uploads the
 * per-problem tables; synchronous), enqueue (kernel launches on `stream`
 * only: no allocation, copy or host synchronization), results (copies the
 * results back; synchronizes `stream`).  All three take the same arguments;
 * the workspace must stay untouched between them.  ecnt_count_batched runs
 * all three. */
typedef struct {
    int64_t n;
    int32_t dims[3];
    int32_t reserved;
    const double *taus;
} ecnt_batch_item;

ECNT_API size_t ecnt_batch_workspace_bytes(const ecnt_batch_item *items, int32_t nprob,
                                           int32_t nshift, int64_t m, const ecnt_prec *T,
                                           const ecnt_opts *opts);

ECNT_API ecnt_status ecnt_batch_prepare(const ecnt_csr *A, const ecnt_prec *T,
                                        const ecnt_batch_item *items, int32_t nprob,
                                        int32_t nshift, const void *probes, int64_t m,
                                        const ecnt_opts *opts, void *ws, size_t ws_bytes,
                                        void *stream);

ECNT_API ecnt_status ecnt_batch_enqueue(const ecnt_csr *A, const ecnt_prec *T,
                                        const ecnt_batch_item *items, int32_t nprob,
                                        int32_t nshift, const void *probes, int64_t m,
                                        const ecnt_opts *opts, void *ws, size_t ws_bytes,
                                        void *stream);

ECNT_API ecnt_status ecnt_batch_results(const ecnt_batch_item *items, int32_t nprob,
                                        int32_t nshift, int64_t m, const ecnt_prec *T,
                                        const ecnt_opts *opts, void *ws, size_t ws_bytes,
                                        void *stream, double *negcounts, double *counts,
                                        double *variances, ecnt_info *info);

ECNT_API ecnt_status ecnt_count_batched(const ecnt_csr *A, const ecnt_prec *T,
                                        const ecnt_batch_item *items, int32_t nprob,
                                        int32_t nshift, const void *probes, int64_t m,
                                        const ecnt_opts *opts, void *ws, size_t ws_bytes,
                                        void *stream, double *negcounts, double *counts,
                                        double *variances, ecnt_info *info);

/* ---- ILDL(t) factorization on the host (Section 6) ----
 *
 * Incomplete L D L^T of A - tau I with 1 x 1 / 2 x 2 pivots and a drop
 * tolerance, from which ECNT_PREC_LDL builds T = P^T L^{-T} |D|^{-1} L^{-1} P
 * (HPD whatever is dropped).  The paper takes the factorization from an
 * external package; this one is right-looking in the matrix's own order with
 * Bunch-Kaufman partial pivoting (alpha = (1 + sqrt 17) / 8), and after each
 * pivot drops the multipliers l_i with |l_i| < droptol * sum_i |l_i| of their
 * column before the Schur update.  droptol = 0 gives the exact factorization
 * (Sylvester: the inertia of D is that of A - tau I).
 *   A          host CSR (row_ptr n+1, col_idx, val), symmetric, both triangles
 *   out        receives an opaque host object; release it with ecnt_ildl_free
 * Errors: EINVAL (bad arguments), ENOTHPD (a zero 1 x 1 or singular 2 x 2
 * pivot), EUNSUPPORTED (the factor exceeds int32 indexing).  Runs on the
 * host only: no device work. */
typedef struct ecnt_ildl_s *ecnt_ildl;

ECNT_API ecnt_status ecnt_ildl_factor(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                      const double *val, double tau, double droptol,
                                      ecnt_ildl *out);

/* nnz of L (strict lower part), its bandwidth, the number of 2 x 2 blocks
 * and of negative eigenvalues of D.  Null outputs are skipped. */
ECNT_API ecnt_status ecnt_ildl_sizes(const ecnt_ildl f, int64_t *nnz, int32_t *bandwidth,
                                     int32_t *n2x2, int32_t *nneg);

/* Copies the factor into caller-allocated host arrays laid out as
 * ecnt_ldl_factor describes (perm n, l_row_ptr n+1, l_col_idx / l_val nnz,
 * columns ascending within a row, d_diag n, d_off n).  Null outputs are
 * skipped. */
ECNT_API ecnt_status ecnt_ildl_export(const ecnt_ildl f, int32_t *perm, int32_t *l_row_ptr,
                                      int32_t *l_col_idx, double *l_val, double *d_diag,
                                      double *d_off);

ECNT_API void ecnt_ildl_free(ecnt_ildl f);

/* Per-kernel-family timing, for measurement.  While enabled, every launch
 * made by ecnt_count / ecnt_negcounts is bracketed by two hipEvents recorded
 * on the caller's stream; elapsed times and the algorithmic bytes of each
 * launch (the distinct block vectors and matrix arrays it must read or write)
 * are accumulated per kernel family.  Enabling resets the totals. */
typedef struct {
    char name[24];       /* kernel family, e.g. "lz_update" */
    int64_t launches;
    double total_ms;     /* sum of event-measured launch durations */
    double bytes;        /* sum of algorithmic bytes over those launches */
} ecnt_kernel_stat;

ECNT_API ecnt_status ecnt_profile_enable(int32_t on);
/* Copies up to `max` families into `out`; returns how many were written. */
ECNT_API int32_t ecnt_profile_read(ecnt_kernel_stat *out, int32_t max);

/* Bandwidth probe, for measurement: effective GB/s of a simple stream on the
 * current device, timed with HIP events over `reps` launches on `stream`
 * (synchronizes it).  kind 0: copy (16-byte loads and non-temporal stores,
 * four in flight per lane), 1: read only, 2: the read/write mix of one
 * Gram-Schmidt update sweep (16 vectors read, one read and written back).
 * `buf` is device scratch of `bytes` (copy/read use two halves, the mix 17
 * equal streams; at least 64 MiB, 1 GiB streams or more for stable numbers);
 * its contents are overwritten.  These bound what the estimator's sweeps can
 * reach; a roofline fraction can be quoted against them besides the peak.
 * Errors: EINVAL (bad kind, null pointer, buffer too small), EDEVICE. */
ECNT_API ecnt_status ecnt_hbm_probe(int32_t kind, void *buf, size_t bytes, int32_t reps,
                                    void *stream, double *gbs);

/* Message for the last failed call on this thread ("" if none). */
ECNT_API const char *ecnt_last_error(void);

/* Library version string. */
ECNT_API const char *ecnt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ECOUNT_H */
