/*
 * Lanczos oracle for the preconditioned eigenvalue-count estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written directly from the paper (Vecharynski & Yang, "Preconditioned
 * iterative methods for eigenvalue counts"), used to check the GPU library.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code with the GPU library.
 *
 * What it computes, per probe vector v_j and one shift tau (Section 3.1,
 * Algorithm 1; Section 3.2, Algorithm 2 steps 3-4): the k-step Lanczos
 * decomposition of C = M (A - tau I) M^* (Section 2, eq. negi_T) started at
 * q_1 = v/|v|,
 *
 *   C Q_k = Q_k J_k + beta_{k+1} q_{k+1} e_k^T      (eq. lan)
 *
 * built one column at a time: the coefficients of C q_i along q_{i-1} (beta_i,
 * already known) and q_i (alpha_i, taken first) are removed, the remainder
 * is projected off the whole basis q_1..q_i (full reorthogonalization: one
 * classical Gram-Schmidt pass that does not update alpha_i), and its norm
 * and direction give beta_{i+1} and q_{i+1}.
 *
 * It returns alpha_1..alpha_k, beta_1..beta_{k+1} (beta_1 = 0) and |v|^2.
 * The quadrature (eigendecomposition of J_k and the weighted count) is done
 * by the Python half of the oracle.
 *
 * Breakdown (not discussed in the paper): when
 *   beta_{i+1} <= 1e3 * eps * max(|alpha_1|..|alpha_i|, beta_2..beta_i)
 * the Krylov space is invariant; the run stops with k_used = i and J_i is
 * used (Proposition 1 makes the quadrature exact in that case).
 *
 * Preconditioners M (T = M^* M, all symmetric here):
 *   kind 0: M = I.
 *   kind 1: Jacobi, M_tau = |diag(A) - tau|^(-1/2), built per shift.
 *   kind 2: M = sum_{j=0}^{d} c_j T_j(B), B = (2 (L + sI) - (lo + hi) I)/(hi - lo),
 *           L the Dirichlet Laplacian of the grid `dims` (diagonal 2*ndim,
 *           neighbours -1), evaluated by Clenshaw's recurrence.
 *   kind 3: factored ILDL preconditioner of one shift (Section 6):
 *           P (A - tau I) P^T ~ L D L^T, T = P^T L^{-T} |D|^{-1} L^{-1} P,
 *           M = |D|^{-1/2} L^{-1} P, M^* = P^T L^{-T} |D|^{-1/2}; this M is
 *           not symmetric, so C = M (A - tau I) M^* applies M^* first.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    int prec_kind;
    int ndim;
    int dims[3];
    double s, lo, hi;
    int degree;
    const double *coef;
    double tau;
    const double *jac; /* |a_rr - tau|^(-1/2), kind 1 only */
    /* kind 3: P, strictly lower L (CSR, rows), |D|^(-1/2) by blocks */
    const int32_t *perm;
    const int32_t *l_rp, *l_ci;
    const double *l_val;
    const double *e_diag, *e_off; /* e_off[i] = E_{i+1,i} at the first row of a 2x2 block, else 0 */
} op_t;

/* y = (A - tau I) x */
static void shifted_matvec(const op_t *P, const double *x, double *y)
{
    for (int64_t r = 0; r < P->n; ++r) {
        double acc = 0.0;
        for (int32_t p = P->row_ptr[r]; p < P->row_ptr[r + 1]; ++p)
            acc += P->val[p] * x[P->col_idx[p]];
        y[r] = acc - P->tau * x[r];
    }
}

/* y = L x, L the Dirichlet Laplacian on the grid (missing neighbours are 0) */
static void laplacian(const op_t *P, const double *x, double *y)
{
    int nd = P->ndim;
    int64_t d[3] = {1, 1, 1};
    for (int a = 0; a < nd; ++a) d[3 - nd + a] = P->dims[a];
    /* d[0] x d[1] x d[2] with the last axis contiguous */
    for (int64_t i0 = 0; i0 < d[0]; ++i0)
        for (int64_t i1 = 0; i1 < d[1]; ++i1)
            for (int64_t i2 = 0; i2 < d[2]; ++i2) {
                int64_t r = (i0 * d[1] + i1) * d[2] + i2;
                double acc = 2.0 * nd * x[r];
                if (i2 > 0) acc -= x[r - 1];
                if (i2 + 1 < d[2]) acc -= x[r + 1];
                if (nd >= 2) {
                    if (i1 > 0) acc -= x[r - d[2]];
                    if (i1 + 1 < d[1]) acc -= x[r + d[2]];
                }
                if (nd >= 3) {
                    if (i0 > 0) acc -= x[r - d[1] * d[2]];
                    if (i0 + 1 < d[0]) acc -= x[r + d[1] * d[2]];
                }
                y[r] = acc;
            }
}

/* y = B x with B = (2 (L + sI) - (lo + hi) I) / (hi - lo) */
static void cheb_B(const op_t *P, const double *x, double *y)
{
    laplacian(P, x, y);
    double inv = 1.0 / (P->hi - P->lo);
    for (int64_t r = 0; r < P->n; ++r)
        y[r] = (2.0 * (y[r] + P->s * x[r]) - (P->lo + P->hi) * x[r]) * inv;
}

/* y = M x.  work: 3 vectors of n. */
static void apply_M(const op_t *P, const double *x, double *y, double *work)
{
    int64_t n = P->n;
    if (P->prec_kind == 0) {
        memcpy(y, x, (size_t)n * sizeof(double));
        return;
    }
    if (P->prec_kind == 1) {
        for (int64_t r = 0; r < n; ++r) y[r] = P->jac[r] * x[r];
        return;
    }
    /* Clenshaw: b_{d+1} = b_{d+2} = 0;
     *           b_j = c_j x + 2 B b_{j+1} - b_{j+2}, j = d..1;
     *           M x = c_0 x + B b_1 - b_2. */
    double *b1 = work, *b2 = work + n, *Bb = work + 2 * n; /* b1 = b_{j+1}, b2 = b_{j+2} */
    memset(b1, 0, (size_t)n * sizeof(double));
    memset(b2, 0, (size_t)n * sizeof(double));
    for (int j = P->degree; j >= 1; --j) {
        cheb_B(P, b1, Bb);
        for (int64_t r = 0; r < n; ++r) {
            double bj = P->coef[j] * x[r] + 2.0 * Bb[r] - b2[r];
            b2[r] = b1[r];
            b1[r] = bj;
        }
    }
    cheb_B(P, b1, Bb);
    for (int64_t r = 0; r < n; ++r) y[r] = P->coef[0] * x[r] + Bb[r] - b2[r];
}

/* z = |D|^(-1/2) y, block by block (kind 3) */
static void apply_E(const op_t *P, const double *y, double *z)
{
    int64_t n = P->n;
    for (int64_t i = 0; i < n; ++i) {
        if (i + 1 < n && P->e_off[i] != 0.0) {
            z[i] = P->e_diag[i] * y[i] + P->e_off[i] * y[i + 1];
            z[i + 1] = P->e_off[i] * y[i] + P->e_diag[i + 1] * y[i + 1];
            ++i;
        } else {
            z[i] = P->e_diag[i] * y[i];
        }
    }
}

/* y = M x = |D|^(-1/2) L^{-1} P x (kind 3): forward substitution by rows */
static void apply_M_ldl(const op_t *P, const double *x, double *y, double *work)
{
    int64_t n = P->n;
    double *f = work;
    for (int64_t i = 0; i < n; ++i) {
        double acc = x[P->perm[i]];
        for (int32_t p = P->l_rp[i]; p < P->l_rp[i + 1]; ++p) acc -= P->l_val[p] * f[P->l_ci[p]];
        f[i] = acc;
    }
    apply_E(P, f, y);
}

/* y = M^* x = P^T L^{-T} |D|^(-1/2) x (kind 3): back substitution with L^T,
 * taking the rows of L as columns of L^T */
static void apply_Mstar_ldl(const op_t *P, const double *x, double *y, double *work)
{
    int64_t n = P->n;
    double *z = work;
    apply_E(P, x, z);
    for (int64_t i = n - 1; i >= 0; --i) {
        const double zi = z[i]; /* final: every l_ji z_i term with j > i is already removed */
        for (int32_t p = P->l_rp[i]; p < P->l_rp[i + 1]; ++p) z[P->l_ci[p]] -= P->l_val[p] * zi;
        y[P->perm[i]] = zi;
    }
}

/* y = M (A - tau I) M^* x.  work: 5 vectors of n. */
static void apply_C(const op_t *P, const double *x, double *y, double *work)
{
    double *t = work, *u = work + P->n, *mw = work + 2 * P->n;
    if (P->prec_kind == 3) {
        apply_Mstar_ldl(P, x, t, mw);
        shifted_matvec(P, t, u);
        apply_M_ldl(P, u, y, mw);
        return;
    }
    apply_M(P, x, t, mw);
    shifted_matvec(P, t, u);
    apply_M(P, u, y, mw);
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t r = 0; r < n; ++r) s += a[r] * b[r];
    return s;
}

/* Column i of the Lanczos relation C Q_k = Q_k J_k + beta_{k+1} q_{k+1} e_k^T
 * (Section 3.1, eq. lan): C q_i = beta_i q_{i-1} + alpha_i q_i + beta_{i+1} q_{i+1}.
 * Forms the part of C q_i that is not along q_{i-1} and q_i:
 *   w = C q_i - beta_i q_{i-1},  alpha_i = q_i^T w,  w <- w - alpha_i q_i
 * and returns alpha_i (the diagonal entry of J_k). */
static double relation_residual(const op_t *P, const double *Q, int i, double beta_i, double *w,
                                double *work)
{
    const int64_t n = P->n;
    const double *qi = Q + (size_t)(i - 1) * n;
    apply_C(P, qi, w, work);
    if (i > 1) {
        const double *qm = Q + (size_t)(i - 2) * n;
        for (int64_t r = 0; r < n; ++r) w[r] -= beta_i * qm[r];
    }
    const double a = dot(n, qi, w);
    for (int64_t r = 0; r < n; ++r) w[r] -= a * qi[r];
    return a;
}

/* w <- (I - Q Q^T) w for the nq columns of Q (the full reorthogonalization of
 * Section 3.1): one classical Gram-Schmidt pass, every coefficient
 * h_l = q_l^T w taken from the incoming w, then w -= sum_l h_l q_l. */
static void project_out(int64_t n, const double *Q, int nq, double *w, double *h)
{
    for (int l = 0; l < nq; ++l) h[l] = dot(n, Q + (size_t)l * n, w);
    for (int l = 0; l < nq; ++l) {
        const double *ql = Q + (size_t)l * n;
        for (int64_t r = 0; r < n; ++r) w[r] -= h[l] * ql[r];
    }
}

/* k steps of Lanczos with full reorthogonalization on C from v (Section 3.1,
 * Algorithm 1): the columns of the relation above, one at a time, each
 * residual projected off the whole basis before it is normalized into the
 * next basis vector.  Q: n x (k+1), column i holds q_{i+1}.  Returns the steps
 * taken (fewer than k when the Krylov space is invariant). */
static int lanczos_one(const op_t *P, const double *v, int k, double *alpha, double *beta,
                       double *nu_out, double *Q, double *w, double *h, double *work)
{
    const int64_t n = P->n;
    const double nu = dot(n, v, v);
    *nu_out = nu;
    const double inv = 1.0 / sqrt(nu);
    for (int64_t r = 0; r < n; ++r) Q[r] = v[r] * inv; /* q_1 = v / |v| */
    beta[0] = 0.0;                                        /* beta_1 = 0, q_0 = 0 */
    double scale = 0.0;   /* largest |alpha_l|, beta_l so far (breakdown test) */
    for (int i = 1; i <= k; ++i) {
        const double a = relation_residual(P, Q, i, beta[i - 1], w, work);
        alpha[i - 1] = a;
        project_out(n, Q, i, w, h);
        const double b = sqrt(dot(n, w, w));
        beta[i] = b;   /* beta_{i+1} */
        if (fabs(a) > scale) scale = fabs(a);
        if (i > 1 && beta[i - 1] > scale) scale = beta[i - 1];
        if (b <= 1e3 * DBL_EPSILON * scale) return i; /* invariant Krylov space */
        double *qn = Q + (size_t)i * n;
        for (int64_t r = 0; r < n; ++r) qn[r] = w[r] / b;
    }
    return k;
}

/* Algorithm 1 for every column of V, OpenMP over probes. */
static int run_probes(const op_t *P, const double *V, int64_t m, int k, int nthreads,
                      double *alpha, double *beta, int32_t *k_used, double *nu)
{
    int64_t n = P->n;
    memset(alpha, 0, (size_t)m * k * sizeof(double));
    memset(beta, 0, (size_t)m * (k + 1) * sizeof(double));
    int failed = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *Q = (double *)malloc((size_t)n * (k + 1) * sizeof(double));
        double *w = (double *)malloc((size_t)n * sizeof(double));
        double *v = (double *)malloc((size_t)n * sizeof(double));
        double *work = (double *)malloc((size_t)n * 6 * sizeof(double));
        double *h = (double *)malloc((size_t)(k + 1) * sizeof(double));
        if (!Q || !w || !v || !work || !h) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t j = 0; j < m; ++j) {
                for (int64_t r = 0; r < n; ++r) v[r] = V[r * m + j];
                k_used[j] = lanczos_one(P, v, k, alpha + j * k, beta + j * (k + 1), nu + j, Q, w,
                                        h, work);
            }
        }
        free(Q);
        free(w);
        free(v);
        free(work);
        free(h);
    }
    return failed ? -1 : 0;
}

/*
 * Run Algorithm 1 for every probe j = 0..m-1 at shift tau.
 *   V      n x m row-major probe block (v_j is column j)
 *   alpha  m x k        (row j: alpha_1..alpha_k of probe j; unused tail = 0)
 *   beta   m x (k+1)    (row j: beta_1 = 0, beta_2..beta_{k+1})
 *   k_used m            (k, or the step at which the Krylov space became invariant)
 *   nu     m            |v_j|^2
 * Returns 0, or -1 on bad arguments / allocation failure, -2 if the Jacobi
 * preconditioner is singular (a_rr = tau).
 */
int oracle_lanczos(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                   int prec_kind, int ndim, const int32_t *dims, double s, double lo, double hi,
                   int degree, const double *coef, double tau, const double *V, int64_t m, int k,
                   int nthreads, double *alpha, double *beta, int32_t *k_used, double *nu)
{
    if (n < 1 || m < 1 || k < 1 || k > n) return -1;
    op_t P;
    memset(&P, 0, sizeof P);
    P.n = n;
    P.row_ptr = row_ptr;
    P.col_idx = col_idx;
    P.val = val;
    P.prec_kind = prec_kind;
    P.ndim = ndim;
    for (int a = 0; a < ndim && a < 3; ++a) P.dims[a] = dims[a];
    P.s = s;
    P.lo = lo;
    P.hi = hi;
    P.degree = degree;
    P.coef = coef;
    P.tau = tau;
    double *jac = NULL;
    if (prec_kind == 1) {
        jac = (double *)malloc((size_t)n * sizeof(double));
        if (!jac) return -1;
        for (int64_t r = 0; r < n; ++r) {
            double arr = 0.0;
            for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
                if (col_idx[p] == r) arr = val[p];
            double d = fabs(arr - tau);
            if (d == 0.0) {
                free(jac);
                return -2;
            }
            jac[r] = 1.0 / sqrt(d);
        }
        P.jac = jac;
    }
    int rc = run_probes(&P, V, m, k, nthreads, alpha, beta, k_used, nu);
    free(jac);
    return rc;
}

/*
 * Dense preconditioned operator C = M (A - tau I) M for small n, built column
 * by column with the same operator code (used by moment tests of the oracle).
 */
int oracle_dense_operator(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const double *val, int prec_kind, int ndim, const int32_t *dims, double s,
                          double lo, double hi, int degree, const double *coef, double tau,
                          double *Cout /* n x n row-major */)
{
    op_t P;
    memset(&P, 0, sizeof P);
    P.n = n;
    P.row_ptr = row_ptr;
    P.col_idx = col_idx;
    P.val = val;
    P.prec_kind = prec_kind;
    P.ndim = ndim;
    for (int a = 0; a < ndim && a < 3; ++a) P.dims[a] = dims[a];
    P.s = s;
    P.lo = lo;
    P.hi = hi;
    P.degree = degree;
    P.coef = coef;
    P.tau = tau;
    double *jac = NULL;
    if (prec_kind == 1) {
        jac = (double *)malloc((size_t)n * sizeof(double));
        for (int64_t r = 0; r < n; ++r) {
            double arr = 0.0;
            for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
                if (col_idx[p] == r) arr = val[p];
            jac[r] = 1.0 / sqrt(fabs(arr - tau));
        }
        P.jac = jac;
    }
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    double *work = (double *)malloc((size_t)n * 6 * sizeof(double));
    for (int64_t c = 0; c < n; ++c) {
        e[c] = 1.0;
        apply_C(&P, e, y, work);
        e[c] = 0.0;
        for (int64_t r = 0; r < n; ++r) Cout[r * n + c] = y[r];
    }
    free(e);
    free(y);
    free(work);
    free(jac);
    return 0;
}

/*
 * Forward-mode tangent of Algorithm 1 (used to check gradients of the
 * smoothed estimator).  The matrix depends on a direction (du, dtau) as
 * A - tau I -> A + t diag(du) - (tau + t dtau) I, with M independent of both
 * (no preconditioner or the Laplacian polynomial), so
 *   dC x = M (du .* (M x) - dtau * (M x)).
 * Every line of Algorithm 1 is differentiated in its literal order; the
 * outputs are alpha, beta as in oracle_lanczos and their derivatives
 * dalpha (m x k), dbeta (m x (k+1)).
 */
static int lanczos_tangent_one(const op_t *P, const double *du, double dtau, const double *v, int k,
                               double *alpha, double *beta, double *dalpha, double *dbeta,
                               double *nu_out, double *Q, double *dQ, double *w, double *dw,
                               double *h, double *work)
{
    int64_t n = P->n;
    double *t = work + 5 * n, *u = work + 6 * n, *y2 = work + 7 * n;
    double nu = dot(n, v, v);
    *nu_out = nu;
    double inv = 1.0 / sqrt(nu);
    for (int64_t r = 0; r < n; ++r) {
        Q[r] = v[r] * inv;
        dQ[r] = 0.0;
    }
    beta[0] = 0.0;
    dbeta[0] = 0.0;
    double scale = 0.0;
    for (int i = 1; i <= k; ++i) {
        const double *qi = Q + (size_t)(i - 1) * n, *dqi = dQ + (size_t)(i - 1) * n;
        /* w = C q_i ;  dw = dC q_i + C dq_i */
        apply_C(P, qi, w, work);
        apply_C(P, dqi, dw, work);
        apply_M(P, qi, t, work + 2 * n);
        for (int64_t r = 0; r < n; ++r) u[r] = du[r] * t[r] - dtau * t[r];
        apply_M(P, u, y2, work + 2 * n);
        for (int64_t r = 0; r < n; ++r) dw[r] += y2[r];
        if (i > 1) {
            const double *qm = Q + (size_t)(i - 2) * n, *dqm = dQ + (size_t)(i - 2) * n;
            for (int64_t r = 0; r < n; ++r) {
                w[r] -= beta[i - 1] * qm[r];
                dw[r] -= dbeta[i - 1] * qm[r] + beta[i - 1] * dqm[r];
            }
        }
        double a = dot(n, qi, w);
        double da = dot(n, dqi, w) + dot(n, qi, dw);
        alpha[i - 1] = a;
        dalpha[i - 1] = da;
        for (int64_t r = 0; r < n; ++r) {
            w[r] -= a * qi[r];
            dw[r] -= da * qi[r] + a * dqi[r];
        }
        /* one classical Gram-Schmidt pass: h = Q^T w, w -= Q h */
        double *dh = h + (k + 1);
        for (int l = 0; l < i; ++l) {
            const double *ql = Q + (size_t)l * n, *dql = dQ + (size_t)l * n;
            h[l] = dot(n, ql, w);
            dh[l] = dot(n, dql, w) + dot(n, ql, dw);
        }
        for (int l = 0; l < i; ++l) {
            const double *ql = Q + (size_t)l * n, *dql = dQ + (size_t)l * n;
            for (int64_t r = 0; r < n; ++r) {
                w[r] -= h[l] * ql[r];
                dw[r] -= dh[l] * ql[r] + h[l] * dql[r];
            }
        }
        double b = sqrt(dot(n, w, w));
        double db = dot(n, w, dw) / b;
        beta[i] = b;
        dbeta[i] = db;
        if (fabs(a) > scale) scale = fabs(a);
        if (i > 1 && beta[i - 1] > scale) scale = beta[i - 1];
        if (b <= 1e3 * DBL_EPSILON * scale) return i;
        double *qn = Q + (size_t)i * n, *dqn = dQ + (size_t)i * n;
        for (int64_t r = 0; r < n; ++r) {
            qn[r] = w[r] / b;
            dqn[r] = dw[r] / b - w[r] * db / (b * b);
        }
    }
    return k;
}

int oracle_lanczos_tangent(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                           const double *val, int prec_kind, int ndim, const int32_t *dims,
                           double s, double lo, double hi, int degree, const double *coef,
                           double tau, const double *du, double dtau, const double *V, int64_t m,
                           int k, int nthreads, double *alpha, double *beta, double *dalpha,
                           double *dbeta, int32_t *k_used, double *nu)
{
    if (n < 1 || m < 1 || k < 1 || k > n) return -1;
    if (prec_kind == 1) return -3; /* M would depend on diag(A) and tau */
    op_t P;
    memset(&P, 0, sizeof P);
    P.n = n;
    P.row_ptr = row_ptr;
    P.col_idx = col_idx;
    P.val = val;
    P.prec_kind = prec_kind;
    P.ndim = ndim;
    for (int a = 0; a < ndim && a < 3; ++a) P.dims[a] = dims[a];
    P.s = s;
    P.lo = lo;
    P.hi = hi;
    P.degree = degree;
    P.coef = coef;
    P.tau = tau;
    memset(alpha, 0, (size_t)m * k * sizeof(double));
    memset(beta, 0, (size_t)m * (k + 1) * sizeof(double));
    memset(dalpha, 0, (size_t)m * k * sizeof(double));
    memset(dbeta, 0, (size_t)m * (k + 1) * sizeof(double));
    int failed = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *Q = (double *)malloc((size_t)n * (k + 1) * sizeof(double));
        double *dQ = (double *)malloc((size_t)n * (k + 1) * sizeof(double));
        double *w = (double *)malloc((size_t)n * sizeof(double));
        double *dw = (double *)malloc((size_t)n * sizeof(double));
        double *v = (double *)malloc((size_t)n * sizeof(double));
        double *work = (double *)malloc((size_t)n * 8 * sizeof(double));
        double *h = (double *)malloc((size_t)2 * (k + 1) * sizeof(double));
        if (!Q || !dQ || !w || !dw || !v || !work || !h) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t j = 0; j < m; ++j) {
                for (int64_t r = 0; r < n; ++r) v[r] = V[r * m + j];
                k_used[j] = lanczos_tangent_one(&P, du, dtau, v, k, alpha + j * k,
                                                beta + j * (k + 1), dalpha + j * k,
                                                dbeta + j * (k + 1), nu + j, Q, dQ, w, dw, h, work);
            }
        }
        free(Q);
        free(dQ);
        free(w);
        free(dw);
        free(v);
        free(work);
        free(h);
    }
    return failed ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * Arnoldi estimator for an unfactored preconditioner (Section 4, Algorithms
 * 3 and 4).  The operator is C = T (A - tau I) with
 *   kind 0: T = I,
 *   kind 1: T = |diag(A) - tau|^(-1) (the square of the Jacobi M above),
 *   kind 2: T = sum_j c_j T_j(B), the series given (Clenshaw, as apply_M).
 * Per probe, Algorithm 3 with modified Gram-Schmidt:
 *   q_1 = v/|v|; for j = 1..k: w = C q_j; for i = 1..j: h_ij = q_i^T w,
 *   w = w - h_ij q_i; h_{j+1,j} = |w|; q_{j+1} = w / h_{j+1,j}.
 * The quadrature (eigendecomposition of H_k) is done by the Python half.
 * Breakdown: when h_{j+1,j} <= 1e3 * eps * max |h_il| so far, the Krylov
 * space is invariant; the run stops with k_used = j.
 * ------------------------------------------------------------------------ */

/* y = T x (see above); work: 3 vectors of n */
static void apply_T(const op_t *P, const double *x, double *y, double *work)
{
    if (P->prec_kind == 1) {
        for (int64_t r = 0; r < P->n; ++r) y[r] = P->jac[r] * P->jac[r] * x[r];
        return;
    }
    apply_M(P, x, y, work); /* kind 0: copy; kind 2: the series */
}

/* H: (k+1) x k row-major, row i column l holds h_{i+1,l+1} */
static int arnoldi_one(const op_t *P, const double *v, int k, double *H, double *nu_out,
                       double *Q, double *w, double *u, double *work)
{
    int64_t n = P->n;
    double nu = dot(n, v, v);
    *nu_out = nu;
    double inv = 1.0 / sqrt(nu);
    for (int64_t r = 0; r < n; ++r) Q[r] = v[r] * inv;
    double scale = 0.0;
    for (int j = 1; j <= k; ++j) {
        const double *qj = Q + (size_t)(j - 1) * n;
        shifted_matvec(P, qj, u);
        apply_T(P, u, w, work);
        for (int i = 1; i <= j; ++i) {
            const double *qi = Q + (size_t)(i - 1) * n;
            double h = dot(n, qi, w);
            H[(size_t)(i - 1) * k + (j - 1)] = h;
            for (int64_t r = 0; r < n; ++r) w[r] -= h * qi[r];
            if (fabs(h) > scale) scale = fabs(h);
        }
        double b = sqrt(dot(n, w, w));
        H[(size_t)j * k + (j - 1)] = b;
        if (b <= 1e3 * DBL_EPSILON * scale) return j;
        if (b > scale) scale = b;
        double *qn = Q + (size_t)j * n;
        for (int64_t r = 0; r < n; ++r) qn[r] = w[r] / b;
    }
    return k;
}

/*
 * Algorithm 3 for every probe j = 0..m-1 at shift tau.
 *   V      n x m row-major probe block
 *   H      m x (k+1) x k (per probe as in arnoldi_one; unused entries 0)
 *   k_used m, nu m (|v_j|^2)
 * Returns 0, -1 on bad arguments / allocation failure, -2 if kind 1 is
 * singular (a_rr = tau).
 */
int oracle_arnoldi(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                   int prec_kind, int ndim, const int32_t *dims, double s, double lo, double hi,
                   int degree, const double *coef, double tau, const double *V, int64_t m, int k,
                   int nthreads, double *H, int32_t *k_used, double *nu)
{
    if (n < 1 || m < 1 || k < 1 || k > n) return -1;
    op_t P;
    memset(&P, 0, sizeof P);
    P.n = n;
    P.row_ptr = row_ptr;
    P.col_idx = col_idx;
    P.val = val;
    P.prec_kind = prec_kind;
    P.ndim = ndim;
    for (int a = 0; a < ndim && a < 3; ++a) P.dims[a] = dims[a];
    P.s = s;
    P.lo = lo;
    P.hi = hi;
    P.degree = degree;
    P.coef = coef;
    P.tau = tau;
    double *jac = NULL;
    if (prec_kind == 1) {
        jac = (double *)malloc((size_t)n * sizeof(double));
        if (!jac) return -1;
        for (int64_t r = 0; r < n; ++r) {
            double arr = 0.0;
            for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
                if (col_idx[p] == r) arr = val[p];
            double d = fabs(arr - tau);
            if (d == 0.0) {
                free(jac);
                return -2;
            }
            jac[r] = 1.0 / sqrt(d);
        }
        P.jac = jac;
    }
    memset(H, 0, (size_t)m * (k + 1) * k * sizeof(double));
    int failed = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *Q = (double *)malloc((size_t)n * (k + 1) * sizeof(double));
        double *w = (double *)malloc((size_t)n * sizeof(double));
        double *u = (double *)malloc((size_t)n * sizeof(double));
        double *v = (double *)malloc((size_t)n * sizeof(double));
        double *work = (double *)malloc((size_t)n * 3 * sizeof(double));
        if (!Q || !w || !u || !v || !work) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t j = 0; j < m; ++j) {
                for (int64_t r = 0; r < n; ++r) v[r] = V[r * m + j];
                k_used[j] = arnoldi_one(&P, v, k, H + (size_t)j * (k + 1) * k, nu + j, Q, w, u,
                                        work);
            }
        }
        free(Q);
        free(w);
        free(u);
        free(v);
        free(work);
    }
    free(jac);
    return failed ? -1 : 0;
}

/*
 * |D|^(-1/2) block by block: 1 / sqrt|d| for a 1x1 block; for a 2x2 block
 * [[a, b], [b, c]] (b != 0) the spectral form sum_i |mu_i|^(-1/2) v_i v_i^T.
 */
static void abs_invsqrt_blocks(int64_t n, const double *d_diag, const double *d_off,
                               double *e_diag, double *e_off)
{
    for (int64_t i = 0; i < n; ++i) {
        e_off[i] = 0.0;
        if (i + 1 < n && d_off[i] != 0.0) {
            const double a = d_diag[i], b = d_off[i], c = d_diag[i + 1];
            const double mid = 0.5 * (a + c), rad = hypot(0.5 * (a - c), b);
            const double mu1 = mid + rad, mu2 = mid - rad;
            /* eigenvector of mu1: (b, mu1 - a) or (mu1 - c, b), whichever is longer */
            double vx = b, vy = mu1 - a;
            const double ux = mu1 - c, uy = b;
            if (hypot(ux, uy) > hypot(vx, vy)) {
                vx = ux;
                vy = uy;
            }
            const double len = hypot(vx, vy);
            vx /= len;
            vy /= len;
            const double f1 = 1.0 / sqrt(fabs(mu1)), f2 = 1.0 / sqrt(fabs(mu2));
            e_diag[i] = f1 * vx * vx + f2 * vy * vy;
            e_diag[i + 1] = f1 * vy * vy + f2 * vx * vx;
            e_off[i] = (f1 - f2) * vx * vy;
            e_off[i + 1] = 0.0;
            ++i;
        } else {
            e_diag[i] = 1.0 / sqrt(fabs(d_diag[i]));
        }
    }
}

static void fill_ldl(op_t *P, int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *val, double tau, const int32_t *perm, const int32_t *l_rp,
                     const int32_t *l_ci, const double *l_val, const double *e_diag,
                     const double *e_off)
{
    memset(P, 0, sizeof *P);
    P->n = n;
    P->row_ptr = row_ptr;
    P->col_idx = col_idx;
    P->val = val;
    P->prec_kind = 3;
    P->tau = tau;
    P->perm = perm;
    P->l_rp = l_rp;
    P->l_ci = l_ci;
    P->l_val = l_val;
    P->e_diag = e_diag;
    P->e_off = e_off;
}

/*
 * Algorithm 1 with the factored ILDL preconditioner of shift tau (kind 3):
 * perm, L (strictly lower, CSR), D (d_diag, d_off as oracle_ildl writes
 * them).  Outputs as oracle_lanczos.  Returns 0, -1 (bad arguments), -2 (a
 * zero pivot in D).
 */
int oracle_lanczos_ldl(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *val, double tau, const int32_t *perm, const int32_t *l_rp,
                       const int32_t *l_ci, const double *l_val, const double *d_diag,
                       const double *d_off, const double *V, int64_t m, int k, int nthreads,
                       double *alpha, double *beta, int32_t *k_used, double *nu)
{
    if (n < 1 || m < 1 || k < 1 || k > n) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (d_diag[i] == 0.0 && !(i > 0 && d_off[i - 1] != 0.0) && d_off[i] == 0.0) return -2;
    double *e = (double *)malloc((size_t)n * 2 * sizeof(double));
    if (!e) return -1;
    abs_invsqrt_blocks(n, d_diag, d_off, e, e + n);
    op_t P;
    fill_ldl(&P, n, row_ptr, col_idx, val, tau, perm, l_rp, l_ci, l_val, e, e + n);
    int rc = run_probes(&P, V, m, k, nthreads, alpha, beta, k_used, nu);
    free(e);
    return rc;
}

/* Dense C = M (A - tau I) M^* with the ILDL preconditioner (small n only). */
int oracle_dense_operator_ldl(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              const double *val, double tau, const int32_t *perm,
                              const int32_t *l_rp, const int32_t *l_ci, const double *l_val,
                              const double *d_diag, const double *d_off, double *Cout)
{
    double *e = (double *)malloc((size_t)n * 2 * sizeof(double));
    double *x = (double *)calloc((size_t)n, sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    double *work = (double *)malloc((size_t)n * 6 * sizeof(double));
    if (!e || !x || !y || !work) {
        free(e);
        free(x);
        free(y);
        free(work);
        return -1;
    }
    abs_invsqrt_blocks(n, d_diag, d_off, e, e + n);
    op_t P;
    fill_ldl(&P, n, row_ptr, col_idx, val, tau, perm, l_rp, l_ci, l_val, e, e + n);
    for (int64_t c = 0; c < n; ++c) {
        x[c] = 1.0;
        apply_C(&P, x, y, work);
        x[c] = 0.0;
        for (int64_t r = 0; r < n; ++r) Cout[r * n + c] = y[r];
    }
    free(e);
    free(x);
    free(y);
    free(work);
    return 0;
}

/* |D|^(-1/2) as the oracle forms it (for the pins of the block formula). */
int oracle_abs_invsqrt_blocks(int64_t n, const double *d_diag, const double *d_off,
                              double *e_diag, double *e_off)
{
    abs_invsqrt_blocks(n, d_diag, d_off, e_diag, e_off);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Y = C X for an n x m block (both row-major, column j = one vector), column
 * by column with apply_C; C = M (A - tau I) M^* with preconditioner kinds
 * 0..2.  Used by the block-Lanczos oracle, which does its own recurrence in
 * numpy.  Returns 0, -1 on bad arguments or allocation failure, -2 if the
 * Jacobi preconditioner is singular.
 */
int oracle_apply_operator(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const double *val, int prec_kind, int ndim, const int32_t *dims,
                          double s, double lo, double hi, int degree, const double *coef,
                          double tau, const double *X, int64_t m, int nthreads, double *Y)
{
    if (n < 1 || m < 1 || prec_kind < 0 || prec_kind > 2) return -1;
    op_t P;
    memset(&P, 0, sizeof P);
    P.n = n;
    P.row_ptr = row_ptr;
    P.col_idx = col_idx;
    P.val = val;
    P.prec_kind = prec_kind;
    P.ndim = ndim;
    for (int a = 0; a < ndim && a < 3; ++a) P.dims[a] = dims[a];
    P.s = s;
    P.lo = lo;
    P.hi = hi;
    P.degree = degree;
    P.coef = coef;
    P.tau = tau;
    double *jac = NULL;
    if (prec_kind == 1) {
        jac = (double *)malloc((size_t)n * sizeof(double));
        if (!jac) return -1;
        for (int64_t r = 0; r < n; ++r) {
            double arr = 0.0;
            for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
                if (col_idx[p] == r) arr = val[p];
            double d = fabs(arr - tau);
            if (d == 0.0) {
                free(jac);
                return -2;
            }
            jac[r] = 1.0 / sqrt(d);
        }
        P.jac = jac;
    }
    int failed = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *x = (double *)malloc((size_t)n * sizeof(double));
        double *y = (double *)malloc((size_t)n * sizeof(double));
        double *work = (double *)malloc((size_t)n * 6 * sizeof(double));
        if (!x || !y || !work) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t j = 0; j < m; ++j) {
                for (int64_t r = 0; r < n; ++r) x[r] = X[r * m + j];
                apply_C(&P, x, y, work);
                for (int64_t r = 0; r < n; ++r) Y[r * m + j] = y[r];
            }
        }
        free(x);
        free(y);
        free(work);
    }
    free(jac);
    return failed ? -1 : 0;
}
