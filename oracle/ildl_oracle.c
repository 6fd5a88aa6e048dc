/*
 * ILDL(t) oracle: incomplete LDL^T factorization of K = A - tau I with
 * Bunch-Kaufman 1x1 / 2x2 pivoting and a drop tolerance, and the HPD
 * preconditioner built from it.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64, written from the paper
 * (Vecharynski & Yang, "Preconditioned iterative methods for eigenvalue
 * counts", Section 6: T = L^{-*} |D|^{-1} L^{-1} from an ILDL(t) of A - tau I,
 * the absolute value taken block by block so that T is HPD).  The paper
 * delegates the factorization itself to an external package; the pivoting
 * rule (Bunch-Kaufman partial pivoting, alpha = (1 + sqrt 17)/8), the
 * dropping rule and the natural ordering used here are this project's
 * reading of it.  Shares no code with the GPU library.
 *
 * Algorithm (right-looking, on a DENSE n x n array, so that every step can
 * be checked by eye):
 *   S = P K P^T, the active (Schur) matrix, symmetric, both triangles kept.
 *   for k = 0, 1, ...:
 *     lambda = max_{i>k} |S_ik|, r = smallest such i.
 *     1x1 pivot at k    if lambda == 0 or |S_kk| >= alpha lambda, or
 *                       |S_kk| sigma >= alpha lambda^2 with
 *                       sigma = max_{i>=k, i!=r} |S_ir|;
 *     else 1x1 after swapping r <-> k     if |S_rr| >= alpha sigma;
 *     else 2x2 pivot on (k, k+1) after swapping r <-> k+1.
 *     multipliers: l_i = S_ik / d (1x1), [l1_i l2_i] = [S_ik S_i,k+1] D^{-1}
 *     (2x2); each multiplier column is then thinned: an entry with
 *     |l_i| < t * sum_i |l_i| (sum over the column before thinning, in row
 *     order) is set to 0.
 *     Schur update with the thinned multipliers, for i >= j beyond the pivot:
 *       1x1: S_ij -= (l_i * d) * l_j
 *       2x2: S_ij -= (l1_i a + l2_i b) * l1_j + (l1_i b + l2_i c) * l2_j
 *     and S_ji = S_ij.
 * With t = 0 nothing is dropped and P K P^T = L D L^T up to rounding
 * (Sylvester: the inertia of D is that of K).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ALPHA_BK 0.6403882032022076   /* (1 + sqrt(17)) / 8 */

/*
 * Factor K = A - tau I (A: n x n CSR, both triangles).
 * Outputs:
 *   perm   n (caller-allocated): row i of P K P^T is row perm[i] of K
 *   d_diag n (caller-allocated): D_ii
 *   d_off  n (caller-allocated): d_off[i] = D_{i+1,i} when rows i, i+1 form a
 *          2x2 block, else 0
 *   *l_rp, *l_ci, *l_val: the strictly lower part of L (unit diagonal not
 *          stored) in CSR, non-zeros only, allocated here with malloc; free
 *          them with oracle_free.  *nnz_out: their number of entries.
 * Returns 0, -1 on bad arguments / allocation failure, -3 on a zero 1x1 pivot
 * or a singular 2x2 pivot.
 */
void oracle_free(void *p) { free(p); }

int oracle_ildl(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                double tau, double droptol, int32_t *perm, double *d_diag, double *d_off,
                int64_t *nnz_out, int32_t **l_rp, int32_t **l_ci, double **l_val)
{
    if (n < 1 || droptol < 0.0) return -1;
    *l_rp = NULL;
    *l_ci = NULL;
    *l_val = NULL;
    *nnz_out = 0;
    double *S = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    double *l1 = (double *)malloc((size_t)n * sizeof(double));
    double *l2 = (double *)malloc((size_t)n * sizeof(double));
    int64_t *idx = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!S || !l1 || !l2 || !idx) {
        free(S);
        free(l1);
        free(l2);
        free(idx);
        return -1;
    }
#define AT(i, j) S[(size_t)(i) * (size_t)n + (size_t)(j)]
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) AT(r, col_idx[p]) += val[p];
        AT(r, r) -= tau;
    }
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    memset(d_diag, 0, (size_t)n * sizeof(double));
    memset(d_off, 0, (size_t)n * sizeof(double));
    int rc = 0;

    /* symmetric interchange of active indices a, b (both >= k): rows over all
     * columns (this also permutes the rows of the L columns already formed),
     * columns over the active rows only */
#define SWAP_IDX(a, b, k)                                                      \
    do {                                                                       \
        if ((a) != (b)) {                                                      \
            for (int64_t c_ = 0; c_ < n; ++c_) {                               \
                double t_ = AT(a, c_);                                         \
                AT(a, c_) = AT(b, c_);                                         \
                AT(b, c_) = t_;                                                \
            }                                                                  \
            for (int64_t r_ = (k); r_ < n; ++r_) {                             \
                double t_ = AT(r_, a);                                         \
                AT(r_, a) = AT(r_, b);                                         \
                AT(r_, b) = t_;                                                \
            }                                                                  \
            int32_t p_ = perm[a];                                              \
            perm[a] = perm[b];                                                 \
            perm[b] = p_;                                                      \
        }                                                                      \
    } while (0)

    int64_t k = 0;
    while (k < n) {
        /* pivot choice (Bunch-Kaufman partial pivoting) */
        double lambda = 0.0;
        int64_t r = -1;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(AT(k, i)) > lambda) {
                lambda = fabs(AT(k, i));
                r = i;
            }
        int two = 0;
        if (lambda > 0.0 && fabs(AT(k, k)) < ALPHA_BK * lambda) {
            double sigma = 0.0;
            for (int64_t i = k; i < n; ++i)
                if (i != r && fabs(AT(r, i)) > sigma) sigma = fabs(AT(r, i));
            if (fabs(AT(k, k)) * sigma >= ALPHA_BK * lambda * lambda) {
                /* 1x1 at k */
            } else if (fabs(AT(r, r)) >= ALPHA_BK * sigma) {
                SWAP_IDX(r, k, k);
            } else {
                SWAP_IDX(r, k + 1, k);
                two = 1;
            }
        }
        if (!two) {
            const double d = AT(k, k);
            if (d == 0.0) {
                rc = -3;
                break;
            }
            d_diag[k] = d;
            double nrm = 0.0;
            for (int64_t i = k + 1; i < n; ++i) {   /* S_ik read from row k (symmetry) */
                l1[i] = AT(k, i) / d;
                nrm += fabs(l1[i]);
            }
            const double thr = droptol * nrm;
            int64_t cnt = 0;
            for (int64_t i = k + 1; i < n; ++i) {
                if (fabs(l1[i]) < thr) l1[i] = 0.0;
                if (l1[i] != 0.0) idx[cnt++] = i;
            }
            for (int64_t a = 0; a < cnt; ++a) {
                const int64_t i = idx[a];
                const double u = l1[i] * d;
                for (int64_t b = 0; b <= a; ++b) {
                    const int64_t j = idx[b];
                    AT(i, j) -= u * l1[j];
                    AT(j, i) = AT(i, j);
                }
            }
            for (int64_t i = k + 1; i < n; ++i) {
                AT(i, k) = l1[i];   /* column k of L */
                AT(k, i) = 0.0;
            }
            k += 1;
        } else {
            const double a = AT(k, k), b = AT(k + 1, k), c = AT(k + 1, k + 1);
            const double det = a * c - b * b;
            if (det == 0.0) {
                rc = -3;
                break;
            }
            d_diag[k] = a;
            d_diag[k + 1] = c;
            d_off[k] = b;
            double n1 = 0.0, n2 = 0.0;
            for (int64_t i = k + 2; i < n; ++i) {
                const double s1 = AT(k, i), s2 = AT(k + 1, i);
                l1[i] = (s1 * c - s2 * b) / det;
                l2[i] = (s2 * a - s1 * b) / det;
                n1 += fabs(l1[i]);
                n2 += fabs(l2[i]);
            }
            const double t1 = droptol * n1, t2 = droptol * n2;
            int64_t cnt = 0;
            for (int64_t i = k + 2; i < n; ++i) {
                if (fabs(l1[i]) < t1) l1[i] = 0.0;
                if (fabs(l2[i]) < t2) l2[i] = 0.0;
                if (l1[i] != 0.0 || l2[i] != 0.0) idx[cnt++] = i;
            }
            for (int64_t p = 0; p < cnt; ++p) {
                const int64_t i = idx[p];
                const double w1 = l1[i] * a + l2[i] * b;
                const double w2 = l1[i] * b + l2[i] * c;
                for (int64_t q = 0; q <= p; ++q) {
                    const int64_t j = idx[q];
                    AT(i, j) -= w1 * l1[j] + w2 * l2[j];
                    AT(j, i) = AT(i, j);
                }
            }
            for (int64_t i = k + 2; i < n; ++i) {
                AT(i, k) = l1[i];
                AT(i, k + 1) = l2[i];
                AT(k, i) = 0.0;
                AT(k + 1, i) = 0.0;
            }
            AT(k + 1, k) = 0.0;   /* inside D, not L */
            k += 2;
        }
    }
    if (rc == 0) {
        int64_t nnz = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < i; ++j) nnz += AT(i, j) != 0.0;
        int32_t *rp = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
        int32_t *ci = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
        double *lv = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
        if (!rp || !ci || !lv) {
            free(rp);
            free(ci);
            free(lv);
            rc = -1;
        } else {
            int64_t e = 0;
            rp[0] = 0;
            for (int64_t i = 0; i < n; ++i) {
                for (int64_t j = 0; j < i; ++j)
                    if (AT(i, j) != 0.0) {
                        ci[e] = (int32_t)j;
                        lv[e] = AT(i, j);
                        ++e;
                    }
                rp[i + 1] = (int32_t)e;
            }
            *l_rp = rp;
            *l_ci = ci;
            *l_val = lv;
            *nnz_out = nnz;
        }
    }
#undef SWAP_IDX
#undef AT
    free(S);
    free(l1);
    free(l2);
    free(idx);
    return rc;
}
