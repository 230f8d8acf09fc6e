/*
 * TEST INFRASTRUCTURE ONLY: a plain, slow FP64 CPU oracle for the submatrix
 * sign method.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  It shares no code with the GPU path.
 *
 * What it computes (Lass, Schade, Kuehne, Plessl, "A Submatrix-Based Method
 * for Approximate Matrix Function Evaluation in the Quantum Chemistry Code
 * CP2K"):
 *
 *   - Submatrix method (Sec. III-A, three-step overview; Sec. IV-C applies it
 *     per block column and to combined block columns): for a group g of
 *     block columns, the principal submatrix keeps every block row that is
 *     stored in any member column; the matrix function is evaluated on that
 *     dense submatrix and only the group's own columns are copied back, into
 *     the stored blocks of the input pattern.
 *   - Matrix sign by eigendecomposition (Sec. IV-F, Eq. eigendecompsym):
 *     sign(A) = Q signum(Lambda) Q^T, with the extension that an eigenvalue
 *     on the imaginary axis (here: zero) maps to 0 (Eq. signevext).
 *   - Density matrix for an orthogonalised K (Eq. DsignSym with S = I):
 *     D = (I - sign(K - mu I)) / 2; at finite temperature the signum is
 *     replaced by the Fermi function (Sec. IV-F, last paragraph), i.e.
 *     D = Q f(Lambda) Q^T with f(x) = 1 / (1 + exp(x / kT)).
 *   - Electron count N = Tr D (Sec. IV-G, no spin factor) and band energy
 *     E = Tr(D K) (Eq. bandenergy), both over the stored blocks.
 *
 * The symmetric eigensolver is the cyclic-by-row two-sided Jacobi method
 * with Rutishauser's stable rotation update (Golub & Van Loan, Matrix
 * Computations, Sec. 8.5), written out plainly.
 *
 * Storage conventions: dense matrices are column-major; the block-sparse
 * input is block-compressed-sparse-column with both triangles stored, block
 * (I, J) a dense column-major b_I x b_J array at the running offset of the
 * preceding blocks in storage order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_INVALID -1
#define ORACLE_E_JACOBI -2
#define ORACLE_E_NOMEM -3
#define ORACLE_E_NOT_SYMMETRIC -4

typedef struct {
    int32_t n;          /* submatrix dimension n_g                          */
    int32_t nrow_blk;   /* |R(g)|                                           */
    int32_t sweeps;     /* Jacobi sweeps used                               */
    int32_t n_neg;      /* eigenvalues below -tau0                          */
    int32_t n_zero;     /* eigenvalues with |lambda| <= tau0                */
    int32_t pad;
    double min_abs_lambda;  /* min |lambda| of K_sub - mu I                  */
    double max_abs_lambda;
    double inf_norm;        /* ||K_sub - mu I||_inf (max row sum)            */
    double eig_residual;    /* max |A Q - Q Lambda|                          */
    double orth_residual;   /* max |Q^T Q - I|                               */
} oracle_group_info;

int32_t oracle_abi_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Cyclic Jacobi eigensolver                                                 */
/* ------------------------------------------------------------------------ */

/*
 * Eigen-decomposition of the symmetric n x n matrix a (column-major,
 * overwritten).  On return lam[k] are the eigenvalues in ascending order and
 * column k of q (n x n, column-major) is the matching unit eigenvector.
 * Sweeps continue until max_{p != q} |a_pq| <= 1e-15 * max_p |a_pp| or
 * max_sweeps is reached.  Returns the number of sweeps, or -1 if it did not
 * converge.
 */
int32_t oracle_jacobi(int32_t n, double *a, double *lam, double *q, int32_t max_sweeps)
{
    for (int64_t i = 0; i < (int64_t)n * n; i++) q[i] = 0.0;
    for (int32_t i = 0; i < n; i++) q[i + (int64_t)i * n] = 1.0;

    int32_t sweep;
    int converged = 0;
    for (sweep = 0; sweep <= max_sweeps; sweep++) {
        double off = 0.0, dmax = 0.0;
        for (int32_t j = 0; j < n; j++) {
            double d = fabs(a[j + (int64_t)j * n]);
            if (d > dmax) dmax = d;
            for (int32_t i = 0; i < n; i++) {
                if (i == j) continue;
                double v = fabs(a[i + (int64_t)j * n]);
                if (v > off) off = v;
            }
        }
        if (off <= 1e-15 * dmax) { converged = 1; break; }
        if (sweep == max_sweeps) break;
        const double skip = 1e-18 * dmax;

        /* one cyclic-by-row sweep over p < q */
        for (int32_t p = 0; p < n - 1; p++) {
            for (int32_t r = p + 1; r < n; r++) {
                double *colp = a + (int64_t)p * n;
                double *colr = a + (int64_t)r * n;
                double apq = colr[p];
                if (fabs(apq) <= skip) continue;
                /* rotation that zeroes a_pr (G&VL sym.schur2) */
                double theta = (colr[r] - colp[p]) / (2.0 * apq);
                double t = (theta >= 0.0)
                    ? 1.0 / (theta + sqrt(1.0 + theta * theta))
                    : -1.0 / (-theta + sqrt(1.0 + theta * theta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                double tau = s / (1.0 + c);
                /* Rutishauser's update of every other row/column entry */
                for (int32_t k = 0; k < n; k++) {
                    if (k == p || k == r) continue;
                    double akp = colp[k];
                    double akr = colr[k];
                    double nkp = akp - s * (akr + tau * akp);
                    double nkr = akr + s * (akp - tau * akr);
                    colp[k] = nkp;
                    colr[k] = nkr;
                    a[p + (int64_t)k * n] = nkp;   /* keep both triangles */
                    a[r + (int64_t)k * n] = nkr;
                }
                colp[p] -= t * apq;
                colr[r] += t * apq;
                colr[p] = 0.0;
                colp[r] = 0.0;
                /* accumulate Q <- Q J */
                double *qp = q + (int64_t)p * n;
                double *qr = q + (int64_t)r * n;
                for (int32_t k = 0; k < n; k++) {
                    double x = qp[k], y = qr[k];
                    qp[k] = x - s * (y + tau * x);
                    qr[k] = y + s * (x - tau * y);
                }
            }
        }
    }

    /* eigenvalues from the diagonal, sorted ascending together with Q */
    for (int32_t i = 0; i < n; i++) lam[i] = a[i + (int64_t)i * n];
    for (int32_t i = 1; i < n; i++) {           /* insertion sort: small n */
        int32_t j = i;
        while (j > 0 && lam[j - 1] > lam[j]) {
            double tl = lam[j]; lam[j] = lam[j - 1]; lam[j - 1] = tl;
            double *c0 = q + (int64_t)j * n, *c1 = q + (int64_t)(j - 1) * n;
            for (int32_t k = 0; k < n; k++) { double tv = c0[k]; c0[k] = c1[k]; c1[k] = tv; }
            j--;
        }
    }
    return converged ? sweep : -1;
}

/* ------------------------------------------------------------------------ */
/* Scalar maps applied to the eigenvalues                                    */
/* ------------------------------------------------------------------------ */

/* Occupation of an eigenvalue x of K - mu I.
 * kT == 0: 1 for x < -tau0, 1/2 for |x| <= tau0 (Eq. signevext: sign 0),
 *          0 for x > tau0, i.e. (1 - signum(x)) / 2.
 * kT > 0 : Fermi function 1 / (1 + exp(x / kT)), evaluated without overflow. */
static double occupation(double x, double kT, double tau0)
{
    if (kT > 0.0) {
        double y = x / kT;
        if (y > 0.0) { double e = exp(-y); return e / (1.0 + e); }
        return 1.0 / (1.0 + exp(y));
    }
    if (x < -tau0) return 1.0;
    if (x > tau0) return 0.0;
    return 0.5;
}

/* Sign value of an eigenvalue: signum with signum(|x| <= tau0) = 0. */
static double signum0(double x, double tau0)
{
    if (x < -tau0) return -1.0;
    if (x > tau0) return 1.0;
    return 0.0;
}

static double inf_norm(int32_t n, const double *a)
{
    double best = 0.0;
    for (int32_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int32_t j = 0; j < n; j++) s += fabs(a[i + (int64_t)j * n]);
        if (s > best) best = s;
    }
    return best;
}

/* max|A Q - Q Lambda| and max|Q^T Q - I| for the decomposition of a0 */
static void eig_checks(int32_t n, const double *a0, const double *lam, const double *q,
                       double *res_eig, double *res_orth)
{
    double re = 0.0, ro = 0.0;
    for (int32_t k = 0; k < n; k++) {
        const double *qk = q + (int64_t)k * n;
        for (int32_t i = 0; i < n; i++) {
            double s = 0.0;
            for (int32_t j = 0; j < n; j++) s += a0[i + (int64_t)j * n] * qk[j];
            double d = fabs(s - lam[k] * qk[i]);
            if (d > re) re = d;
        }
        for (int32_t l = 0; l < n; l++) {
            const double *ql = q + (int64_t)l * n;
            double s = 0.0;
            for (int32_t i = 0; i < n; i++) s += qk[i] * ql[i];
            double d = fabs(s - (k == l ? 1.0 : 0.0));
            if (d > ro) ro = d;
        }
    }
    *res_eig = re;
    *res_orth = ro;
}

/* tau0 of the zero-eigenvalue convention: 1e-14 * ||A||_inf */
static double zero_tol(int32_t n, const double *a) { return 1e-14 * inf_norm(n, a); }

/*
 * Dense maps of a symmetric matrix (column-major, not modified):
 *   mode 0: S = sign(A) = Q signum0(Lambda) Q^T
 *   mode 1: D = Q occupation(Lambda) Q^T  (kT as given)
 * Optionally returns the eigenvalues (ascending) and eigenvectors.
 */
int32_t oracle_dense_map(int32_t n, const double *a, int32_t mode, double kT,
                         double *out, double *lam_out, double *q_out)
{
    if (n < 0 || (n > 0 && (!a || !out))) return ORACLE_E_INVALID;
    if (n == 0) return ORACLE_OK;
    double *w = malloc(sizeof(double) * (size_t)n * n);
    double *q = q_out ? q_out : malloc(sizeof(double) * (size_t)n * n);
    double *lam = lam_out ? lam_out : malloc(sizeof(double) * (size_t)n);
    double *f = malloc(sizeof(double) * (size_t)n);
    if (!w || !q || !lam || !f) return ORACLE_E_NOMEM;
    memcpy(w, a, sizeof(double) * (size_t)n * n);
    double tau0 = zero_tol(n, a);
    int32_t sw = oracle_jacobi(n, w, lam, q, 60);
    for (int32_t k = 0; k < n; k++)
        f[k] = (mode == 0) ? signum0(lam[k], tau0) : occupation(lam[k], kT, tau0);
    for (int32_t j = 0; j < n; j++)
        for (int32_t i = 0; i < n; i++) {
            double s = 0.0;
            for (int32_t k = 0; k < n; k++)
                s += q[i + (int64_t)k * n] * f[k] * q[j + (int64_t)k * n];
            out[i + (int64_t)j * n] = s;
        }
    free(w); free(f);
    if (!q_out) free(q);
    if (!lam_out) free(lam);
    return sw < 0 ? ORACLE_E_JACOBI : ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* The submatrix method on a block-sparse matrix                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t nblk;
    const int32_t *blk_size;
    const int64_t *col_ptr;
    const int32_t *row_idx;
    const double *values;
    int64_t *val_off;      /* [nnzb + 1] */
} bsc_view;

static int64_t find_block(const bsc_view *k, int32_t i, int32_t j)
{
    /* storage position of block (i, j), or -1; rows ascending per column */
    int64_t lo = k->col_ptr[j], hi = k->col_ptr[j + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int32_t r = k->row_idx[mid];
        if (r == i) return mid;
        if (r < i) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Row set of a group (submatrix step 1, generalised to a group of block
 * columns as the union of the member columns' stored block rows, ascending).
 * rows_out has room for nblk entries; returns |R(g)|.
 */
static int32_t group_rows(const bsc_view *k, const int32_t *cols, int32_t ncols,
                          char *mark, int32_t *rows_out)
{
    int32_t m = 0;
    for (int32_t c = 0; c < ncols; c++) {
        int32_t j = cols[c];
        for (int64_t p = k->col_ptr[j]; p < k->col_ptr[j + 1]; p++) mark[k->row_idx[p]] = 1;
    }
    for (int32_t i = 0; i < k->nblk; i++)
        if (mark[i]) { rows_out[m++] = i; mark[i] = 0; }
    return m;
}

/*
 * One group: assemble A_g = K[R(g), R(g)] - mu I, decompose, form the
 * group's own columns of D_g = Q occ(Lambda) Q^T and copy them into the
 * stored blocks of those columns.  lam/q (optional, n_g and n_g^2 doubles)
 * receive the decomposition; rows_out (optional, nblk ints) receives R(g).
 */
static int32_t solve_group(const bsc_view *k, const int32_t *cols, int32_t ncols,
                           double mu, double kT, double *d_values,
                           oracle_group_info *info, double *lam_keep, double *q_keep,
                           int32_t *rows_keep)
{
    int32_t nblk = k->nblk;
    char *mark = calloc((size_t)nblk, 1);
    int32_t *rows = malloc(sizeof(int32_t) * (size_t)nblk);
    int32_t *pos = malloc(sizeof(int32_t) * (size_t)nblk);    /* block -> index in R(g) */
    if (!mark || !rows || !pos) return ORACLE_E_NOMEM;
    int32_t m = group_rows(k, cols, ncols, mark, rows);
    for (int32_t i = 0; i < nblk; i++) pos[i] = -1;
    int64_t *off = malloc(sizeof(int64_t) * (size_t)(m + 1));   /* o_I in the submatrix */
    off[0] = 0;
    for (int32_t t = 0; t < m; t++) { pos[rows[t]] = t; off[t + 1] = off[t] + k->blk_size[rows[t]]; }
    int32_t n = (int32_t)off[m];

    /* A_g: stored blocks of K restricted to R(g) x R(g), zero elsewhere */
    double *a = calloc((size_t)n * n, sizeof(double));
    double *a0 = malloc(sizeof(double) * (size_t)n * n);
    double *lam = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n * n);
    double *f = malloc(sizeof(double) * (size_t)n);
    if (!a || !a0 || !lam || !q || !f) return ORACLE_E_NOMEM;
    for (int32_t tc = 0; tc < m; tc++) {
        int32_t jc = rows[tc];
        int32_t bj = k->blk_size[jc];
        for (int32_t tr = 0; tr < m; tr++) {
            int32_t ir = rows[tr];
            int64_t p = find_block(k, ir, jc);
            if (p < 0) continue;
            int32_t bi = k->blk_size[ir];
            const double *blk = k->values + k->val_off[p];
            for (int32_t cc = 0; cc < bj; cc++)
                for (int32_t rr = 0; rr < bi; rr++)
                    a[(off[tr] + rr) + (off[tc] + cc) * (int64_t)n] = blk[rr + cc * (int64_t)bi];
        }
    }
    for (int32_t i = 0; i < n; i++) a[i + (int64_t)i * n] -= mu;
    memcpy(a0, a, sizeof(double) * (size_t)n * n);

    int32_t sweeps = oracle_jacobi(n, a, lam, q, 60);
    double tau0 = zero_tol(n, a0);
    info->n = n;
    info->nrow_blk = m;
    info->sweeps = sweeps;
    info->inf_norm = inf_norm(n, a0);
    info->n_neg = 0; info->n_zero = 0;
    info->min_abs_lambda = INFINITY; info->max_abs_lambda = 0.0;
    for (int32_t l = 0; l < n; l++) {
        double x = lam[l];
        if (x < -tau0) info->n_neg++;
        else if (fabs(x) <= tau0) info->n_zero++;
        if (fabs(x) < info->min_abs_lambda) info->min_abs_lambda = fabs(x);
        if (fabs(x) > info->max_abs_lambda) info->max_abs_lambda = fabs(x);
        f[l] = occupation(x, kT, tau0);
    }
    eig_checks(n, a0, lam, q, &info->eig_residual, &info->orth_residual);

    /* own columns of D_g, copied into the stored blocks (I, J), J in g */
    if (d_values) {
        for (int32_t c = 0; c < ncols; c++) {
            int32_t jc = cols[c];
            int32_t bj = k->blk_size[jc];
            int64_t oj = off[pos[jc]];
            for (int64_t p = k->col_ptr[jc]; p < k->col_ptr[jc + 1]; p++) {
                int32_t ir = k->row_idx[p];
                int32_t bi = k->blk_size[ir];
                int64_t oi = off[pos[ir]];
                double *dst = d_values + k->val_off[p];
                for (int32_t cc = 0; cc < bj; cc++)
                    for (int32_t rr = 0; rr < bi; rr++) {
                        int64_t gi = oi + rr, gj = oj + cc;
                        double s = 0.0;
                        for (int32_t l = 0; l < n; l++)
                            s += q[gi + (int64_t)l * n] * f[l] * q[gj + (int64_t)l * n];
                        dst[rr + cc * (int64_t)bi] = s;
                    }
            }
        }
    }
    if (lam_keep) memcpy(lam_keep, lam, sizeof(double) * (size_t)n);
    if (q_keep) memcpy(q_keep, q, sizeof(double) * (size_t)n * n);
    if (rows_keep) memcpy(rows_keep, rows, sizeof(int32_t) * (size_t)m);

    free(mark); free(rows); free(pos); free(off);
    free(a); free(a0); free(lam); free(q); free(f);
    return sweeps < 0 ? ORACLE_E_JACOBI : ORACLE_OK;
}

static int32_t make_view(bsc_view *v, int32_t nblk, const int32_t *blk_size,
                         const int64_t *col_ptr, const int32_t *row_idx, const double *values)
{
    if (nblk < 0 || !blk_size || !col_ptr || !row_idx || !values) return ORACLE_E_INVALID;
    v->nblk = nblk; v->blk_size = blk_size; v->col_ptr = col_ptr;
    v->row_idx = row_idx; v->values = values;
    int64_t nnzb = col_ptr[nblk];
    v->val_off = malloc(sizeof(int64_t) * (size_t)(nnzb + 1));
    if (!v->val_off) return ORACLE_E_NOMEM;
    v->val_off[0] = 0;
    for (int32_t j = 0; j < nblk; j++)
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++)
            v->val_off[p + 1] = v->val_off[p] + (int64_t)blk_size[row_idx[p]] * blk_size[j];
    return ORACLE_OK;
}

/*
 * Step 1 of the method reads K as the symmetric matrix it is (the Kohn-Sham
 * matrix of Sec. II-A, orthogonalised, so that Eq. DsignSym applies): every
 * stored block (I, J) must have its mirror (J, I) stored, with
 * max|K_IJ - K_JI^T| <= 1e-12 max|K|.  The submatrix assembly reads both
 * triangles, so an asymmetric input is refused rather than silently used.
 */
static int32_t check_symmetric(const bsc_view *k)
{
    double amax = 0.0, dmax = 0.0;
    for (int32_t j = 0; j < k->nblk; j++)
        for (int64_t p = k->col_ptr[j]; p < k->col_ptr[j + 1]; p++) {
            int32_t i = k->row_idx[p];
            int64_t q = find_block(k, j, i);
            if (q < 0) return ORACLE_E_NOT_SYMMETRIC;
            int32_t bi = k->blk_size[i], bj = k->blk_size[j];
            const double *a = k->values + k->val_off[p];      /* bi x bj, column-major */
            const double *b = k->values + k->val_off[q];      /* bj x bi */
            for (int32_t c = 0; c < bj; c++)
                for (int32_t r = 0; r < bi; r++) {
                    double x = a[r + (int64_t)c * bi], y = b[c + (int64_t)r * bj];
                    if (!isfinite(x)) return ORACLE_E_INVALID;
                    if (fabs(x) > amax) amax = fabs(x);
                    if (fabs(x - y) > dmax) dmax = fabs(x - y);
                }
        }
    return dmax <= 1e-12 * amax ? ORACLE_OK : ORACLE_E_NOT_SYMMETRIC;
}

/* Dimension n_g and |R(g)| of every group (no decomposition). */
int32_t oracle_group_dims(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr,
                          const int32_t *row_idx, int32_t ngroups, const int32_t *grp_ptr,
                          const int32_t *grp_blocks, int32_t *n_out, int32_t *m_out)
{
    if (nblk < 0 || ngroups < 0 || !blk_size || !col_ptr || !row_idx || !grp_ptr) return ORACLE_E_INVALID;
    bsc_view v = {nblk, blk_size, col_ptr, row_idx, NULL, NULL};
    char *mark = calloc((size_t)nblk + 1, 1);
    int32_t *rows = malloc(sizeof(int32_t) * ((size_t)nblk + 1));
    for (int32_t g = 0; g < ngroups; g++) {
        int32_t m = group_rows(&v, grp_blocks + grp_ptr[g], grp_ptr[g + 1] - grp_ptr[g], mark, rows);
        int64_t n = 0;
        for (int32_t t = 0; t < m; t++) n += blk_size[rows[t]];
        if (n_out) n_out[g] = (int32_t)n;
        if (m_out) m_out[g] = m;
    }
    free(mark); free(rows);
    return ORACLE_OK;
}

/*
 * The whole method.  For every group listed in `which` (all groups when
 * which == NULL), writes the group's own block columns of D into d_values
 * (K's layout; other entries are left untouched) and its info record.
 * n_out / e_out receive N = sum of the diagonals of the written diagonal
 * blocks and E = sum over the written blocks of <D_IJ, K_IJ>, accumulated
 * in storage order after all groups are done.
 */
int32_t oracle_submatrix(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr,
                         const int32_t *row_idx, const double *values,
                         int32_t ngroups, const int32_t *grp_ptr, const int32_t *grp_blocks,
                         double mu, double kT, const int32_t *which, int32_t nwhich,
                         int32_t nthreads, double *d_values, double *n_out, double *e_out,
                         oracle_group_info *info)
{
    bsc_view v;
    int32_t st = make_view(&v, nblk, blk_size, col_ptr, row_idx, values);
    if (st) return st;
    if (ngroups < 0 || !grp_ptr || !grp_blocks || !d_values || kT < 0.0) { free(v.val_off); return ORACLE_E_INVALID; }
    st = check_symmetric(&v);
    if (st) { free(v.val_off); return st; }
    int32_t njobs = which ? nwhich : ngroups;
    int32_t status = ORACLE_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < njobs; t++) {
        int32_t g = which ? which[t] : t;
        oracle_group_info gi;
        memset(&gi, 0, sizeof gi);
        int32_t s = solve_group(&v, grp_blocks + grp_ptr[g], grp_ptr[g + 1] - grp_ptr[g],
                                mu, kT, d_values, &gi, NULL, NULL, NULL);
        if (info) info[t] = gi;
        if (s != ORACLE_OK) {
#pragma omp critical
            status = s;
        }
    }
    /* reductions over the written columns, fixed (storage) order */
    double n_acc = 0.0, e_acc = 0.0;
    for (int32_t t = 0; t < njobs; t++) {
        int32_t g = which ? which[t] : t;
        for (int32_t c = grp_ptr[g]; c < grp_ptr[g + 1]; c++) {
            int32_t j = grp_blocks[c];
            int32_t bj = blk_size[j];
            for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++) {
                int32_t i = row_idx[p];
                int32_t bi = blk_size[i];
                const double *dv = d_values + v.val_off[p];
                const double *kv = values + v.val_off[p];
                for (int64_t e = 0; e < (int64_t)bi * bj; e++) e_acc += dv[e] * kv[e];
                if (i == j)
                    for (int32_t r = 0; r < bi; r++) n_acc += dv[r + (int64_t)r * bi];
            }
        }
    }
    if (n_out) *n_out = n_acc;
    if (e_out) *e_out = e_acc;
    free(v.val_off);
    return status;
}

/*
 * Decomposition of one group's shifted submatrix, for derivative and
 * mu-search checks: rows_out (nblk ints) gets R(g), lam_out (n_g) and
 * q_out (n_g^2, column-major) the eigenpairs of K[R(g), R(g)] - mu I.
 * Call oracle_group_dims first to size the outputs.
 */
int32_t oracle_group_eig(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr,
                         const int32_t *row_idx, const double *values,
                         int32_t ncols, const int32_t *cols, double mu,
                         int32_t *rows_out, double *lam_out, double *q_out,
                         oracle_group_info *info)
{
    bsc_view v;
    int32_t st = make_view(&v, nblk, blk_size, col_ptr, row_idx, values);
    if (st) return st;
    oracle_group_info gi;
    memset(&gi, 0, sizeof gi);
    st = solve_group(&v, cols, ncols, mu, 0.0, NULL, &gi, lam_out, q_out, rows_out);
    if (info) *info = gi;
    free(v.val_off);
    return st;
}
