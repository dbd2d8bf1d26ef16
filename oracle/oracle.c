/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, single-threaded FP64 sparse Cholesky used only to check the
 * GPU library.  Only the tests, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no code, header or table with the library.
 *
 * What it computes (the plain definition the multifrontal method reaches up
 * to rounding; Tacho section of the paper, three-phase interface of the
 * Trilinos section):
 *   given SPD A and the library's final permutation p (new -> old),
 *   C[i][j] = A[p[i]][p[j]], C = L L^T with L lower triangular and a positive
 *   diagonal, and x = P^T L^{-T} L^{-1} P b.
 *
 * Symbolic quantities (defined on the pattern of C, explicit zeros counted,
 * no cancellation, diagonal always present):
 *   parent(j) = min{ i > j : L_ij != 0 }, -1 for a root   (elimination tree)
 *   eta_j     = #{ i >= j : L_ij != 0 }                      (column count)
 *   fundamental supernodes: j and j+1 share one iff parent(j) = j+1,
 *   eta_j = eta_{j+1} + 1 and j+1 has exactly one child; relaxed supernodes
 *   merge those along chains while few explicit zeros are added (below).
 *
 * Numeric values are read from the original lower triangle (row >= col).
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so
 * every multiply and subtract rounds separately).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOTSPD -3
#define ORACLE_ENOMEM -4

/* Upper triangle of C in compressed columns: column j holds rows i < j. */
static int upper_pattern(int64_t n, const int64_t *rowptr, const int32_t *colind,
                         const int32_t *pinv, int64_t **up_out, int32_t **ui_out) {
    int64_t *up = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!up) return ORACLE_ENOMEM;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            int64_t i = pinv[r], j = pinv[colind[k]];
            if (i < j) up[j + 1]++;
        }
    for (int64_t j = 0; j < n; ++j) up[j + 1] += up[j];
    int32_t *ui = (int32_t *)malloc(sizeof(int32_t) * (size_t)(up[n] > 0 ? up[n] : 1));
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!ui || !next) { free(up); free(ui); free(next); return ORACLE_ENOMEM; }
    for (int64_t j = 0; j < n; ++j) next[j] = up[j];
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            int64_t i = pinv[r], j = pinv[colind[k]];
            if (i < j) ui[next[j]++] = (int32_t)i;
        }
    free(next);
    *up_out = up;
    *ui_out = ui;
    return ORACLE_OK;
}

static int32_t *inverse_perm(int64_t n, const int32_t *perm) {
    int32_t *pinv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!pinv) return NULL;
    for (int64_t i = 0; i < n; ++i) pinv[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (perm[i] < 0 || perm[i] >= n || pinv[perm[i]] != -1) { free(pinv); return NULL; }
        pinv[perm[i]] = (int32_t)i;
    }
    return pinv;
}

/* Elimination tree (Liu), with path compression through `anc`. */
static void etree_upper(int64_t n, const int64_t *up, const int32_t *ui, int32_t *parent,
                        int32_t *anc) {
    for (int64_t j = 0; j < n; ++j) {
        parent[j] = -1;
        anc[j] = -1;
        for (int64_t p = up[j]; p < up[j + 1]; ++p) {
            int32_t i = ui[p];
            while (i != -1 && i < j) {
                int32_t inext = anc[i];
                anc[i] = (int32_t)j;
                if (inext == -1) { parent[i] = (int32_t)j; break; }
                i = inext;
            }
        }
    }
}

/* Row structure of row j of L (columns k < j with L_jk != 0): union of the
 * etree paths from each i with C_ji != 0 up to j.  Returns the count;
 * `mark` must not hold j on entry for any node. */
static int64_t row_reach(int64_t j, const int64_t *up, const int32_t *ui, const int32_t *parent,
                         int32_t *mark, int32_t *out) {
    int64_t cnt = 0;
    mark[j] = (int32_t)j;
    for (int64_t p = up[j]; p < up[j + 1]; ++p) {
        int32_t k = ui[p];
        while (k != -1 && mark[k] != j) {
            mark[k] = (int32_t)j;
            out[cnt++] = k;
            k = parent[k];
        }
    }
    return cnt;
}

/* parent[n], colcount[n] (eta_j, diagonal included). */
int oracle_symbolic(int64_t n, const int64_t *rowptr, const int32_t *colind, const int32_t *perm,
                    int32_t *parent, int64_t *colcount) {
    if (n < 0) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    int32_t *pinv = inverse_perm(n, perm);
    if (!pinv) return ORACLE_EINVAL;
    int64_t *up;
    int32_t *ui;
    int rc = upper_pattern(n, rowptr, colind, pinv, &up, &ui);
    if (rc) { free(pinv); return rc; }
    int32_t *work = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * 2);
    if (!work) { free(pinv); free(up); free(ui); return ORACLE_ENOMEM; }
    int32_t *mark = work, *reach = work + n;
    etree_upper(n, up, ui, parent, mark);
    for (int64_t j = 0; j < n; ++j) { colcount[j] = 1; mark[j] = -1; }
    for (int64_t j = 0; j < n; ++j) {
        int64_t cnt = row_reach(j, up, ui, parent, mark, reach);
        for (int64_t t = 0; t < cnt; ++t) colcount[reach[t]]++;
    }
    free(work);
    free(pinv);
    free(up);
    free(ui);
    return ORACLE_OK;
}

/* Fundamental supernodes from the etree and column counts.
 * super_ptr[nsuper+1]: first column of each supernode; super_parent[nsuper]:
 * supernode holding parent(last column), -1 for a root.  Arrays sized n+1 / n. */
int oracle_supernodes(int64_t n, const int32_t *parent, const int64_t *colcount,
                      int32_t *super_ptr, int32_t *super_parent, int64_t *nsuper_out) {
    if (n < 0) return ORACLE_EINVAL;
    int32_t *nchild = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *col2super = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!nchild || !col2super) { free(nchild); free(col2super); return ORACLE_ENOMEM; }
    for (int64_t j = 0; j < n; ++j)
        if (parent[j] >= 0) nchild[parent[j]]++;
    int64_t ns = 0;
    for (int64_t j = 0; j < n; ++j) {
        int joins = j > 0 && parent[j - 1] == j && colcount[j - 1] == colcount[j] + 1 &&
                    nchild[j] == 1;
        if (!joins) super_ptr[ns++] = (int32_t)j;
        col2super[j] = (int32_t)(ns - 1);
    }
    super_ptr[ns] = (int32_t)n;
    for (int64_t s = 0; s < ns; ++s) {
        int32_t last = super_ptr[s + 1] - 1;
        super_parent[s] = parent[last] < 0 ? -1 : col2super[parent[last]];
    }
    *nsuper_out = ns;
    free(nchild);
    free(col2super);
    return ORACLE_OK;
}

/* Relaxed supernodes: the reading taken of the paper's "dense supernodal
 * blocks" (Tacho section).  Walk the fundamental supernodes in column order;
 * supernode p joins the group that ends at column f_p - 1 when that group's
 * last column has parent f_p and the merged dense block (w columns, order
 * m = w + eta_{l_p - 1} - 1, padded = sum over its columns of the rows at or
 * below the column) has at most padded/2 (m <= 16), padded/5 (m <= 64) or
 * padded/20 entries that are structurally zero. */
int oracle_relaxed_supernodes(int64_t n, const int32_t *parent, const int64_t *colcount,
                              int32_t *super_ptr, int32_t *super_parent, int64_t *nsuper_out) {
    if (n < 0) return ORACLE_EINVAL;
    int32_t *fptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *fpar = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *col2super = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!fptr || !fpar || !col2super) { free(fptr); free(fpar); free(col2super); return ORACLE_ENOMEM; }
    int64_t nf = 0;
    int rc = oracle_supernodes(n, parent, colcount, fptr, fpar, &nf);
    if (rc) { free(fptr); free(fpar); free(col2super); return rc; }
    int64_t ns = 0;
    long long group_true = 0; /* structural entries of the open group */
    for (int64_t p = 0; p < nf; ++p) {
        int64_t f = fptr[p], l = fptr[p + 1];
        long long ptrue = 0;
        for (int64_t j = f; j < l; ++j) ptrue += colcount[j];
        int merge = 0;
        if (ns > 0 && parent[f - 1] == f) {
            int64_t g = super_ptr[ns - 1];
            long long m = (long long)(l - g) + colcount[l - 1] - 1;
            long long padded = 0;
            for (int64_t j = g; j < l; ++j) padded += m - (j - g);
            long long zeros = padded - (group_true + ptrue);
            long long div = m <= 16 ? 2 : (m <= 64 ? 5 : 20);
            merge = zeros * div <= padded;
        }
        if (merge) {
            group_true += ptrue;
        } else {
            super_ptr[ns++] = (int32_t)f;
            group_true = ptrue;
        }
    }
    super_ptr[ns] = (int32_t)n;
    for (int64_t s = 0; s < ns; ++s)
        for (int32_t j = super_ptr[s]; j < super_ptr[s + 1]; ++j) col2super[j] = (int32_t)s;
    for (int64_t s = 0; s < ns; ++s) {
        int32_t last = super_ptr[s + 1] - 1;
        super_parent[s] = parent[last] < 0 ? -1 : col2super[parent[last]];
    }
    *nsuper_out = ns;
    free(fptr);
    free(fpar);
    free(col2super);
    return ORACLE_OK;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Left-looking numeric factorization.  Lp[n+1] must hold the prefix sums of
 * the column counts (from oracle_symbolic); Li/Lx are filled, each column
 * sorted ascending with the diagonal first.  On a non-positive or NaN pivot
 * returns ORACLE_ENOTSPD with *fail_index = p[j] (original numbering). */
int oracle_factor(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *values,
                  const int32_t *perm, const int32_t *parent, const int64_t *Lp, int32_t *Li,
                  double *Lx, int64_t *fail_index) {
    if (n < 0) return ORACLE_EINVAL;
    *fail_index = -1;
    if (n == 0) return ORACLE_OK;
    int32_t *pinv = inverse_perm(n, perm);
    if (!pinv) return ORACLE_EINVAL;
    int64_t *up;
    int32_t *ui;
    int rc = upper_pattern(n, rowptr, colind, pinv, &up, &ui);
    if (rc) { free(pinv); return rc; }

    /* Lower triangle of C with values, column j holds rows i >= j. */
    int64_t *cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
            if (r >= colind[k]) {
                int64_t a = pinv[r], b = pinv[colind[k]];
                cp[(a < b ? a : b) + 1]++;
            }
    for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cp[n] > 0 ? cp[n] : 1));
    double *cx = (double *)malloc(sizeof(double) * (size_t)(cp[n] > 0 ? cp[n] : 1));
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *reach = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *x = (double *)calloc((size_t)n, sizeof(double));
    for (int64_t j = 0; j < n; ++j) next[j] = cp[j];
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
            if (r >= colind[k]) {
                int64_t a = pinv[r], b = pinv[colind[k]];
                int64_t col = a < b ? a : b, row = a < b ? b : a;
                ci[next[col]] = (int32_t)row;
                cx[next[col]] = values[k];
                next[col]++;
            }

    /* Structure of L: row j of L is row_reach(j); appending j to every
     * column in it, for j ascending, leaves each column sorted. */
    for (int64_t j = 0; j < n; ++j) { next[j] = Lp[j] + 1; Li[Lp[j]] = (int32_t)j; mark[j] = -1; }
    for (int64_t j = 0; j < n; ++j) {
        int64_t cnt = row_reach(j, up, ui, parent, mark, reach);
        for (int64_t t = 0; t < cnt; ++t) Li[next[reach[t]]++] = (int32_t)j;
    }

    /* Numeric: x = C[j:, j] - sum_k L[j:, k] L_jk, then scale. */
    for (int64_t j = 0; j < n; ++j) { next[j] = Lp[j] + 1; mark[j] = -1; }
    rc = ORACLE_OK;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t p = cp[j]; p < cp[j + 1]; ++p) x[ci[p]] = cx[p];
        int64_t cnt = row_reach(j, up, ui, parent, mark, reach);
        qsort(reach, (size_t)cnt, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < cnt; ++t) {
            int32_t k = reach[t];
            int64_t pos = next[k]; /* Li[pos] == j */
            double ljk = Lx[pos];
            for (int64_t p = pos; p < Lp[k + 1]; ++p) {
                double prod = Lx[p] * ljk;
                x[Li[p]] = x[Li[p]] - prod;
            }
            next[k] = pos + 1;
        }
        double d = x[j];
        if (!(d > 0.0)) {
            *fail_index = perm[j];
            rc = ORACLE_ENOTSPD;
            break;
        }
        double ljj = sqrt(d);
        Lx[Lp[j]] = ljj;
        x[j] = 0.0;
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
            Lx[p] = x[Li[p]] / ljj;
            x[Li[p]] = 0.0;
        }
    }
    free(pinv); free(up); free(ui); free(cp); free(ci); free(cx);
    free(next); free(mark); free(reach); free(x);
    return rc;
}

/* x = P^T L^{-T} L^{-1} P b for nrhs column-major columns (leading dim ld).
 * Column-oriented forward then backward substitution, one column at a time.
 * x may alias b. */
int oracle_solve(int64_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
                 const int32_t *perm, int64_t nrhs, const double *b, int64_t ldb, double *x,
                 int64_t ldx) {
    if (n < 0 || nrhs < 0 || ldb < n || ldx < n) return ORACLE_EINVAL;
    double *z = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!z) return ORACLE_ENOMEM;
    for (int64_t c = 0; c < nrhs; ++c) {
        const double *bc = b + c * ldb;
        double *xc = x + c * ldx;
        for (int64_t i = 0; i < n; ++i) z[i] = bc[perm[i]];
        for (int64_t j = 0; j < n; ++j) {
            z[j] = z[j] / Lx[Lp[j]];
            for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
                double prod = Lx[p] * z[j];
                z[Li[p]] = z[Li[p]] - prod;
            }
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            double s = z[j];
            for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
                double prod = Lx[p] * z[Li[p]];
                s = s - prod;
            }
            z[j] = s / Lx[Lp[j]];
        }
        for (int64_t i = 0; i < n; ++i) xc[perm[i]] = z[i];
    }
    free(z);
    return ORACLE_OK;
}
