/*
 * oracle.c -- plain, serial FP64 reference for sparse Cholesky LL^T and the
 * forward/back triangular solves on a fixed symmetric pattern.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this.  It shares no code, header or table with
 * the GPU library, and the GPU library never calls it.
 *
 * What it computes.  The paper (Sec. 3.3) singles out computations whose
 * control flow is fixed by the sparsity structure and whose values change
 * from run to run; numeric Cholesky of an SPD matrix on a fixed pattern is
 * one (no pivoting, only + - * / sqrt).  The paper itself does not define the
 * factorization, so the oracle is the textbook definition written out:
 *
 *   A^ = P A P^T  (A^_ij = A_{perm[i], perm[j]}),   A^ = L L^T,
 *   L_ik = (A^_ik - sum_{m<k} L_im L_km) / L_kk     (k < i)
 *   L_ii = sqrt(A^_ii - sum_{k<i} L_ik^2)
 *
 * evaluated row by row ("up-looking"): row i of L is a sparse triangular
 * solve with the rows above it.  Every sum runs over ascending k with plain
 * "t -= a*b" so the result does not depend on the compiler (built with
 * -O2 -ffp-contract=off -fno-fast-math).
 *
 * Symbolic part (structural, explicit zeros count, nothing is dropped):
 *   parent(j) = min { i > j : L_ij != 0 }            (elimination tree)
 *   struct(L_i,:) = union over k with A^_ik != 0, k < i, of the etree path
 *                   from k up to (not including) i, plus i  (row subtree)
 *   the column structure is the transpose; rows sorted ascending.
 * The etree uses Liu's ancestor-compression algorithm.
 *
 * Indices are 0-based; a failed pivot is reported 1-based (LAPACK style).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Rows of A^ restricted to k <= i:  for row i, entries (k, value-index). */
typedef struct {
    int64_t n;
    int64_t *rp;   /* n+1 */
    int32_t *rk;   /* column k of each entry, k <= i, sorted ascending */
    int64_t *rv;   /* index into the caller's value array */
} rows_t;

static void rows_free(rows_t *r) {
    free(r->rp); free(r->rk); free(r->rv);
    r->rp = NULL; r->rk = NULL; r->rv = NULL;
}

/* Build the rows of the permuted lower triangle.  Returns 0 or -1 (OOM). */
static int rows_build(int64_t n, const int64_t *colptr, const int32_t *rowind,
                      const int32_t *perm, rows_t *out) {
    int64_t nnz = colptr[n];
    int32_t *pinv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    out->n = n;
    out->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    out->rk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    out->rv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!pinv || !out->rp || !out->rk || !out->rv || !fill) {
        free(pinv); free(fill); rows_free(out); return -1;
    }
    for (int64_t k = 0; k < n; k++) pinv[perm ? perm[k] : k] = (int32_t)k;
    /* count entries per new row (the larger of the two new indices) */
    for (int64_t c = 0; c < n; c++)
        for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
            int32_t i = pinv[rowind[p]], j = pinv[c];
            int32_t hi = i > j ? i : j;
            out->rp[hi + 1]++;
        }
    for (int64_t i = 0; i < n; i++) out->rp[i + 1] += out->rp[i];
    memcpy(fill, out->rp, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t c = 0; c < n; c++)
        for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
            int32_t i = pinv[rowind[p]], j = pinv[c];
            int32_t hi = i > j ? i : j, lo = i > j ? j : i;
            int64_t q = fill[hi]++;
            out->rk[q] = lo;
            out->rv[q] = p;
        }
    /* sort each row by column (insertion sort: rows are short) */
    for (int64_t i = 0; i < n; i++) {
        for (int64_t a = out->rp[i] + 1; a < out->rp[i + 1]; a++) {
            int32_t kk = out->rk[a]; int64_t vv = out->rv[a];
            int64_t b = a - 1;
            while (b >= out->rp[i] && out->rk[b] > kk) {
                out->rk[b + 1] = out->rk[b]; out->rv[b + 1] = out->rv[b]; b--;
            }
            out->rk[b + 1] = kk; out->rv[b + 1] = vv;
        }
    }
    free(pinv); free(fill);
    return 0;
}

/*
 * Symbolic analysis.  Outputs parent[n] and Lcolptr[n+1] (column counts
 * include the diagonal).  If Lrowind is non-NULL it must hold Lcolptr[n]
 * entries and receives the row indices of every column, ascending, diagonal
 * first.  Only rows i < nrows are considered (nrows = n for the whole
 * matrix; a smaller value gives the pattern of the leading nrows x nrows
 * block).  Returns 0, or -1 on allocation failure.
 */
int or_symbolic(int64_t n, const int64_t *colptr, const int32_t *rowind,
                const int32_t *perm, int64_t nrows, int32_t *parent,
                int64_t *Lcolptr, int32_t *Lrowind) {
    rows_t R;
    if (nrows > n || nrows < 0) nrows = n;
    if (rows_build(n, colptr, rowind, perm, &R)) return -1;
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!anc || !mark || !cnt) { free(anc); free(mark); free(cnt); rows_free(&R); return -1; }

    /* etree: Liu's algorithm with path compression through anc[] */
    for (int64_t i = 0; i < n; i++) {
        parent[i] = -1; anc[i] = -1;
        if (i >= nrows) continue;
        for (int64_t p = R.rp[i]; p < R.rp[i + 1]; p++) {
            int32_t k = R.rk[p];
            while (k != -1 && k < i) {
                int32_t next = anc[k];
                anc[k] = (int32_t)i;
                if (next == -1) parent[k] = (int32_t)i;
                k = next;
            }
        }
    }
    /* column counts by walking every row subtree once */
    for (int64_t i = 0; i < n; i++) mark[i] = -1;
    for (int64_t i = 0; i < nrows; i++) {
        mark[i] = (int32_t)i;
        cnt[i]++; /* diagonal */
        for (int64_t p = R.rp[i]; p < R.rp[i + 1]; p++) {
            int32_t k = R.rk[p];
            while (k != -1 && k < i && mark[k] != i) {
                mark[k] = (int32_t)i;
                cnt[k]++;
                k = parent[k];
            }
        }
    }
    Lcolptr[0] = 0;
    for (int64_t j = 0; j < n; j++) Lcolptr[j + 1] = Lcolptr[j] + cnt[j];
    if (Lrowind) {
        /* rows visit columns in ascending i, so columns come out sorted */
        int64_t *fill = cnt; /* reuse as fill pointers */
        for (int64_t j = 0; j < n; j++) fill[j] = Lcolptr[j];
        for (int64_t i = 0; i < n; i++) mark[i] = -1;
        for (int64_t i = 0; i < nrows; i++) {
            mark[i] = (int32_t)i;
            for (int64_t p = R.rp[i]; p < R.rp[i + 1]; p++) {
                int32_t k = R.rk[p];
                while (k != -1 && k < i && mark[k] != i) {
                    mark[k] = (int32_t)i;
                    /* the diagonal of column k was written when row k ran */
                    Lrowind[fill[k]++] = (int32_t)i;
                    k = parent[k];
                }
            }
            Lrowind[fill[i]++] = (int32_t)i; /* diagonal: first in column i */
        }
    }
    free(anc); free(mark); free(cnt); rows_free(&R);
    return 0;
}

/*
 * Numeric up-looking factorization of rows 0..nrows-1 of A^ = P A P^T.
 * vals: the caller's values in the order of (colptr, rowind).
 * Lcolptr/Lrowind: from or_symbolic with the same nrows.
 * Lx receives the values in that pattern.  Returns 0 on success, i+1 if the
 * pivot of row i fails d > 0 (d <= 0 or NaN; rows after it are not
 * computed), -1 on allocation failure.
 */
int or_factor(int64_t n, const int64_t *colptr, const int32_t *rowind,
              const double *vals, const int32_t *perm, int64_t nrows,
              const int32_t *parent, const int64_t *Lcolptr,
              const int32_t *Lrowind, double *Lx) {
    rows_t R;
    if (nrows > n || nrows < 0) nrows = n;
    if (rows_build(n, colptr, rowind, perm, &R)) return -1;
    double *x = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *pat = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!x || !mark || !pat || !next) {
        free(x); free(mark); free(pat); free(next); rows_free(&R); return -1;
    }
    int info = 0;
    for (int64_t j = 0; j < n; j++) { mark[j] = -1; next[j] = Lcolptr[j] + 1; }
    for (int64_t i = 0; i < nrows && !info; i++) {
        /* row pattern of L (without i): the row subtree */
        int64_t np = 0;
        mark[i] = (int32_t)i;
        double d = 0.0;
        for (int64_t p = R.rp[i]; p < R.rp[i + 1]; p++) {
            int32_t k = R.rk[p];
            if (k == i) { d = vals[R.rv[p]]; continue; }
            x[k] = vals[R.rv[p]];
            while (k != -1 && k < i && mark[k] != i) {
                mark[k] = (int32_t)i;
                pat[np++] = k;
                k = parent[k];
            }
        }
        /* ascending order of k is a topological order of the row subtree */
        for (int64_t a = 1; a < np; a++) {
            int32_t v = pat[a]; int64_t b = a - 1;
            while (b >= 0 && pat[b] > v) { pat[b + 1] = pat[b]; b--; }
            pat[b + 1] = v;
        }
        for (int64_t a = 0; a < np; a++) {
            int32_t k = pat[a];
            double lkk = Lx[Lcolptr[k]];
            double lik = x[k] / lkk;
            x[k] = 0.0;
            /* subtract L_rk * L_ik from the not-yet-finished entries r < i */
            for (int64_t q = Lcolptr[k] + 1; q < next[k]; q++)
                x[Lrowind[q]] -= Lx[q] * lik;
            d -= lik * lik;
            Lx[next[k]] = lik;
            next[k]++;
        }
        if (!(d > 0.0)) { info = (int)(i + 1); break; }
        Lx[Lcolptr[i]] = sqrt(d);
    }
    free(x); free(mark); free(pat); free(next); rows_free(&R);
    return info;
}

/*
 * Solve A x = b with the factor:  y = L^{-1} (P b),  z = L^{-T} y,
 * x = P^T z.  b is [nrhs][n] (each right-hand side contiguous), overwritten
 * with x.  Forward: column-oriented; backward: dot products down each
 * column of L.
 */
void or_solve(int64_t n, const int64_t *Lcolptr, const int32_t *Lrowind,
              const double *Lx, const int32_t *perm, double *b, int64_t nrhs) {
    double *y = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    if (!y) return;
    for (int64_t r = 0; r < nrhs; r++) {
        double *bb = b + r * n;
        for (int64_t k = 0; k < n; k++) y[k] = bb[perm ? perm[k] : k];
        for (int64_t j = 0; j < n; j++) {
            double yj = y[j] / Lx[Lcolptr[j]];
            y[j] = yj;
            for (int64_t q = Lcolptr[j] + 1; q < Lcolptr[j + 1]; q++)
                y[Lrowind[q]] -= Lx[q] * yj;
        }
        for (int64_t j = n - 1; j >= 0; j--) {
            double t = y[j];
            for (int64_t q = Lcolptr[j] + 1; q < Lcolptr[j + 1]; q++)
                t -= Lx[q] * y[Lrowind[q]];
            y[j] = t / Lx[Lcolptr[j]];
        }
        for (int64_t k = 0; k < n; k++) bb[perm ? perm[k] : k] = y[k];
    }
    free(y);
}

/*
 * y = A x for the symmetric matrix given by its lower CSC triangle
 * (original numbering).  x, y are [nrhs][n].
 */
void or_spmv(int64_t n, const int64_t *colptr, const int32_t *rowind,
             const double *vals, const double *x, double *y, int64_t nrhs) {
    for (int64_t r = 0; r < nrhs; r++) {
        const double *xx = x + r * n;
        double *yy = y + r * n;
        for (int64_t i = 0; i < n; i++) yy[i] = 0.0;
        for (int64_t c = 0; c < n; c++)
            for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
                int32_t i = rowind[p];
                yy[i] += vals[p] * xx[c];
                if (i != c) yy[c] += vals[p] * xx[i];
            }
    }
}

/*
 * Estimate of ||A^{-1}||_1 from solves with the factor (Hager 1984, with
 * Higham's 1988 safeguards as used by LAPACK's one-norm estimators).  It
 * maximizes the convex function f(x) = ||A^{-1} x||_1 over the unit ball of
 * the one-norm by a gradient ascent that only visits vertices e_j:
 *   x = (1/n, ..., 1/n)
 *   repeat: y = A^{-1} x,  xi = sign(y),  z = A^{-T} xi (A symmetric, so one
 *           more solve with the same factor);
 *           if max_j |z_j| <= z^T x (no vertex improves), stop with ||y||_1;
 *           else x = e_j with j = argmax |z_j| (stop when j repeats)
 * at most five times; the estimate is a lower bound of ||A^{-1}||_1.  It is
 * then compared with 2 ||A^{-1} v||_1 / (3n) for the alternating vector
 * v_i = (-1)^i (1 + i/(n-1)), which catches matrices where the ascent stops
 * at a poor vertex, and the larger of the two is returned.  Returns -1 on
 * allocation failure.
 */
double or_inv_norm1_est(int64_t n, const int64_t *Lcolptr, const int32_t *Lrowind,
                        const double *Lx, const int32_t *perm) {
    if (n <= 0) return 0.0;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y) { free(x); free(y); return -1.0; }
    for (int64_t i = 0; i < n; i++) x[i] = 1.0 / (double)n;
    double est = 0.0;
    int64_t jlast = -1;
    for (int it = 0; it < 5; it++) {
        memcpy(y, x, sizeof(double) * (size_t)n);
        or_solve(n, Lcolptr, Lrowind, Lx, perm, y, 1);       /* y = A^{-1} x */
        double ny = 0.0;
        for (int64_t i = 0; i < n; i++) ny += fabs(y[i]);
        if (ny <= est && it > 0) break;                       /* no progress */
        est = ny;
        for (int64_t i = 0; i < n; i++) y[i] = y[i] >= 0.0 ? 1.0 : -1.0;
        or_solve(n, Lcolptr, Lrowind, Lx, perm, y, 1);       /* z = A^{-T} xi */
        double ztx = 0.0, zmax = -1.0;
        int64_t j = 0;
        for (int64_t i = 0; i < n; i++) {
            ztx += y[i] * x[i];
            if (fabs(y[i]) > zmax) { zmax = fabs(y[i]); j = i; }
        }
        if (zmax <= ztx || j == jlast) break;
        jlast = j;
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
        x[j] = 1.0;
    }
    /* alternating-sign test vector */
    for (int64_t i = 0; i < n; i++) {
        double mag = 1.0 + (n > 1 ? (double)i / (double)(n - 1) : 0.0);
        x[i] = (i % 2 == 0) ? mag : -mag;
    }
    or_solve(n, Lcolptr, Lrowind, Lx, perm, x, 1);
    double alt = 0.0;
    for (int64_t i = 0; i < n; i++) alt += fabs(x[i]);
    alt = 2.0 * alt / (3.0 * (double)n);
    free(x); free(y);
    return alt > est ? alt : est;
}
