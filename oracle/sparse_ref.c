/*
 * Oracle helper: textbook incomplete factorizations and triangular solves on a
 * generic CSR matrix, in FP64.  TEST INFRASTRUCTURE ONLY -- only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load this file.
 *
 * These are the three sequential preconditioners compared in Section 3 of the
 * paper (items 3-5 of its preconditioner list): ILU with no fill-in, IC with
 * no fill-in and SOR (read as its symmetric form, SSOR, since PCG needs a
 * symmetric M).  Nothing here knows about the phase-unwrapping stencil: the
 * matrix arrives as CSR with column indices sorted ascending in every row and
 * the diagonal present in every row.
 *
 *   ILU(0): Gaussian elimination (IKJ order) with every update that falls
 *           outside the sparsity pattern of A dropped.  Stored in place:
 *           strict lower part = unit-lower L, diagonal + upper part = U.
 *   IC(0):  Cholesky A ~ L L^T with L restricted to the lower pattern of A.
 *   SSOR:   M = (D/w + L)(D/w)^{-1}(D/w + L^T) / (2 - w).
 *
 * Build: gcc -O2 -fPIC -shared -o liblp_oracle_sparse.so sparse_ref.c -lm
 */
#include <math.h>
#include <stddef.h>

/* position of column c in row r, or -1 (linear scan: rows hold a few entries) */
static ptrdiff_t find_col(const int* rowptr, const int* col, int r, int c)
{
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q)
        if (col[q] == c) return q;
    return -1;
}

/* ILU(0), IKJ variant.  lu: output array with the pattern of a.
 * A finished pivot below pivot_floor * a_ii is replaced by a_ii.
 * Returns the number of replaced pivots, or -(row+1) when a row has no diagonal. */
int orc_ilu0(int n, const int* rowptr, const int* col, const double* a, double pivot_floor,
             double* lu)
{
    int hits = 0;
    for (int q = 0; q < rowptr[n]; ++q) lu[q] = a[q];
    for (int i = 0; i < n; ++i) {
        for (int q = rowptr[i]; q < rowptr[i + 1] && col[q] < i; ++q) {
            int k = col[q];
            ptrdiff_t kk = find_col(rowptr, col, k, k);
            if (kk < 0 || lu[kk] == 0.0) return -(k + 1);
            lu[q] /= lu[kk];
            /* row_i -= l_ik * row_k, restricted to the pattern of row i, for columns > k */
            for (int t = q + 1; t < rowptr[i + 1]; ++t) {
                ptrdiff_t kj = find_col(rowptr, col, k, col[t]);
                if (kj >= 0) lu[t] -= lu[q] * lu[kj];
            }
        }
        ptrdiff_t ii = find_col(rowptr, col, i, i);
        if (ii < 0) return -(i + 1);
        if (lu[ii] < pivot_floor * a[ii]) { lu[ii] = a[ii]; ++hits; }
    }
    return hits;
}

/* Solve (L U) s = r with the in-place ILU(0) factors. */
void orc_lu_solve(int n, const int* rowptr, const int* col, const double* lu,
                  const double* r, double* s)
{
    for (int i = 0; i < n; ++i) {            /* L y = r, L unit lower */
        double v = r[i];
        for (int q = rowptr[i]; q < rowptr[i + 1] && col[q] < i; ++q) v -= lu[q] * s[col[q]];
        s[i] = v;
    }
    for (int i = n - 1; i >= 0; --i) {       /* U s = y */
        double v = s[i], d = 0.0;
        for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            if (col[q] > i) v -= lu[q] * s[col[q]];
            else if (col[q] == i) d = lu[q];
        }
        s[i] = v / d;
    }
}

/* IC(0): row-oriented Cholesky restricted to the lower pattern.
 * l: output array with the pattern of a; only entries with col <= row are set.
 * A squared diagonal below pivot_floor * a_ii is replaced by a_ii.
 * Returns the number of replaced pivots, or -(row+1) when a row has no diagonal. */
int orc_ic0(int n, const int* rowptr, const int* col, const double* a, double pivot_floor,
            double* l)
{
    int hits = 0;
    for (int q = 0; q < rowptr[n]; ++q) l[q] = 0.0;
    for (int i = 0; i < n; ++i) {
        double diag_acc = 0.0;
        ptrdiff_t ii = -1;
        for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            int k = col[q];
            if (k > i) break;
            if (k == i) { ii = q; break; }
            /* l_ik = (a_ik - sum_{j<k} l_ij l_kj) / l_kk over the common lower pattern */
            double v = a[q];
            for (int t = rowptr[i]; t < q; ++t) {
                ptrdiff_t kj = find_col(rowptr, col, k, col[t]);
                if (kj >= 0) v -= l[t] * l[kj];
            }
            ptrdiff_t kk = find_col(rowptr, col, k, k);
            l[q] = v / l[kk];
            diag_acc += l[q] * l[q];
        }
        if (ii < 0) return -(i + 1);
        double d = a[ii] - diag_acc;
        if (d < pivot_floor * a[ii]) { d = a[ii]; ++hits; }
        l[ii] = sqrt(d);
    }
    return hits;
}

/* Solve (L L^T) s = r with the IC(0) factor. */
void orc_llt_solve(int n, const int* rowptr, const int* col, const double* l,
                   const double* r, double* s)
{
    for (int i = 0; i < n; ++i) {            /* L y = r */
        double v = r[i], d = 1.0;
        for (int q = rowptr[i]; q < rowptr[i + 1] && col[q] <= i; ++q) {
            if (col[q] < i) v -= l[q] * s[col[q]];
            else d = l[q];
        }
        s[i] = v / d;
    }
    for (int i = n - 1; i >= 0; --i) {       /* L^T s = y, column-oriented over row i of L */
        double d = 1.0;
        ptrdiff_t ii = find_col(rowptr, col, i, i);
        if (ii >= 0) d = l[ii];
        s[i] /= d;
        for (int q = rowptr[i]; q < rowptr[i + 1] && col[q] < i; ++q) s[col[q]] -= l[q] * s[i];
    }
}

/* SSOR(w): s = M^{-1} r with M = (D/w + L)(D/w)^{-1}(D/w + L^T) / (2 - w),
 * L the strict lower part of a (symmetric a assumed). */
void orc_ssor_solve(int n, const int* rowptr, const int* col, const double* a, double w,
                    const double* r, double* s)
{
    for (int i = 0; i < n; ++i) {            /* (D/w + L) y = r */
        double v = r[i], d = 0.0;
        for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            if (col[q] < i) v -= a[q] * s[col[q]];
            else if (col[q] == i) d = a[q];
        }
        s[i] = v / (d / w);
    }
    for (int i = 0; i < n; ++i) {            /* z = (D/w) y */
        ptrdiff_t ii = find_col(rowptr, col, i, i);
        s[i] *= a[ii] / w;
    }
    for (int i = n - 1; i >= 0; --i) {       /* (D/w + L^T) t = z, using row i's upper part = L^T */
        double v = s[i], d = 0.0;
        for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            if (col[q] > i) v -= a[q] * s[col[q]];
            else if (col[q] == i) d = a[q];
        }
        s[i] = v / (d / w);
    }
    for (int i = 0; i < n; ++i) s[i] *= (2.0 - w);
}
