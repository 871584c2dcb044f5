/* Oracle 3x3 point-block ILU on a given pattern and its triangular solves --
 * test infrastructure.
 *
 * Plain, unblocked C written for readability, not speed.  The matrix is in
 * block-CSR form (3x3 blocks stored row-major, 9 doubles each) with column
 * indices sorted inside every block row; diagpos[i] is the position of the
 * diagonal block of row i.  The sparsity pattern is the given one -- the
 * 81-point block pattern for ILU(0), the level-k pattern (computed by the
 * caller) for ILU(k) -- and no entry outside it is created, in the IKJ order
 *     for i: for k < i in row i (ascending): a_ik <- a_ik * inv(a_kk)
 *                                             a_ij <- a_ij - a_ik * a_kj  (j > k, j in row i)
 * Diagonal blocks are inverted by Gauss-Jordan elimination with partial
 * pivoting; the inverses are returned in dinv (the diagonal blocks of vals keep
 * U_ii itself).
 */
#include <math.h>
#include <string.h>

static void mul33(const double *a, const double *b, double *c) {
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s)
      c[3 * r + s] = a[3 * r + 0] * b[0 + s] + a[3 * r + 1] * b[3 + s] + a[3 * r + 2] * b[6 + s];
}

/* Gauss-Jordan with partial pivoting on [A | I]; returns 0 if singular. */
static int inv33(const double *a, double *out) {
  double m[3][6];
  for (int r = 0; r < 3; ++r) {
    for (int s = 0; s < 3; ++s) {
      m[r][s] = a[3 * r + s];
      m[r][3 + s] = (r == s) ? 1.0 : 0.0;
    }
  }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
    if (!(fabs(m[piv][col]) > 0.0)) return 0;
    if (piv != col)
      for (int s = 0; s < 6; ++s) { double t = m[col][s]; m[col][s] = m[piv][s]; m[piv][s] = t; }
    double d = m[col][col];
    for (int s = 0; s < 6; ++s) m[col][s] /= d;
    for (int r = 0; r < 3; ++r) {
      if (r == col) continue;
      double f = m[r][col];
      for (int s = 0; s < 6; ++s) m[r][s] -= f * m[col][s];
    }
  }
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) out[3 * r + s] = m[r][3 + s];
  return 1;
}

int oracle_inv33(const double *a, double *out) { return inv33(a, out); }

/* Returns 0 on success, 1 + row index of a singular pivot otherwise. */
int oracle_bilu0(int nrows, const int *indptr, const int *indices, const int *diagpos,
                 double *vals, double *dinv) {
  double L[9], T[9];
  for (int i = 0; i < nrows; ++i) {
    for (int p = indptr[i]; p < diagpos[i]; ++p) {
      int k = indices[p];
      mul33(vals + 9 * (long)p, dinv + 9 * (long)k, L);
      memcpy(vals + 9 * (long)p, L, sizeof(L));
      int pi = p + 1;
      for (int q = diagpos[k] + 1; q < indptr[k + 1]; ++q) {
        int j = indices[q];
        while (pi < indptr[i + 1] && indices[pi] < j) ++pi;
        if (pi < indptr[i + 1] && indices[pi] == j) {
          mul33(L, vals + 9 * (long)q, T);
          for (int e = 0; e < 9; ++e) vals[9 * (long)pi + e] -= T[e];
        }
      }
    }
    if (!inv33(vals + 9 * (long)diagpos[i], dinv + 9 * (long)i)) return 1 + i;
  }
  return 0;
}

/* z = U^{-1} L^{-1} r with L unit lower (blocks left of the diagonal). */
void oracle_bilu0_solve(int nrows, const int *indptr, const int *indices, const int *diagpos,
                        const double *vals, const double *dinv, const double *r, double *z) {
  double *y = z; /* forward result stored in z, then overwritten backward */
  for (int i = 0; i < nrows; ++i) {
    double s[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
    for (int p = indptr[i]; p < diagpos[i]; ++p) {
      const double *a = vals + 9 * (long)p;
      const double *x = y + 3 * (long)indices[p];
      for (int c = 0; c < 3; ++c) s[c] -= a[3 * c] * x[0] + a[3 * c + 1] * x[1] + a[3 * c + 2] * x[2];
    }
    y[3 * i] = s[0]; y[3 * i + 1] = s[1]; y[3 * i + 2] = s[2];
  }
  for (int i = nrows - 1; i >= 0; --i) {
    double s[3] = {y[3 * i], y[3 * i + 1], y[3 * i + 2]};
    for (int p = diagpos[i] + 1; p < indptr[i + 1]; ++p) {
      const double *a = vals + 9 * (long)p;
      const double *x = z + 3 * (long)indices[p];
      for (int c = 0; c < 3; ++c) s[c] -= a[3 * c] * x[0] + a[3 * c + 1] * x[1] + a[3 * c + 2] * x[2];
    }
    const double *d = dinv + 9 * (long)i;
    for (int c = 0; c < 3; ++c) z[3 * i + c] = d[3 * c] * s[0] + d[3 * c + 1] * s[1] + d[3 * c + 2] * s[2];
  }
}

/* Symbolic ILU(level) on a block pattern (test infrastructure).
 *
 * Input: the level-0 pattern in block CSR (indptr0, indices0, columns sorted,
 * diagonal included), n rows.  For every row i, in order: the entries of the
 * level-0 pattern get level 0; the columns k < i of the row are taken in
 * ascending order (fill columns k < i join as they appear) and every entry
 * (k, j), j > k, of the already computed row k offers (i, j) the level
 * lev(i, k) + lev(k, j) + 1; entries whose smallest offered level is <= level
 * are kept.  Output: indptr[n + 1], indices and levs (sorted columns) with
 * room for `cap` entries.  Returns the number of entries, or -1 if cap is too
 * small (or out of memory). */
#include <stdlib.h>

static void heap_push(int *h, int *len, int v) {
  int i = (*len)++;
  h[i] = v;
  while (i > 0) {
    int p = (i - 1) / 2;
    if (h[p] <= h[i]) break;
    int t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static int heap_pop(int *h, int *len) {
  int top = h[0];
  h[0] = h[--(*len)];
  int i = 0;
  for (;;) {
    int l = 2 * i + 1, r = l + 1, m = i;
    if (l < *len && h[l] < h[m]) m = l;
    if (r < *len && h[r] < h[m]) m = r;
    if (m == i) break;
    int t = h[m]; h[m] = h[i]; h[i] = t;
    i = m;
  }
  return top;
}

static int cmp_int(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}

long oracle_iluk_symbolic(int n, const int *indptr0, const int *indices0, int level, long cap, long *indptr,
                          int *indices, int *levs) {
  int *lev = malloc(sizeof(int) * (size_t)n);
  int *done = malloc(sizeof(int) * (size_t)n);
  int *touched = malloc(sizeof(int) * (size_t)n);
  int *heap = malloc(sizeof(int) * (size_t)n);
  if (!lev || !done || !touched || !heap) {
    free(lev); free(done); free(touched); free(heap);
    return -1;
  }
  for (int j = 0; j < n; ++j) { lev[j] = -1; done[j] = -1; }
  long nnz = 0;
  indptr[0] = 0;
  for (int i = 0; i < n; ++i) {
    int nt = 0, hl = 0;
    for (int p = indptr0[i]; p < indptr0[i + 1]; ++p) {
      int j = indices0[p];
      lev[j] = 0;
      touched[nt++] = j;
      if (j < i) heap_push(heap, &hl, j);
    }
    while (hl > 0) {
      int k = heap_pop(heap, &hl);
      if (done[k] == i) continue;
      done[k] = i;
      int lik = lev[k];
      for (long q = indptr[k]; q < indptr[k + 1]; ++q) {
        int j = indices[q];
        if (j <= k) continue;
        int cand = lik + levs[q] + 1;
        if (cand > level) continue;
        if (lev[j] < 0) {
          lev[j] = cand;
          touched[nt++] = j;
          if (j < i) heap_push(heap, &hl, j);
        } else if (cand < lev[j]) {
          lev[j] = cand;
        }
      }
    }
    qsort(touched, (size_t)nt, sizeof(int), cmp_int);
    if (nnz + nt > cap) {
      free(lev); free(done); free(touched); free(heap);
      return -1;
    }
    for (int t = 0; t < nt; ++t) {
      indices[nnz + t] = touched[t];
      levs[nnz + t] = lev[touched[t]];
      lev[touched[t]] = -1;
    }
    nnz += nt;
    indptr[i + 1] = nnz;
  }
  free(lev); free(done); free(touched); free(heap);
  return nnz;
}
