/*
 * Observation generator for the synthetic inverse problems: a forward solve
 * of the convection-diffusion model (eq. (1) of the paper: dC/dt =
 * div(a grad C) - v.grad C + f, C = 0 on the Dirichlet faces, zero flux on the
 * others, C(., 0) = 0) on a node-centred finite-volume mesh, advanced by the
 * Douglas alternating-direction scheme (theta = 1/2).  It is deliberately a
 * different discretisation, on a finer mesh, from the space-time finite
 * elements the inversion uses (Section 4 produces its data by a forward solve
 * on a finer mesh), and it holds none of the inversion's arithmetic.
 *
 * Space: nodes i = 0..n-1 per axis with spacing h; dual cells (half cells on
 * the boundary).  Per axis d, for a node g that is not a Dirichlet node,
 *   (L_d C)_g = sum over its axis neighbours nb of a_mid/(h^2 w_g) (C_nb - C_g)
 *               - v_d (central difference inside, one-sided on the faces)
 * with w_g = 1/2 on the first and last node of the axis, 1 elsewhere, and
 * a_mid the coefficient at the edge midpoint.  Dirichlet nodes hold C = 0
 * (their rows of L_d are zero and their columns are dropped).
 *
 * Time (Douglas scheme for C' = L C + f with L = L_x + L_y + L_z):
 *   Y_0 = C^k + dt (L C^k + (f^k + f^{k+1}) / 2)
 *   (I - dt/2 L_d) Y_d = Y_{d-1} - dt/2 L_d C^k,  d = x, y, z
 *   C^{k+1} = Y_z
 * The tridiagonal systems along each grid line are solved by the Thomas
 * algorithm with factors computed once.  Lines are independent, so the result
 * does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double *lo, *di, *hi;   /* (L_d C)_g = lo C_{g-s} + di C_g + hi C_{g+s} */
  double *cp, *m, *a;     /* Thomas factors of I - dt/2 L_d                */
} axis_t;

static void axis_free(axis_t *A) {
  free(A->lo); free(A->di); free(A->hi); free(A->cp); free(A->m); free(A->a);
}

/* Coefficients of L_d.  nn: nodes per axis; d: the axis; amid: coefficient at
 * the midpoints of the edges along d, indexed like the lower node of the edge
 * on a grid with nn[d]-1 nodes along d. */
static int axis_build(axis_t *A, const int nn[3], int d, double h, double v, const double *amid,
                      const unsigned char *dir, double dt) {
  const long N = (long)nn[0] * nn[1] * nn[2];
  A->lo = calloc(N, sizeof(double));
  A->di = calloc(N, sizeof(double));
  A->hi = calloc(N, sizeof(double));
  A->cp = calloc(N, sizeof(double));
  A->m = calloc(N, sizeof(double));
  A->a = calloc(N, sizeof(double));
  if (!A->lo || !A->di || !A->hi || !A->cp || !A->m || !A->a) return -1;
  const long s = d == 0 ? 1 : d == 1 ? nn[0] : (long)nn[0] * nn[1];
  int en[3] = {nn[0], nn[1], nn[2]};
  en[d] -= 1;   /* edge grid */
#pragma omp parallel for schedule(static)
  for (long g = 0; g < N; ++g) {
    const int pos[3] = {(int)(g % nn[0]), (int)((g / nn[0]) % nn[1]), (int)(g / ((long)nn[0] * nn[1]))};
    const int p = pos[d], n = nn[d];
    if (dir[g] || n < 2) continue;
    const double w = (p == 0 || p == n - 1) ? 0.5 : 1.0;
    double lo = 0.0, hi = 0.0, di = 0.0;
    if (p > 0) {
      int e[3] = {pos[0], pos[1], pos[2]};
      e[d] = p - 1;
      const double c = amid[e[0] + (long)en[0] * (e[1] + (long)en[1] * e[2])] / (h * h * w);
      lo += c;
      di -= c;
    }
    if (p < n - 1) {
      int e[3] = {pos[0], pos[1], pos[2]};
      e[d] = p;
      const double c = amid[e[0] + (long)en[0] * (e[1] + (long)en[1] * e[2])] / (h * h * w);
      hi += c;
      di -= c;
    }
    if (v != 0.0) {
      if (p == 0) {
        hi -= v / h;
        di += v / h;
      } else if (p == n - 1) {
        lo += v / h;
        di -= v / h;
      } else {
        hi -= v / (2.0 * h);
        lo += v / (2.0 * h);
      }
    }
    if (p > 0 && dir[g - s]) lo = 0.0;
    if (p < n - 1 && dir[g + s]) hi = 0.0;
    A->lo[g] = lo;
    A->di[g] = di;
    A->hi[g] = hi;
  }
  /* Thomas factors of I - dt/2 L_d along every line */
  const long nl = N / nn[d];
#pragma omp parallel for schedule(static)
  for (long l = 0; l < nl; ++l) {
    long g0;
    if (d == 0) g0 = l * nn[0];
    else if (d == 1) g0 = (l % nn[0]) + (l / nn[0]) * (long)nn[0] * nn[1];
    else g0 = l;
    double cprev = 0.0;
    for (int p = 0; p < nn[d]; ++p) {
      const long g = g0 + p * s;
      const double a = -0.5 * dt * A->lo[g], b = 1.0 - 0.5 * dt * A->di[g], c = -0.5 * dt * A->hi[g];
      const double piv = b - (p > 0 ? a * cprev : 0.0);
      A->m[g] = 1.0 / piv;
      A->cp[g] = c / piv;
      A->a[g] = p > 0 ? a : 0.0;
      cprev = A->cp[g];
    }
  }
  return 0;
}

/* y = L_d x */
static void axis_apply(const axis_t *A, const int nn[3], int d, const double *x, double *y) {
  const long N = (long)nn[0] * nn[1] * nn[2];
  const long s = d == 0 ? 1 : d == 1 ? nn[0] : (long)nn[0] * nn[1];
#pragma omp parallel for schedule(static)
  for (long g = 0; g < N; ++g) {
    double acc = A->di[g] * x[g];
    if (A->lo[g] != 0.0) acc += A->lo[g] * x[g - s];
    if (A->hi[g] != 0.0) acc += A->hi[g] * x[g + s];
    y[g] = acc;
  }
}

/* x = (I - dt/2 L_d)^{-1} r along every line (in place on r). */
static void axis_solve(const axis_t *A, const int nn[3], int d, double *r) {
  const long s = d == 0 ? 1 : d == 1 ? nn[0] : (long)nn[0] * nn[1];
  const int n = nn[d];
  if (d == 0) {
    const long nl = (long)nn[1] * nn[2];
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nl; ++l) {
      double *x = r + l * nn[0];
      const double *m = A->m + l * nn[0], *a = A->a + l * nn[0], *cp = A->cp + l * nn[0];
      x[0] *= m[0];
      for (int p = 1; p < n; ++p) x[p] = (x[p] - a[p] * x[p - 1]) * m[p];
      for (int p = n - 2; p >= 0; --p) x[p] -= cp[p] * x[p + 1];
    }
    return;
  }
  /* y and z: sweep whole rows of x at a time (contiguous inner loop) */
  const int outer = d == 1 ? nn[2] : nn[1];
  const long ostride = d == 1 ? (long)nn[0] * nn[1] : nn[0];
#pragma omp parallel for schedule(static)
  for (int o = 0; o < outer; ++o) {
    const long base = o * ostride;
    for (int i = 0; i < nn[0]; ++i) r[base + i] *= A->m[base + i];
    for (int p = 1; p < n; ++p) {
      const long g = base + p * s;
      for (int i = 0; i < nn[0]; ++i) r[g + i] = (r[g + i] - A->a[g + i] * r[g - s + i]) * A->m[g + i];
    }
    for (int p = n - 2; p >= 0; --p) {
      const long g = base + p * s;
      for (int i = 0; i < nn[0]; ++i) r[g + i] -= A->cp[g + i] * r[g + s + i];
    }
  }
}

/* f(x, t) = I(t) sum_k amp exp(-|x - c_k(t)|^2 / w^2), c_k(t) = p_k + t (q_k - p_k),
 * I(t) = sin(pi t) or 1; zero on Dirichlet nodes. */
static void source(const int nn[3], const double h[3], double t, int nsrc, const double *p, const double *q,
                   double w, double amp, int sin_int, const unsigned char *dir, double *f) {
  const double I = sin_int ? sin(M_PI * t) : 1.0;
  double c[3 * 16];
  for (int k = 0; k < nsrc; ++k)
    for (int e = 0; e < 3; ++e) c[3 * k + e] = p[3 * k + e] + t * (q[3 * k + e] - p[3 * k + e]);
  const double iw2 = 1.0 / (w * w);
#pragma omp parallel for schedule(static) collapse(2)
  for (int kz = 0; kz < nn[2]; ++kz)
    for (int jy = 0; jy < nn[1]; ++jy) {
      const double Y = jy * h[1], Z = kz * h[2];
      const long base = (long)nn[0] * (jy + (long)nn[1] * kz);
      for (int ix = 0; ix < nn[0]; ++ix) {
        const double X = ix * h[0];
        double acc = 0.0;
        for (int k = 0; k < nsrc; ++k) {
          const double dx = X - c[3 * k], dy = Y - c[3 * k + 1], dz = Z - c[3 * k + 2];
          acc += amp * exp(-(dx * dx + dy * dy + dz * dz) * iw2);
        }
        f[base + ix] = dir[base + ix] ? 0.0 : I * acc;
      }
    }
}

/* Forward solve; writes C at the sensor nodes after every `out_every` steps
 * (row 0 = the initial state, zero): out[(nsteps/out_every + 1) * nsens].
 * Returns 0, or -1 on bad arguments / allocation failure. */
int fv_forward(const int *nn, const double *h, double T, int nsteps, int out_every, const double *ax,
               const double *ay, const double *az, const double *v, const unsigned char *dir, int nsrc,
               const double *p, const double *q, double w, double amp, int sin_int, int nsens, const int *sens,
               double *out) {
  if (nsteps < 1 || out_every < 1 || nsteps % out_every || nsrc < 0 || nsrc > 16) return -1;
  const long N = (long)nn[0] * nn[1] * nn[2];
  const double dt = T / nsteps;
  axis_t A[3];
  memset(A, 0, sizeof(A));
  const double *amid[3] = {ax, ay, az};
  int rc = 0;
  for (int d = 0; d < 3 && rc == 0; ++d) rc = axis_build(&A[d], nn, d, h[d], v[d], amid[d], dir, dt);
  double *C = calloc(N, sizeof(double)), *Y = calloc(N, sizeof(double)), *f0 = calloc(N, sizeof(double)),
         *f1 = calloc(N, sizeof(double)), *LC[3];
  for (int d = 0; d < 3; ++d) LC[d] = calloc(N, sizeof(double));
  if (rc || !C || !Y || !f0 || !f1 || !LC[0] || !LC[1] || !LC[2]) rc = -1;
  if (rc == 0) {
    for (int s = 0; s < nsens; ++s) out[s] = 0.0;
    source(nn, h, 0.0, nsrc, p, q, w, amp, sin_int, dir, f0);
    for (int k = 0; k < nsteps; ++k) {
      source(nn, h, (k + 1) * dt, nsrc, p, q, w, amp, sin_int, dir, f1);
      for (int d = 0; d < 3; ++d) axis_apply(&A[d], nn, d, C, LC[d]);
#pragma omp parallel for schedule(static)
      for (long g = 0; g < N; ++g)
        Y[g] = C[g] + dt * (LC[0][g] + LC[1][g] + LC[2][g] + 0.5 * (f0[g] + f1[g])) - 0.5 * dt * LC[0][g];
      axis_solve(&A[0], nn, 0, Y);
      for (int d = 1; d < 3; ++d) {
#pragma omp parallel for schedule(static)
        for (long g = 0; g < N; ++g) Y[g] -= 0.5 * dt * LC[d][g];
        axis_solve(&A[d], nn, d, Y);
      }
      double *tmp = C;
      C = Y;
      Y = tmp;
      tmp = f0;
      f0 = f1;
      f1 = tmp;
      if ((k + 1) % out_every == 0) {
        double *row = out + (long)((k + 1) / out_every) * nsens;
        for (int s = 0; s < nsens; ++s) row[s] = C[sens[s]];
      }
    }
  }
  free(C); free(Y); free(f0); free(f1);
  for (int d = 0; d < 3; ++d) { free(LC[d]); axis_free(&A[d]); }
  return rc;
}
