/*
 * Falicov-Kimball impurity update in extended precision (oracle; TEST
 * INFRASTRUCTURE ONLY: only the test suite calls it, through
 * oracle/impurity.py).
 *
 * The same steps as oracle.impurity.update, in the same order (Sec. II: eq.
 * effective_medium, eq. dynamical_mean_field with the point-split chemical
 * potential shifts of the M display, eq. g_imp_solve, Dyson again), carried
 * out in long double complex (64-bit significand) instead of complex128:
 *   g_r   = G_loc W,   s_r = Sigma W                 (right-weighted kernels)
 *   g0inv = inv(g_r) + s_r                           (effective medium)
 *   a_m   = g0inv + i W^-1 (M(mu + d_m) - M(mu))     (m = 0, 1)
 *   g_imp = (1 - w1) inv(a_0) + w1 inv(a_1)
 *   Sigma_new = (g0inv - inv(g_imp)) W^-1
 * The last line subtracts two matrices of order 1/dt to leave one of order
 * Sigma, so the complex128 evaluation loses about log10(|g0inv| / |Sigma|)
 * digits on top of the inversions' rounding; the 11 extra bits here keep the
 * reference far below the 1e-10 parity bar at N_c in the thousands.
 *
 * Inverses: textbook Gauss-Jordan elimination with partial pivoting (largest
 * modulus in the column), row interchanges recorded and undone on the columns
 * at the end.  Rows of the elimination are spread over OpenMP threads.
 *
 * Layout: every matrix is n x n, row-major, interleaved (re, im) doubles;
 * w holds n complex weights (re, im).  Returns 0, or 1 for an exactly zero
 * pivot, 2 for an allocation failure.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

/* In-place inverse of the n x n complex matrix (re, im split). */
static int gj_inverse(int n, ld* re, ld* im, int* perm_row) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    ld best = -1.0L;
    for (int i = k; i < n; ++i) {
      const ld a = hypotl(re[(size_t)i * n + k], im[(size_t)i * n + k]);
      if (a > best) {
        best = a;
        p = i;
      }
    }
    if (best == 0.0L) return 1;
    perm_row[k] = p;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        ld t = re[(size_t)k * n + j];
        re[(size_t)k * n + j] = re[(size_t)p * n + j];
        re[(size_t)p * n + j] = t;
        t = im[(size_t)k * n + j];
        im[(size_t)k * n + j] = im[(size_t)p * n + j];
        im[(size_t)p * n + j] = t;
      }
    }
    /* scale the pivot row by 1 / pivot; the pivot column takes 1 / pivot */
    const ld pr = re[(size_t)k * n + k], pi = im[(size_t)k * n + k];
    const ld den = pr * pr + pi * pi;
    const ld ir = pr / den, ii = -pi / den;
    re[(size_t)k * n + k] = 1.0L;
    im[(size_t)k * n + k] = 0.0L;
    for (int j = 0; j < n; ++j) {
      const ld xr = re[(size_t)k * n + j], xi = im[(size_t)k * n + j];
      re[(size_t)k * n + j] = xr * ir - xi * ii;
      im[(size_t)k * n + j] = xr * ii + xi * ir;
    }
    /* eliminate column k from every other row */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const ld fr = re[(size_t)i * n + k], fi = im[(size_t)i * n + k];
      if (fr == 0.0L && fi == 0.0L) continue;
      re[(size_t)i * n + k] = 0.0L;
      im[(size_t)i * n + k] = 0.0L;
      ld* ri = re + (size_t)i * n;
      ld* mi = im + (size_t)i * n;
      const ld* rk = re + (size_t)k * n;
      const ld* mk = im + (size_t)k * n;
      for (int j = 0; j < n; ++j) {
        ri[j] -= fr * rk[j] - fi * mk[j];
        mi[j] -= fr * mk[j] + fi * rk[j];
      }
    }
  }
  /* the result is inv(P A) = inv(A) P^-1: undo the interchanges on the
     columns, last one first */
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm_row[k];
    if (p == k) continue;
    for (int i = 0; i < n; ++i) {
      ld t = re[(size_t)i * n + k];
      re[(size_t)i * n + k] = re[(size_t)i * n + p];
      re[(size_t)i * n + p] = t;
      t = im[(size_t)i * n + k];
      im[(size_t)i * n + k] = im[(size_t)i * n + p];
      im[(size_t)i * n + p] = t;
    }
  }
  return 0;
}

/* Inverse of an n x n complex128 matrix in extended precision (for the pins
   of this file's elimination); out may alias a. */
int oracle_inverse_ld(int n, const double* a, double* out) {
  const size_t nn = (size_t)n * n;
  ld* re = malloc(sizeof(ld) * nn);
  ld* im = malloc(sizeof(ld) * nn);
  int* perm = malloc(sizeof(int) * (size_t)n);
  if (!re || !im || !perm) {
    free(re); free(im); free(perm);
    return 2;
  }
  for (size_t e = 0; e < nn; ++e) {
    re[e] = a[2 * e];
    im[e] = a[2 * e + 1];
  }
  const int s = gj_inverse(n, re, im, perm);
  for (size_t e = 0; e < nn && s == 0; ++e) {
    out[2 * e] = (double)re[e];
    out[2 * e + 1] = (double)im[e];
  }
  free(re); free(im); free(perm);
  return s;
}

/* Entry (j, j-1) and the corner (0, n-1) of i W^-1 (M(mu + d) - M(mu)): the
   paper's M has subdiagonal -(1 + i W_j mu) and corner +(1 + i W_0 mu). */
static void shift_entry(ld wr, ld wi, ld d, int corner, ld* sr, ld* si) {
  /* M(mu + d) - M(mu) at the entry: -/+ i W d (mu cancels) */
  const ld sign = corner ? 1.0L : -1.0L;
  const ld dr = sign * (-wi * d), di = sign * (wr * d);   /* sign * i W d */
  /* i (dr + i di) / W */
  const ld nr = -di, ni = dr;
  const ld den = wr * wr + wi * wi;
  *sr = (nr * wr + ni * wi) / den;
  *si = (ni * wr - nr * wi) / den;
}

int oracle_impurity_update_ld(int n, const double* gloc, const double* sigma,
                              const double* w, double d0, double d1, double w1,
                              double* out) {
  const size_t nn = (size_t)n * n;
  ld* buf = malloc(sizeof(ld) * nn * 10);
  int* perm = malloc(sizeof(int) * (size_t)n);
  if (!buf || !perm) {
    free(buf); free(perm);
    return 2;
  }
  ld *g0r = buf, *g0i = buf + nn, *a0r = buf + 2 * nn, *a0i = buf + 3 * nn;
  ld *a1r = buf + 4 * nn, *a1i = buf + 5 * nn, *gir = buf + 6 * nn, *gii = buf + 7 * nn;
  ld *tr = buf + 8 * nn, *ti = buf + 9 * nn;
  int status = 0;
  /* g_r = G_loc W (right weighting: column j times W_j) */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t e = (size_t)i * n + j;
      const ld gr = gloc[2 * e], gi = gloc[2 * e + 1];
      const ld wr = w[2 * j], wi = w[2 * j + 1];
      g0r[e] = gr * wr - gi * wi;
      g0i[e] = gr * wi + gi * wr;
    }
  /* g0inv = inv(g_r) + Sigma W */
  if ((status = gj_inverse(n, g0r, g0i, perm)) != 0) goto done;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t e = (size_t)i * n + j;
      const ld sr = sigma[2 * e], si = sigma[2 * e + 1];
      const ld wr = w[2 * j], wi = w[2 * j + 1];
      g0r[e] += sr * wr - si * wi;
      g0i[e] += sr * wi + si * wr;
    }
  /* a_m = g0inv + the point-split shift by d_m */
  memcpy(a0r, g0r, sizeof(ld) * nn);
  memcpy(a0i, g0i, sizeof(ld) * nn);
  memcpy(a1r, g0r, sizeof(ld) * nn);
  memcpy(a1i, g0i, sizeof(ld) * nn);
  for (int j = 0; j < n; ++j) {
    const int corner = (j == 0);
    const int col = corner ? n - 1 : j - 1;
    if (n == 1) break;
    const size_t e = (size_t)j * n + col;
    ld sr, si;
    shift_entry(w[2 * j], w[2 * j + 1], d0, corner, &sr, &si);
    a0r[e] += sr;
    a0i[e] += si;
    shift_entry(w[2 * j], w[2 * j + 1], d1, corner, &sr, &si);
    a1r[e] += sr;
    a1i[e] += si;
  }
  if ((status = gj_inverse(n, a0r, a0i, perm)) != 0) goto done;
  if ((status = gj_inverse(n, a1r, a1i, perm)) != 0) goto done;
  /* g_imp = (1 - w1) inv(a0) + w1 inv(a1) */
  for (size_t e = 0; e < nn; ++e) {
    gir[e] = (1.0L - w1) * a0r[e] + (ld)w1 * a1r[e];
    gii[e] = (1.0L - w1) * a0i[e] + (ld)w1 * a1i[e];
  }
  if ((status = gj_inverse(n, gir, gii, perm)) != 0) goto done;
  /* Sigma_new W = g0inv - inv(g_imp); Sigma_new = that / W (column j) */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t e = (size_t)i * n + j;
      tr[e] = g0r[e] - gir[e];
      ti[e] = g0i[e] - gii[e];
      const ld wr = w[2 * j], wi = w[2 * j + 1];
      const ld den = wr * wr + wi * wi;
      out[2 * e] = (double)((tr[e] * wr + ti[e] * wi) / den);
      out[2 * e + 1] = (double)((ti[e] * wr - tr[e] * wi) / den);
    }
done:
  free(buf);
  free(perm);
  return status;
}
