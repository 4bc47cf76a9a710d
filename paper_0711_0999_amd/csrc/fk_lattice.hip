// Lattice-step kernels around the batched inversion (gfx950):
//   build      A_k = G0_k^-1 - W Sigma W, with the exact sparse G0_k^-1 of the
//              sampled noninteracting function (Sec. II, eq. g_contour_non_final2)
//   reduce     G_loc += sum_k rho_k G_k            (eq. g_loc), fixed order
//   current    j(t_i) += sum_k rho_k ebar_k(t_i) Re[i G_k[i, 2N_t - i]]   (eq. current_def)
//   norms      max |A - B| and non-finite detection
//   impurity   the elementwise pieces of the Falicov-Kimball update
//              (eqs. effective_medium, dynamical_mean_field, g_imp_solve)
// All of them are HBM-streaming kernels: consecutive threads touch consecutive
// complex elements of a row.
#include "fk_internal.h"
#include "fk_kernels.h"

namespace fk {

// ------------------------------------------------------------ Sigma_t ------
// sigt[i][j] = W_i sigma[i][j] W_j  (both contour integrals of eq. dyson)
__global__ void k_sigma_weight(const c64* __restrict__ sigma,
                               const c64* __restrict__ w, c64* __restrict__ sigt,
                               int n) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (e / n) * n);
    const c64 s = sigma[e], wi = w[i], wj = w[j];
    c64 t;
    t.re = wi.re * s.re - wi.im * s.im;
    t.im = wi.re * s.im + wi.im * s.re;
    c64 r;
    r.re = t.re * wj.re - t.im * wj.im;
    r.im = t.re * wj.im + t.im * wj.re;
    sigt[e] = r;
  }
}

// -------------------------------------------------------------- build ------
// Per point k: the subdiagonal of G0_k^-1 is -i exp(-i q_i) with
// q_i = eps da_i + ebar dg_i - mu dz_i (differences of the antiderivative
// tables between contour points i and i-1), the diagonal is i, and the corner
// (0, N-1) is i exp(-beta (eps - mu) - i q_c), q_c = eps (a_0 - a_{N-1}) +
// ebar (g_0 - g_{N-1}) - mu (z_0 - z_{N-1}).
__device__ inline c64 cexp_minus_i(c64 q, double extra_real) {
  // exp(-i q + extra_real) for complex q = a + i b: exp(b + extra) (cos a - i sin a)
  const double m = exp(q.im + extra_real);
  double s, c;
  sincos(q.re, &s, &c);
  c64 r;
  r.re = m * c;
  r.im = -m * s;
  return r;
}

// Subdiagonal entry T[i][i-1] (i >= 1) and corner T[0][n-1] of G0_k^-1.
__device__ inline c64 t_sub(const PointTables& tab, int k, int i) {
  const double eps = tab.eps[k], ebar = tab.ebar[k];
  const c64 da = tab.da[i], dg = tab.dg[i], dz = tab.dz[i];
  c64 q;
  q.re = eps * da.re + ebar * dg.re - tab.mu * dz.re;
  q.im = eps * da.im + ebar * dg.im - tab.mu * dz.im;
  const c64 ex = cexp_minus_i(q, 0.0);
  return c64{ex.im, -ex.re};  // -i * ex
}
__device__ inline c64 t_corner(const PointTables& tab, int k) {
  const double eps = tab.eps[k], ebar = tab.ebar[k];
  c64 q;
  q.re = eps * tab.ca.re + ebar * tab.cg.re - tab.mu * tab.cz.re;
  q.im = eps * tab.ca.im + ebar * tab.cg.im - tab.mu * tab.cz.im;
  const c64 ex = cexp_minus_i(q, -tab.beta * (eps - tab.mu));
  return c64{-ex.im, ex.re};  // +i * ex
}

// tsub[m][i] = T_k[i][i-1] (i >= 1), tcor[m] = T_k[0][n-1] for k = k0 + m
__global__ void k_ttab(const PointTables tab, int k0, int nmat, int n,
                       c64* __restrict__ tsub, c64* __restrict__ tcor) {
  const int m = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gridDim.x * blockDim.x) {
    tsub[(size_t)m * n + i] = (i >= 1) ? t_sub(tab, k0 + m, i) : c64{0.0, 0.0};
    if (i == 0) tcor[m] = t_corner(tab, k0 + m);
  }
}

hipError_t launch_ttab(const PointTables& tab, int k0, int nmat, int n,
                       c64* tsub, c64* tcor, hipStream_t st) {
  hipLaunchKernelGGL(k_ttab, dim3((n + 255) / 256, nmat), dim3(256), 0, st, tab,
                     k0, nmat, n, tsub, tcor);
  return hipGetLastError();
}

// One thread per column j of row i = blockIdx.y: the row of -Sigma~ is read
// once and written to the matrices m = blockIdx.z, blockIdx.z + gridDim.z, ...
// with i on the diagonal and the point's sub-diagonal / corner entry added.
template <typename TO>
__global__ void k_build(const c64* __restrict__ sigt,
                        const PointTables tab, int k0, int nmat,
                        cplx<TO>* __restrict__ xbuf, size_t mat_stride, int ld,
                        int n) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const c64 s = sigt[(size_t)i * n + j];
  c64 a;
  a.re = -s.re;
  a.im = -s.im;
  if (j == i) a.im += 1.0;
  const bool sub = j != i && (j == i - 1 || (i == 0 && j == n - 1));
  for (int m = blockIdx.z; m < nmat; m += gridDim.z) {
    c64 v = a;
    if (sub) {
      const c64 t = (j == i - 1) ? t_sub(tab, k0 + m, i) : t_corner(tab, k0 + m);
      v.re += t.re;
      v.im += t.im;
    }
    cplx<TO> o;
    o.re = (TO)v.re;
    o.im = (TO)v.im;
    xbuf[(size_t)m * mat_stride + (size_t)i * ld + j] = o;
  }
}

// ------------------------------------------------------------- reduce ------
// out[a][b] += sum_m coef[m] X_m[piv_m[a]][rowcol_m[b]]   (m in fixed order)
template <typename TI>
__global__ void k_reduce(const cplx<TI>* __restrict__ xbuf, size_t mat_stride,
                         int ld, const int* __restrict__ pivbuf,
                         const int* __restrict__ rowcolbuf, int istride,
                         const double* __restrict__ coef, int nmat, int n,
                         c64* __restrict__ out, int accumulate) {
  const int a = blockIdx.y;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n;
       b += gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int m = 0; m < nmat; ++m) {
      const int r = pivbuf[(size_t)m * istride + a];
      const int c = rowcolbuf[(size_t)m * istride + b];
      if (r < 0 || c < 0 || r >= n || c >= n) {  // incomplete inversion
        re = im = __builtin_nan("");
        continue;
      }
      const cplx<TI> v = xbuf[(size_t)m * mat_stride + (size_t)r * ld + c];
      const double w = coef[m];
      re += w * (double)v.re;
      im += w * (double)v.im;
    }
    c64 o = accumulate ? out[(size_t)a * n + b] : c64{0.0, 0.0};
    o.re += re;
    o.im += im;
    out[(size_t)a * n + b] = o;
  }
}

// j(t_i) += sum_m rho_m vel_m(i) Re[i G_m[i][2 n_t - i]],
// vel_m(i) = ebar cos(E t_i) + eps sin(E t_i) for t_i > 0, else ebar.
template <typename TI>
__global__ void k_current(const cplx<TI>* __restrict__ xbuf, size_t mat_stride,
                          int ld, const int* __restrict__ pivbuf,
                          const int* __restrict__ rowcolbuf, int istride,
                          const PointTables tab, int k0, int nmat, int n_t,
                          int n, double* __restrict__ cur) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_t) return;
  const int pcol = 2 * n_t - i;
  const double ct = tab.cos_et[i], st = tab.sin_et[i];
  const bool on = tab.t_pos[i] != 0;
  double acc = 0.0;
  for (int m = 0; m < nmat; ++m) {
    const int k = k0 + m;
    const int r = pivbuf[(size_t)m * istride + i];
    const int c = rowcolbuf[(size_t)m * istride + pcol];
    if (r < 0 || c < 0 || r >= n || c >= n) {
      acc = __builtin_nan("");
      continue;
    }
    const cplx<TI> v = xbuf[(size_t)m * mat_stride + (size_t)r * ld + c];
    const double vel = on ? tab.ebar[k] * ct + tab.eps[k] * st : tab.ebar[k];
    acc += tab.rho[k] * vel * (-(double)v.im);  // Re[i g] = -Im g
  }
  cur[i] += acc;
}

// Equal-time entries of G_loc: less[i] = G[i][2 N_t - i] (G^<(t_i, t_i)) and
// greater[i] = G[2 N_t - i][i] (G^>(t_i, t_i)), i < N_t.
__global__ void k_equal_time(const c64* __restrict__ g, int n_t, int n,
                             c64* __restrict__ less, c64* __restrict__ greater) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_t) return;
  const int p = 2 * n_t - i;
  less[i] = g[(size_t)i * n + p];
  greater[i] = g[(size_t)p * n + i];
}

hipError_t launch_equal_time(const c64* g, int n_t, int n, c64* less, c64* greater,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_equal_time, dim3((n_t + 127) / 128), dim3(128), 0, st, g, n_t,
                     n, less, greater);
  return hipGetLastError();
}

// ------------------------------------------------ spectral functions ------
// Retarded pair f_d = G^R(t_{i+d}, t_{i-d}) = G^> - G^< of the local G on the
// contour, with G^>(t_a, t_b) = G[p(a)][b], G^<(t_a, t_b) = G[a][p(b)] and
// p(k) = 2 N_t - k (Sec. II: the retarded function from the two real branches).
__device__ inline c64 retarded_pair(const c64* __restrict__ g, int n_t, int n,
                                    int i, int d) {
  const int a = i + d, b = i - d;
  const c64 gg = g[(size_t)(2 * n_t - a) * n + b];
  const c64 gl = g[(size_t)a * n + (2 * n_t - b)];
  c64 f;
  f.re = gg.re - gl.re;
  f.im = gg.im - gl.im;
  return f;
}

// Nonequilibrium DOS (Sec. II, eqs. gr_omega and dos_def) at the average times
// T = t_i, i = tix[r], and the frequencies w[q]: one thread per frequency and
// time (times strided over the grid's y dimension),
//   rho = -(h / pi) Im sum_{d=0}^{D} c_d e^{i w d h} f_d,
// h = 2 dt, D = min(i, N_t - 1 - i), trapezoid weights c_0 = c_D = 1/2 (c_0 =
// 1/2 alone when D = 0), 1 in between.
__global__ void k_wigner_dos(const c64* __restrict__ g, int n_t, int n, double h,
                             const int* __restrict__ tix, int n_T,
                             const double* __restrict__ w, int n_w,
                             double* __restrict__ dos) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_w) return;
  const double om = w[q];
  for (int r = blockIdx.y; r < n_T; r += gridDim.y) {
    const int i = tix[r];
    const int dmax = min(i, n_t - 1 - i);
    double acc = 0.0;
    for (int d = 0; d <= dmax; ++d) {
      const c64 f = retarded_pair(g, n_t, n, i, d);
      double sn, cs;
      sincos(om * (d * h), &sn, &cs);
      const double c = (d == 0 || d == dmax) ? 0.5 : 1.0;
      acc += c * (sn * f.re + cs * f.im);
    }
    dos[(size_t)r * n_w + q] = -h * acc / 3.14159265358979323846;
  }
}

// Equal-time moments (Sec. II, moments paragraph) at T = t_i, i = tix[r]
// (3 <= i <= N_t - 4): with f_d as above and h = 2 dt,
//   mu0 = i f_0,  mu1 = -(-3 f_0 + 4 f_1 - f_2) / (2 h),
//   mu2 = -i (2 f_0 - 5 f_1 + 4 f_2 - f_3) / h^2;
// mu[3 r + m] = mu_m.
__global__ void k_moments(const c64* __restrict__ g, int n_t, int n, double h,
                          const int* __restrict__ tix, int n_T, c64* __restrict__ mu) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_T) return;
  const int i = tix[r];
  const c64 f0 = retarded_pair(g, n_t, n, i, 0), f1 = retarded_pair(g, n_t, n, i, 1);
  const c64 f2 = retarded_pair(g, n_t, n, i, 2), f3 = retarded_pair(g, n_t, n, i, 3);
  c64 m0, m1, m2;
  m0.re = -f0.im;
  m0.im = f0.re;
  m1.re = -(-3.0 * f0.re + 4.0 * f1.re - f2.re) / (2.0 * h);
  m1.im = -(-3.0 * f0.im + 4.0 * f1.im - f2.im) / (2.0 * h);
  const double d2r = (2.0 * f0.re - 5.0 * f1.re + 4.0 * f2.re - f3.re) / (h * h);
  const double d2i = (2.0 * f0.im - 5.0 * f1.im + 4.0 * f2.im - f3.im) / (h * h);
  m2.re = d2i;     // -i (d2r + i d2i)
  m2.im = -d2r;
  mu[3 * r] = m0;
  mu[3 * r + 1] = m1;
  mu[3 * r + 2] = m2;
}

hipError_t launch_wigner_dos(const c64* g, int n_t, int n, double dt, const int* tix,
                             int n_T, const double* w, int n_w, double* dos,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_wigner_dos, dim3((n_w + 127) / 128, n_T < 4096 ? n_T : 4096),
                     dim3(128), 0, st, g, n_t, n, 2.0 * dt, tix, n_T, w, n_w, dos);
  return hipGetLastError();
}

hipError_t launch_moments(const c64* g, int n_t, int n, double dt, const int* tix,
                          int n_T, c64* mu, hipStream_t st) {
  hipLaunchKernelGGL(k_moments, dim3((n_T + 127) / 128), dim3(128), 0, st, g, n_t, n,
                     2.0 * dt, tix, n_T, mu);
  return hipGetLastError();
}

// -------------------------------------------------------------- norms ------
// bits of the max of |a - b| (or |a| when b == nullptr) as an unsigned 64-bit
// key: non-negative doubles order like their bit patterns, NaN above +Inf.
__global__ void k_maxabs(const c64* __restrict__ a, const c64* __restrict__ b,
                         size_t total, unsigned long long* __restrict__ key) {
  double m = 0.0;
  bool bad = false;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    c64 d = a[e];
    if (b) {
      d.re -= b[e].re;
      d.im -= b[e].im;
    }
    const double v = sqrt(d.re * d.re + d.im * d.im);
    if (!(v <= 1.79769313486231570815e308)) bad = true;
    else if (v > m) m = v;
  }
  unsigned long long k = bad ? 0x7ff8000000000000ULL
                             : (unsigned long long)__double_as_longlong(m);
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(k, off);
    k = o > k ? o : k;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(key, k);
}

// ----------------------------------------------------------- impurity ------
// dst[i][j] = src[i][j] * W_j  (right weighting), stored into an inversion slot
__global__ void k_right_weight(const c64* __restrict__ src,
                               const c64* __restrict__ w, c64* __restrict__ dst,
                               int ld, int n) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (e / n) * n);
    const c64 s = src[e], wj = w[j];
    c64 r;
    r.re = s.re * wj.re - s.im * wj.im;
    r.im = s.re * wj.im + s.im * wj.re;
    dst[(size_t)i * ld + j] = r;
  }
}

// g0inv += sigma * W (right-weighted Sigma added to the inverse already there)
__global__ void k_add_right_weighted(c64* __restrict__ g0inv,
                                     const c64* __restrict__ sigma,
                                     const c64* __restrict__ w, int n) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e - (e / n) * n);
    const c64 s = sigma[e], wj = w[j];
    c64 g = g0inv[e];
    g.re += s.re * wj.re - s.im * wj.im;
    g.im += s.re * wj.im + s.im * wj.re;
    g0inv[e] = g;
  }
}

// slot_m = g0inv + d_m S for m = 0, 1 (S[j][j-1] = 1, S[0][n-1] = -1);
// x1 may be null (one slot)
__global__ void k_shifted_pair(const c64* __restrict__ g0inv, double d0,
                               double d1, c64* __restrict__ x0,
                               c64* __restrict__ x1, int ld, int n) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (e / n) * n);
    double s = 0.0;
    if (j == i - 1) s = 1.0;
    if (i == 0 && j == n - 1) s = (n == 1) ? 0.0 : -1.0;
    c64 a = g0inv[e], b = g0inv[e];
    a.re += d0 * s;
    b.re += d1 * s;
    x0[(size_t)i * ld + j] = a;
    if (x1) x1[(size_t)i * ld + j] = b;
  }
}

// slot[i][j] += delta_ij + d (S X)[i][j], (S X)[i][j] = s_i X[i - 1 mod n][j]
// (s_0 = -1, else 1): the sparse part of I + (Sigma W + d S) X, X natural.
__global__ void k_add_identity_shift(c64* __restrict__ slot, int ld,
                                     const c64* __restrict__ x, double d, int n) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int k = (i == 0) ? n - 1 : i - 1;
  const double sg = (i == 0) ? -d : d;
  const c64 v = x[(size_t)k * n + j];
  c64 a = slot[(size_t)i * ld + j];
  a.re += sg * v.re + (j == i ? 1.0 : 0.0);
  a.im += sg * v.im;
  slot[(size_t)i * ld + j] = a;
}

hipError_t launch_add_identity_shift(c64* slot, int ld, const c64* x, double d, int n,
                                     hipStream_t st) {
  hipLaunchKernelGGL(k_add_identity_shift, dim3((n + 255) / 256, n), dim3(256), 0, st,
                     slot, ld, x, d, n);
  return hipGetLastError();
}

// Falicov-Kimball self-energy from the one inverse X = C^-1, C = G0^-1 + d_c S:
// sigma_new W = -h S + gam S X S (the two-inversion form of the paper's
// G0^-1 - G_imp^-1), sigma_new[i][j] = that / W_j, and the running max of
// |sigma_new - sigma_old| via the key of k_maxabs.  (S X S)[i][j] =
// s_i t_j X[i - 1 mod n][j + 1 mod n] with s_0 = t_{n-1} = -1, else 1.
__global__ void k_sigma_fk(const c64* __restrict__ x, const c64* __restrict__ w,
                           c64* __restrict__ sigma, int n, double h, double gam,
                           unsigned long long* __restrict__ key) {
  const size_t total = (size_t)n * n;
  double mx = 0.0;
  bool bad = false;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (e / n) * n);
    const int k = (i == 0) ? n - 1 : i - 1, l = (j == n - 1) ? 0 : j + 1;
    const double sg = gam * ((i == 0) ? -1.0 : 1.0) * ((j == n - 1) ? -1.0 : 1.0);
    const c64 v = x[(size_t)k * n + l];
    c64 d{sg * v.re, sg * v.im};
    if (j == i - 1) d.re -= h;
    else if (i == 0 && j == n - 1) d.re += h;
    const c64 wj = w[j];
    const double den = wj.re * wj.re + wj.im * wj.im;
    c64 sv;
    sv.re = (d.re * wj.re + d.im * wj.im) / den;
    sv.im = (d.im * wj.re - d.re * wj.im) / den;
    const c64 old = sigma[e];
    const double dr = sv.re - old.re, di = sv.im - old.im;
    const double a = sqrt(dr * dr + di * di);
    if (!(a <= 1.79769313486231570815e308)) bad = true;
    else if (a > mx) mx = a;
    sigma[e] = sv;
  }
  unsigned long long kk = bad ? 0x7ff8000000000000ULL
                              : (unsigned long long)__double_as_longlong(mx);
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(kk, off);
    kk = o > kk ? o : kk;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(key, kk);
}

// ------------------------------------------------------------ launchers ----
static inline int grid_for(size_t total, int block) {
  size_t g = (total + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_sigma_weight(const c64* sigma, const c64* w, c64* sigt, int n,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_weight, dim3(grid_for((size_t)n * n, 256)),
                     dim3(256), 0, st, sigma, w, sigt, n);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_build(const c64* sigt, const PointTables& tab, int k0,
                        int nmat, cplx<TO>* xbuf, size_t mat_stride, int ld,
                        int n, hipStream_t st) {
  if (nmat <= 0) return hipSuccess;
  const int gz = nmat < 16 ? nmat : 16;
  hipLaunchKernelGGL(k_build<TO>, dim3((n + 255) / 256, n, gz), dim3(256), 0, st, sigt,
                     tab, k0, nmat, xbuf, mat_stride, ld, n);
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_reduce(const cplx<TI>* xbuf, size_t mat_stride, int ld,
                         const int* piv, const int* rowcol, int istride,
                         const double* coef, int nmat, int n, c64* out,
                         int accumulate, hipStream_t st) {
  const int bx = (n + 255) / 256;
  hipLaunchKernelGGL(k_reduce<TI>, dim3(bx, n), dim3(256), 0, st, xbuf,
                     mat_stride, ld, piv, rowcol, istride, coef, nmat, n, out,
                     accumulate);
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_current(const cplx<TI>* xbuf, size_t mat_stride, int ld,
                          const int* piv, const int* rowcol, int istride,
                          const PointTables& tab, int k0, int nmat, int n_t,
                          int n, double* cur, hipStream_t st) {
  hipLaunchKernelGGL(k_current<TI>, dim3((n_t + 127) / 128), dim3(128), 0, st,
                     xbuf, mat_stride, ld, piv, rowcol, istride, tab, k0, nmat,
                     n_t, n, cur);
  return hipGetLastError();
}

hipError_t launch_maxabs(const c64* a, const c64* b, size_t total,
                         unsigned long long* key, hipStream_t st) {
  hipLaunchKernelGGL(k_maxabs, dim3(grid_for(total, 256) > 2048 ? 2048 : grid_for(total, 256)),
                     dim3(256), 0, st, a, b, total, key);
  return hipGetLastError();
}

hipError_t launch_right_weight(const c64* src, const c64* w, c64* dst, int ld,
                               int n, hipStream_t st) {
  hipLaunchKernelGGL(k_right_weight, dim3(grid_for((size_t)n * n, 256)),
                     dim3(256), 0, st, src, w, dst, ld, n);
  return hipGetLastError();
}

hipError_t launch_add_right_weighted(c64* g0inv, const c64* sigma, const c64* w,
                                     int n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_right_weighted, dim3(grid_for((size_t)n * n, 256)),
                     dim3(256), 0, st, g0inv, sigma, w, n);
  return hipGetLastError();
}

hipError_t launch_shifted_pair(const c64* g0inv, double d0, double d1, c64* x0,
                               c64* x1, int ld, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_shifted_pair, dim3(grid_for((size_t)n * n, 256)),
                     dim3(256), 0, st, g0inv, d0, d1, x0, x1, ld, n);
  return hipGetLastError();
}

hipError_t launch_sigma_fk(const c64* x, const c64* w, c64* sigma, int n, double h,
                           double gam, unsigned long long* key, hipStream_t st) {
  const int g = grid_for((size_t)n * n, 256);
  hipLaunchKernelGGL(k_sigma_fk, dim3(g > 2048 ? 2048 : g), dim3(256), 0, st, x, w,
                     sigma, n, h, gam, key);
  return hipGetLastError();
}

template hipError_t launch_build<double>(const c64*, const PointTables&, int,
                                         int, c64*, size_t, int, int,
                                         hipStream_t);
template hipError_t launch_build<float>(const c64*, const PointTables&, int,
                                        int, c32*, size_t, int, int,
                                        hipStream_t);
template hipError_t launch_reduce<double>(const c64*, size_t, int, const int*,
                                          const int*, int, const double*, int,
                                          int, c64*, int, hipStream_t);
template hipError_t launch_reduce<float>(const c32*, size_t, int, const int*,
                                         const int*, int, const double*, int,
                                         int, c64*, int, hipStream_t);
template hipError_t launch_current<double>(const c64*, size_t, int, const int*,
                                           const int*, int, const PointTables&,
                                           int, int, int, int, double*,
                                           hipStream_t);
template hipError_t launch_current<float>(const c32*, size_t, int, const int*,
                                          const int*, int, const PointTables&,
                                          int, int, int, int, double*,
                                          hipStream_t);

}  // namespace fk
