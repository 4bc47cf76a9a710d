// Launchers of the lattice-step and impurity kernels (fk_lattice.hip).
#pragma once

#include "fk_internal.h"

namespace fk {

// Device tables shared by all points of one context.  Per point k: eps, ebar,
// rho.  Per contour point i >= 1: da/dg/dz = differences of the antiderivative
// tables alpha, gamma and of z between points i and i-1 (complex).  Corner
// differences ca/cg/cz = value at point 0 minus value at point N_c - 1.
// Upper-branch tables (i < N_t): cos(E t_i), sin(E t_i), t_i > 0.
struct PointTables {
  const double* eps;
  const double* ebar;
  const double* rho;
  const c64* da;
  const c64* dg;
  const c64* dz;
  c64 ca, cg, cz;
  double mu, beta;
  const double* cos_et;
  const double* sin_et;
  const int* t_pos;
};

hipError_t launch_sigma_weight(const c64* sigma, const c64* w, c64* sigt, int n,
                               hipStream_t st);
template <typename TO>
hipError_t launch_build(const c64* sigt, const PointTables& tab, int k0,
                        int nmat, cplx<TO>* xbuf, size_t mat_stride, int ld,
                        int n, hipStream_t st);
template <typename TI>
hipError_t launch_reduce(const cplx<TI>* xbuf, size_t mat_stride, int ld,
                         const int* piv, const int* rowcol, int istride,
                         const double* coef, int nmat, int n, c64* out,
                         int accumulate, hipStream_t st);
template <typename TI>
hipError_t launch_current(const cplx<TI>* xbuf, size_t mat_stride, int ld,
                          const int* piv, const int* rowcol, int istride,
                          const PointTables& tab, int k0, int nmat, int n_t,
                          int n, double* cur, hipStream_t st);
hipError_t launch_maxabs(const c64* a, const c64* b, size_t total,
                         unsigned long long* key, hipStream_t st);
// Nonequilibrium DOS rho(t_i, w) (dos[r * n_w + q], i = tix[r]) and equal-time
// moments mu_m(t_i) (mu[3 r + m]) of the local G on the contour; the time
// indices must satisfy 0 <= i < N_t (DOS) and 3 <= i <= N_t - 4 (moments).
hipError_t launch_wigner_dos(const c64* g, int n_t, int n, double dt, const int* tix,
                             int n_T, const double* w, int n_w, double* dos,
                             hipStream_t st);
hipError_t launch_moments(const c64* g, int n_t, int n, double dt, const int* tix,
                          int n_T, c64* mu, hipStream_t st);
hipError_t launch_equal_time(const c64* g, int n_t, int n, c64* less, c64* greater,
                             hipStream_t st);
hipError_t launch_right_weight(const c64* src, const c64* w, c64* dst, int ld,
                               int n, hipStream_t st);
hipError_t launch_add_right_weighted(c64* g0inv, const c64* sigma, const c64* w,
                                     int n, hipStream_t st);
hipError_t launch_shifted_pair(const c64* g0inv, double d0, double d1, c64* x0,
                               c64* x1, int ld, int n, hipStream_t st);
// slot += I + d S X (X natural, n x n; slot with leading dimension ld)
hipError_t launch_add_identity_shift(c64* slot, int ld, const c64* x, double d, int n,
                                     hipStream_t st);
// sigma_new = (-h S + gam S X S) W^-1 from X = (G0^-1 + d_c S)^-1 (natural layout)
hipError_t launch_sigma_fk(const c64* x, const c64* w, c64* sigma, int n, double h,
                           double gam, unsigned long long* key, hipStream_t st);

hipError_t launch_ttab(const PointTables& tab, int k0, int nmat, int n,
                       c64* tsub, c64* tcor, hipStream_t st);
template <typename TI>
hipError_t launch_unpermute(const cplx<TI>* x, size_t xstride, int ld,
                            const int* piv, const int* rowcol, int n, int nmat,
                            c64* out, hipStream_t st);
hipError_t launch_bgemm(c64* C, const c64* Cin, double beta, const c64* A,
                        size_t sA, const c64* B, int n, int nmat,
                        hipStream_t st);
hipError_t launch_residual(c64* P, const c64* X, const c64* tsub,
                           const c64* tcor, int n, int nmat,
                           unsigned long long* key, hipStream_t st);

}  // namespace fk
