// C ABI of the fkdmft library: contour, quadrature, context, the lattice step
// (batched Gauss-Jordan inversion of every point matrix), the Falicov-Kimball
// impurity update and the self-consistency loop.  See include/fkdmft.h.
#include "../../include/fkdmft.h"
#include "fk_internal.h"
#include "fk_kernels.h"
#include "fk_ctx.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace fk;

// ============================================================ static scratch
// Staging memory of fk_wigner_dos_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel or a copy (on the host it only stands in for the symbol):
// its device address is looked up once per device with hipGetSymbolAddress
// while that device is current (fk_create) and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Look up this device's scratch address once (dev must be current).
hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
  }
  return g_scratch_err[dev];
}

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_done[dev] ? g_scratch_ptr[dev] : nullptr;
}
}  // namespace

// ===================================================================== host ==
namespace {

// Sturm-sequence count of eigenvalues below x of the symmetric tridiagonal
// Jacobi matrix of the normalized Hermite weight (zero diagonal, off-diagonal
// b_k = sqrt(k/2), k = 1..n-1).
int sturm_count(int n, double x) {
  int cnt = 0;
  double q = -x;
  if (q < 0) ++cnt;
  for (int k = 1; k < n; ++k) {
    const double b2 = 0.5 * k;
    if (q == 0.0) q = 1e-300;
    q = -x - b2 / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}


bool integral_ratio(double span, double step, int* out) {
  if (!(step > 0.0) || !(span > 0.0)) return false;
  const double r = span / step;
  const double m = floor(r + 0.5);
  if (m < 1.0 || m > 1e7) return false;
  if (fabs(r - m) > 1e-9 * std::max(1.0, fabs(r))) return false;
  *out = (int)m;
  return true;
}

fk_status build_contour(const fk_contour* c, ContourInfo* ci) {
  if (!c) return FK_EINVAL;
  if (!(c->t_max > c->t_min)) return FK_EINVAL;
  int n_t, n_tau;
  if (!integral_ratio(c->t_max - c->t_min, c->dt, &n_t)) return FK_EINVAL;
  if (!integral_ratio(c->beta, c->dtau, &n_tau)) return FK_EINVAL;
  ci->n_t = n_t;
  ci->n_tau = n_tau;
  ci->n_c = 2 * n_t + n_tau;
  const int n = ci->n_c;
  ci->zr.assign(n, 0.0);
  ci->zi.assign(n, 0.0);
  ci->wr.assign(n, 0.0);
  ci->wi.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    if (j < n_t) {                    // upper real branch, leftpoint weight +dt
      ci->zr[j] = c->t_min + j * c->dt;
      ci->wr[j] = c->dt;
    } else if (j < 2 * n_t) {         // lower real branch, weight -dt
      ci->zr[j] = c->t_max - (j - n_t) * c->dt;
      ci->wr[j] = -c->dt;
    } else {                          // imaginary branch, weight -i dtau
      ci->zr[j] = c->t_min;
      ci->zi[j] = -c->dtau * (j - 2 * n_t);
      ci->wi[j] = -c->dtau;
    }
  }
  return FK_OK;
}

}  // namespace

extern "C" fk_status fk_gauss_hermite(int n, double* x, double* w) {
  if (n < 1 || n > 150 || !x || !w) return FK_EINVAL;
  std::vector<double> xs(n), ws(n);
  const double bound = 2.0 * sqrt(0.5 * (n > 1 ? n - 1 : 1)) + 1.0;
  for (int k = 0; k < n; ++k) {
    // k-th eigenvalue (ascending): count(x) <= k below it, > k above it
    double lo = -bound, hi = bound;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(n, mid) > k) hi = mid;
      else lo = mid;
    }
    xs[k] = 0.5 * (lo + hi);
  }
  for (int k = 0; k < n; ++k) {
    // Christoffel weight 1 / sum_j p_j(x)^2 with orthonormal p_j
    const double t = xs[k];
    double pm = 0.0, p = 1.0, s = 1.0;
    for (int j = 1; j < n; ++j) {
      const double bj = sqrt(0.5 * j);
      const double bjm = sqrt(0.5 * (j - 1));
      const double pn = (t * p - bjm * pm) / bj;
      pm = p;
      p = pn;
      s += p * p;
    }
    ws[k] = 1.0 / s;
  }
  for (int k = 0; k < n; ++k) {   // the weight is even: symmetrize
    x[k] = 0.5 * (xs[k] - xs[n - 1 - k]);
    w[k] = 0.5 * (ws[k] + ws[n - 1 - k]);
  }
  return FK_OK;
}

extern "C" fk_status fk_contour_build(const fk_contour* c, int* dims, double* z,
                                      double* W) {
  if (!dims) return FK_EINVAL;
  ContourInfo ci;
  fk_status s = build_contour(c, &ci);
  if (s != FK_OK) return s;
  dims[0] = ci.n_t;
  dims[1] = ci.n_tau;
  dims[2] = ci.n_c;
  for (int j = 0; j < ci.n_c; ++j) {
    if (z) {
      z[2 * j] = ci.zr[j];
      z[2 * j + 1] = ci.zi[j];
    }
    if (W) {
      W[2 * j] = ci.wr[j];
      W[2 * j + 1] = ci.wi[j];
    }
  }
  return FK_OK;
}

extern "C" fk_status fk_update_plan(int n, int S, int q, int* out6) {
  if (n < 1 || n > kMaxN || S < 0 || q < 0 || q >= kPhases || !out6) return FK_EINVAL;
  const PhasePlan pl = phase_plan(n, S, q);
  out6[0] = pl.jb;
  out6[1] = pl.kw;
  out6[2] = pl.b0;
  out6[3] = pl.lo;
  out6[4] = pl.hi;
  out6[5] = block_brow(n, S);
  return FK_OK;
}

extern "C" fk_status fk_extrapolate_to_zero(int n_steps, const double* steps, int len,
                                            const double* values, double* out) {
  if (n_steps < 1 || len < 0 || !steps || (len > 0 && (!values || !out)))
    return FK_EINVAL;
  for (int k = 0; k < n_steps; ++k) {
    if (!std::isfinite(steps[k]) || !(steps[k] > 0.0)) return FK_EINVAL;
    for (int m = 0; m < k; ++m)
      if (steps[m] == steps[k]) return FK_EINVAL;
  }
  // w_k = prod_{m != k} h_m / (h_m - h_k): the value at h = 0 of the
  // interpolating polynomial through (h_k, f_k) is sum_k w_k f_k
  std::vector<double> w(n_steps, 1.0);
  for (int k = 0; k < n_steps; ++k)
    for (int m = 0; m < n_steps; ++m)
      if (m != k) w[k] *= steps[m] / (steps[m] - steps[k]);
  for (int e = 0; e < len; ++e) {
    double acc = 0.0;
    for (int k = 0; k < n_steps; ++k) acc += w[k] * values[(size_t)k * len + e];
    out[e] = acc;
  }
  return FK_OK;
}

extern "C" const char* fk_status_string(fk_status s) {
  switch (s) {
    case FK_OK: return "FK_OK";
    case FK_EINVAL: return "FK_EINVAL";
    case FK_ENOMEM: return "FK_ENOMEM";
    case FK_EDEVICE: return "FK_EDEVICE";
    case FK_ESINGULAR: return "FK_ESINGULAR";
    case FK_ENONFINITE: return "FK_ENONFINITE";
    case FK_ENOTCONV: return "FK_ENOTCONV";
    case FK_ESTATE: return "FK_ESTATE";
    default: return "FK_UNKNOWN";
  }
}



namespace {

fk_status set_err(fk_ctx* c, fk_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIPCHK(ctx, expr)                                                    \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return set_err((ctx), e_ == hipErrorOutOfMemory ? FK_ENOMEM : FK_EDEVICE, \
                     "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                     __LINE__);                                              \
  } while (0)

template <typename T> int batch_cap_for(fk_ctx* c) {
  const size_t per = sizeof(cplx<T>) * ((size_t)c->ci.n_c + kBRows) * c->ci.n_c +
                     2 * sizeof(int) * (size_t)c->ci.n_c;
  size_t cap = c->batch_bytes / per;
  if (c->want_batch > 0) cap = (size_t)c->want_batch;
  if (cap < 1) cap = 1;
  if (cap > (size_t)c->npts) cap = (size_t)c->npts;
  // equalize the batches so the last one is not a small tail
  const size_t nb = (c->npts + cap - 1) / cap;
  cap = (c->npts + nb - 1) / nb;
  return (int)cap;
}

template <typename T> Batch<T>& lattice_batch(fk_ctx* c);
template <> Batch<double>& lattice_batch<double>(fk_ctx* c) { return c->b64; }
template <> Batch<float>& lattice_batch<float>(fk_ctx* c) { return c->b32; }

template <typename T> fk_status ensure_batch(fk_ctx* c) {
  Batch<T>& b = lattice_batch<T>(c);
  const int cap = batch_cap_for<T>(c);
  if (b.x && b.cap == cap && b.variant == c->variant) return FK_OK;
  HIPCHK(c, batch_alloc(b, cap, c->ci.n_c, c->variant));
  return FK_OK;
}

fk_status check_status(fk_ctx* c, const int* d_status, int nmat, int k0,
                       const char* what) {
  std::vector<int> s(nmat);
  HIPCHK(c, hipMemcpyAsync(s.data(), d_status, sizeof(int) * nmat,
                           hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int m = 0; m < nmat; ++m) {
    if (s[m] > 0)
      return set_err(c, FK_ESINGULAR, "%s: zero pivot at column %d of matrix %d",
                     what, s[m] - 1, k0 + m);
    if (s[m] < 0)
      return set_err(c, FK_ENONFINITE,
                     "%s: non-finite pivot at column %d of matrix %d", what,
                     -s[m] - 1, k0 + m);
  }
  return FK_OK;
}

double read_key(fk_ctx* c, fk_status* st) {
  unsigned long long k = 0;
  hipError_t e = hipMemcpyAsync(&k, c->d_key, sizeof k, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) {
    *st = set_err(c, FK_EDEVICE, "read norm: %s", hipGetErrorString(e));
    return 0.0;
  }
  *st = FK_OK;
  double v;
  memcpy(&v, &k, sizeof v);
  return v;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

// Lattice step in precision T (T = double: FP64 path).
// The batch left by an earlier step and G_loc are stale from here on: both are
// marked invalid before any device work and valid again only on success.
void invalidate_results(fk_ctx* c) {
  c->last_prec = -1;
  c->have_gloc = false;
}

template <typename T> fk_status lattice_step(fk_ctx* c, double* ir_out) {
  invalidate_results(c);
  fk_status s = ensure_batch<T>(c);
  if (s != FK_OK) return s;
  Batch<T>& b = lattice_batch<T>(c);
  const int n = c->ci.n_c;
  for (double& t : c->times) t = 0.0;
  int launches = 0;
  HIPCHK(c, launch_sigma_weight(c->d_sigma, c->d_w, c->d_sigt, n, c->st));
  HIPCHK(c, fill_f64(c->d_cur, 0.0, (size_t)c->ci.n_t, c->st));
  for (int k0 = 0; k0 < c->npts; k0 += b.cap) {
    const int nmat = std::min(b.cap, c->npts - k0);
    HIPCHK(c, hipEventRecord(c->ev[0], c->st));
    HIPCHK(c, launch_build<T>(c->d_sigt, c->tab, k0, nmat, b.x, b.stride, b.ld,
                              n, c->st));
    HIPCHK(c, hipEventRecord(c->ev[1], c->st));
    Aux ax = c->aux;
    ax.clk = c->clk.on ? &c->clk : nullptr;
    HIPCHK(c, batch_invert<T>(b, nmat, c->st, ax, &launches, &c->ev[6]));
    HIPCHK(c, hipEventRecord(c->ev[2], c->st));
    HIPCHK(c, launch_reduce<T>(b.x, b.stride, b.ld, b.piv, b.rowcol, n,
                               c->d_rho + k0, nmat, n, c->d_gloc, k0 > 0 ? 1 : 0,
                               c->st));
    HIPCHK(c, launch_current<T>(b.x, b.stride, b.ld, b.piv, b.rowcol, n, c->tab,
                                k0, nmat, c->ci.n_t, n, c->d_cur, c->st));
    HIPCHK(c, hipEventRecord(c->ev[3], c->st));
    s = check_status(c, b.status, nmat, k0, "lattice inversion");
    if (s != FK_OK) return s;
    if (c->clk.on) clock_collect(c->clk);
    c->times[0] += elapsed(c->ev[0], c->ev[1]);
    c->times[1] += elapsed(c->ev[1], c->ev[2]);
    c->times[3] += elapsed(c->ev[2], c->ev[3]);
    c->times[6] += elapsed(c->ev[6], c->ev[7]);
  }
  c->times[5] = launches;
  // non-finite check of G_loc
  HIPCHK(c, fill_u64(c->d_key, 0ULL, 1, c->st));
  HIPCHK(c, launch_maxabs(c->d_gloc, nullptr, (size_t)n * n, c->d_key, c->st));
  double mx = read_key(c, &s);
  if (s != FK_OK) return s;
  if (!(mx <= std::numeric_limits<double>::max()))
    return set_err(c, FK_ENONFINITE, "G_loc has non-finite entries");
  if (ir_out) *ir_out = 0.0;
  c->last_nmat = std::min(b.cap, c->npts - (c->npts - 1) / b.cap * b.cap);
  c->last_k0 = c->npts - c->last_nmat;
  c->last_prec = sizeof(T) == sizeof(double) ? 0 : 1;
  c->have_gloc = true;
  return FK_OK;
}

// Mixed lattice step: complex64 build and inversion, then ir_steps FP64
// refinement steps X <- X + X (I - A X), FP64 reduction.
fk_status lattice_step_mixed(fk_ctx* c, double* ir_out) {
  invalidate_results(c);
  const int n = c->ci.n_c, ir = c->ir_steps;
  const size_t nn = (size_t)n * n;
  // batch size: complex64 matrix + side buffer, plus three FP64 matrices when
  // refining
  const size_t per = sizeof(c32) * (nn + (size_t)kBRows * n) + 2 * sizeof(int) * n +
                     (ir > 0 ? 3 * sizeof(c64) * nn + sizeof(c64) * (n + 1) : 0);
  size_t cap = c->batch_bytes / per;
  if (c->want_batch > 0) cap = (size_t)c->want_batch;
  cap = std::max<size_t>(1, std::min<size_t>(cap, c->npts));
  const size_t nb = (c->npts + cap - 1) / cap;
  cap = (c->npts + nb - 1) / nb;
  Batch<float>& b = c->b32;
  if (!b.x || b.cap != (int)cap || b.variant != c->variant)
    HIPCHK(c, batch_alloc(b, (int)cap, n, c->variant));
  if (ir > 0 && c->ir_cap != (int)cap) {
    c->ir_cap = 0;   // counts as allocated only once every buffer is
    c64** bufs[] = {&c->ir_x, &c->ir_p, &c->ir_y};
    for (c64** q : bufs) {
      if (*q) (void)hipFree(*q);
      *q = nullptr;
      HIPCHK(c, hipMalloc(q, sizeof(c64) * nn * cap));
    }
    if (c->ir_tsub) (void)hipFree(c->ir_tsub);
    if (c->ir_tcor) (void)hipFree(c->ir_tcor);
    c->ir_tsub = c->ir_tcor = nullptr;
    HIPCHK(c, hipMalloc(&c->ir_tsub, sizeof(c64) * (size_t)n * cap));
    HIPCHK(c, hipMalloc(&c->ir_tcor, sizeof(c64) * cap));
    c->ir_cap = (int)cap;
  }
  for (double& t : c->times) t = 0.0;
  int launches = 0;
  double resid = 0.0;
  fk_status s;
  HIPCHK(c, launch_sigma_weight(c->d_sigma, c->d_w, c->d_sigt, n, c->st));
  HIPCHK(c, fill_f64(c->d_cur, 0.0, (size_t)c->ci.n_t, c->st));
  for (int k0 = 0; k0 < c->npts; k0 += b.cap) {
    const int nmat = std::min(b.cap, c->npts - k0);
    HIPCHK(c, hipEventRecord(c->ev[0], c->st));
    HIPCHK(c, launch_build<float>(c->d_sigt, c->tab, k0, nmat, b.x, b.stride, b.ld,
                                  n, c->st));
    HIPCHK(c, hipEventRecord(c->ev[1], c->st));
    Aux ax = c->aux;
    ax.clk = c->clk.on ? &c->clk : nullptr;
    HIPCHK(c, batch_invert<float>(b, nmat, c->st, ax, &launches, &c->ev[6]));
    HIPCHK(c, hipEventRecord(c->ev[2], c->st));
    if (ir == 0) {
      HIPCHK(c, hipEventRecord(c->ev[3], c->st));
      HIPCHK(c, launch_reduce<float>(b.x, b.stride, b.ld, b.piv, b.rowcol, n,
                                     c->d_rho + k0, nmat, n, c->d_gloc,
                                     k0 > 0 ? 1 : 0, c->st));
      HIPCHK(c, launch_current<float>(b.x, b.stride, b.ld, b.piv, b.rowcol, n,
                                      c->tab, k0, nmat, c->ci.n_t, n, c->d_cur,
                                      c->st));
    } else {
      HIPCHK(c, launch_ttab(c->tab, k0, nmat, n, c->ir_tsub, c->ir_tcor, c->st));
      HIPCHK(c, launch_unpermute<float>(b.x, b.stride, b.ld, b.piv, b.rowcol, n,
                                        nmat, c->ir_x, c->st));
      c64* X = c->ir_x;
      c64* Y = c->ir_y;
      for (int it = 0; it < ir; ++it) {
        HIPCHK(c, fill_u64(c->d_key, 0ULL, 1, c->st));
        HIPCHK(c, launch_bgemm(c->ir_p, nullptr, 0.0, c->d_sigt, 0, X, n, nmat,
                               c->st));
        HIPCHK(c, launch_residual(c->ir_p, X, c->ir_tsub, c->ir_tcor, n, nmat,
                                  c->d_key, c->st));
        HIPCHK(c, launch_bgemm(Y, X, 1.0, X, nn, c->ir_p, n, nmat, c->st));
        std::swap(X, Y);
        const double r = read_key(c, &s);
        if (s != FK_OK) return s;
        // the last step's residual R = I - A X is that of the iterate entering
        // it; the returned X + X R has the residual R^2 exactly (Newton), whose
        // entries are at most N_c max|R|^2: that bound is reported
        if (it == ir - 1) resid = std::max(resid, (double)n * r * r);
      }
      HIPCHK(c, hipEventRecord(c->ev[3], c->st));
      HIPCHK(c, launch_reduce<double>(X, nn, n, c->d_iota, c->d_iota, 0,
                                      c->d_rho + k0, nmat, n, c->d_gloc,
                                      k0 > 0 ? 1 : 0, c->st));
      HIPCHK(c, launch_current<double>(X, nn, n, c->d_iota, c->d_iota, 0, c->tab,
                                       k0, nmat, c->ci.n_t, n, c->d_cur, c->st));
    }
    HIPCHK(c, hipEventRecord(c->ev[4], c->st));
    s = check_status(c, b.status, nmat, k0, "complex64 inversion");
    if (s != FK_OK) return s;
    if (c->clk.on) clock_collect(c->clk);
    c->times[0] += elapsed(c->ev[0], c->ev[1]);
    c->times[1] += elapsed(c->ev[1], c->ev[2]);
    c->times[2] += elapsed(c->ev[2], c->ev[3]);
    c->times[3] += elapsed(c->ev[3], c->ev[4]);
    c->times[6] += elapsed(c->ev[6], c->ev[7]);
  }
  c->times[5] = launches;
  HIPCHK(c, fill_u64(c->d_key, 0ULL, 1, c->st));
  HIPCHK(c, launch_maxabs(c->d_gloc, nullptr, nn, c->d_key, c->st));
  const double mx = read_key(c, &s);
  if (s != FK_OK) return s;
  if (!(mx <= std::numeric_limits<double>::max()))
    return set_err(c, FK_ENONFINITE, "G_loc has non-finite entries");
  if (ir_out) *ir_out = resid;
  c->have_gloc = true;
  return FK_OK;
}

fk_status impurity(fk_ctx* c, double* dsig) {
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "impurity update before a lattice step");
  const int n = c->ci.n_c;
  Batch<double>& b = c->imp;
  if (!b.x) HIPCHK(c, batch_alloc(b, 1, n));
  int launches = 0;
  fk_status s;
  HIPCHK(c, hipEventRecord(c->ev[4], c->st));
  // G0^-1 = (G_loc W)^-1 + Sigma W.  G_imp = (1 - w1) A0^-1 + w1 A1^-1 with
  // A_m = G0^-1 + d_m S has the inverse A1 C^-1 A0, C = (1 - w1) A1 + w1 A0 =
  // G0^-1 + d_c S, so that
  //   Sigma_new W = G0^-1 - G_imp^-1 = -h S + w1 (1 - w1) (d0 - d1)^2 S C^-1 S,
  // h = (1 - w1) d0 + w1 d1; and with X = G_loc W, Y = Sigma W + d_c S,
  //   C^-1 = (X^-1 + Y)^-1 = X (I + Y X)^-1:
  // one inversion and two products instead of the paper's four inversions.
  double d0, d1;
  if (c->m.convention == 0) {
    d0 = 0.5 * c->m.U;
    d1 = -0.5 * c->m.U;
  } else {
    d0 = 0.0;
    d1 = -c->m.U;
  }
  const double w1 = c->m.w1;
  const double dc = (1.0 - w1) * d1 + w1 * d0, h = (1.0 - w1) * d0 + w1 * d1;
  const double gam = w1 * (1.0 - w1) * (d0 - d1) * (d0 - d1);
  c64* X = c->d_g0inv;   // impurity scratch
  HIPCHK(c, launch_right_weight(c->d_gloc, c->d_w, X, n, n, c->st));
  HIPCHK(c, launch_right_weight(c->d_sigma, c->d_w, c->d_tmp, n, n, c->st));
  HIPCHK(c, launch_bgemm(b.x, nullptr, 0.0, c->d_tmp, 0, X, n, 1, c->st));
  HIPCHK(c, launch_add_identity_shift(b.x, b.ld, X, dc, n, c->st));
  HIPCHK(c, batch_invert<double>(b, 1, c->st, c->aux, &launches));
  if ((s = check_status(c, b.status, 1, 0, "inverse of I + (Sigma W + d S) G_loc W")) !=
      FK_OK)
    return s;
  HIPCHK(c, launch_reduce<double>(b.x, b.stride, b.ld, b.piv, b.rowcol, n,
                                  c->d_coef, 1, n, c->d_tmp, 0, c->st));
  HIPCHK(c, launch_bgemm(b.x, nullptr, 0.0, X, 0, c->d_tmp, n, 1, c->st));
  HIPCHK(c, fill_u64(c->d_key, 0ULL, 1, c->st));
  HIPCHK(c, launch_sigma_fk(b.x, c->d_w, c->d_sigma, n, h, gam, c->d_key, c->st));
  HIPCHK(c, hipEventRecord(c->ev[5], c->st));
  double mx = read_key(c, &s);
  if (s != FK_OK) return s;
  c->times[4] = elapsed(c->ev[4], c->ev[5]);
  if (!(mx <= std::numeric_limits<double>::max()))
    return set_err(c, FK_ENONFINITE, "Sigma has non-finite entries");
  if (dsig) *dsig = mx;
  return FK_OK;
}

fk_status copy_matrix_in(fk_ctx* c, c64* dst, const double* src, int on_device) {
  if (!src) return set_err(c, FK_EINVAL, "NULL matrix pointer");
  const size_t bytes = sizeof(c64) * (size_t)c->ci.n_c * c->ci.n_c;
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

fk_status copy_matrix_out(fk_ctx* c, double* dst, const c64* src, int on_device) {
  if (!dst) return set_err(c, FK_EINVAL, "NULL matrix pointer");
  const size_t bytes = sizeof(c64) * (size_t)c->ci.n_c * c->ci.n_c;
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

void free_ctx(fk_ctx* c) {
  c64* cs[] = {c->d_w, c->d_sigma, c->d_sigt, c->d_gloc, c->d_gprev,
               c->d_g0inv, c->d_tmp, c->d_da, c->d_dg, c->d_dz};
  for (c64* p : cs)
    if (p) (void)hipFree(p);
  double* ds[] = {c->d_cur, c->d_eps, c->d_ebar, c->d_rho, c->d_cos, c->d_sin,
                  c->d_coef};
  for (double* p : ds)
    if (p) (void)hipFree(p);
  if (c->d_tpos) (void)hipFree(c->d_tpos);
  c64* irs[] = {c->ir_x, c->ir_p, c->ir_y, c->ir_tsub, c->ir_tcor};
  for (c64* p : irs)
    if (p) (void)hipFree(p);
  if (c->d_iota) (void)hipFree(c->d_iota);
  if (c->d_key) (void)hipFree(c->d_key);
  batch_free(c->b64);
  batch_free(c->b32);
  batch_free(c->imp);
  for (hipEvent_t& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->clk.ev)
    if (e) (void)hipEventDestroy(e);
  if (c->aux.evN) (void)hipEventDestroy(c->aux.evN);
  if (c->aux.evP) (void)hipEventDestroy(c->aux.evP);
  if (c->aux.st2) (void)hipStreamDestroy(c->aux.st2);
  if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
}

template <typename P> hipError_t upload(P** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

}  // namespace

// ================================================================== C ABI ==
extern "C" fk_status fk_create(const fk_contour* cont, const fk_model* mod,
                               void* hip_stream, fk_ctx** out) {
  if (!cont || !mod || !out) return FK_EINVAL;
  *out = nullptr;
  ContourInfo ci;
  if (build_contour(cont, &ci) != FK_OK) return FK_EINVAL;
  if (mod->n_eps < 1 || mod->n_eps > 150 || mod->n_ebar < 1 || mod->n_ebar > 150)
    return FK_EINVAL;
  if (mod->gh_average != 0 && mod->gh_average != 1) return FK_EINVAL;
  if (mod->gh_average && (mod->n_eps > 149 || mod->n_ebar > 149)) return FK_EINVAL;
  if (mod->convention != 0 && mod->convention != 1) return FK_EINVAL;
  if (!(mod->w1 >= 0.0 && mod->w1 <= 1.0)) return FK_EINVAL;
  if (!std::isfinite(mod->U) || !std::isfinite(mod->E) || !std::isfinite(mod->mu))
    return FK_EINVAL;
  if (ci.n_c > kMaxN || ci.n_c < 3) return FK_EINVAL;

  int ndev = 0, dev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return FK_EDEVICE;
  if (hipGetDevice(&dev) != hipSuccess) return FK_EDEVICE;
  // the no-allocation entry point's staging array on this device (its
  // failure only disables fk_wigner_dos_noalloc, which then reports it)
  (void)scratch_setup(dev);

  fk_ctx* c = new (std::nothrow) fk_ctx();
  if (!c) return FK_ENOMEM;
  for (hipEvent_t& e : c->ev) e = nullptr;
  c->c = *cont;
  c->m = *mod;
  c->ci = ci;
  c->dev = dev;
  const int n = ci.n_c, n_t = ci.n_t;

  // quadrature points k = a * n_ebar + b of the n_eps x n_ebar product rule;
  // with gh_average the (n_eps + 1) x (n_ebar + 1) rule follows, and every
  // weight is halved: the average of the two rules (Sec. II, the quadrature
  // paragraph: N and N + 1 points)
  const int nrules = mod->gh_average ? 2 : 1;
  c->npts = 0;
  for (int q = 0; q < nrules; ++q) {
    const int na = mod->n_eps + q, nb = mod->n_ebar + q;
    std::vector<double> xa(na), wa(na), xb(nb), wb(nb);
    fk_gauss_hermite(na, xa.data(), wa.data());
    fk_gauss_hermite(nb, xb.data(), wb.data());
    const double scale = nrules == 2 ? 0.5 : 1.0;
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < nb; ++b) {
        c->eps.push_back(xa[a]);
        c->ebar.push_back(xb[b]);
        c->rho.push_back(scale * wa[a] * wb[b]);
      }
    c->npts += na * nb;
  }

  // antiderivative tables alpha, gamma of the band phase (eq.
  // g_contour_non_final2): sin(Et)/E and (cos Et - 1)/E for real t > 0,
  // otherwise alpha = z and gamma = 0.
  std::vector<c64> alpha(n), gamma(n), zc(n);
  const double E = mod->E;
  for (int j = 0; j < n; ++j) {
    zc[j] = c64{ci.zr[j], ci.zi[j]};
    alpha[j] = zc[j];
    gamma[j] = c64{0.0, 0.0};
    if (E != 0.0 && j < 2 * n_t && ci.zr[j] > 0.0) {
      const double t = ci.zr[j];
      alpha[j] = c64{sin(E * t) / E, 0.0};
      const double h = sin(0.5 * E * t);
      gamma[j] = c64{-2.0 * h * h / E, 0.0};
    }
  }
  std::vector<c64> da(n), dg(n), dz(n);
  da[0] = dg[0] = dz[0] = c64{0.0, 0.0};
  for (int j = 1; j < n; ++j) {
    da[j] = c64{alpha[j].re - alpha[j - 1].re, alpha[j].im - alpha[j - 1].im};
    dg[j] = c64{gamma[j].re - gamma[j - 1].re, gamma[j].im - gamma[j - 1].im};
    dz[j] = c64{zc[j].re - zc[j - 1].re, zc[j].im - zc[j - 1].im};
  }
  std::vector<double> cs(n_t), sn(n_t);
  std::vector<int> tp(n_t);
  for (int i = 0; i < n_t; ++i) {
    const double t = ci.zr[i];
    cs[i] = cos(E * t);
    sn[i] = sin(E * t);
    tp[i] = t > 0.0 ? 1 : 0;
  }
  std::vector<c64> w(n);
  for (int j = 0; j < n; ++j) w[j] = c64{ci.wr[j], ci.wi[j]};
  const double coef[3] = {1.0, 1.0 - mod->w1, mod->w1};

  hipError_t e = hipSuccess;
  if (hip_stream) {
    c->st = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking);
    c->own_stream = (e == hipSuccess);
  }
  const size_t mat = sizeof(c64) * (size_t)n * n;
  if (e == hipSuccess) e = upload(&c->d_w, w.data(), sizeof(c64) * n);
  if (e == hipSuccess) e = hipMalloc(&c->d_sigma, mat);
  if (e == hipSuccess) e = hipMemset(c->d_sigma, 0, mat);
  if (e == hipSuccess) e = hipMalloc(&c->d_sigt, mat);
  if (e == hipSuccess) e = hipMalloc(&c->d_gloc, mat);
  if (e == hipSuccess) e = hipMalloc(&c->d_gprev, mat);
  if (e == hipSuccess) e = hipMalloc(&c->d_g0inv, mat);
  if (e == hipSuccess) e = hipMalloc(&c->d_tmp, mat);
  if (e == hipSuccess) e = hipMalloc(&c->d_cur, sizeof(double) * n_t);
  if (e == hipSuccess) e = upload(&c->d_eps, c->eps.data(), sizeof(double) * c->npts);
  if (e == hipSuccess) e = upload(&c->d_ebar, c->ebar.data(), sizeof(double) * c->npts);
  if (e == hipSuccess) e = upload(&c->d_rho, c->rho.data(), sizeof(double) * c->npts);
  if (e == hipSuccess) e = upload(&c->d_da, da.data(), sizeof(c64) * n);
  if (e == hipSuccess) e = upload(&c->d_dg, dg.data(), sizeof(c64) * n);
  if (e == hipSuccess) e = upload(&c->d_dz, dz.data(), sizeof(c64) * n);
  if (e == hipSuccess) e = upload(&c->d_cos, cs.data(), sizeof(double) * n_t);
  if (e == hipSuccess) e = upload(&c->d_sin, sn.data(), sizeof(double) * n_t);
  if (e == hipSuccess) e = upload(&c->d_tpos, tp.data(), sizeof(int) * n_t);
  if (e == hipSuccess) e = upload(&c->d_coef, coef, sizeof coef);
  if (e == hipSuccess) e = hipMalloc(&c->d_key, sizeof(unsigned long long));
  if (e == hipSuccess) {
    std::vector<int> iota(n);
    for (int j = 0; j < n; ++j) iota[j] = j;
    e = upload(&c->d_iota, iota.data(), sizeof(int) * n);
  }
  for (hipEvent_t& ev : c->ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux.st2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->aux.evN, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->aux.evP, hipEventDisableTiming);
  if (e != hipSuccess) {
    const fk_status s = (e == hipErrorOutOfMemory) ? FK_ENOMEM : FK_EDEVICE;
    free_ctx(c);
    delete c;
    return s;
  }
  c->tab.eps = c->d_eps;
  c->tab.ebar = c->d_ebar;
  c->tab.rho = c->d_rho;
  c->tab.da = c->d_da;
  c->tab.dg = c->d_dg;
  c->tab.dz = c->d_dz;
  c->tab.ca = c64{alpha[0].re - alpha[n - 1].re, alpha[0].im - alpha[n - 1].im};
  c->tab.cg = c64{gamma[0].re - gamma[n - 1].re, gamma[0].im - gamma[n - 1].im};
  c->tab.cz = c64{zc[0].re - zc[n - 1].re, zc[0].im - zc[n - 1].im};
  c->tab.mu = mod->mu;
  c->tab.beta = cont->beta;
  c->tab.cos_et = c->d_cos;
  c->tab.sin_et = c->d_sin;
  c->tab.t_pos = c->d_tpos;

  size_t bb = (size_t)24 << 30;
  if (const char* s = getenv("FKDMFT_BATCH_BYTES")) {
    const double v = atof(s);
    if (v > 0) bb = (size_t)v;
  }
  c->batch_bytes = bb;
  if (const char* s = getenv("FKDMFT_LOOKAHEAD")) c->aux.lookahead = atoi(s) != 0;
  *out = c;
  return FK_OK;
}

extern "C" fk_status fk_destroy(fk_ctx* c) {
  if (!c) return FK_OK;
  if (c->st) (void)hipStreamSynchronize(c->st);
  free_ctx(c);
  delete c;
  return FK_OK;
}

extern "C" const char* fk_last_error(const fk_ctx* c) {
  return c ? c->err.c_str() : "NULL context";
}

extern "C" fk_status fk_dims(const fk_ctx* c, int* n_t, int* n_tau, int* n_c) {
  if (!c) return FK_EINVAL;
  if (n_t) *n_t = c->ci.n_t;
  if (n_tau) *n_tau = c->ci.n_tau;
  if (n_c) *n_c = c->ci.n_c;
  return FK_OK;
}

extern "C" fk_status fk_contour_points(const fk_ctx* c, double* z, double* W) {
  if (!c) return FK_EINVAL;
  int dims[3];
  return fk_contour_build(&c->c, dims, z, W);
}

extern "C" fk_status fk_points(const fk_ctx* c, int* n_points, double* eps,
                               double* ebar, double* rho) {
  if (!c) return FK_EINVAL;
  if (n_points) *n_points = c->npts;
  for (int k = 0; k < c->npts; ++k) {
    if (eps) eps[k] = c->eps[k];
    if (ebar) ebar[k] = c->ebar[k];
    if (rho) rho[k] = c->rho[k];
  }
  return FK_OK;
}

extern "C" fk_status fk_set_batch(fk_ctx* c, int batch, int* used) {
  if (!c || batch < 0) return FK_EINVAL;
  c->want_batch = batch;
  c->last_prec = -1;   // the batch buffers are freed
  batch_free(c->b64);
  batch_free(c->b32);
  fk_status s = ensure_batch<double>(c);
  if (s != FK_OK) return s;
  if (used) *used = c->b64.cap;
  return FK_OK;
}

extern "C" fk_status fk_set_sigma(fk_ctx* c, const double* sigma, int on_device) {
  if (!c) return FK_EINVAL;
  return copy_matrix_in(c, c->d_sigma, sigma, on_device);
}

extern "C" fk_status fk_get_sigma(const fk_ctx* cc, double* sigma, int on_device) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c) return FK_EINVAL;
  return copy_matrix_out(c, sigma, c->d_sigma, on_device);
}

extern "C" fk_status fk_get_gloc(const fk_ctx* cc, double* gloc, int on_device) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c) return FK_EINVAL;
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "no lattice step yet");
  return copy_matrix_out(c, gloc, c->d_gloc, on_device);
}

extern "C" fk_status fk_set_refinement(fk_ctx* c, int ir_steps) {
  if (!c || ir_steps < 0 || ir_steps > 4) return FK_EINVAL;
  c->ir_steps = ir_steps;
  return FK_OK;
}

extern "C" fk_status fk_set_switch(fk_ctx* c, double switch_tol) {
  if (!c || !(switch_tol >= 0.0)) return FK_EINVAL;
  c->switch_tol = switch_tol;
  return FK_OK;
}

extern "C" fk_status fk_compute_gloc(fk_ctx* c, fk_precision prec, double* ir_out) {
  if (!c) return FK_EINVAL;
  if (prec == FK_FP64) return lattice_step<double>(c, ir_out);
  if (prec == FK_MIXED) return lattice_step_mixed(c, ir_out);
  return set_err(c, FK_EINVAL, "unknown precision %d", (int)prec);
}

extern "C" fk_status fk_get_current(const fk_ctx* cc, double* t, double* j,
                                    double* n_t_out) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c) return FK_EINVAL;
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "no lattice step yet");
  const int n_t = c->ci.n_t, n = c->ci.n_c;
  if (t)
    for (int i = 0; i < n_t; ++i) t[i] = c->ci.zr[i];
  if (j) {
    HIPCHK(c, hipMemcpyAsync(j, c->d_cur, sizeof(double) * n_t,
                             hipMemcpyDeviceToHost, c->st));
  }
  if (n_t_out) {
    // n(t_i) = Re[-i G^<(t_i, t_i)] = Im G_loc[i][2 N_t - i]
    std::vector<c64> less(n_t);
    HIPCHK(c, launch_equal_time(c->d_gloc, n_t, n, c->d_tmp, c->d_tmp + n_t, c->st));
    HIPCHK(c, hipMemcpyAsync(less.data(), c->d_tmp, sizeof(c64) * n_t,
                             hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (int i = 0; i < n_t; ++i) n_t_out[i] = less[i].im;
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

extern "C" fk_status fk_get_zeroth_moment(const fk_ctx* cc, double* m0) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c || !m0) return FK_EINVAL;
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "no lattice step yet");
  const int n_t = c->ci.n_t, n = c->ci.n_c;
  std::vector<c64> lg(2 * (size_t)n_t);
  HIPCHK(c, launch_equal_time(c->d_gloc, n_t, n, c->d_tmp, c->d_tmp + n_t, c->st));
  HIPCHK(c, hipMemcpyAsync(lg.data(), c->d_tmp, sizeof(c64) * 2 * n_t,
                           hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int i = 0; i < n_t; ++i) {   // G^> - G^<
    m0[2 * i] = lg[n_t + i].re - lg[i].re;
    m0[2 * i + 1] = lg[n_t + i].im - lg[i].im;
  }
  return FK_OK;
}

namespace {
// Device copies of small host arrays for the spectral functions: one
// allocation per call (post-processing, outside the iteration), freed on return.
struct CallBuffer {
  void* p = nullptr;
  ~CallBuffer() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

extern "C" fk_status fk_wigner_dos(const fk_ctx* cc, int n_T, const int* t_index,
                                   int n_w, const double* omega, double* dos) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c || !t_index || !omega || !dos || n_T < 1 || n_w < 1) return FK_EINVAL;
  const int n_t = c->ci.n_t, n = c->ci.n_c;
  for (int r = 0; r < n_T; ++r)
    if (t_index[r] < 0 || t_index[r] >= n_t)
      return set_err(c, FK_EINVAL, "time index %d outside [0, N_t)", t_index[r]);
  for (int q = 0; q < n_w; ++q)
    if (!std::isfinite(omega[q])) return set_err(c, FK_EINVAL, "non-finite frequency");
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "no lattice step yet");
  const size_t bi = sizeof(int) * (size_t)n_T, bw = sizeof(double) * (size_t)n_w;
  const size_t bo = sizeof(double) * (size_t)n_T * n_w;
  const size_t off_w = (bi + 255) / 256 * 256, off_o = off_w + (bw + 255) / 256 * 256;
  CallBuffer buf;
  HIPCHK(c, hipMalloc(&buf.p, off_o + bo));
  char* base = static_cast<char*>(buf.p);
  HIPCHK(c, hipMemcpyAsync(base, t_index, bi, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(base + off_w, omega, bw, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, launch_wigner_dos(c->d_gloc, n_t, n, c->c.dt, reinterpret_cast<int*>(base),
                              n_T, reinterpret_cast<double*>(base + off_w), n_w,
                              reinterpret_cast<double*>(base + off_o), c->st));
  HIPCHK(c, hipMemcpyAsync(dos, base + off_o, bo, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

extern "C" fk_status fk_wigner_dos_noalloc(const fk_ctx* cc, int n_T, const int* t_index,
                                           int n_w, const double* omega, double* dos) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c || !t_index || !omega || !dos || n_T < 1 || n_w < 1) return FK_EINVAL;
  const int n_t = c->ci.n_t, n = c->ci.n_c;
  for (int r = 0; r < n_T; ++r)
    if (t_index[r] < 0 || t_index[r] >= n_t)
      return set_err(c, FK_EINVAL, "time index %d outside [0, N_t)", t_index[r]);
  for (int q = 0; q < n_w; ++q)
    if (!std::isfinite(omega[q])) return set_err(c, FK_EINVAL, "non-finite frequency");
  // staging layout in the static array: time indices, frequencies, result,
  // each segment 256-byte aligned
  const size_t bi = sizeof(int) * (size_t)n_T, bw = sizeof(double) * (size_t)n_w;
  const size_t bo = sizeof(double) * (size_t)n_T * n_w;
  const size_t off_w = (bi + 255) / 256 * 256, off_o = off_w + (bw + 255) / 256 * 256;
  if (off_o + bo > kScratchBytes)
    return set_err(c, FK_EINVAL,
                   "fk_wigner_dos_noalloc: %d times x %d frequencies need %zu bytes of "
                   "staging, above its %zu-byte static scratch", n_T, n_w, off_o + bo,
                   kScratchBytes);
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "no lattice step yet");
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr(c->dev));
  if (!base)
    return set_err(c, FK_EDEVICE, "static scratch of device %d unavailable: %s", c->dev,
                   hipGetErrorString(c->dev >= 0 && c->dev < kMaxDevices
                                         ? g_scratch_err[c->dev] : hipErrorInvalidDevice));
  HIPCHK(c, hipMemcpyAsync(base, t_index, bi, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(base + off_w, omega, bw, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, launch_wigner_dos(c->d_gloc, n_t, n, c->c.dt, reinterpret_cast<int*>(base),
                              n_T, reinterpret_cast<double*>(base + off_w), n_w,
                              reinterpret_cast<double*>(base + off_o), c->st));
  HIPCHK(c, hipMemcpyAsync(dos, base + off_o, bo, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

extern "C" fk_status fk_equal_time_moments(const fk_ctx* cc, int n_T, const int* t_index,
                                           double* mu) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c || !t_index || !mu || n_T < 1) return FK_EINVAL;
  const int n_t = c->ci.n_t, n = c->ci.n_c;
  for (int r = 0; r < n_T; ++r)
    if (t_index[r] < 3 || t_index[r] > n_t - 4)
      return set_err(c, FK_EINVAL, "time index %d outside [3, N_t - 4]", t_index[r]);
  if (!c->have_gloc) return set_err(c, FK_ESTATE, "no lattice step yet");
  const size_t bi = sizeof(int) * (size_t)n_T, off_o = (bi + 255) / 256 * 256;
  const size_t bo = sizeof(c64) * 3 * (size_t)n_T;
  CallBuffer buf;
  HIPCHK(c, hipMalloc(&buf.p, off_o + bo));
  char* base = static_cast<char*>(buf.p);
  HIPCHK(c, hipMemcpyAsync(base, t_index, bi, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, launch_moments(c->d_gloc, n_t, n, c->c.dt, reinterpret_cast<int*>(base), n_T,
                           reinterpret_cast<c64*>(base + off_o), c->st));
  HIPCHK(c, hipMemcpyAsync(mu, base + off_o, bo, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

extern "C" fk_status fk_impurity_update(fk_ctx* c, double* max_dsigma_out) {
  if (!c) return FK_EINVAL;
  return impurity(c, max_dsigma_out);
}

namespace {
// One self-consistency iteration (the it-th of a run): lattice step, delta =
// max |G_loc - G_loc of the previous iteration| from the second iteration on,
// impurity update (dsig: max |Sigma_new - Sigma|, nullable).  In a mixed run the
// low-precision phase ends below switch_tol, or as soon as delta stops
// contracting below 100 switch_tol (it has reached the complex64 noise floor).
fk_status iteration(fk_ctx* c, int it, bool* low, double* delta, double* prev_delta,
                    double* hist, double* dsig) {
  if (*low) c->low_iters++;
  fk_status s = fk_compute_gloc(c, *low ? FK_MIXED : FK_FP64, nullptr);
  if (s != FK_OK) return s;
  if (it > 1) {
    HIPCHK(c, fill_u64(c->d_key, 0ULL, 1, c->st));
    HIPCHK(c, launch_maxabs(c->d_gloc, c->d_gprev, (size_t)c->ci.n_c * c->ci.n_c,
                            c->d_key, c->st));
    *delta = read_key(c, &s);
    if (s != FK_OK) return s;
  }
  if (hist) hist[it - 1] = *delta;
  HIPCHK(c, hipMemcpyAsync(c->d_gprev, c->d_gloc,
                           sizeof(c64) * (size_t)c->ci.n_c * c->ci.n_c,
                           hipMemcpyDeviceToDevice, c->st));
  s = impurity(c, dsig);
  if (s != FK_OK) return s;
  // leave the complex64 phase below switch_tol, or when delta stops
  // contracting close to the complex64 noise floor (a stall far above it, as in
  // the first iterations of a slowly contracting loop, is not a precision limit)
  if (*low && (*delta < c->switch_tol ||
               (it > 2 && *delta < 100.0 * c->switch_tol && *delta > 0.95 * *prev_delta)))
    *low = false;
  *prev_delta = *delta;
  return FK_OK;
}
}  // namespace

extern "C" fk_status fk_iterate(fk_ctx* c, int max_iter, double tol,
                                fk_precision prec, int* iters_out,
                                double* delta_out, double* hist) {
  if (!c || max_iter < 1) return FK_EINVAL;
  c->low_iters = 0;
  double delta = std::numeric_limits<double>::infinity();
  double prev_delta = delta;
  bool low = (prec == FK_MIXED);
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    fk_status s = iteration(c, it, &low, &delta, &prev_delta, hist, nullptr);
    if (s != FK_OK) return s;
    if (delta < tol) break;
  }
  if (it > max_iter) it = max_iter;
  if (iters_out) *iters_out = it;
  if (delta_out) *delta_out = delta;
  if (tol > 0.0 && !(delta < tol))
    return set_err(c, FK_ENOTCONV, "not converged after %d iterations (delta %.3e)",
                   max_iter, delta);
  return FK_OK;
}

extern "C" fk_status fk_iterate_judged(fk_ctx* c, const double* fallback_dev,
                                       double accept, int max_iter, double tol,
                                       fk_precision prec, int* iters_out,
                                       double* delta_out, double* hist,
                                       int* outcome) {
  if (!c || max_iter < 2 || !(accept > 0.0)) return FK_EINVAL;
  c->low_iters = 0;
  const size_t nn = (size_t)c->ci.n_c * c->ci.n_c;
  const c64* fb = reinterpret_cast<const c64*>(fallback_dev);
  fk_status s;
  // size of the proposed move away from the fallback start
  HIPCHK(c, fill_u64(c->d_key, 0ULL, 1, c->st));
  HIPCHK(c, launch_maxabs(c->d_sigma, fb, nn, c->d_key, c->st));
  const double move = read_key(c, &s);
  if (s != FK_OK) return s;
  double delta = std::numeric_limits<double>::infinity();
  double prev_delta = delta;
  bool low = (prec == FK_MIXED);
  int result = 0;   // 0 accepted, 1 rejected by the first residual, 2 abandoned later
  int it = 0, base = 0;
  bool judged = false;
  int rising = 0;
  if (!(move <= std::numeric_limits<double>::max())) result = 1;
  if (move == 0.0) judged = true;   // the start is the fallback itself
  for (it = 1; result == 0 && it <= max_iter; ++it) {
    double dsig = 0.0;
    const double before = delta;
    const bool was_low = low;
    s = iteration(c, it, &low, &delta, &prev_delta, hist, judged ? nullptr : &dsig);
    if (s == FK_ENONFINITE || s == FK_ESINGULAR) {
      result = judged ? 2 : 1;
      judged = true;   // the failed iteration is counted
      break;
    }
    if (s != FK_OK) return s;
    if (!judged) {
      judged = true;
      // accept the start if one iteration moves Sigma by at most `accept` times
      // the distance between the start and the fallback
      if (!(dsig <= accept * move)) {
        result = 1;
        break;
      }
    }
    if (delta < tol) break;
    // abandon a start whose FP64 iteration grows three times in a row
    rising = (it > 2 && !was_low && delta > before) ? rising + 1 : 0;
    if (rising >= 3) {
      result = 2;
      break;
    }
  }
  if (result != 0) {
    // restart from the fallback; the iterations spent so far are counted
    base = judged ? std::min(it, max_iter) : 0;
    if (fb)
      HIPCHK(c, hipMemcpyAsync(c->d_sigma, fb, sizeof(c64) * nn, hipMemcpyDeviceToDevice,
                               c->st));
    else
      HIPCHK(c, fill_f64(reinterpret_cast<double*>(c->d_sigma), 0.0, 2 * nn, c->st));
    delta = prev_delta = std::numeric_limits<double>::infinity();
    low = (prec == FK_MIXED);
    for (it = 1; base + it <= max_iter; ++it) {
      s = iteration(c, it, &low, &delta, &prev_delta, hist ? hist + base : nullptr,
                    nullptr);
      if (s != FK_OK) return s;
      if (delta < tol) break;
    }
    it = std::min(base + it, max_iter);
  } else if (it > max_iter) {
    it = max_iter;
  }
  if (iters_out) *iters_out = it;
  if (delta_out) *delta_out = delta;
  if (outcome) *outcome = result;
  if (tol > 0.0 && !(delta < tol))
    return set_err(c, FK_ENOTCONV, "not converged after %d iterations (delta %.3e)",
                   max_iter, delta);
  return FK_OK;
}

extern "C" fk_status fk_get_point_green(const fk_ctx* cc, int k, double* g,
                                        int on_device) {
  fk_ctx* c = const_cast<fk_ctx*>(cc);
  if (!c || !g) return FK_EINVAL;
  if (c->last_prec != 0 || k < c->last_k0 || k >= c->last_k0 + c->last_nmat)
    return set_err(c, FK_ESTATE,
                   "point %d is not in the FP64 lattice batch left by the last step "
                   "(points %d..%d)", k, c->last_k0, c->last_k0 + c->last_nmat - 1);
  const int n = c->ci.n_c, m = k - c->last_k0;
  Batch<double>& b = c->b64;
  c64* dst = on_device ? reinterpret_cast<c64*>(g) : c->d_tmp;
  HIPCHK(c, launch_unpermute<double>(b.x + b.stride * m, b.stride, b.ld,
                                     b.piv + (size_t)m * n, b.rowcol + (size_t)m * n,
                                     n, 1, dst, c->st));
  if (!on_device)
    HIPCHK(c, hipMemcpyAsync(g, c->d_tmp, sizeof(c64) * (size_t)n * n,
                             hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return FK_OK;
}

extern "C" fk_status fk_low_iterations(const fk_ctx* c, int* n) {
  if (!c || !n) return FK_EINVAL;
  *n = c->low_iters;
  return FK_OK;
}

extern "C" fk_status fk_set_kernel_clock(fk_ctx* c, int on) {
  if (!c) return FK_EINVAL;
  KernelClock& k = c->clk;
  if (on && k.ev.empty()) {
    k.ev.assign(2 * (kMaxN / kNBO + 2), nullptr);
    for (hipEvent_t& e : k.ev) HIPCHK(c, hipEventCreate(&e));
  }
  k.on = on != 0;
  k.used = 0;
  k.flops.clear();
  k.ms = k.flop = 0.0;
  k.launches = 0;
  return FK_OK;
}

extern "C" fk_status fk_kernel_clock(const fk_ctx* c, double* out3) {
  if (!c || !out3) return FK_EINVAL;
  out3[0] = c->clk.ms;
  out3[1] = (double)c->clk.launches;
  out3[2] = c->clk.flop;
  return FK_OK;
}

extern "C" fk_status fk_timings(const fk_ctx* c, double* out7) {
  if (!c || !out7) return FK_EINVAL;
  for (int i = 0; i < 7; ++i) out7[i] = c->times[i];
  return FK_OK;
}

// ================================================================ autotuner
namespace {
double matrix_bytes(const fk_ctx* c) {
  const double n = c->ci.n_c;
  return 16.0 * (n * n + kBRows * n) + 8.0 * n;
}
}  // namespace

extern "C" fk_status fk_set_tuning(fk_ctx* c, const fk_tuning* t) {
  if (!c || !t || (t->tile_rows != 64 && t->tile_rows != 128) || t->batch < 0)
    return FK_EINVAL;
  c->variant = t->tile_rows == 128 ? 1 : 0;
  c->aux.lookahead = t->lookahead != 0;
  if (t->batch > 0) c->want_batch = t->batch;
  c->last_prec = -1;   // the next step may reallocate the batch
  c->tuned = *t;
  return FK_OK;
}

extern "C" fk_status fk_get_tuning(const fk_ctx* c, fk_tuning* t) {
  if (!c || !t) return FK_EINVAL;
  fk_tuning r = c->tuned;
  r.tile_rows = c->variant == 1 ? 128 : 64;
  r.lookahead = c->aux.lookahead ? 1 : 0;
  r.batch = c->b64.cap > 0 ? c->b64.cap : c->want_batch;
  r.chunk_bytes = r.batch * matrix_bytes(c);
  *t = r;
  return FK_OK;
}

extern "C" fk_status fk_autotune(fk_ctx* c, double max_bytes, int keep,
                                 fk_tuning* best) {
  if (!c || !(max_bytes > 0)) return FK_EINVAL;
  const double mb = matrix_bytes(c);
  int cap_max = (int)std::min<double>(c->npts, std::floor(max_bytes / mb));
  if (cap_max < 1) return set_err(c, FK_ENOMEM, "max_bytes below one matrix");
  // candidate batch sizes: the points split evenly into k batches for the
  // smallest k the byte budget allows and the next three (no short last
  // batch), the budget's quarter, and whole multiples of the compute-unit
  // count (the panel runs one workgroup per matrix, so a batch that fills the
  // CUs exactly avoids a partial round of panel workgroups)
  std::vector<int> caps;
  auto add_cap = [&](int b) {
    if (b >= 1 && b <= cap_max && std::find(caps.begin(), caps.end(), b) == caps.end())
      caps.push_back(b);
  };
  const int kmin = (c->npts + cap_max - 1) / cap_max;
  for (int k = kmin; k < kmin + 4 && k <= c->npts; ++k) add_cap((c->npts + k - 1) / k);
  add_cap(std::max(1, cap_max / 4));
  int dev = 0, ncu = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  for (int k = 1; k <= 3 && ncu > 0; ++k)
    if (k * ncu < c->npts) add_cap(k * ncu);
  const int n = c->ci.n_c;
  c->last_prec = -1;   // the trials overwrite and free the batch buffers
  HIPCHK(c, launch_sigma_weight(c->d_sigma, c->d_w, c->d_sigt, n, c->st));
  int trials = 0;
  fk_status s;
  // one schedule: build and invert one batch twice, the second timed; the
  // estimate is that time per batch times the number of batches
  auto time_one = [&](int variant, int cap, int la, double* est) -> fk_status {
    c->variant = variant;
    c->want_batch = cap;
    c->aux.lookahead = la != 0;
    batch_free(c->b64);
    fk_status st;
    if ((st = ensure_batch<double>(c)) != FK_OK) return st;
    Batch<double>& b = c->b64;
    const int nmat = b.cap;
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      HIPCHK(c, launch_build<double>(c->d_sigt, c->tab, 0, nmat, b.x, b.stride, b.ld, n,
                                     c->st));
      HIPCHK(c, hipEventRecord(c->ev[0], c->st));
      HIPCHK(c, batch_invert<double>(b, nmat, c->st, c->aux, nullptr));
      HIPCHK(c, hipEventRecord(c->ev[1], c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
      ms = elapsed(c->ev[0], c->ev[1]);
    }
    if ((st = check_status(c, b.status, nmat, 0, "autotune inversion")) != FK_OK) return st;
    *est = (double)ms * ((c->npts + nmat - 1) / nmat);
    ++trials;
    return FK_OK;
  };
  struct Cand {
    int variant, cap, la;
    double est;
  };
  // first pass: every schedule once.  The look-ahead stream counts only when
  // it wins clearly: one batch timed once cannot resolve smaller differences
  std::vector<Cand> cands;
  for (int variant : {0, 1})
    for (int cap : caps) {
      double est_plain = 0.0;
      for (int la : {0, 1}) {
        double est = 0.0;
        if ((s = time_one(variant, cap, la, &est)) != FK_OK) return s;
        if (!la) est_plain = est;
        if (!la || est < 0.98 * est_plain) cands.push_back({variant, cap, la, est});
      }
    }
  // second pass: the three fastest again, slowest first, on a device whose
  // clocks have settled under the first pass's load (the first trials of a
  // cold device run faster than the same work does in a long run); the
  // choice uses these times only
  std::sort(cands.begin(), cands.end(),
            [](const Cand& a, const Cand& b2) { return a.est < b2.est; });
  if (cands.size() > 3) cands.resize(3);
  std::reverse(cands.begin(), cands.end());
  fk_tuning bestt{64, 1, 0, 0.0, std::numeric_limits<double>::infinity(), 0};
  for (const Cand& cd : cands) {
    double est = 0.0;
    if ((s = time_one(cd.variant, cd.cap, cd.la, &est)) != FK_OK) return s;
    if (est < bestt.est_step_ms) {
      bestt.tile_rows = cd.variant ? 128 : 64;
      bestt.batch = c->b64.cap;
      bestt.lookahead = cd.la;
      bestt.chunk_bytes = c->b64.cap * mb;
      bestt.est_step_ms = est;
    }
  }
  bestt.trials = trials;
  batch_free(c->b64);
  if ((s = fk_set_tuning(c, &bestt)) != FK_OK) return s;
  if (keep && (s = ensure_batch<double>(c)) != FK_OK) return s;
  if (best) *best = bestt;
  return FK_OK;
}
