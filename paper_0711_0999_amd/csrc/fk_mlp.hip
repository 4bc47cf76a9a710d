// Learned warm start of the self-consistency loop (gfx950): a fully connected
// tanh network evaluated pointwise on contour pairs (t_i, t_j), trained on
// solutions that the plain iteration produced, with its own forward, backward
// and Adam kernels.  Training runs in FP32 on the f32 matrix cores; inference
// can run in BF16 (bf16 matrix cores, FP32 accumulation).
//
// Also here: the rank-r randomized sketch of a self-energy (singular values of
// Y = Sigma Omega, Omega supplied by the caller), the per-pair feature rows,
// the training targets and the application of a predicted correction.
#include "fk_ctx.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

using namespace fk;

static constexpr int kWsFeatures = FK_WS_FEATURES;

namespace fk {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ inline short f2bf(float x) {  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C[M x N] = epi(op(A)[M x K] op(B)[K x N]) (+ beta C).  TA = 0: A[m][k] at
// A[m lda + k], TA = 1: at A[k lda + m]; TB = 0: B[k][n] at B[k ldb + n],
// TB = 1: at B[n ldb + k].  EPI 0: plain, 1: + bias[n] then tanh, 2: + bias[n].
// BF = 1 rounds both operands to bf16 and uses the bf16 matrix cores.
// 64 x 64 tiles, 2 x 2 waves of 32 x 32, K chunks of 16 through LDS.
template <int TA, int TB, int EPI, int BF>
__global__ __launch_bounds__(256, 2) void k_gemm32(
    const float* __restrict__ A, int lda, const float* __restrict__ B, int ldb,
    float* __restrict__ C, int ldc, const float* __restrict__ bias, int M,
    int N, int K, float beta) {
  constexpr int T = 64, KC = 16, AP = KC + 1, BP = T + 1;
  __shared__ float As[T * AP];
  __shared__ float Bs[KC * BP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  const int ntn = (N + T - 1) / T;
  const int r0 = (blockIdx.x / ntn) * T, c0 = (blockIdx.x % ntn) * T;
  v4f acc[2][2];
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[ii][jj] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int i = e / KC, k = e % KC;                 // A: 64 rows x 16 k
      const int m = r0 + i, kk = k0 + k;
      float a = 0.f;
      if (m < M && kk < K) a = TA ? A[(size_t)kk * lda + m] : A[(size_t)m * lda + kk];
      As[i * AP + k] = a;
      const int k2 = e / T, c = e % T;                  // B: 16 k x 64 cols
      const int n = c0 + c, kb = k0 + k2;
      float b = 0.f;
      if (n < N && kb < K) b = TB ? B[(size_t)n * ldb + kb] : B[(size_t)kb * ldb + n];
      Bs[k2 * BP + c] = b;
    }
    __syncthreads();
    if (BF) {
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          v4s av, bv;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            av[t] = f2bf(As[(32 * wr + 16 * ii + li) * AP + 4 * lk + t]);
            bv[t] = f2bf(Bs[(4 * lk + t) * BP + 32 * wc + 16 * jj + li]);
          }
          acc[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[ii][jj], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int k = 0; k < KC; k += 4)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const float a = As[(32 * wr + 16 * ii + li) * AP + k + lk];
            const float b = Bs[(k + lk) * BP + 32 * wc + 16 * jj + li];
            acc[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[ii][jj], 0, 0, 0);
          }
    }
  }
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = r0 + 32 * wr + 16 * ii + 4 * lk + v;   // f32 accumulator rows
        const int n = c0 + 32 * wc + 16 * jj + li;
        if (m < M && n < N) {
          float y = acc[ii][jj][v];
          if (EPI >= 1) y += bias[n];
          if (EPI == 1) y = tanhf(y);
          if (beta != 0.f) y += beta * C[(size_t)m * ldc + n];
          C[(size_t)m * ldc + n] = y;
        }
      }
}

template <int TA, int TB, int EPI, int BF>
hipError_t gemm32(const float* A, int lda, const float* B, int ldb, float* C,
                  int ldc, const float* bias, int M, int N, int K, float beta,
                  hipStream_t st) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  hipLaunchKernelGGL((k_gemm32<TA, TB, EPI, BF>), dim3(tiles), dim3(256), 0, st,
                     A, lda, B, ldb, C, ldc, bias, M, N, K, beta);
  return hipGetLastError();
}

// dZ = dH * (1 - H^2) (tanh derivative), in place
__global__ void k_tanh_back(float* __restrict__ d, const float* __restrict__ h,
                            size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    d[e] *= 1.f - h[e] * h[e];
}

// dY = 2 (Y - T) / rows; per-block partial sums of (Y - T)^2
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                      float* __restrict__ d, size_t n, float inv_rows,
                      double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const float r = y[e] - t[e];
    d[e] = 2.f * r * inv_rows;
    acc += (double)r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// db[n] = sum over rows of dZ[r][n]
__global__ void k_colsum(const float* __restrict__ d, int rows, int cols,
                         float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += d[(size_t)r * cols + c];
  out[c] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, size_t n,
                       float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// Minibatch gather: slot q of step `step` takes row SplitMix64(seed + q') mod
// rows, q' = step * batch + q (Steele, Lea & Flood 2014).
__device__ inline unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_gather_rows(const float* __restrict__ x, const float* __restrict__ t,
                              long long rows, int d_in, int d_out, int batch,
                              unsigned long long seed, long long step,
                              float* __restrict__ xs, float* __restrict__ ts) {
  const int q = blockIdx.x;
  const unsigned long long h =
      splitmix64(seed * 0xD1B54A32D192ED03ull + (unsigned long long)(step * batch + q));
  const long long r = (long long)(h % (unsigned long long)rows);
  for (int c = threadIdx.x; c < d_in; c += blockDim.x)
    xs[(size_t)q * d_in + c] = x[(size_t)r * d_in + c];
  for (int c = threadIdx.x; c < d_out; c += blockDim.x)
    ts[(size_t)q * d_out + c] = t[(size_t)r * d_out + c];
}

// Y[i][r] = sum_j d_i Sigma[i][j] d_j Omega[j][r] with d_j = sqrt(|W_j|): the
// range sketch of the symmetrically weighted kernel, whose singular values
// approximate those of the contour integral operator and so do not grow with N_c.
__global__ void k_sketch(const c64* __restrict__ s, const c64* __restrict__ w,
                         const double* __restrict__ om, int n, int r,
                         c64* __restrict__ y) {
  const int i = blockIdx.x;
  const double di = sqrt(hypot(w[i].re, w[i].im));
  for (int q = threadIdx.x; q < r; q += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < n; ++j) {
      const c64 a = s[(size_t)i * n + j];
      const double o = sqrt(hypot(w[j].re, w[j].im)) * om[(size_t)j * r + q];
      re += a.re * o;
      im += a.im * o;
    }
    y[(size_t)i * r + q] = c64{di * re, di * im};
  }
}

// Z[j][q] = sum_i conj(d_i Sigma[i][j] d_j) Q[i][q]: Z = (D Sigma D)^H Q
__global__ void k_sketch_adj(const c64* __restrict__ s, const c64* __restrict__ w,
                             const c64* __restrict__ qm, int n, int r,
                             c64* __restrict__ z) {
  const int j = blockIdx.x;
  const double dj = sqrt(hypot(w[j].re, w[j].im));
  for (int q = threadIdx.x; q < r; q += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int i = 0; i < n; ++i) {
      const c64 a = s[(size_t)i * n + j];
      const double di = sqrt(hypot(w[i].re, w[i].im));
      const c64 b = qm[(size_t)i * r + q];
      // conj(a) b
      re += di * (a.re * b.re + a.im * b.im);
      im += di * (a.re * b.im - a.im * b.re);
    }
    z[(size_t)j * r + q] = c64{dj * re, dj * im};
  }
}

// Feature row of the pair (i, j) = idx / n (T = t_max - t_min; t+ = max(t, 0)
// on the real branches, 0 on the imaginary one):
//   [glob (ng) | branch one-hot i (3) | branch one-hot j (3) | t_i/T | tau_i/beta |
//    t_j/T | tau_j/beta | [i >= j] | [i - j >= 2] | (t_i - t_j)/T |
//    max(t_i, t_j, 0)/T | sin E t_i+ | cos E t_i+ | sin E t_j+ | cos E t_j+ |
//    s Re Sigma_prev | s Im Sigma_prev |
//    sin, cos (pi k t_i/T), k = 1..8 | same for t_j | sin, cos (pi k tau_i/beta),
//    k = 1, 2 | same for tau_j | 0 ...]
// The second step flag marks where the discrete self-energy of the point-split
// impurity update jumps across the diagonal, two contour indices below it.
constexpr int kFourierT = 8, kFourierTau = 2;   // harmonics of t/T and tau/beta
static_assert(20 + 4 * kFourierT + 4 * kFourierTau == kWsFeatures, "feature count");
struct FeatGeo {
  const c64* z;       // contour points (device)
  int n, n_t;
  double tspan, beta, E;
};
__global__ void k_features(FeatGeo g, const c64* __restrict__ sprev,
                           const float* __restrict__ glob, int ng,
                           const long long* __restrict__ idx, long long rows,
                           float scale, float* __restrict__ x, int d_in) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < rows;
       r += (long long)gridDim.x * blockDim.x) {
    const long long p = idx ? idx[r] : r;
    float* row = x + (size_t)r * d_in;
    if (p < 0 || p >= (long long)g.n * g.n) {   // pair index out of range
      for (int q = 0; q < d_in; ++q) row[q] = __builtin_nanf("");
      continue;
    }
    const int i = (int)(p / g.n), j = (int)(p - (p / g.n) * g.n);
    int c = 0;
    for (int q = 0; q < ng; ++q) row[c++] = glob[q];
    const int bi = i < g.n_t ? 0 : (i < 2 * g.n_t ? 1 : 2);
    const int bj = j < g.n_t ? 0 : (j < 2 * g.n_t ? 1 : 2);
    for (int q = 0; q < 3; ++q) row[c++] = (bi == q) ? 1.f : 0.f;
    for (int q = 0; q < 3; ++q) row[c++] = (bj == q) ? 1.f : 0.f;
    const double ti = bi < 2 ? g.z[i].re : 0.0, taui = bi == 2 ? -g.z[i].im : 0.0;
    const double tj = bj < 2 ? g.z[j].re : 0.0, tauj = bj == 2 ? -g.z[j].im : 0.0;
    row[c++] = (float)(ti / g.tspan);
    row[c++] = (float)(taui / g.beta);
    row[c++] = (float)(tj / g.tspan);
    row[c++] = (float)(tauj / g.beta);
    row[c++] = i >= j ? 1.f : 0.f;
    row[c++] = i - j >= 2 ? 1.f : 0.f;
    row[c++] = (float)((ti - tj) / g.tspan);
    row[c++] = (float)(fmax(fmax(ti, tj), 0.0) / g.tspan);
    const double pi = g.E * fmax(ti, 0.0), pj = g.E * fmax(tj, 0.0);
    row[c++] = (float)sin(pi);
    row[c++] = (float)cos(pi);
    row[c++] = (float)sin(pj);
    row[c++] = (float)cos(pj);
    const c64 sp = sprev[p];
    row[c++] = (float)(scale * sp.re);
    row[c++] = (float)(scale * sp.im);
    // Fourier features of the four coordinates
    const double xs[4] = {ti / g.tspan, tj / g.tspan, taui / g.beta, tauj / g.beta};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int kmax = a < 2 ? kFourierT : kFourierTau;
      for (int k = 1; k <= kmax; ++k) {
        double sn, cs;
        sincospi(k * xs[a], &sn, &cs);
        row[c++] = (float)sn;
        row[c++] = (float)cs;
      }
    }
    for (; c < d_in; ++c) row[c] = 0.f;
  }
}

// t = scale (Sigma_new - Sigma_prev) at the listed pairs
__global__ void k_targets(const c64* __restrict__ sprev, const c64* __restrict__ snew,
                          const long long* __restrict__ idx, long long rows,
                          long long total, float scale, float* __restrict__ t) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < rows;
       r += (long long)gridDim.x * blockDim.x) {
    const long long p = idx ? idx[r] : r;
    if (p < 0 || p >= total) {
      t[2 * r] = t[2 * r + 1] = __builtin_nanf("");
      continue;
    }
    t[2 * r] = (float)(scale * (snew[p].re - sprev[p].re));
    t[2 * r + 1] = (float)(scale * (snew[p].im - sprev[p].im));
  }
}

// Sigma = Sigma_prev + y / scale at every pair (y: n*n rows of 2)
// Sigma = Sigma_prev + y / scale; with keep_pre the pairs whose contour points
// both lie before the field is switched on (upper-branch indices below a,
// lower-branch indices from b on, every imaginary-branch index) keep Sigma_prev.
__global__ void k_apply(const c64* __restrict__ sprev, const float* __restrict__ y,
                        int n, int a, int b, int keep_pre, double inv_scale,
                        c64* __restrict__ sigma) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const bool pre = keep_pre && (i < a || i >= b) && (j < a || j >= b);
    sigma[e] = pre ? sprev[e]
                   : c64{sprev[e].re + inv_scale * y[2 * e], sprev[e].im + inv_scale * y[2 * e + 1]};
  }
}

}  // namespace fk

// ====================================================================== MLP
struct fk_mlp {
  int d_in = 0, width = 0, depth = 0, d_out = 0;
  std::vector<std::pair<int, int>> shapes;   // (out, in) per layer
  std::vector<size_t> woff, boff;            // offsets of W_l, b_l in params
  size_t np = 0;
  float* p = nullptr;    // params
  float* g = nullptr;    // gradient
  float* m = nullptr;    // Adam moments
  float* v = nullptr;
  long long step = 0;
  // work buffers for a batch of up to cap rows: activations per layer, deltas
  int cap = 0;
  std::vector<float*> h;
  float* d0 = nullptr;
  float* d1 = nullptr;
  float* xs = nullptr;   // gathered minibatch
  float* ts = nullptr;
  double* partial = nullptr;
  hipStream_t st = nullptr;
  std::string err;
};

namespace {
fk_status merr(fk_mlp* a, fk_status s, const char* fmt, ...) {
  if (a) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    a->err = buf;
  }
  return s;
}
#define MCHK(a, expr)                                                       \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return merr((a), e_ == hipErrorOutOfMemory ? FK_ENOMEM : FK_EDEVICE,   \
                  "%s: %s", #expr, hipGetErrorString(e_));                  \
  } while (0)

void free_work(fk_mlp* a) {
  // h[0] is the caller's input (or the gathered minibatch), never owned here
  for (size_t l = 1; l < a->h.size(); ++l)
    if (a->h[l]) (void)hipFree(a->h[l]);
  a->h.clear();
  if (a->d0) (void)hipFree(a->d0);
  if (a->d1) (void)hipFree(a->d1);
  if (a->partial) (void)hipFree(a->partial);
  if (a->xs) (void)hipFree(a->xs);
  if (a->ts) (void)hipFree(a->ts);
  a->xs = a->ts = nullptr;
  a->d0 = a->d1 = nullptr;
  a->partial = nullptr;
  a->cap = 0;
}

fk_status ensure_work(fk_mlp* a, int rows) {
  if (rows <= a->cap) return FK_OK;
  free_work(a);
  a->h.assign(a->depth + 1, nullptr);
  for (int l = 1; l <= a->depth; ++l)
    MCHK(a, hipMalloc(&a->h[l], sizeof(float) * (size_t)rows * a->shapes[l - 1].first));
  const size_t dw = (size_t)std::max(a->width, a->d_out);
  MCHK(a, hipMalloc(&a->d0, sizeof(float) * (size_t)rows * dw));
  MCHK(a, hipMalloc(&a->d1, sizeof(float) * (size_t)rows * dw));
  MCHK(a, hipMalloc(&a->partial, sizeof(double) * 1024));
  MCHK(a, hipMalloc(&a->xs, sizeof(float) * (size_t)rows * a->d_in));
  MCHK(a, hipMalloc(&a->ts, sizeof(float) * (size_t)rows * a->d_out));
  a->cap = rows;
  return FK_OK;
}

// forward pass; activations kept in a->h (h[0] = x, not owned)
hipError_t forward(fk_mlp* a, const float* x, int rows, bool bf16, float* out) {
  a->h[0] = const_cast<float*>(x);
  hipError_t e = hipSuccess;
  for (int l = 0; l < a->depth; ++l) {
    const int o = a->shapes[l].first, in = a->shapes[l].second;
    const float* W = a->p + a->woff[l];
    const float* b = a->p + a->boff[l];
    float* y = (l == a->depth - 1 && out) ? out : a->h[l + 1];
    const bool last = l == a->depth - 1;
    if (bf16)
      e = last ? gemm32<0, 1, 2, 1>(a->h[l], in, W, in, y, o, b, rows, o, in, 0.f, a->st)
               : gemm32<0, 1, 1, 1>(a->h[l], in, W, in, y, o, b, rows, o, in, 0.f, a->st);
    else
      e = last ? gemm32<0, 1, 2, 0>(a->h[l], in, W, in, y, o, b, rows, o, in, 0.f, a->st)
               : gemm32<0, 1, 1, 0>(a->h[l], in, W, in, y, o, b, rows, o, in, 0.f, a->st);
    if (e != hipSuccess) return e;
  }
  return e;
}

// loss and gradient of a batch into a->g; returns the loss in *loss
fk_status loss_grad(fk_mlp* a, const float* x, const float* t, int rows,
                    double* loss) {
  fk_status s = ensure_work(a, rows);
  if (s != FK_OK) return s;
  MCHK(a, forward(a, x, rows, false, nullptr));
  const int L = a->depth;
  const int dout = a->shapes[L - 1].first;
  const size_t ny = (size_t)rows * dout;
  int gb = (int)std::min<size_t>((ny + 255) / 256, 1024);
  hipLaunchKernelGGL(k_mse, dim3(gb), dim3(256), 0, a->st, a->h[L], t, a->d0, ny,
                     1.f / rows, a->partial);
  MCHK(a, hipGetLastError());
  float* d = a->d0;   // delta of the current layer's output (pre-activation)
  float* dn = a->d1;
  for (int l = L - 1; l >= 0; --l) {
    const int o = a->shapes[l].first, in = a->shapes[l].second;
    if (l < L - 1) {
      const size_t n = (size_t)rows * o;
      hipLaunchKernelGGL(k_tanh_back, dim3((int)std::min<size_t>((n + 255) / 256, 4096)),
                         dim3(256), 0, a->st, d, a->h[l + 1], n);
      MCHK(a, hipGetLastError());
    }
    // dW = d^T h_l  (o x in), db = column sums of d
    MCHK(a, (gemm32<1, 0, 0, 0>(d, o, a->h[l], in, a->g + a->woff[l], in, nullptr,
                                o, in, rows, 0.f, a->st)));
    hipLaunchKernelGGL(k_colsum, dim3((o + 255) / 256), dim3(256), 0, a->st, d, rows,
                       o, a->g + a->boff[l]);
    MCHK(a, hipGetLastError());
    if (l > 0) {   // d_{l-1} = d W_l  (rows x in)
      MCHK(a, (gemm32<0, 0, 0, 0>(d, o, a->p + a->woff[l], in, dn, in, nullptr, rows,
                                  in, o, 0.f, a->st)));
      std::swap(d, dn);
    }
  }
  if (loss) {
    std::vector<double> part(gb);
    MCHK(a, hipMemcpyAsync(part.data(), a->partial, sizeof(double) * gb,
                           hipMemcpyDeviceToHost, a->st));
    MCHK(a, hipStreamSynchronize(a->st));
    double sum = 0.0;
    for (double q : part) sum += q;
    *loss = sum / rows;
  }
  return FK_OK;
}
}  // namespace

extern "C" fk_status fk_mlp_create(int d_in, int width, int depth, int d_out,
                                   const float* params, fk_mlp** out) {
  if (d_in < 1 || width < 1 || depth < 2 || d_out < 1 || !params || !out)
    return FK_EINVAL;
  fk_mlp* a = new (std::nothrow) fk_mlp();
  if (!a) return FK_ENOMEM;
  a->d_in = d_in;
  a->width = width;
  a->depth = depth;
  a->d_out = d_out;
  std::vector<int> dims{d_in};
  for (int l = 0; l < depth - 1; ++l) dims.push_back(width);
  dims.push_back(d_out);
  size_t off = 0;
  for (int l = 0; l < depth; ++l) {
    a->shapes.push_back({dims[l + 1], dims[l]});
    a->woff.push_back(off);
    off += (size_t)dims[l + 1] * dims[l];
    a->boff.push_back(off);
    off += dims[l + 1];
  }
  a->np = off;
  hipError_t e = hipStreamCreateWithFlags(&a->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&a->p, sizeof(float) * off);
  if (e == hipSuccess) e = hipMalloc(&a->g, sizeof(float) * off);
  if (e == hipSuccess) e = hipMalloc(&a->m, sizeof(float) * off);
  if (e == hipSuccess) e = hipMalloc(&a->v, sizeof(float) * off);
  if (e == hipSuccess) e = hipMemcpy(a->p, params, sizeof(float) * off, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(a->m, 0, sizeof(float) * off);
  if (e == hipSuccess) e = hipMemset(a->v, 0, sizeof(float) * off);
  if (e != hipSuccess) {
    fk_mlp_destroy(a);
    return e == hipErrorOutOfMemory ? FK_ENOMEM : FK_EDEVICE;
  }
  *out = a;
  return FK_OK;
}

extern "C" fk_status fk_mlp_destroy(fk_mlp* a) {
  if (!a) return FK_OK;
  if (a->st) (void)hipStreamSynchronize(a->st);
  free_work(a);
  float* ps[] = {a->p, a->g, a->m, a->v};
  for (float* q : ps)
    if (q) (void)hipFree(q);
  if (a->st) (void)hipStreamDestroy(a->st);
  delete a;
  return FK_OK;
}

extern "C" const char* fk_mlp_last_error(const fk_mlp* a) {
  return a ? a->err.c_str() : "NULL network";
}

extern "C" fk_status fk_mlp_n_params(const fk_mlp* a, long long* n) {
  if (!a || !n) return FK_EINVAL;
  *n = (long long)a->np;
  return FK_OK;
}

extern "C" fk_status fk_mlp_get_params(const fk_mlp* a, float* params) {
  if (!a || !params) return FK_EINVAL;
  fk_mlp* b = const_cast<fk_mlp*>(a);
  MCHK(b, hipMemcpyAsync(params, a->p, sizeof(float) * a->np, hipMemcpyDeviceToHost, a->st));
  MCHK(b, hipStreamSynchronize(a->st));
  return FK_OK;
}

extern "C" fk_status fk_mlp_set_params(fk_mlp* a, const float* params) {
  if (!a || !params) return FK_EINVAL;
  MCHK(a, hipMemcpyAsync(a->p, params, sizeof(float) * a->np, hipMemcpyHostToDevice, a->st));
  MCHK(a, hipMemsetAsync(a->m, 0, sizeof(float) * a->np, a->st));
  MCHK(a, hipMemsetAsync(a->v, 0, sizeof(float) * a->np, a->st));
  MCHK(a, hipStreamSynchronize(a->st));
  a->step = 0;
  return FK_OK;
}

extern "C" fk_status fk_mlp_forward(fk_mlp* a, const float* x_dev, int rows,
                                    float* y_dev, int bf16) {
  if (!a || !x_dev || !y_dev || rows < 1) return FK_EINVAL;
  // evaluate in slices of at most 65536 rows to bound the work buffers
  const int slice = 65536;
  fk_status s = ensure_work(a, std::min(rows, slice));
  if (s != FK_OK) return s;
  for (int r0 = 0; r0 < rows; r0 += slice) {
    const int nr = std::min(slice, rows - r0);
    MCHK(a, forward(a, x_dev + (size_t)r0 * a->d_in, nr, bf16 != 0,
                    y_dev + (size_t)r0 * a->d_out));
  }
  MCHK(a, hipStreamSynchronize(a->st));
  return FK_OK;
}

extern "C" fk_status fk_mlp_loss_grad(fk_mlp* a, const float* x_dev,
                                      const float* t_dev, int rows, double* loss,
                                      float* grad_host) {
  if (!a || !x_dev || !t_dev || rows < 1) return FK_EINVAL;
  fk_status s = loss_grad(a, x_dev, t_dev, rows, loss);
  if (s != FK_OK) return s;
  if (grad_host) {
    MCHK(a, hipMemcpyAsync(grad_host, a->g, sizeof(float) * a->np, hipMemcpyDeviceToHost,
                           a->st));
  }
  MCHK(a, hipStreamSynchronize(a->st));
  return FK_OK;
}

// Adam steps on minibatches sampled with replacement (see the header).
extern "C" fk_status fk_mlp_train(fk_mlp* a, const float* x_dev, const float* t_dev,
                                  int rows, int batch, int steps, float lr,
                                  unsigned long long seed, double* loss_hist) {
  if (!a || !x_dev || !t_dev || rows < 1 || batch < 1 || steps < 1 || !(lr > 0))
    return FK_EINVAL;
  fk_status st = ensure_work(a, batch);
  if (st != FK_OK) return st;
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(k_gather_rows, dim3(batch), dim3(64), 0, a->st, x_dev, t_dev,
                       (long long)rows, a->d_in, a->d_out, batch, seed, (long long)s,
                       a->xs, a->ts);
    MCHK(a, hipGetLastError());
    double loss = 0.0;
    st = loss_grad(a, a->xs, a->ts, batch, loss_hist ? &loss : nullptr);
    if (st != FK_OK) return st;
    if (loss_hist) loss_hist[s] = loss;
    a->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)a->step), c2 = 1.f - powf(b2, (float)a->step);
    hipLaunchKernelGGL(k_adam, dim3((int)std::min<size_t>((a->np + 255) / 256, 4096)),
                       dim3(256), 0, a->st, a->p, a->g, a->m, a->v, a->np, lr, b1, b2,
                       1e-8f, c1, c2);
    MCHK(a, hipGetLastError());
  }
  MCHK(a, hipStreamSynchronize(a->st));
  return FK_OK;
}

// ============================================================ warm-start I/O
namespace {
fk_status ws_geo(fk_ctx* c, FeatGeo* g, c64** dz) {
  const int n = c->ci.n_c;
  std::vector<c64> z(n);
  for (int j = 0; j < n; ++j) z[j] = c64{c->ci.zr[j], c->ci.zi[j]};
  hipError_t e = hipMalloc(dz, sizeof(c64) * n);
  if (e == hipSuccess) e = hipMemcpy(*dz, z.data(), sizeof(c64) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return FK_EDEVICE;
  g->z = *dz;
  g->n = n;
  g->n_t = c->ci.n_t;
  g->tspan = c->c.t_max - c->c.t_min;
  g->beta = c->c.beta;
  g->E = c->m.E;
  return FK_OK;
}
}  // namespace

namespace {
// Eigenvalues (descending) of a Hermitian r x r matrix given as its real
// symmetric embedding [[Re G, -Im G], [Im G, Re G]] (2r x 2r, every eigenvalue
// twice), by cyclic Jacobi rotations.
std::vector<double> hermitian_eigenvalues(std::vector<double>& a, int r) {
  const int m2 = 2 * r;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < m2; ++p)
      for (int q = 0; q < m2; ++q)
        (p == q ? diag : off) += a[(size_t)p * m2 + q] * a[(size_t)p * m2 + q];
    if (off <= 1e-30 * std::max(diag, 1e-300)) break;
    for (int p = 0; p < m2; ++p)
      for (int q = p + 1; q < m2; ++q) {
        const double apq = a[(size_t)p * m2 + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = (a[(size_t)q * m2 + q] - a[(size_t)p * m2 + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k2 = 0; k2 < m2; ++k2) {   // columns p, q
          const double kp = a[(size_t)k2 * m2 + p], kq = a[(size_t)k2 * m2 + q];
          a[(size_t)k2 * m2 + p] = cs * kp - sn * kq;
          a[(size_t)k2 * m2 + q] = sn * kp + cs * kq;
        }
        for (int k2 = 0; k2 < m2; ++k2) {   // rows p, q
          const double pk = a[(size_t)p * m2 + k2], qk = a[(size_t)q * m2 + k2];
          a[(size_t)p * m2 + k2] = cs * pk - sn * qk;
          a[(size_t)q * m2 + k2] = sn * pk + cs * qk;
        }
      }
  }
  std::vector<double> ev(m2);
  for (int p = 0; p < m2; ++p) ev[p] = a[(size_t)p * m2 + p];
  std::sort(ev.begin(), ev.end(), [](double x, double y) { return x > y; });
  std::vector<double> out(r);
  for (int p = 0; p < r; ++p) out[p] = ev[2 * p];
  return out;
}

// Orthonormalizes the r columns of y (n x r, row-major) in place by modified
// Gram-Schmidt, applied twice; columns that the earlier ones already span (norm
// below 1e-13 of the largest input column) become zero.
void orthonormalize(std::vector<c64>& y, int n, int r) {
  double ymax = 0.0;
  for (int q = 0; q < r; ++q) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const c64 v = y[(size_t)i * r + q];
      s += v.re * v.re + v.im * v.im;
    }
    ymax = std::max(ymax, std::sqrt(s));
  }
  std::vector<char> dead(r, 0);
  for (int pass = 0; pass < 2; ++pass)
    for (int q = 0; q < r; ++q) {
      if (dead[q]) continue;
      for (int p = 0; p < q; ++p) {
        if (dead[p]) continue;
        double cr = 0.0, ci = 0.0;   // <Q_p, y_q> = sum conj(Q_p) y_q
        for (int i = 0; i < n; ++i) {
          const c64 a = y[(size_t)i * r + p], b = y[(size_t)i * r + q];
          cr += a.re * b.re + a.im * b.im;
          ci += a.re * b.im - a.im * b.re;
        }
        for (int i = 0; i < n; ++i) {
          const c64 a = y[(size_t)i * r + p];
          c64& b = y[(size_t)i * r + q];
          b.re -= cr * a.re - ci * a.im;
          b.im -= cr * a.im + ci * a.re;
        }
      }
      double s = 0.0;
      for (int i = 0; i < n; ++i) {
        const c64 v = y[(size_t)i * r + q];
        s += v.re * v.re + v.im * v.im;
      }
      const double nrm = std::sqrt(s);
      if (!(nrm > 1e-13 * ymax)) {
        dead[q] = 1;
        for (int i = 0; i < n; ++i) y[(size_t)i * r + q] = c64{0.0, 0.0};
        continue;
      }
      for (int i = 0; i < n; ++i) {
        y[(size_t)i * r + q].re /= nrm;
        y[(size_t)i * r + q].im /= nrm;
      }
    }
}
}  // namespace

// Randomized SVD of D Sigma D: Y = D Sigma D Omega on the device, Q = an
// orthonormal basis of range(Y) on the host, Z = (D Sigma D)^H Q on the device,
// singular values of B = Z^H = Q^H D Sigma D from the eigenvalues of Z^H Z.
extern "C" fk_status fk_ws_sketch(fk_ctx* c, const double* sigma_dev, int rank,
                                  const double* omega_host, double* sv_out) {
  if (!c || !sigma_dev || rank < 1 || rank > 256 || !omega_host || !sv_out)
    return FK_EINVAL;
  const int n = c->ci.n_c, r = rank;
  const c64* sg = reinterpret_cast<const c64*>(sigma_dev);
  double* om = nullptr;
  c64* y = nullptr;
  c64* qd = nullptr;
  std::vector<c64> yh((size_t)n * r);
  hipError_t e = hipMalloc(&om, sizeof(double) * (size_t)n * r);
  if (e == hipSuccess) e = hipMalloc(&y, sizeof(c64) * (size_t)n * r);
  if (e == hipSuccess) e = hipMalloc(&qd, sizeof(c64) * (size_t)n * r);
  if (e == hipSuccess)
    e = hipMemcpyAsync(om, omega_host, sizeof(double) * (size_t)n * r,
                       hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sketch, dim3(n), dim3(64), 0, c->st, sg, c->d_w, om, n, r, y);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(yh.data(), y, sizeof(c64) * yh.size(), hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e == hipSuccess) {
    orthonormalize(yh, n, r);
    e = hipMemcpyAsync(qd, yh.data(), sizeof(c64) * yh.size(), hipMemcpyHostToDevice, c->st);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sketch_adj, dim3(n), dim3(64), 0, c->st, sg, c->d_w, qd, n, r, y);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(yh.data(), y, sizeof(c64) * yh.size(), hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (om) (void)hipFree(om);
  if (y) (void)hipFree(y);
  if (qd) (void)hipFree(qd);
  if (e != hipSuccess) return FK_EDEVICE;
  // Gram matrix Z^H Z, Hermitian r x r, as its real symmetric embedding
  const int m2 = 2 * r;
  std::vector<double> a((size_t)m2 * m2, 0.0);
  for (int p = 0; p < r; ++p)
    for (int q = 0; q < r; ++q) {
      double sr = 0, si = 0;
      for (int i = 0; i < n; ++i) {
        const c64 u = yh[(size_t)i * r + p], v = yh[(size_t)i * r + q];
        sr += u.re * v.re + u.im * v.im;   // conj(u) v
        si += u.re * v.im - u.im * v.re;
      }
      a[(size_t)p * m2 + q] = sr;
      a[(size_t)(p + r) * m2 + (q + r)] = sr;
      a[(size_t)p * m2 + (q + r)] = -si;
      a[(size_t)(p + r) * m2 + q] = si;
    }
  const std::vector<double> ev = hermitian_eigenvalues(a, r);
  for (int p = 0; p < r; ++p) sv_out[p] = std::sqrt(std::max(ev[p], 0.0));
  return FK_OK;
}

extern "C" fk_status fk_ws_features(fk_ctx* c, const double* sigma_prev_dev,
                                    const float* glob_host, int n_glob,
                                    const long long* idx_dev, long long rows,
                                    double scale, float* x_dev, int d_in) {
  if (!c || !sigma_prev_dev || !x_dev || rows < 1 || n_glob < 0 ||
      d_in < n_glob + kWsFeatures)
    return FK_EINVAL;
  FeatGeo g;
  c64* dz = nullptr;
  float* dg = nullptr;
  if (ws_geo(c, &g, &dz) != FK_OK) return FK_EDEVICE;
  hipError_t e = hipMalloc(&dg, sizeof(float) * std::max(n_glob, 1));
  if (e == hipSuccess && n_glob)
    e = hipMemcpyAsync(dg, glob_host, sizeof(float) * n_glob, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) {
    const int grid = (int)std::min<long long>((rows + 255) / 256, 8192);
    hipLaunchKernelGGL(k_features, dim3(grid), dim3(256), 0, c->st, g,
                       reinterpret_cast<const c64*>(sigma_prev_dev), dg, n_glob,
                       idx_dev, rows, (float)scale, x_dev, d_in);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (dz) (void)hipFree(dz);
  if (dg) (void)hipFree(dg);
  return e == hipSuccess ? FK_OK : FK_EDEVICE;
}

extern "C" fk_status fk_ws_targets(fk_ctx* c, const double* sigma_prev_dev,
                                   const double* sigma_new_dev,
                                   const long long* idx_dev, long long rows,
                                   double scale, float* t_dev) {
  if (!c || !sigma_prev_dev || !sigma_new_dev || !t_dev || rows < 1) return FK_EINVAL;
  const int grid = (int)std::min<long long>((rows + 255) / 256, 8192);
  hipLaunchKernelGGL(k_targets, dim3(grid), dim3(256), 0, c->st,
                     reinterpret_cast<const c64*>(sigma_prev_dev),
                     reinterpret_cast<const c64*>(sigma_new_dev), idx_dev, rows,
                     (long long)c->ci.n_c * c->ci.n_c, (float)scale, t_dev);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  return e == hipSuccess ? FK_OK : FK_EDEVICE;
}

extern "C" fk_status fk_ws_apply(fk_ctx* c, const double* sigma_prev_dev,
                                 const float* y_dev, double scale, int keep_pre_field) {
  if (!c || !sigma_prev_dev || !y_dev || !(scale != 0.0)) return FK_EINVAL;
  const int n = c->ci.n_c, n_t = c->ci.n_t;
  // the branches run t_min -> t_max and back; the field acts from t = 0 on
  // (a small tolerance for the rounding of t_min + j dt at t = 0)
  const double tiny = 1e-9 * c->c.dt;
  int a = 0, b = 2 * n_t;
  while (a < n_t && c->ci.zr[a] <= tiny) ++a;
  while (b > n_t && c->ci.zr[b - 1] <= tiny) --b;
  const size_t total = (size_t)n * n;
  const int grid = (int)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_apply, dim3(grid), dim3(256), 0, c->st,
                     reinterpret_cast<const c64*>(sigma_prev_dev), y_dev, n, a, b,
                     keep_pre_field ? 1 : 0, 1.0 / scale, c->d_sigma);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  return e == hipSuccess ? FK_OK : FK_EDEVICE;
}
