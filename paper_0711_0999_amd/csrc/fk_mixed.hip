// FP64 iterative refinement of complex64 inverses (gfx950).
//
// With X ~ A^-1 from the complex64 Gauss-Jordan inversion of A = G0^-1 - W
// Sigma W, one refinement step is Newton's step for the inverse
//     R = I - A X  (FP64),     X <- X + X R  (FP64),
// which squares the relative error.  A X = T X - Sigma_t X with T = G0^-1 the
// bidiagonal-plus-corner matrix, so the residual costs one dense complex GEMM
// with the shared left operand Sigma_t plus an O(N^2) sparse product, and the
// correction one more dense GEMM.
#include "fk_internal.h"
#include "fk_kernels.h"

namespace fk {

typedef double v4d __attribute__((ext_vector_type(4)));

// out[m][a][b] = X[m][piv_m[a]][rowcol_m[b]] in FP64 (undo the logical pivoting)
template <typename TI>
__global__ void k_unpermute(const cplx<TI>* __restrict__ x, size_t xstride,
                            int ld, const int* __restrict__ piv,
                            const int* __restrict__ rowcol, int n,
                            c64* __restrict__ out) {
  const int m = blockIdx.z, a = blockIdx.y;
  const int r = piv[(size_t)m * n + a];
  const cplx<TI>* src = x + (size_t)m * xstride + (size_t)r * ld;
  c64* dst = out + (size_t)m * n * n + (size_t)a * n;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n;
       b += gridDim.x * blockDim.x) {
    const cplx<TI> v = src[rowcol[(size_t)m * n + b]];
    dst[b] = c64{(double)v.re, (double)v.im};
  }
}

// C[m] = beta Cin[m] + A[m] B[m] for n x n complex128 matrices (leading
// dimension n).  sA = 0 shares A across the batch.  64 x 64 tiles, 2 x 2 waves
// of 32 x 32, K in double-buffered chunks of 16, f64 matrix cores, three real
// products per complex one (Gauss: Re = P1 - P2, Im = P3 - P1 - P2 with
// P1 = Re a Re b, P2 = Im a Im b, P3 = (Re a + Im a)(Re b + Im b)).
constexpr int kGT = 64, kGK = 16;
__global__ __launch_bounds__(256, 2) void k_bgemm(
    c64* __restrict__ C, const c64* __restrict__ Cin, double beta,
    const c64* __restrict__ A, size_t sA, const c64* __restrict__ B, int n,
    int nmat) {
  constexpr int AP = kGK + 1, BP = kGT + 1;
  __shared__ c64 As[2][kGT * AP];
  __shared__ c64 Bs[2][kGK * BP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  const int nt = (n + kGT - 1) / kGT;
  const int per_m = nt * nt;
  const int nitems = per_m * nmat;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
  const int chunk = (nitems + 7) >> 3;
  const int lo = xcd * chunk, hi = min(nitems, lo + chunk);
  const size_t ss = (size_t)n * n;
  const int nch = (n + kGK - 1) / kGK;
  for (int it = lo + slot; it < hi; it += per) {
    const int m = it / per_m, t = it - (it / per_m) * per_m;
    const int tc = t / nt, tr = t - (t / nt) * nt;
    const int r0 = tr * kGT, c0 = tc * kGT;
    const c64* am = A + sA * m;
    const c64* bm = B + ss * m;
    v4d p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          p1[ii][jj][v] = 0.0;
          p2[ii][jj][v] = 0.0;
          p3[ii][jj][v] = 0.0;
        }
    c64 pa[4], pb[4];
    auto load = [&](int kb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + q * 256;
        const int i = e / kGK, k = e % kGK;
        pa[q] = am[(size_t)min(r0 + i, n - 1) * n + min(kb + k, n - 1)];
        const int kk = e / kGT, c = e % kGT;
        pb[q] = bm[(size_t)min(kb + kk, n - 1) * n + min(c0 + c, n - 1)];
      }
    };
    auto stash = [&](int buf, int kb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + q * 256;
        const int i = e / kGK, k = e % kGK;
        c64 a = pa[q];
        if (!(r0 + i < n && kb + k < n)) a = c64{0.0, 0.0};
        As[buf][i * AP + k] = a;
        const int kk = e / kGT, c = e % kGT;
        c64 b = pb[q];
        if (!(kb + kk < n && c0 + c < n)) b = c64{0.0, 0.0};
        Bs[buf][kk * BP + c] = b;
      }
    };
    load(0);
    stash(0, 0);
    __syncthreads();
    for (int kc = 0; kc < nch; ++kc) {
      const int buf = kc & 1;
      const bool more = kc + 1 < nch;
      if (more) load((kc + 1) * kGK);
#pragma unroll
      for (int k = 0; k < kGK; k += 4) {
        double ar[2], ai[2], as_[2], br[2], bi[2], bs_[2];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
          const c64 a = As[buf][(32 * wr + 16 * ii + li) * AP + k + lk];
          ar[ii] = a.re;
          ai[ii] = a.im;
          as_[ii] = a.re + a.im;
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const c64 b = Bs[buf][(k + lk) * BP + 32 * wc + 16 * jj + li];
          br[jj] = b.re;
          bi[jj] = b.im;
          bs_[jj] = b.re + b.im;
        }
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            p1[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ii], br[jj], p1[ii][jj], 0, 0, 0);
            p2[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[ii], bi[jj], p2[ii][jj], 0, 0, 0);
            p3[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(as_[ii], bs_[jj], p3[ii][jj], 0, 0, 0);
          }
      }
      if (more) stash(buf ^ 1, (kc + 1) * kGK);
      __syncthreads();
    }
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 32 * wr + 16 * ii + lk + 4 * v;  // f64 layout
          const int col = c0 + 32 * wc + 16 * jj + li;
          if (row < n && col < n) {
            const size_t e = ss * m + (size_t)row * n + col;
            c64 c{0.0, 0.0};
            if (beta != 0.0) c = Cin[e];
            const double q1 = p1[ii][jj][v], q2 = p2[ii][jj][v];
            C[e] = c64{(q1 - q2) + beta * c.re, ((p3[ii][jj][v] - q1) - q2) + beta * c.im};
          }
        }
  }
}

// R = I - T X + P in place of P (P = Sigma_t X), T = i I + sub-diagonal tsub
// + corner tcor at (0, n-1); running max |R| into key.
__global__ void k_residual(c64* __restrict__ P, const c64* __restrict__ X,
                           const c64* __restrict__ tsub,
                           const c64* __restrict__ tcor, int n, int nmat,
                           unsigned long long* __restrict__ key) {
  const size_t ss = (size_t)n * n, total = ss * nmat;
  double mx = 0.0;
  bool bad = false;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / ss);
    const size_t f = e - (size_t)m * ss;
    const int i = (int)(f / n), j = (int)(f - (f / n) * n);
    const c64* xm = X + ss * m;
    const c64 xv = xm[f];
    c64 tx{-xv.im, xv.re};  // i * X[i][j]
    const c64 t = (i >= 1) ? tsub[(size_t)m * n + i] : tcor[m];
    const c64 xo = xm[(size_t)((i >= 1) ? i - 1 : n - 1) * n + j];
    tx.re += t.re * xo.re - t.im * xo.im;
    tx.im += t.re * xo.im + t.im * xo.re;
    c64 r = P[e];
    r.re += (i == j ? 1.0 : 0.0) - tx.re;
    r.im -= tx.im;
    P[e] = r;
    const double a = sqrt(r.re * r.re + r.im * r.im);
    if (!(a <= 1.79769313486231570815e308)) bad = true;
    else if (a > mx) mx = a;
  }
  unsigned long long k = bad ? 0x7ff8000000000000ULL
                             : (unsigned long long)__double_as_longlong(mx);
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(k, off);
    k = o > k ? o : k;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(key, k);
}

template <typename TI>
hipError_t launch_unpermute(const cplx<TI>* x, size_t xstride, int ld,
                            const int* piv, const int* rowcol, int n, int nmat,
                            c64* out, hipStream_t st) {
  hipLaunchKernelGGL(k_unpermute<TI>, dim3((n + 255) / 256, n, nmat), dim3(256),
                     0, st, x, xstride, ld, piv, rowcol, n, out);
  return hipGetLastError();
}

hipError_t launch_bgemm(c64* C, const c64* Cin, double beta, const c64* A,
                        size_t sA, const c64* B, int n, int nmat,
                        hipStream_t st) {
  const int nt = (n + kGT - 1) / kGT;
  const long long items = (long long)nt * nt * nmat;
  const int grid = (int)(8 * ((items + 7) / 8));
  hipLaunchKernelGGL(k_bgemm, dim3(grid), dim3(256), 0, st, C, Cin, beta, A,
                     sA, B, n, nmat);
  return hipGetLastError();
}

hipError_t launch_residual(c64* P, const c64* X, const c64* tsub,
                           const c64* tcor, int n, int nmat,
                           unsigned long long* key, hipStream_t st) {
  size_t g = ((size_t)n * n * nmat + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_residual, dim3((int)g), dim3(256), 0, st, P, X, tsub,
                     tcor, n, nmat, key);
  return hipGetLastError();
}

template hipError_t launch_unpermute<float>(const c32*, size_t, int, const int*,
                                            const int*, int, int, c64*,
                                            hipStream_t);
template hipError_t launch_unpermute<double>(const c64*, size_t, int,
                                             const int*, const int*, int, int,
                                             c64*, hipStream_t);

}  // namespace fk
