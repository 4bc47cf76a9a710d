// Batched blocked in-place Gauss-Jordan inversion with partial pivoting, for
// gfx950.  This is the hot loop of the lattice step: every (eps, ebar) point
// needs the inverse of the dense complex matrix G0_k^-1 - W Sigma W (the
// "matrix inversion" of the paper's integrand, Sec. II, eq. g_loc).
//
// Algorithm (one step per kNB-column panel, all matrices of the batch in one
// launch):
//   * The panel columns of step s were factored by the previous launch: for
//     each panel column c a pivot row piv[c] was chosen among the rows not yet
//     pivoted (largest |re|+|im|), and the panel now holds the transformed
//     identity columns M = E[:, P] of the elementary Gauss-Jordan transforms.
//   * Every other column stripe (kNB columns, all rows) is owned by one
//     workgroup, which applies the deferred rank-kNB update
//         C <- mask_P(C) + M * B,   B = old values of the pivot rows P,
//     (mask_P zeroes the pivot rows) on the matrix cores (complex product as
//     four real MFMA products), row tile by row tile.
//   * The workgroup that owns the stripe of step s+1 then factors it as the
//     next panel (look-ahead): kIB columns at a time in registers with a
//     workgroup-wide pivot search, the rest of the panel updated through LDS.
// Rows are never swapped: with r = piv and rinv = rowcol, the inverse is
// inv(A)[a][b] = X[r[a]][rinv[b]], which the reduction kernels read directly.
#include "fk_internal.h"

#include <float.h>
#include <limits.h>

namespace fk {

// 16x16x4 matrix-core products.  Operands: lane l holds A[l%16][l/16] and
// B[l/16][l%16].  The accumulator layout differs between the two precisions
// (measured on gfx950): register v of lane l holds D[row][l%16] with
//   f64: row = (l/16) + 4 v      f32: row = 4 (l/16) + v.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int drow(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int drow(int lk, int v) { return 4 * lk + v; }
};

template <typename T> __device__ inline T big_value();
template <> __device__ inline double big_value<double>() { return DBL_MAX; }
template <> __device__ inline float big_value<float>() { return FLT_MAX; }

constexpr int kPitch = kNB + 1;            // padded LDS row (complex elements)
constexpr int kRPT = kMaxN / kThreads;     // panel rows per thread
static_assert(kMaxN % kThreads == 0, "kMaxN must be a multiple of kThreads");

// ---------------------------------------------------------------- update ---
// C <- mask(C) + M B on the stripe [c0, c0+cw) of one matrix, all rows.
template <typename T>
__device__ void update_stripe(cplx<T>* __restrict__ x, int ld, int n,
                              const int* __restrict__ piv,
                              const int* __restrict__ rowcol, int step, int q,
                              unsigned char* smem) {
  typedef typename Mfma<T>::v4 v4;
  cplx<T>* Bs = reinterpret_cast<cplx<T>*>(smem);   // [kNB][kPitch]
  cplx<T>* Ms = Bs + kNB * kPitch;                   // [kTM][kPitch]
  const int tid = threadIdx.x;
  const int j0 = step * kNB;
  const int w = min(kNB, n - j0);
  const int c0 = q * kNB;
  const int cw = min(kNB, n - c0);

  // old pivot rows of this stripe; zero-padded to kNB x kNB.  All loads use
  // clamped (in-range) addresses and are masked afterwards, so that they are
  // issued together instead of one branch-guarded round trip at a time.
  {
    int pr[kNB * kNB / kThreads];
#pragma unroll
    for (int t = 0; t < kNB * kNB / kThreads; ++t) {
      const int l = (tid + t * kThreads) / kNB;
      pr[t] = piv[j0 + min(l, w - 1)];
    }
    cplx<T> bv[kNB * kNB / kThreads];
#pragma unroll
    for (int t = 0; t < kNB * kNB / kThreads; ++t) {
      const int e = tid + t * kThreads;
      const int c = e % kNB;
      bv[t] = x[(size_t)pr[t] * ld + c0 + min(c, cw - 1)];
    }
#pragma unroll
    for (int t = 0; t < kNB * kNB / kThreads; ++t) {
      const int e = tid + t * kThreads;
      const int l = e / kNB, c = e % kNB;
      cplx<T> v = bv[t];
      if (!(l < w && c < cw)) v.re = v.im = T(0);
      Bs[l * kPitch + c] = v;
    }
  }

  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  for (int r0 = 0; r0 < n; r0 += kTM) {
    __syncthreads();  // Bs written / previous Ms consumed
    constexpr int kML = kTM * kNB / kThreads;
    cplx<T> mv[kML];
#pragma unroll
    for (int t = 0; t < kML; ++t) {
      const int e = tid + t * kThreads;
      const int i = e / kNB, l = e % kNB;
      mv[t] = x[(size_t)min(r0 + i, n - 1) * ld + j0 + min(l, w - 1)];
    }
    int rcv[2][4];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v);
        rcv[ii][v] = rowcol[min(row, n - 1)];
      }
    cplx<T> cv[2][2][4];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v);
          const int col = 32 * wc + 16 * jj + li;
          cv[ii][jj][v] = x[(size_t)min(row, n - 1) * ld + c0 + min(col, cw - 1)];
        }
#pragma unroll
    for (int t = 0; t < kML; ++t) {
      const int e = tid + t * kThreads;
      const int i = e / kNB, l = e % kNB;
      cplx<T> v = mv[t];
      if (!(r0 + i < n && l < w)) v.re = v.im = T(0);
      Ms[i * kPitch + l] = v;
    }
    v4 cr[2][2], ci[2][2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v);
          const int col = 32 * wc + 16 * jj + li;
          const int rc = rcv[ii][v];
          const bool keep = row < n && col < cw && !(rc >= j0 && rc < j0 + w);
          cr[ii][jj][v] = keep ? cv[ii][jj][v].re : T(0);
          ci[ii][jj][v] = keep ? cv[ii][jj][v].im : T(0);
        }
    __syncthreads();  // Ms ready
#pragma unroll 4
    for (int k = 0; k < kNB; k += 4) {
      T ar[2], ai[2], an[2], br[2], bi[2];
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const cplx<T> a = Ms[(32 * wr + 16 * ii + li) * kPitch + k + lk];
        ar[ii] = a.re;
        ai[ii] = a.im;
        an[ii] = -a.im;
      }
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const cplx<T> b = Bs[(k + lk) * kPitch + 32 * wc + 16 * jj + li];
        br[jj] = b.re;
        bi[jj] = b.im;
      }
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          cr[ii][jj] = Mfma<T>::run(ar[ii], br[jj], cr[ii][jj]);
          cr[ii][jj] = Mfma<T>::run(an[ii], bi[jj], cr[ii][jj]);
          ci[ii][jj] = Mfma<T>::run(ar[ii], bi[jj], ci[ii][jj]);
          ci[ii][jj] = Mfma<T>::run(ai[ii], br[jj], ci[ii][jj]);
        }
    }
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v);
          const int col = 32 * wc + 16 * jj + li;
          if (row < n && col < cw) {
            cplx<T> c;
            c.re = cr[ii][jj][v];
            c.im = ci[ii][jj][v];
            x[(size_t)row * ld + c0 + col] = c;
          }
        }
  }
}

// ----------------------------------------------------------------- panel ---
template <typename T>
__device__ inline void cmul_sub(cplx<T>& acc, const cplx<T>& a, const cplx<T>& b) {
  acc.re -= a.re * b.re - a.im * b.im;
  acc.im -= a.re * b.im + a.im * b.re;
}
template <typename T>
__device__ inline cplx<T> cmul(const cplx<T>& a, const cplx<T>& b) {
  cplx<T> r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}

// Factor the stripe q (columns [c0, c0+cw), all rows) as a Gauss-Jordan panel.
template <typename T>
__device__ void factor_panel(cplx<T>* __restrict__ x, int ld, int n,
                             int* __restrict__ piv, int* __restrict__ rowcol,
                             int q, int* __restrict__ status,
                             unsigned char* smem) {
  cplx<T>* Mi = reinterpret_cast<cplx<T>*>(smem);   // [kMaxN][kIB]
  cplx<T>* Bo = Mi + kMaxN * kIB;                    // [kIB][kNB]
  cplx<T>* prow = Bo + kIB * kNB;                    // [kIB]
  T* redv = reinterpret_cast<T*>(prow + kIB);        // [4]
  int* redi = reinterpret_cast<int*>(redv + 4);      // [4]
  int* pvt = redi + 4;                               // [kIB]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = q * kNB;
  const int cw = min(kNB, n - c0);
  const T inf_key = big_value<T>();

  bool pvd[kRPT];
#pragma unroll
  for (int i = 0; i < kRPT; ++i) {
    const int r = tid + i * kThreads;
    pvd[i] = (r < n) ? (rowcol[r] >= 0) : true;
  }

  for (int b0 = 0; b0 < cw; b0 += kIB) {
    const int iw = min(kIB, cw - b0);
    cplx<T> v[kRPT][kIB];
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int r = min(tid + i * kThreads, n - 1);
#pragma unroll
      for (int l = 0; l < kIB; ++l)
        v[i][l] = x[(size_t)r * ld + c0 + b0 + min(l, iw - 1)];
    }
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int r = tid + i * kThreads;
#pragma unroll
      for (int l = 0; l < kIB; ++l)
        if (!(r < n && l < iw)) v[i][l].re = v[i][l].im = T(0);
    }
#pragma unroll
    for (int l = 0; l < kIB; ++l) {
      if (l >= iw) break;
      // ---- pivot search: largest |re|+|im| among unpivoted rows
      T best = T(-1);
      int bidx = INT_MAX;
#pragma unroll
      for (int i = 0; i < kRPT; ++i) {
        const int r = tid + i * kThreads;
        if (r < n && !pvd[i]) {
          T a = fabs(v[i][l].re) + fabs(v[i][l].im);
          if (!(a <= inf_key)) a = inf_key;  // NaN / Inf win and get flagged
          if (a > best || (a == best && r < bidx)) {
            best = a;
            bidx = r;
          }
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const T ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bidx, off);
        if (ob > best || (ob == best && oi < bidx)) {
          best = ob;
          bidx = oi;
        }
      }
      if (lane == 0) {
        redv[wave] = best;
        redi[wave] = bidx;
      }
      __syncthreads();
      best = redv[0];
      bidx = redi[0];
#pragma unroll
      for (int wv = 1; wv < kThreads / 64; ++wv) {
        const T ob = redv[wv];
        const int oi = redi[wv];
        if (ob > best || (ob == best && oi < bidx)) {
          best = ob;
          bidx = oi;
        }
      }
      const int p = bidx;  // always a valid unpivoted row: fewer than n pivots so far
      const int col = c0 + b0 + l;
      if (tid == 0 && (best == T(0) || best == inf_key))
        atomicCAS(status, 0, best == T(0) ? (1 + col) : -(1 + col));
      if ((p % kThreads) == tid) {
        const int i = p / kThreads;
#pragma unroll
        for (int ii = 0; ii < kRPT; ++ii)
          if (ii == i) {
#pragma unroll
            for (int l2 = 0; l2 < kIB; ++l2) prow[l2] = v[ii][l2];
            pvd[ii] = true;
          }
        piv[col] = p;
        rowcol[p] = col;
        pvt[l] = p;
      }
      __syncthreads();
      // ---- eliminate column l from every other row (Gauss-Jordan)
      const cplx<T> pv = prow[l];
      const T den = pv.re * pv.re + pv.im * pv.im;
      cplx<T> inv;
      inv.re = pv.re / den;
      inv.im = -pv.im / den;
      cplx<T> ps[kIB];
#pragma unroll
      for (int l2 = 0; l2 < kIB; ++l2) ps[l2] = cmul(prow[l2], inv);
      ps[l] = inv;
#pragma unroll
      for (int i = 0; i < kRPT; ++i) {
        const int r = tid + i * kThreads;
        if (r < n) {
          if (r == p) {
#pragma unroll
            for (int l2 = 0; l2 < kIB; ++l2) v[i][l2] = ps[l2];
          } else {
            const cplx<T> m = v[i][l];
#pragma unroll
            for (int l2 = 0; l2 < kIB; ++l2)
              if (l2 != l) cmul_sub(v[i][l2], m, ps[l2]);
            cplx<T> nm = cmul(m, inv);
            nm.re = -nm.re;
            nm.im = -nm.im;
            v[i][l] = nm;
          }
        }
      }
      __syncthreads();  // redv / prow reused by the next column
    }
    // ---- inner block done: write it back and keep it in LDS
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int r = tid + i * kThreads;
      if (r < n) {
#pragma unroll
        for (int l = 0; l < kIB; ++l) {
          if (l < iw) x[(size_t)r * ld + c0 + b0 + l] = v[i][l];
          Mi[r * kIB + l] = v[i][l];  // zero beyond iw
        }
      }
    }
    // old values of this block's pivot rows in the other panel columns
    for (int e = tid; e < kIB * kNB; e += kThreads) {
      const int l = e / kNB, c = e - (e / kNB) * kNB;
      cplx<T> t = {T(0), T(0)};
      if (l < iw && c < cw && (c < b0 || c >= b0 + iw))
        t = x[(size_t)pvt[l] * ld + c0 + c];
      Bo[e] = t;
    }
    __syncthreads();
    // rank-iw update of the other panel columns (row-major, coalesced); the
    // loads of kBat elements are issued before any of them is stored.
    constexpr int kBat = 8;
    const int total = n * cw;
    int pv0[kIB];
#pragma unroll
    for (int l = 0; l < kIB; ++l) pv0[l] = (l < iw) ? pvt[l] : -1;
    for (int e0 = tid; e0 < total; e0 += kThreads * kBat) {
      cplx<T> old[kBat];
#pragma unroll
      for (int b = 0; b < kBat; ++b) {
        const int e = min(e0 + b * kThreads, total - 1);
        const int r = e / cw, c = e - (e / cw) * cw;
        old[b] = x[(size_t)r * ld + c0 + c];
      }
#pragma unroll
      for (int b = 0; b < kBat; ++b) {
        const int e = e0 + b * kThreads;
        if (e >= total) break;
        const int r = e / cw, c = e - (e / cw) * cw;
        if (c >= b0 && c < b0 + iw) continue;
        bool isp = false;
#pragma unroll
        for (int l = 0; l < kIB; ++l) isp |= (pv0[l] == r);
        cplx<T> acc = old[b];
        if (isp) acc.re = acc.im = T(0);
#pragma unroll
        for (int l = 0; l < kIB; ++l) {
          const cplx<T> mm = Mi[r * kIB + l];
          const cplx<T> bb = Bo[l * kNB + c];
          acc.re += mm.re * bb.re - mm.im * bb.im;
          acc.im += mm.re * bb.im + mm.im * bb.re;
        }
        x[(size_t)r * ld + c0 + c] = acc;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- kernel ---
// Work items are split into 8 contiguous chunks, one per XCD (workgroups are
// dispatched round-robin over the 8 XCDs), so the stripes of one matrix share
// that XCD's L2 when they read the panel.
template <typename T>
__global__ __launch_bounds__(kThreads, 1) void gje_step_kernel(
    cplx<T>* __restrict__ xbuf, int* __restrict__ pivbuf,
    int* __restrict__ rowcolbuf, const MatDesc* __restrict__ descs,
    const WorkItem* __restrict__ items, int nitems, int step,
    int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per = gridDim.x >> 3;
  const int chunk = (nitems + 7) >> 3;
  const int lo = xcd * chunk;
  const int hi = min(nitems, lo + chunk);
  for (int it = lo + slot; it < hi; it += per) {
    const WorkItem wi = items[it];
    const MatDesc d = descs[wi.mat];
    cplx<T>* x = xbuf + d.xoff;
    int* piv = pivbuf + d.ioff;
    int* rowcol = rowcolbuf + d.ioff;
    if (step >= 0 && wi.stripe != step)
      update_stripe<T>(x, d.ld, d.n, piv, rowcol, step, wi.stripe, smem);
    if (wi.stripe == step + 1 && wi.stripe * kNB < d.n) {
      __syncthreads();
      factor_panel<T>(x, d.ld, d.n, piv, rowcol, wi.stripe,
                      status + d.status_idx, smem);
    }
    __syncthreads();
  }
}

template <typename T> size_t gje_lds_bytes() {
  const size_t upd = sizeof(cplx<T>) * (size_t)(kNB + kTM) * kPitch;
  const size_t pan = sizeof(cplx<T>) * ((size_t)kMaxN * kIB + kIB * kNB + kIB) +
                     4 * sizeof(T) + 4 * sizeof(int) + kIB * sizeof(int);
  return upd > pan ? upd : pan;
}

template <typename T>
hipError_t gje_step(cplx<T>* xbuf, int* pivbuf, int* rowcolbuf,
                    const MatDesc* descs, const WorkItem* items, int nitems,
                    int step, int* status, int grid, hipStream_t st) {
  static bool attr_set = false;
  const size_t lds = gje_lds_bytes<T>();
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&gje_step_kernel<T>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (nitems <= 0) return hipSuccess;
  if (grid <= 0 || (grid & 7)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gje_step_kernel<T>, dim3(grid), dim3(kThreads), lds, st,
                     xbuf, pivbuf, rowcolbuf, descs, items, nitems, step,
                     status);
  return hipGetLastError();
}

template hipError_t gje_step<double>(c64*, int*, int*, const MatDesc*,
                                     const WorkItem*, int, int, int*, int,
                                     hipStream_t);
template hipError_t gje_step<float>(c32*, int*, int*, const MatDesc*,
                                    const WorkItem*, int, int, int*, int,
                                    hipStream_t);
template size_t gje_lds_bytes<double>();
template size_t gje_lds_bytes<float>();

}  // namespace fk
