// Batched blocked in-place Gauss-Jordan inversion with partial pivoting, for
// gfx950.  This is the hot loop of the lattice step: every (eps, ebar) point
// needs the inverse of the dense complex matrix G0_k^-1 - W Sigma W (the
// "matrix inversion" of the integrand of eq. g_loc, Sec. II).
//
// Outer step S handles the block of kNBO = 128 columns starting at J0 = S*kNBO:
//   panel   (one 512-thread workgroup per matrix) eliminates the block's two
//           64-column inner panels in turn.  For each column the pivot is the
//           largest |re|+|im| among the rows not yet pivoted; kIB columns are
//           eliminated in registers at a time, the rest of the inner panel is
//           updated in coalesced passes, and the other inner panel receives
//           the rank-64 transform on the matrix cores.  Afterwards the block
//           holds the transformed identity columns M = E[:, P] of all
//           elementary Gauss-Jordan transforms of the step.
//   gather  copies the pivot rows P of the step (their values before the
//           step) into a side buffer B.
//   update  every other column tile: C <- mask_P(C) + M B (K = 128), a batched
//           complex GEMM on the matrix cores (four real products per complex
//           one), double-buffered K chunks in LDS, two workgroups per CU.
// The host runs the update of the next block's columns first and factors that
// block on a second stream while the big update of the current step runs.
// Rows are never swapped: with r = piv and rinv = rowcol the inverse is
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

template <typename T>
__device__ inline cplx<T> cmul(const cplx<T>& a, const cplx<T>& b) {
  cplx<T> r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
template <typename T>
__device__ inline void cfma(cplx<T>& acc, const cplx<T>& a, const cplx<T>& b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}

constexpr int kPW = kPanelThreads / 64;          // waves of the panel kernel
constexpr int kRPT = kMaxN / kPanelThreads;      // panel rows per thread
constexpr int kPitch = kNB + 1;                  // padded LDS row (elements)
static_assert(kMaxN % kPanelThreads == 0, "kMaxN");
static_assert(kNBO == 2 * kNB && kTile == kNB, "block sizes");

// ------------------------------------------------------ panel: inner update
// C <- mask(C) + M B on the 64-column stripe q of one matrix, with M the
// columns of inner panel p (already eliminated) and B the old values of p's
// pivot rows in stripe q (read before any write: this workgroup owns q).
// The kPW waves form (kPW/4) x 4 blocks of (16 kRB) x 16 over each 64 x 64 tile.
constexpr int kRB = kTile / (16 * (kPW / 4));   // 16-row blocks per wave
static_assert(kPW % 4 == 0 && kRB >= 1, "panel waves");
template <typename T>
__device__ __forceinline__ void inner_update(cplx<T>* __restrict__ x, int ld, int n,
                             const int* __restrict__ piv,
                             const int* __restrict__ rowcol, int p, int q,
                             unsigned char* smem) {
  typedef typename Mfma<T>::v4 v4;
  cplx<T>* Bs = reinterpret_cast<cplx<T>*>(smem);   // [kNB][kPitch]
  cplx<T>* Ms = Bs + kNB * kPitch;                   // [kTile][kPitch]
  const int tid = threadIdx.x;
  const int j0 = p * kNB, w = min(kNB, n - j0);
  const int c0 = q * kNB, cw = min(kNB, n - c0);
  constexpr int kL = kNB * kNB / kPanelThreads;     // elements per thread
  {
    int pr[kL];
    cplx<T> bv[kL];
#pragma unroll
    for (int t = 0; t < kL; ++t) {
      const int l = (tid + t * kPanelThreads) / kNB;
      pr[t] = piv[j0 + min(l, w - 1)];
    }
#pragma unroll
    for (int t = 0; t < kL; ++t) {
      const int c = (tid + t * kPanelThreads) % kNB;
      bv[t] = x[(size_t)pr[t] * ld + c0 + min(c, cw - 1)];
    }
#pragma unroll
    for (int t = 0; t < kL; ++t) {
      const int e = tid + t * kPanelThreads;
      const int l = e / kNB, c = e % kNB;
      cplx<T> v = bv[t];
      if (!(l < w && c < cw)) v.re = v.im = T(0);
      Bs[l * kPitch + c] = v;
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int li = lane & 15, lk = lane >> 4;
  const int col = 16 * wc + li;
  for (int r0 = 0; r0 < n; r0 += kTile) {
    __syncthreads();
    cplx<T> mv[kL];
#pragma unroll
    for (int t = 0; t < kL; ++t) {
      const int e = tid + t * kPanelThreads;
      const int i = e / kNB, l = e % kNB;
      mv[t] = x[(size_t)min(r0 + i, n - 1) * ld + j0 + min(l, w - 1)];
    }
    int rcv[kRB][4];
    cplx<T> cv[kRB][4];
#pragma unroll
    for (int ii = 0; ii < kRB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * (kRB * wr + ii) + Mfma<T>::drow(lk, v);
        rcv[ii][v] = rowcol[min(row, n - 1)];
        cv[ii][v] = x[(size_t)min(row, n - 1) * ld + c0 + min(col, cw - 1)];
      }
#pragma unroll
    for (int t = 0; t < kL; ++t) {
      const int e = tid + t * kPanelThreads;
      const int i = e / kNB, l = e % kNB;
      cplx<T> v = mv[t];
      if (!(r0 + i < n && l < w)) v.re = v.im = T(0);
      Ms[i * kPitch + l] = v;
    }
    v4 cr[kRB], ci[kRB];
#pragma unroll
    for (int ii = 0; ii < kRB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * (kRB * wr + ii) + Mfma<T>::drow(lk, v);
        const bool keep = row < n && col < cw &&
                          !(rcv[ii][v] >= j0 && rcv[ii][v] < j0 + w);
        cr[ii][v] = keep ? cv[ii][v].re : T(0);
        ci[ii][v] = keep ? cv[ii][v].im : T(0);
      }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kNB; k += 4) {
      const cplx<T> b = Bs[(k + lk) * kPitch + col];
#pragma unroll
      for (int ii = 0; ii < kRB; ++ii) {
        const cplx<T> a = Ms[(16 * (kRB * wr + ii) + li) * kPitch + k + lk];
        cr[ii] = Mfma<T>::run(a.re, b.re, cr[ii]);
        ci[ii] = Mfma<T>::run(a.re, b.im, ci[ii]);
        cr[ii] = Mfma<T>::run(-a.im, b.im, cr[ii]);
        ci[ii] = Mfma<T>::run(a.im, b.re, ci[ii]);
      }
    }
#pragma unroll
    for (int ii = 0; ii < kRB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * (kRB * wr + ii) + Mfma<T>::drow(lk, v);
        if (row < n && col < cw) {
          cplx<T> c;
          c.re = cr[ii][v];
          c.im = ci[ii][v];
          x[(size_t)row * ld + c0 + col] = c;
        }
      }
  }
}

// Column groups updated per batch of loads in the panel's rank-kIB updates
// (bounded by registers: kIB complex values per group).
template <typename T> struct GroupBatch { static constexpr int value = 4; };
template <> struct GroupBatch<float> { static constexpr int value = 7; };

// ---------------------------------------------------- panel: factorization
// Eliminate the columns of inner panel q (all rows) with partial pivoting.
template <typename T>
__device__ __forceinline__ void factor_panel(cplx<T>* __restrict__ x, int ld, int n,
                             int* __restrict__ piv, int* __restrict__ rowcol,
                             int q, int* __restrict__ status,
                             unsigned char* smem) {
  cplx<T>* Bo = reinterpret_cast<cplx<T>*>(smem);   // [kIB][kNB]
  cplx<T>* prow = Bo + kIB * kNB;                    // [kIB]
  T* redv = reinterpret_cast<T*>(prow + kIB);        // [kPW]
  int* redi = reinterpret_cast<int*>(redv + kPW);    // [kPW]
  int* pvt = redi + kPW;                             // [kIB]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = q * kNB, cw = min(kNB, n - c0);
  const T inf_key = big_value<T>();
  constexpr int kGB = GroupBatch<T>::value;

  bool pvd[kRPT];
#pragma unroll
  for (int i = 0; i < kRPT; ++i) {
    const int r = tid + i * kPanelThreads;
    pvd[i] = (r < n) ? (rowcol[min(r, n - 1)] >= 0) : true;
  }
  const int ngroups = (cw + kIB - 1) / kIB;

  for (int b0 = 0; b0 < cw; b0 += kIB) {
    const int iw = min(kIB, cw - b0);
    cplx<T> v[kRPT][kIB];
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int r = min(tid + i * kPanelThreads, n - 1);
#pragma unroll
      for (int l = 0; l < kIB; ++l)
        v[i][l] = x[(size_t)r * ld + c0 + b0 + min(l, iw - 1)];
    }
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int r = tid + i * kPanelThreads;
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
        const int r = tid + i * kPanelThreads;
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
      for (int wv = 1; wv < kPW; ++wv) {
        const T ob = redv[wv];
        const int oi = redi[wv];
        if (ob > best || (ob == best && oi < bidx)) {
          best = ob;
          bidx = oi;
        }
      }
      const int p = bidx;  // a valid unpivoted row: fewer than n pivots so far
      const int col = c0 + b0 + l;
      if (tid == 0 && (best == T(0) || best == inf_key))
        atomicCAS(status, 0, best == T(0) ? (1 + col) : -(1 + col));
      if ((p % kPanelThreads) == tid) {
        const int i = p / kPanelThreads;
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
        const int r = tid + i * kPanelThreads;
        if (r == p) {
#pragma unroll
          for (int l2 = 0; l2 < kIB; ++l2) v[i][l2] = ps[l2];
        } else {
          const cplx<T> m = v[i][l];
#pragma unroll
          for (int l2 = 0; l2 < kIB; ++l2)
            if (l2 != l) {
              v[i][l2].re -= m.re * ps[l2].re - m.im * ps[l2].im;
              v[i][l2].im -= m.re * ps[l2].im + m.im * ps[l2].re;
            }
          const cplx<T> nm = cmul(m, inv);
          v[i][l].re = -nm.re;
          v[i][l].im = -nm.im;
        }
      }
      __syncthreads();  // redv / prow reused by the next column
    }
    // ---- write the eliminated block back; old pivot rows of the other columns
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int r = tid + i * kPanelThreads;
      if (r < n) {
#pragma unroll
        for (int l = 0; l < kIB; ++l)
          if (l < iw) x[(size_t)r * ld + c0 + b0 + l] = v[i][l];
      }
    }
    for (int e = tid; e < kIB * kNB; e += kPanelThreads) {
      const int l = e / kNB, c = e % kNB;
      const bool ok = l < iw && c < cw && (c < b0 || c >= b0 + iw);
      cplx<T> t = x[(size_t)pvt[min(l, iw - 1)] * ld + c0 + min(c, cw - 1)];
      if (!ok) t.re = t.im = T(0);
      Bo[e] = t;
    }
    __syncthreads();
    // ---- rank-iw update of the other column groups of the panel on the rows
    // this thread owns and has just written: each row's eliminated values are
    // read back once (same thread, program order) and applied to every other
    // group of the row.
    const int cur = b0 / kIB;
    int pv0[kIB];
#pragma unroll
    for (int l = 0; l < kIB; ++l) pv0[l] = (l < iw) ? pvt[l] : -1;
#pragma unroll 1
    for (int i = 0; i < kRPT; ++i) {
      const int r = tid + i * kPanelThreads;
      if (r >= n) continue;
      bool isp = false;
#pragma unroll
      for (int l = 0; l < kIB; ++l) isp |= (pv0[l] == r);
      cplx<T> mm[kIB];
#pragma unroll
      for (int l = 0; l < kIB; ++l) mm[l] = x[(size_t)r * ld + c0 + b0 + min(l, iw - 1)];
      // the other groups in batches of kGB whose loads are all in flight
      // together (a group index past the panel reads the current group and
      // stores nothing)
#pragma unroll 1
      for (int q0 = 0; q0 < kNB / kIB - 1; q0 += kGB) {
        cplx<T> od[kGB][kIB];
        int cgs[kGB], gws[kGB];
        bool ok[kGB];
#pragma unroll
        for (int q = 0; q < kGB; ++q) {
          int g = q0 + q;
          g += (g >= cur) ? 1 : 0;
          ok[q] = (q0 + q < kNB / kIB - 1) && g < ngroups;
          cgs[q] = (ok[q] ? g : cur) * kIB;
          gws[q] = min(kIB, cw - cgs[q]);
#pragma unroll
          for (int cc = 0; cc < kIB; ++cc)
            od[q][cc] = x[(size_t)r * ld + c0 + cgs[q] + min(cc, gws[q] - 1)];
        }
#pragma unroll
        for (int q = 0; q < kGB; ++q) {
          if (!ok[q]) continue;
#pragma unroll
          for (int cc = 0; cc < kIB; ++cc) {
            cplx<T> acc = od[q][cc];
            if (isp) acc.re = acc.im = T(0);
#pragma unroll
            for (int l = 0; l < kIB; ++l)
              if (l < iw) cfma(acc, mm[l], Bo[l * kNB + cgs[q] + cc]);
            if (cc < gws[q]) x[(size_t)r * ld + c0 + cgs[q] + cc] = acc;
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kPanelThreads, 1) void k_outer_panel(
    cplx<T>* __restrict__ xbuf, int* __restrict__ pivbuf,
    int* __restrict__ rowcolbuf, const MatDesc* __restrict__ descs, int S,
    int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  const MatDesc d = descs[blockIdx.x];
  const int n = d.n;
  if (S * kNBO >= n) return;
  cplx<T>* x = xbuf + d.xoff;
  int* piv = pivbuf + d.ioff;
  int* rowcol = rowcolbuf + d.ioff;
  int* st = status + d.status_idx;
  const int p0 = 2 * S, p1 = 2 * S + 1;
  factor_panel<T>(x, d.ld, n, piv, rowcol, p0, st, smem);
  if (p1 * kNB < n) {
    __syncthreads();
    inner_update<T>(x, d.ld, n, piv, rowcol, p0, p1, smem);
    __syncthreads();
    factor_panel<T>(x, d.ld, n, piv, rowcol, p1, st, smem);
    __syncthreads();
    inner_update<T>(x, d.ld, n, piv, rowcol, p1, p0, smem);
  }
}

// ------------------------------------------------------------------ gather
template <typename T>
__global__ void k_gather(const cplx<T>* __restrict__ xbuf,
                         cplx<T>* __restrict__ bbuf,
                         const int* __restrict__ pivbuf,
                         const MatDesc* __restrict__ descs, int S) {
  const MatDesc d = descs[blockIdx.y];
  const int l = blockIdx.x;
  const int J0 = S * kNBO;
  if (J0 >= d.n || l >= min(kNBO, d.n - J0)) return;
  const int p = pivbuf[d.ioff + J0 + l];
  const cplx<T>* src = xbuf + d.xoff + (size_t)p * d.ld;
  cplx<T>* dst = bbuf + d.boff + (size_t)l * d.ld;
  for (int c = threadIdx.x; c < d.n; c += blockDim.x) dst[c] = src[c];
}

// ------------------------------------------------------------------ update
// C <- mask_P(C) + M B for the listed tiles of (32 WR) x 64: 2 WR waves as
// WR x 2 blocks of 32 x 32 (WR = 2: 64 x 64 tiles, two workgroups per CU;
// WR = 4: 128 x 64 tiles sharing each B chunk, one workgroup per CU).  K in
// chunks of kKC, double-buffered through LDS with the next chunk's global
// loads in flight during the current chunk's MFMAs.
template <typename T, int WR>
__global__ __launch_bounds__(128 * WR, 4 / WR) void k_update(
    cplx<T>* __restrict__ xbuf, const cplx<T>* __restrict__ bbuf,
    const int* __restrict__ rowcolbuf, const MatDesc* __restrict__ descs,
    const TileItem* __restrict__ items, int nitems, int S) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int TR = 32 * WR, NT = 128 * WR;
  constexpr int AP = kKC + 1, BP = kTile + 1;
  __shared__ cplx<T> As[2][TR * AP];
  __shared__ cplx<T> Bsh[2][kKC * BP];
  constexpr int kLA = TR * kKC / NT;      // chunk loads per thread
  constexpr int kLB = kKC * kTile / NT;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per = gridDim.x >> 3;
  const int chunk = (nitems + 7) >> 3;
  const int lo = xcd * chunk, hi = min(nitems, lo + chunk);

  for (int it = lo + slot; it < hi; it += per) {
    const TileItem ti = items[it];
    const MatDesc d = descs[ti.mat];
    const int n = d.n, ld = d.ld;
    const int J0 = S * kNBO, wO = min(kNBO, n - J0);
    const int nch = (wO + kKC - 1) / kKC;
    const int r0 = ti.tr * TR, c0 = ti.tc * kTile;
    cplx<T>* xm = xbuf + d.xoff;
    const cplx<T>* bm = bbuf + d.boff;
    const int* rowcol = rowcolbuf + d.ioff;

    // pivot-row mask (the C tile itself is read during the last K chunk and
    // added in the epilogue, so the MFMAs start as soon as chunk 0 is in LDS)
    int rcv[2][4];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        rcv[ii][v] = rowcol[min(r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v), n - 1)];
    // chunk 0
    cplx<T> pa[kLA], pb[kLB];
#pragma unroll
    for (int t = 0; t < kLA; ++t) {
      const int e = tid + t * NT;
      const int i = e / kKC, k = e % kKC;
      pa[t] = xm[(size_t)min(r0 + i, n - 1) * ld + J0 + min(k, wO - 1)];
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int e = tid + t * NT;
      const int k = e / kTile, c = e % kTile;
      pb[t] = bm[(size_t)min(k, wO - 1) * ld + min(c0 + c, n - 1)];
    }
    v4 cr[2][2], ci[2][2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cr[ii][jj][v] = T(0);
          ci[ii][jj][v] = T(0);
        }
#pragma unroll
    for (int t = 0; t < kLA; ++t) {
      const int e = tid + t * NT;
      const int i = e / kKC, k = e % kKC;
      cplx<T> v = pa[t];
      if (!(r0 + i < n && k < wO)) v.re = v.im = T(0);
      As[0][i * AP + k] = v;
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int e = tid + t * NT;
      const int k = e / kTile, c = e % kTile;
      cplx<T> v = pb[t];
      if (!(k < wO && c0 + c < n)) v.re = v.im = T(0);
      Bsh[0][k * BP + c] = v;
    }
    __syncthreads();

    // the MFMAs of one K chunk from LDS buffer buf
    auto mfma_chunk = [&](int buf) {
      const cplx<T>* as = As[buf];
      const cplx<T>* bs = Bsh[buf];
#pragma unroll
      for (int k = 0; k < kKC; k += 4) {
        T ar[2], ai[2], an[2], br[2], bi[2];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
          const cplx<T> a = as[(32 * wr + 16 * ii + li) * AP + k + lk];
          ar[ii] = a.re;
          ai[ii] = a.im;
          an[ii] = -a.im;
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const cplx<T> b = bs[(k + lk) * BP + 32 * wc + 16 * jj + li];
          br[jj] = b.re;
          bi[jj] = b.im;
        }
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            cr[ii][jj] = Mfma<T>::run(ar[ii], br[jj], cr[ii][jj]);
            ci[ii][jj] = Mfma<T>::run(ar[ii], bi[jj], ci[ii][jj]);
          }
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            cr[ii][jj] = Mfma<T>::run(an[ii], bi[jj], cr[ii][jj]);
            ci[ii][jj] = Mfma<T>::run(ai[ii], br[jj], ci[ii][jj]);
          }
      }
    };

    for (int kc = 0; kc + 1 < nch; ++kc) {
      const int buf = kc & 1;
      const int kb = (kc + 1) * kKC;
#pragma unroll
      for (int t = 0; t < kLA; ++t) {
        const int e = tid + t * NT;
        const int i = e / kKC, k = e % kKC;
        pa[t] = xm[(size_t)min(r0 + i, n - 1) * ld + J0 + min(kb + k, wO - 1)];
      }
#pragma unroll
      for (int t = 0; t < kLB; ++t) {
        const int e = tid + t * NT;
        const int k = e / kTile, c = e % kTile;
        pb[t] = bm[(size_t)min(kb + k, wO - 1) * ld + min(c0 + c, n - 1)];
      }
      mfma_chunk(buf);
#pragma unroll
      for (int t = 0; t < kLA; ++t) {
        const int e = tid + t * NT;
        const int i = e / kKC, k = e % kKC;
        cplx<T> v = pa[t];
        if (!(r0 + i < n && kb + k < wO)) v.re = v.im = T(0);
        As[buf ^ 1][i * AP + k] = v;
      }
#pragma unroll
      for (int t = 0; t < kLB; ++t) {
        const int e = tid + t * NT;
        const int k = e / kTile, c = e % kTile;
        cplx<T> v = pb[t];
        if (!(kb + k < wO && c0 + c < n)) v.re = v.im = T(0);
        Bsh[buf ^ 1][k * BP + c] = v;
      }
      __syncthreads();
    }
    // last chunk, with the C tile's loads in flight
    cplx<T> cv[2][2][4];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v), n - 1);
          const int col = min(c0 + 32 * wc + 16 * jj + li, n - 1);
          cv[ii][jj][v] = xm[(size_t)row * ld + col];
        }
    mfma_chunk((nch - 1) & 1);
    __syncthreads();   // LDS free for this workgroup's next item
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v);
          const int col = c0 + 32 * wc + 16 * jj + li;
          if (row < n && col < n) {
            const int rc = rcv[ii][v];
            const bool keep = !(rc >= J0 && rc < J0 + wO);
            cplx<T> c;
            c.re = cr[ii][jj][v] + (keep ? cv[ii][jj][v].re : T(0));
            c.im = ci[ii][jj][v] + (keep ? cv[ii][jj][v].im : T(0));
            xm[(size_t)row * ld + col] = c;
          }
        }
  }
}

// --------------------------------------------------------------- launchers
template <typename T> static size_t panel_lds_bytes() {
  const size_t upd = sizeof(cplx<T>) * (size_t)(kNB + kTile) * kPitch;
  const size_t fac = sizeof(cplx<T>) * (kIB * kNB + kIB) + kPW * sizeof(T) +
                     kPW * sizeof(int) + kIB * sizeof(int);
  return upd > fac ? upd : fac;
}

template <typename T>
hipError_t gje_panel(cplx<T>* x, int* piv, int* rowcol, const MatDesc* d,
                     int nmat, int S, int* status, hipStream_t st) {
  static bool attr_set = false;
  const size_t lds = panel_lds_bytes<T>();
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_outer_panel<T>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_outer_panel<T>, dim3(nmat), dim3(kPanelThreads), lds, st,
                     x, piv, rowcol, d, S, status);
  return hipGetLastError();
}

template <typename T>
hipError_t gje_gather(const cplx<T>* x, cplx<T>* bbuf, const int* piv,
                      const MatDesc* d, int nmat, int S, hipStream_t st) {
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather<T>, dim3(kNBO, nmat), dim3(256), 0, st, x, bbuf,
                     piv, d, S);
  return hipGetLastError();
}

template <typename T>
hipError_t gje_update(cplx<T>* x, const cplx<T>* bbuf, const int* rowcol,
                      const MatDesc* d, const TileItem* items, int nitems,
                      int S, int variant, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  // one workgroup per item (a persistent grid of two workgroups per CU
  // measured 4% slower: the dispatcher already overlaps the tiles' prologues)
  const int grid = 8 * ((nitems + 7) / 8);
  if (variant == 1)
    hipLaunchKernelGGL((k_update<T, 4>), dim3(grid), dim3(512), 0, st, x, bbuf,
                       rowcol, d, items, nitems, S);
  else
    hipLaunchKernelGGL((k_update<T, 2>), dim3(grid), dim3(256), 0, st, x, bbuf,
                       rowcol, d, items, nitems, S);
  return hipGetLastError();
}

#define FK_INST(T)                                                            \
  template hipError_t gje_panel<T>(cplx<T>*, int*, int*, const MatDesc*, int, \
                                   int, int*, hipStream_t);                   \
  template hipError_t gje_gather<T>(const cplx<T>*, cplx<T>*, const int*,     \
                                    const MatDesc*, int, int, hipStream_t);   \
  template hipError_t gje_update<T>(cplx<T>*, const cplx<T>*, const int*,     \
                                    const MatDesc*, const TileItem*, int, int, \
                                    int, hipStream_t);
FK_INST(double)
FK_INST(float)

}  // namespace fk
