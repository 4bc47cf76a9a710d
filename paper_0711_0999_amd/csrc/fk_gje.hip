// Batched blocked in-place Gauss-Jordan inversion with partial pivoting, for
// gfx950.  This is the hot loop of the lattice step: every (eps, ebar) point
// needs the inverse of the dense complex matrix G0_k^-1 - W Sigma W (the
// "matrix inversion" of the integrand of eq. g_loc, Sec. II).
//
// Outer step S handles the block of kNBO = 128 columns starting at J0 = S*kNBO:
//   panel   (one 512-thread workgroup per matrix) eliminates the block's
//           four 32-column quarters in turn on the n - J0 rows not pivoted in
//           earlier blocks.  For each column the pivot is the largest
//           |re|+|im| among the rows not yet pivoted; kIB columns are
//           eliminated in registers at a time (one row per thread), the rest
//           of the quarter receives rank-kIB updates (16 lanes per row), and
//           the other quarter of the half and then the other half receive
//           the quarter's (half's) transform on the matrix cores.
//   gather  copies the pivot rows of the step into a side buffer B (their
//           values before the step outside the block, the block's inverse
//           pivot submatrix inside it); B holds the rows of two blocks.
//   fix     the block's columns of the J0 rows pivoted earlier, from that
//           inverse (one small product per row tile).  The block now holds
//           the transformed identity columns M = E[:, P] of all elementary
//           Gauss-Jordan transforms of the step.
//   update  every other column tile: C <- mask_P(C) + M B, a batched complex
//           GEMM on the matrix cores (three real products per complex one),
//           double-buffered K chunks in LDS, two workgroups per CU.  Blocks
//           are applied in groups of kGroup (K up to 512, see block_pos): each
//           block of a group brings the group's earlier blocks' columns up to
//           date and updates the next block's columns; the last one applies
//           all the group's transforms to every other column at once.
// The host runs the update of the next block's columns first; with the
// look-ahead schedule it factors that block on a second stream while the big
// update of the current step runs.
// Rows are never swapped: with r = piv and rinv = rowcol the inverse is
// inv(A)[a][b] = X[r[a]][rinv[b]], which the reduction kernels read directly.
#include "fk_internal.h"

#include <float.h>
#include <limits.h>

#include <atomic>

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
// Panel shapes: rows per thread and register block, (4, 8) up to kSmallN
// rows, (kMaxN / kPanelThreads, 4) beyond (fewer columns per register block
// keep the larger row count in registers).
constexpr int kSmallN = 2048;
constexpr int kRPTs = kSmallN / kPanelThreads, kIBs = kIB;
constexpr int kRPTl = kMaxN / kPanelThreads, kIBl = 4;
constexpr int kPitch = kNB + 1;                  // padded LDS row (elements)
static_assert(kMaxN % kPanelThreads == 0 && kSmallN % kPanelThreads == 0, "kMaxN");
static_assert(kNBO == 2 * kNB && kTile == kNB, "block sizes");

// ------------------------------------------------------ panel: cross update
// C <- mask(C) + M B on the columns [c0, c0 + cw) of one matrix's listed rows,
// with M the already eliminated columns [j0, j0 + w) and B the values of their
// pivot rows in [c0, c0 + cw) (read before any write: this workgroup owns the
// matrix).  KW >= w and CW >= cw are the compile-time widths (32 or 64).  The
// kPW waves form (kPW / (CW/16)) x (CW/16) blocks of (16 RB) x 16 over each
// tile of TRW rows (at least 64).
template <typename T, int KW, int CW>
__device__ __forceinline__ void cross_update(cplx<T>* __restrict__ x, int ld,
                             const int* __restrict__ rows, int m,
                             const int* __restrict__ piv,
                             const int* __restrict__ rowcol, int j0, int w,
                             int c0, int cw, unsigned char* smem) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int NCB = CW / 16, NRW = kPW / NCB;
  constexpr int RB = 1;
  constexpr int TRW = 16 * RB * NRW;
  static_assert(NCB * NRW == kPW && TRW <= kNB + kTile, "waves");
  constexpr int KP = KW + 1, CP = CW + 1;
  cplx<T>* Bs = reinterpret_cast<cplx<T>*>(smem);   // [KW][CP]
  cplx<T>* Ms = Bs + KW * CP;                        // [TRW][KP]
  constexpr int kLB = KW * CW / kPanelThreads;      // B elements per thread
  constexpr int kLM = TRW * KW / kPanelThreads;     // M elements per thread
  static_assert(kLB * kPanelThreads == KW * CW && kLM * kPanelThreads == TRW * KW, "loads");
  static_assert(KW * CP + TRW * KP <= (kNB + kTile) * kPitch, "LDS");
  const int tid = threadIdx.x;
  {
    int pr[kLB];
    cplx<T> bv[kLB];
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int l = (tid + t * kPanelThreads) / CW;
      pr[t] = piv[j0 + min(l, w - 1)];
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int c = (tid + t * kPanelThreads) % CW;
      bv[t] = x[(size_t)pr[t] * ld + c0 + min(c, cw - 1)];
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int e = tid + t * kPanelThreads;
      const int l = e / CW, c = e % CW;
      cplx<T> v = bv[t];
      if (!(l < w && c < cw)) v.re = v.im = T(0);
      Bs[l * CP + c] = v;
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / NCB, wc = wave % NCB;
  const int li = lane & 15, lk = lane >> 4;
  const int col = 16 * wc + li;
  // the tile's M values, its rows' rowcol entries and C values; the next
  // tile's are loaded while the current one is multiplied (the tiles' rows
  // are distinct, and the M columns are not written here)
  cplx<T> mv[kLM];
  int nrc[RB][4];
  cplx<T> ncv[RB][4];
  auto load_tile = [&](int t0) {
#pragma unroll
    for (int t = 0; t < kLM; ++t) {
      const int e = tid + t * kPanelThreads;
      const int i = e / KW, l = e % KW;
      mv[t] = x[(size_t)rows[min(t0 + i, m - 1)] * ld + j0 + min(l, w - 1)];
    }
#pragma unroll
    for (int ii = 0; ii < RB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = t0 + 16 * (RB * wr + ii) + Mfma<T>::drow(lk, v);
        const int r = rows[min(e, m - 1)];
        nrc[ii][v] = rowcol[r];
        ncv[ii][v] = x[(size_t)r * ld + c0 + min(col, cw - 1)];
      }
  };
  load_tile(0);
  for (int r0 = 0; r0 < m; r0 += TRW) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kLM; ++t) {
      const int e = tid + t * kPanelThreads;
      const int i = e / KW, l = e % KW;
      cplx<T> v = mv[t];
      if (!(r0 + i < m && l < w)) v.re = v.im = T(0);
      Ms[i * KP + l] = v;
    }
    // masked C (pivot rows of the block start from zero); the product is
    // formed from three real ones (Gauss) as in the trailing update:
    // P1 = Re a Re b, P2 = Im a Im b, P3 = (Re a + Im a)(Re b + Im b),
    // Re = P1 - P2, Im = P3 - P1 - P2, and C added afterwards
    cplx<T> cv[RB][4];
#pragma unroll
    for (int ii = 0; ii < RB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = r0 + 16 * (RB * wr + ii) + Mfma<T>::drow(lk, v);
        const bool keep = e < m && col < cw &&
                          !(nrc[ii][v] >= j0 && nrc[ii][v] < j0 + w);
        cv[ii][v] = ncv[ii][v];
        if (!keep) cv[ii][v].re = cv[ii][v].im = T(0);
      }
    if (r0 + TRW < m) load_tile(r0 + TRW);
    v4 p1[RB], p2[RB], p3[RB];
#pragma unroll
    for (int ii = 0; ii < RB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) p1[ii][v] = p2[ii][v] = p3[ii][v] = T(0);
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < KW; k += 4) {
      const cplx<T> b = Bs[(k + lk) * CP + col];
      const T bs = b.re + b.im;
#pragma unroll
      for (int ii = 0; ii < RB; ++ii) {
        const cplx<T> a = Ms[(16 * (RB * wr + ii) + li) * KP + k + lk];
        p1[ii] = Mfma<T>::run(a.re, b.re, p1[ii]);
        p2[ii] = Mfma<T>::run(a.im, b.im, p2[ii]);
        p3[ii] = Mfma<T>::run(a.re + a.im, bs, p3[ii]);
      }
    }
#pragma unroll
    for (int ii = 0; ii < RB; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = r0 + 16 * (RB * wr + ii) + Mfma<T>::drow(lk, v);
        if (e < m && col < cw) {
          const T q1 = p1[ii][v], q2 = p2[ii][v];
          cplx<T> c;
          c.re = (q1 - q2) + cv[ii][v].re;
          c.im = ((p3[ii][v] - q1) - q2) + cv[ii][v].im;
          x[(size_t)rows[e] * ld + c0 + col] = c;
        }
      }
  }
}

// ---------------------------------------------------- panel: factorization
// Eliminate the PW (32) columns starting at c0 on the listed rows
// rows[0, m) (the rows not pivoted before this outer block) with partial
// pivoting, IB columns at a time in registers.  Thread tid owns list entries
// tid + i * kPanelThreads, i < RPT; the list is in ascending row order, so a
// tie of pivot keys goes to the lowest row index.
template <typename T, int PW, int RPT, int IB>
__device__ __forceinline__ void factor_panel(cplx<T>* __restrict__ x, int ld, int n,
                             const int* __restrict__ rows, int m,
                             int* __restrict__ piv, int* __restrict__ rowcol,
                             int c0, int* __restrict__ status,
                             unsigned char* smem) {
  static_assert(PW % IB == 0 && PW <= kNB, "panel width");
  cplx<T>* Bo = reinterpret_cast<cplx<T>*>(smem);   // [IB][PW]
  // pivot row and the waves' pivot candidates, double-buffered by column
  // parity so one column's reads never meet the next column's writes
  cplx<T>* prow2 = Bo + IB * PW;                     // [2][IB]
  T* redv2 = reinterpret_cast<T*>(prow2 + 2 * IB);   // [2][kPW]
  int* redi2 = reinterpret_cast<int*>(redv2 + 2 * kPW);  // [2][kPW]
  int* pvt = redi2 + 2 * kPW;                        // [IB]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cw = min(PW, n - c0);
  const T inf_key = big_value<T>();

  // bit i: list entry tid + i kPanelThreads is pivoted (or absent); row ids
  // are re-read from the LDS list where needed (registers go to v)
  unsigned pvd = 0u;
  static_assert(RPT <= 32, "pivot bits");
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int e = tid + i * kPanelThreads;
    if (!(e < m) || rowcol[rows[min(e, m - 1)]] >= 0) pvd |= 1u << i;
  }
  const int ngroups = (cw + IB - 1) / IB;

  for (int b0 = 0; b0 < cw; b0 += IB) {
    const int iw = min(IB, cw - b0);
    cplx<T> v[RPT][IB];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
#pragma unroll
      for (int l = 0; l < IB; ++l)
        v[i][l] = x[(size_t)rows[min(tid + i * kPanelThreads, m - 1)] * ld + c0 + b0 +
                    min(l, iw - 1)];
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int e = tid + i * kPanelThreads;
#pragma unroll
      for (int l = 0; l < IB; ++l)
        if (!(e < m && l < iw)) v[i][l].re = v[i][l].im = T(0);
    }
#pragma unroll
    for (int l = 0; l < IB; ++l) {
      if (l >= iw) break;
      cplx<T>* prow = prow2 + (l & 1) * IB;
      T* redv = redv2 + (l & 1) * kPW;
      int* redi = redi2 + (l & 1) * kPW;
      // ---- pivot search: largest |re|+|im| among unpivoted rows (bidx is
      // a list index)
      T best = T(-1);
      int bidx = INT_MAX;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int e = tid + i * kPanelThreads;
        if (e < m && !((pvd >> i) & 1u)) {
          T a = fabs(v[i][l].re) + fabs(v[i][l].im);
          if (!(a <= inf_key)) a = inf_key;  // NaN / Inf win and get flagged
          if (a > best || (a == best && e < bidx)) {
            best = a;
            bidx = e;
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
      // a valid unpivoted entry: the list holds more rows than this block
      // has columns
      const int pe = bidx;
      const int p = rows[min(pe, m - 1)];
      const int col = c0 + b0 + l;
      if (tid == 0 && (best == T(0) || best == inf_key))
        atomicCAS(status, 0, best == T(0) ? (1 + col) : -(1 + col));
      if ((pe % kPanelThreads) == tid) {
        const int i = pe / kPanelThreads;
#pragma unroll
        for (int ii = 0; ii < RPT; ++ii)
          if (ii == i) {
#pragma unroll
            for (int l2 = 0; l2 < IB; ++l2) prow[l2] = v[ii][l2];
            pvd |= 1u << ii;
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
      // column by column of the register block: the scaled pivot row entry is
      // formed from LDS as it is used (RPT multipliers in registers instead of
      // IB scaled entries; fewer spills in both panel shapes)
      cplx<T> mi[RPT];
#pragma unroll
      for (int i = 0; i < RPT; ++i) mi[i] = v[i][l];
#pragma unroll
      for (int l2 = 0; l2 < IB; ++l2) {
        if (l2 == l) continue;
        const cplx<T> q = cmul(prow[l2], inv);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          if (tid + i * kPanelThreads == pe) {
            v[i][l2] = q;
          } else {
            v[i][l2].re -= mi[i].re * q.re - mi[i].im * q.im;
            v[i][l2].im -= mi[i].re * q.im + mi[i].im * q.re;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (tid + i * kPanelThreads == pe) {
          v[i][l] = inv;
        } else {
          const cplx<T> nm = cmul(mi[i], inv);
          v[i][l].re = -nm.re;
          v[i][l].im = -nm.im;
        }
      }
    }
    // ---- write the eliminated block back; old pivot rows of the other columns
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int e = tid + i * kPanelThreads;
      if (e < m) {
#pragma unroll
        for (int l = 0; l < IB; ++l)
          if (l < iw) x[(size_t)rows[e] * ld + c0 + b0 + l] = v[i][l];
      }
    }
    for (int e = tid; e < IB * PW; e += kPanelThreads) {
      const int l = e / PW, c = e % PW;
      const bool ok = l < iw && c < cw && (c < b0 || c >= b0 + iw);
      cplx<T> t = x[(size_t)pvt[min(l, iw - 1)] * ld + c0 + min(c, cw - 1)];
      if (!ok) t.re = t.im = T(0);
      Bo[e] = t;
    }
    __syncthreads();
    // ---- rank-iw update of the other column groups of the panel: 16 lanes
    // per row (lane k holds columns k and k + 16 of the panel), four rows per
    // wave at a time, so each load and store of a wave covers four rows'
    // contiguous segments instead of one cache line per lane; a row's
    // eliminated values come from the lanes holding them (16-wide shuffles).
    if (ngroups > 1) {
      static_assert(PW == 32 && 16 % IB == 0, "panel lane map");
      const int k16 = lane & 15, rr = lane >> 4;
      const int ca = k16, cb = k16 + 16;
      const bool sta = ca < cw && !(ca >= b0 && ca < b0 + IB);
      const bool stb = cb < cw && !(cb >= b0 && cb < b0 + IB);
      cplx<T> boa[IB], bob[IB];
      int pv0[IB];
#pragma unroll
      for (int l = 0; l < IB; ++l) {
        boa[l] = Bo[l * PW + ca];
        bob[l] = Bo[l * PW + cb];
        pv0[l] = (l < iw) ? pvt[l] : -1;
      }
      const int src0 = b0 & 15;          // lane holding column b0 of the row
      const bool hi = b0 >= 16;          // ... in its second value
      // kRU groups of four rows per wave and trip: their loads are issued
      // together, so a wave waits for memory once per kRU groups (the rows
      // of a trip are distinct; each is read and written by one lane group)
      constexpr int kRU = 4, kStep = 4 * kPW;
#pragma unroll 1
      for (int e0 = 4 * wave; e0 < m; e0 += kStep * kRU) {
        int r[kRU];
        cplx<T> va[kRU], vb[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) r[u] = rows[min(e0 + kStep * u + rr, m - 1)];
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
          va[u] = x[(size_t)r[u] * ld + c0 + min(ca, cw - 1)];
          vb[u] = x[(size_t)r[u] * ld + c0 + min(cb, cw - 1)];
        }
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
          const int e = e0 + kStep * u + rr;
          bool isp = false;
#pragma unroll
          for (int l = 0; l < IB; ++l) isp |= (pv0[l] == r[u]);
          cplx<T> acca = va[u], accb = vb[u];
          if (isp) acca.re = acca.im = accb.re = accb.im = T(0);
          const cplx<T> src = hi ? vb[u] : va[u];
#pragma unroll
          for (int l = 0; l < IB; ++l) {
            if (l < iw) {
              cplx<T> mm;
              mm.re = __shfl(src.re, src0 + l, 16);
              mm.im = __shfl(src.im, src0 + l, 16);
              cfma(acca, mm, boa[l]);
              cfma(accb, mm, bob[l]);
            }
          }
          if (e < m) {
            if (sta) x[(size_t)r[u] * ld + c0 + ca] = acca;
            if (stb) x[(size_t)r[u] * ld + c0 + cb] = accb;
          }
        }
      }
    }
    __syncthreads();
  }
}

// LDS of the panel kernel: the larger of the two phases' buffers, then the
// list of the rows the block works on.
template <typename T> __host__ __device__ constexpr size_t panel_body_bytes() {
  return ((sizeof(cplx<T>) * (size_t)(kNB + kTile) * kPitch >
                   sizeof(cplx<T>) * (kIB * kNB + 2 * kIB) + 2 * kPW * sizeof(T) +
                       2 * kPW * sizeof(int) + kIB * sizeof(int)
               ? sizeof(cplx<T>) * (size_t)(kNB + kTile) * kPitch
               : sizeof(cplx<T>) * (kIB * kNB + 2 * kIB) + 2 * kPW * sizeof(T) +
                     2 * kPW * sizeof(int) + kIB * sizeof(int)) + 15) / 16 * 16;
}
template <typename T> static size_t panel_lds_bytes(int rpt) {
  return panel_body_bytes<T>() + sizeof(int) * (size_t)rpt * kPanelThreads;
}

// Outer block S of one matrix.  Rows pivoted in earlier blocks take no part:
// their columns of this block follow from the block's pivot rows afterwards
// (k_fix), so the panel reads and writes only the n - S kNBO remaining rows.
// RPT kPanelThreads >= n rows; IB columns eliminated in registers at a time.
template <typename T, int RPT, int IB>
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

  // list the unpivoted rows in ascending order (wave ballots, then offsets)
  int* rows = reinterpret_cast<int*>(smem + panel_body_bytes<T>());
  int* cnt = reinterpret_cast<int*>(smem);   // [RPT][kPW], before the panel
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  unsigned long long bal[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + i * kPanelThreads;
    bal[i] = __ballot(r < n && rowcol[min(r, n - 1)] < 0);
    if (lane == 0) cnt[i * kPW + wave] = (int)__popcll(bal[i]);
  }
  __syncthreads();
  int m = 0;   // n - S kNBO unless earlier blocks failed to pivot
  int pos[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    int before = 0;
#pragma unroll
    for (int wv = 0; wv < kPW; ++wv) before += (wv < wave) ? cnt[i * kPW + wv] : 0;
    pos[i] = m + before + (int)__popcll(bal[i] & ((1ull << lane) - 1ull));
#pragma unroll
    for (int wv = 0; wv < kPW; ++wv) m += cnt[i * kPW + wv];
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i)
    if ((bal[i] >> lane) & 1ull) rows[pos[i]] = tid + i * kPanelThreads;
  __syncthreads();
  if (m == 0) return;   // the same for every thread

  // Each 64-column half as two 32-column quarters joined by cross updates,
  // then the halves joined the same way.  Order: Q0, Q0->Q1, Q1, Q1->Q0,
  // L->R, Q2, Q2->Q3, Q3, Q3->Q2, R->L (one call site per kind of step).
  const int ld = d.ld;
  const int J0 = S * kNBO, J1 = J0 + kNB;
#pragma unroll 1
  for (int qi = 0; qi < 4; ++qi) {
    const int c = J0 + 32 * qi;
    if (c >= n) break;
    if (qi == 2) {
      cross_update<T, kNB, kNB>(x, ld, rows, m, piv, rowcol, J0, kNB, J1,
                                min(kNB, n - J1), smem);
      __syncthreads();
    }
    factor_panel<T, 32, RPT, IB>(x, ld, n, rows, m, piv, rowcol, c, st, smem);
    __syncthreads();
    const int dst = (qi & 1) ? c - 32 : c + 32;
    if (dst < n) {
      cross_update<T, 32, 32>(x, ld, rows, m, piv, rowcol, c, min(32, n - c),
                              dst, min(32, n - dst), smem);
      __syncthreads();
    }
  }
  if (J1 < n)
    cross_update<T, kNB, kNB>(x, ld, rows, m, piv, rowcol, J1, min(kNB, n - J1),
                              J0, kNB, smem);
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
  cplx<T>* dst = bbuf + d.boff + (size_t)(block_brow(d.n, S) + l) * d.ld;
  for (int c = threadIdx.x; c < d.n; c += blockDim.x) dst[c] = src[c];
}

// ----------------------------------------------------------------- fix-up
// Rows pivoted in earlier outer blocks skip the panel.  For such a row r the
// block's Gauss-Jordan steps amount to X[r, P] <- -X0[r, P] Minv, with X0 the
// row's values before the block and Minv = X[R, P] the block's pivot rows R in
// pivot order after the panel (the inverse of X0[R, P]), which the gather has
// copied into B.  Those rows are piv[0, J0) in pivot order; one 512-thread
// workgroup takes 64 of them and all of the block's columns, reading its
// rows' X0 before writing, so the product is formed in place.  Eight waves
// as 2 x 4 blocks of 32 x 32, K in chunks of kKC double-buffered in LDS.
template <typename T>
__global__ __launch_bounds__(512, 1) void k_fix(
    cplx<T>* __restrict__ xbuf, const cplx<T>* __restrict__ bbuf,
    const int* __restrict__ pivbuf, const MatDesc* __restrict__ descs, int S) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int TR = 64, TC = kNBO, NT = 512;
  constexpr int AP = kKC + 1, BP = TC + 1;
  __shared__ cplx<T> As[2][TR * AP];
  __shared__ cplx<T> Bsh[2][kKC * BP];
  constexpr int kLA = TR * kKC / NT;
  constexpr int kLB = kKC * TC / NT;
  static_assert(kLA * NT == TR * kKC && kLB * NT == kKC * TC, "fix tile");

  const MatDesc d = descs[blockIdx.y];
  const int n = d.n, ld = d.ld;
  const int J0 = S * kNBO, i0 = blockIdx.x * TR;
  if (J0 >= n || i0 + TR > J0) return;   // J0 is a multiple of TR
  const int wO = min(kNBO, n - J0);
  const int nch = (wO + kKC - 1) / kKC;
  cplx<T>* xm = xbuf + d.xoff;
  const cplx<T>* bm = bbuf + d.boff + (size_t)block_brow(n, S) * ld;
  const int* piv = pivbuf + d.ioff;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int li = lane & 15, lk = lane >> 4;

  int ra[kLA];
#pragma unroll
  for (int t = 0; t < kLA; ++t) ra[t] = piv[i0 + (tid + t * NT) / kKC];
  cplx<T> pa[kLA], pb[kLB];
  auto load = [&](int kb) {
#pragma unroll
    for (int t = 0; t < kLA; ++t) {
      const int k = (tid + t * NT) % kKC;
      pa[t] = xm[(size_t)ra[t] * ld + J0 + min(kb + k, wO - 1)];
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int e = tid + t * NT;
      const int k = e / TC, c = e % TC;
      pb[t] = bm[(size_t)min(kb + k, wO - 1) * ld + J0 + min(c, wO - 1)];
    }
  };
  auto stash = [&](int kb, int buf) {
#pragma unroll
    for (int t = 0; t < kLA; ++t) {
      const int e = tid + t * NT;
      const int i = e / kKC, k = e % kKC;
      cplx<T> v = pa[t];
      if (!(kb + k < wO)) v.re = v.im = T(0);
      As[buf][i * AP + k] = v;
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int e = tid + t * NT;
      const int k = e / TC, c = e % TC;
      cplx<T> v = pb[t];
      if (!(kb + k < wO && c < wO)) v.re = v.im = T(0);
      Bsh[buf][k * BP + c] = v;
    }
  };
  v4 p1[2][2], p2[2][2], p3[2][2];   // three-product form, as k_update
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        p1[ii][jj][v] = T(0);
        p2[ii][jj][v] = T(0);
        p3[ii][jj][v] = T(0);
      }
  load(0);
  stash(0, 0);
  __syncthreads();
  for (int kc = 0; kc < nch; ++kc) {
    const int buf = kc & 1;
    const bool more = kc + 1 < nch;
    if (more) load((kc + 1) * kKC);
    const cplx<T>* as = As[buf];
    const cplx<T>* bs = Bsh[buf];
#pragma unroll
    for (int k = 0; k < kKC; k += 4) {
      T ar[2], ai[2], as_[2], br[2], bi[2], bs_[2];
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const cplx<T> a = as[(32 * wr + 16 * ii + li) * AP + k + lk];
        ar[ii] = a.re;
        ai[ii] = a.im;
        as_[ii] = a.re + a.im;
      }
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const cplx<T> b = bs[(k + lk) * BP + 32 * wc + 16 * jj + li];
        br[jj] = b.re;
        bi[jj] = b.im;
        bs_[jj] = b.re + b.im;
      }
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          p1[ii][jj] = Mfma<T>::run(ar[ii], br[jj], p1[ii][jj]);
          p2[ii][jj] = Mfma<T>::run(ai[ii], bi[jj], p2[ii][jj]);
          p3[ii][jj] = Mfma<T>::run(as_[ii], bs_[jj], p3[ii][jj]);
        }
    }
    if (more) stash((kc + 1) * kKC, buf ^ 1);
    __syncthreads();
  }
  // every global read of the rows is done (last barrier): write in place
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = piv[i0 + 32 * wr + 16 * ii + Mfma<T>::drow(lk, v)];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int col = 32 * wc + 16 * jj + li;
        if (col < wO) {
          cplx<T> c;
          const T q1 = p1[ii][jj][v], q2 = p2[ii][jj][v];
          c.re = q2 - q1;
          c.im = (q1 + q2) - p3[ii][jj][v];
          xm[(size_t)r * ld + J0 + col] = c;
        }
      }
    }
}

// ------------------------------------------------------------------ update
// C <- mask_P(C) + M B for the listed tiles of (32 WR) x 64: 2 WR waves as
// WR x 2 blocks of 32 x 32 (WR = 2: 64 x 64 tiles, two workgroups per CU;
// WR = 4: 128 x 64 tiles sharing each B chunk, one workgroup per CU).  K in
// chunks of kKC, double-buffered through LDS with the next chunk's global
// loads in flight during the current chunk's MFMAs; within a chunk the next
// k-step's operands are read from LDS before the current k-step's MFMAs.
// Interior tiles (whole rows, columns and K chunks) skip every clamp and
// mask.  Each complex product takes three real ones (Gauss): P1 = Re a Re b,
// P2 = Im a Im b and P3 = (Re a + Im a)(Re b + Im b) accumulate separately,
// and the epilogue forms Re = P1 - P2, Im = P3 - P1 - P2: a quarter fewer
// MFMAs than the four-product form, with a normwise (not componentwise) error
// bound of the same order.  The C tile is read in the epilogue.
template <typename T, int WR>
__global__ __launch_bounds__(128 * WR, 4 / WR) void k_update(
    cplx<T>* __restrict__ xbuf, const cplx<T>* __restrict__ bbuf,
    const int* __restrict__ rowcolbuf, const MatDesc* __restrict__ descs,
    const TileItem* __restrict__ items, int nitems) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int TR = 32 * WR, NT = 128 * WR;
  constexpr int AP = kKC + 1, BP = kTile + 1;
  __shared__ cplx<T> As[2][TR * AP];
  __shared__ cplx<T> Bsh[2][kKC * BP];
  constexpr int kLA = TR * kKC / NT;      // chunk loads per thread
  constexpr int kLB = kKC * kTile / NT;
  static_assert(NT % kKC == 0 && NT % kTile == 0, "load map");

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per = gridDim.x >> 3;
  const int chunk = (nitems + 7) >> 3;
  const int lo = xcd * chunk, hi = min(nitems, lo + chunk);
  // this thread's chunk loads: A rows ai0 + t (NT / kKC) at column ak of the
  // chunk, B rows bk0 + t (NT / kTile) at column bc of the tile
  const int ak = tid % kKC, ai0 = tid / kKC;
  const int bc = tid % kTile, bk0 = tid / kTile;
  constexpr int AST = NT / kKC, BST = NT / kTile;

  for (int it = lo + slot; it < hi; it += per) {
    const TileItem ti = items[it];
    const MatDesc d = descs[ti.mat];
    const int n = d.n, ld = d.ld;
    // M = columns [J0, J0 + wO), B = side-buffer rows [b0, b0 + wO)
    const int J0 = ti.jb * kNBO, wO = ti.kw;
    const int nch = (wO + kKC - 1) / kKC;
    const int r0 = ti.tr * TR, c0 = ti.tc * kTile;
    cplx<T>* xm = xbuf + d.xoff;
    const cplx<T>* bm = bbuf + d.boff + (size_t)ti.b0 * ld;
    const int* rowcol = rowcolbuf + d.ioff;
    const bool full = r0 + TR <= n && c0 + kTile <= n && (wO % kKC) == 0;
    const cplx<T>* arow[kLA];
#pragma unroll
    for (int t = 0; t < kLA; ++t)
      arow[t] = xm + (size_t)min(r0 + ai0 + AST * t, n - 1) * ld + J0;
    const cplx<T>* bcol = bm + min(c0 + bc, n - 1);
    cplx<T> pa[kLA], pb[kLB];
    auto gload = [&](int kb) {
      if (full) {
#pragma unroll
        for (int t = 0; t < kLA; ++t) pa[t] = arow[t][kb + ak];
#pragma unroll
        for (int t = 0; t < kLB; ++t) pb[t] = bcol[(size_t)(kb + bk0 + BST * t) * ld];
      } else {
#pragma unroll
        for (int t = 0; t < kLA; ++t) pa[t] = arow[t][min(kb + ak, wO - 1)];
#pragma unroll
        for (int t = 0; t < kLB; ++t)
          pb[t] = bcol[(size_t)min(kb + bk0 + BST * t, wO - 1) * ld];
      }
    };
    auto lstore = [&](int kb, int buf) {
      if (!full) {
#pragma unroll
        for (int t = 0; t < kLA; ++t)
          if (!(r0 + ai0 + AST * t < n && kb + ak < wO)) pa[t].re = pa[t].im = T(0);
#pragma unroll
        for (int t = 0; t < kLB; ++t)
          if (!(kb + bk0 + BST * t < wO && c0 + bc < n)) pb[t].re = pb[t].im = T(0);
      }
#pragma unroll
      for (int t = 0; t < kLA; ++t) As[buf][(ai0 + AST * t) * AP + ak] = pa[t];
#pragma unroll
      for (int t = 0; t < kLB; ++t) Bsh[buf][(bk0 + BST * t) * BP + bc] = pb[t];
    };

    // Edge tiles with at most 16 valid rows (or columns) use a strip layout:
    // wave w multiplies the single 16 x 16 block at columns (rows) 16 w of
    // the strip, a quarter of an interior tile's matrix-core work, instead of
    // a 32 x 32 quarter that lies mostly outside the matrix.  The choice is
    // the same for the whole workgroup.
    const int edge = (n - r0 <= 16) ? 1 : ((n - c0 <= 16) ? 2 : 0);
    const int er0 = edge == 2 ? 16 * wave : 0;   // strip block origin (rows)
    const int ec0 = edge == 1 ? 16 * wave : 0;   // strip block origin (columns)
    // waves whose strip block lies inside the tile (all of them for a
    // 64 x 64 tile; the first four of a 128-row tile's eight in a row strip)
    const bool eact = edge == 1 ? ec0 < kTile : er0 < TR;
    // pivot-row mask of the rows this lane writes
    int rcv[2][4];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = edge ? er0 + 16 * ii : 32 * wr + 16 * ii;
        rcv[ii][v] = rowcol[min(r0 + rr + Mfma<T>::drow(lk, v), n - 1)];
      }
    v4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          p1[ii][jj][v] = T(0);
          p2[ii][jj][v] = T(0);
          p3[ii][jj][v] = T(0);
        }
    gload(0);
    lstore(0, 0);
    __syncthreads();

    // the MFMAs of one K chunk from LDS buffer buf; operands of the next
    // k-step are read before the current k-step's products (ping-pong)
    auto mfma_chunk = [&](int buf) {
      const cplx<T>* as = As[buf];
      const cplx<T>* bs = Bsh[buf];
      cplx<T> a[2][2], b[2][2];
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) a[0][ii] = as[(32 * wr + 16 * ii + li) * AP + lk];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) b[0][jj] = bs[lk * BP + 32 * wc + 16 * jj + li];
#pragma unroll
      for (int s = 0; s < kKC / 4; ++s) {
        const int cur = s & 1;
        if (s + 1 < kKC / 4) {
          const int k = 4 * (s + 1);
#pragma unroll
          for (int ii = 0; ii < 2; ++ii)
            a[cur ^ 1][ii] = as[(32 * wr + 16 * ii + li) * AP + k + lk];
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
            b[cur ^ 1][jj] = bs[(k + lk) * BP + 32 * wc + 16 * jj + li];
        }
        T as_[2], bs_[2];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) as_[ii] = a[cur][ii].re + a[cur][ii].im;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) bs_[jj] = b[cur][jj].re + b[cur][jj].im;
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            p1[ii][jj] = Mfma<T>::run(a[cur][ii].re, b[cur][jj].re, p1[ii][jj]);
            p2[ii][jj] = Mfma<T>::run(a[cur][ii].im, b[cur][jj].im, p2[ii][jj]);
            p3[ii][jj] = Mfma<T>::run(as_[ii], bs_[jj], p3[ii][jj]);
          }
      }
    };

    // strip layout: one 16 x 16 block per wave, accumulated in p*[0][0]
    auto mfma_chunk_edge = [&](int buf) {
      if (!eact) return;
      const cplx<T>* as = As[buf];
      const cplx<T>* bs = Bsh[buf];
#pragma unroll
      for (int s = 0; s < kKC / 4; ++s) {
        const int k = 4 * s;
        const cplx<T> a = as[(er0 + li) * AP + k + lk];
        const cplx<T> b = bs[(k + lk) * BP + ec0 + li];
        p1[0][0] = Mfma<T>::run(a.re, b.re, p1[0][0]);
        p2[0][0] = Mfma<T>::run(a.im, b.im, p2[0][0]);
        p3[0][0] = Mfma<T>::run(a.re + a.im, b.re + b.im, p3[0][0]);
      }
    };

    if (!edge) {
      for (int kc = 0; kc + 1 < nch; ++kc) {
        const int buf = kc & 1;
        gload((kc + 1) * kKC);
        mfma_chunk(buf);
        lstore((kc + 1) * kKC, buf ^ 1);
        __syncthreads();
      }
      mfma_chunk((nch - 1) & 1);
    } else {
      for (int kc = 0; kc + 1 < nch; ++kc) {
        const int buf = kc & 1;
        gload((kc + 1) * kKC);
        mfma_chunk_edge(buf);
        lstore((kc + 1) * kKC, buf ^ 1);
        __syncthreads();
      }
      mfma_chunk_edge((nch - 1) & 1);
    }
    __syncthreads();   // LDS free for this workgroup's next item
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (edge && (ii || jj || !eact)) continue;
          const int row = r0 + (edge ? er0 : 32 * wr + 16 * ii) + Mfma<T>::drow(lk, v);
          const int col = c0 + (edge ? ec0 : 32 * wc + 16 * jj) + li;
          if (row < n && col < n) {
            const int rc = rcv[ii][v];
            const bool keep = !(rc >= J0 && rc < J0 + wO);
            const cplx<T> cv = xm[(size_t)row * ld + col];
            cplx<T> c;
            const T q1 = p1[ii][jj][v], q2 = p2[ii][jj][v];
            c.re = (q1 - q2) + (keep ? cv.re : T(0));
            c.im = ((p3[ii][jj][v] - q1) - q2) + (keep ? cv.im : T(0));
            xm[(size_t)row * ld + col] = c;
          }
        }
  }
}

// --------------------------------------------------------------- launchers
template <typename T>
hipError_t gje_panel(cplx<T>* x, int* piv, int* rowcol, const MatDesc* d,
                     int nmat, int nmax, int S, int* status, hipStream_t st) {
  // the dynamic-LDS limit is a per-device attribute of each kernel: set once
  // per device (outside any graph capture: the first call on a device may
  // pass nmat = 0 for just this)
  static std::atomic<unsigned> attr_set{0u};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  const unsigned bit = dev < 32 ? (1u << dev) : 0u;
  const size_t lds_s = panel_lds_bytes<T>(kRPTs), lds_l = panel_lds_bytes<T>(kRPTl);
  if (!bit || !(attr_set.load() & bit)) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_outer_panel<T, kRPTs, kIBs>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_s);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(
          reinterpret_cast<const void*>(&k_outer_panel<T, kRPTl, kIBl>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_l);
    if (e != hipSuccess) return e;
    attr_set.fetch_or(bit);
  }
  if (nmat <= 0) return hipSuccess;
  if (nmax > kMaxN) return hipErrorInvalidValue;
  if (nmax <= kSmallN)
    hipLaunchKernelGGL((k_outer_panel<T, kRPTs, kIBs>), dim3(nmat), dim3(kPanelThreads),
                       lds_s, st, x, piv, rowcol, d, S, status);
  else
    hipLaunchKernelGGL((k_outer_panel<T, kRPTl, kIBl>), dim3(nmat), dim3(kPanelThreads),
                       lds_l, st, x, piv, rowcol, d, S, status);
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
hipError_t gje_fix(cplx<T>* x, const cplx<T>* bbuf, const int* piv,
                   const MatDesc* d, int nmat, int S, hipStream_t st) {
  if (nmat <= 0 || S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fix<T>, dim3(S * kNBO / 64, nmat), dim3(512), 0, st, x,
                     bbuf, piv, d, S);
  return hipGetLastError();
}

template <typename T>
hipError_t gje_update(cplx<T>* x, const cplx<T>* bbuf, const int* rowcol,
                      const MatDesc* d, const TileItem* items, int nitems,
                      int variant, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  // one workgroup per item (a persistent grid of two workgroups per CU
  // measured 4% slower: the dispatcher already overlaps the tiles' prologues)
  const int grid = 8 * ((nitems + 7) / 8);
  if (variant == 1)
    hipLaunchKernelGGL((k_update<T, 4>), dim3(grid), dim3(512), 0, st, x, bbuf,
                       rowcol, d, items, nitems);
  else
    hipLaunchKernelGGL((k_update<T, 2>), dim3(grid), dim3(256), 0, st, x, bbuf,
                       rowcol, d, items, nitems);
  return hipGetLastError();
}

#define FK_INST(T)                                                            \
  template hipError_t gje_panel<T>(cplx<T>*, int*, int*, const MatDesc*, int, \
                                   int, int, int*, hipStream_t);              \
  template hipError_t gje_gather<T>(const cplx<T>*, cplx<T>*, const int*,     \
                                    const MatDesc*, int, int, hipStream_t);   \
  template hipError_t gje_fix<T>(cplx<T>*, const cplx<T>*, const int*,       \
                                 const MatDesc*, int, int, hipStream_t);      \
  template hipError_t gje_update<T>(cplx<T>*, const cplx<T>*, const int*,     \
                                    const MatDesc*, const TileItem*, int, int, \
                                    hipStream_t);
FK_INST(double)
FK_INST(float)

}  // namespace fk
