// Host-side driver pieces shared by the single-instance context and the
// multi-instance sweep: fill kernels, the inversion batch (uniform or uneven
// matrix sizes) and the blocked Gauss-Jordan schedule.
#pragma once

#include <algorithm>
#include <vector>

#include "fk_internal.h"
#include "fk_kernels.h"

namespace fk {
namespace {


__global__ void k_fill_int(int* p, int v, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}
__global__ void k_fill_f64(double* p, double v, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

hipError_t fill_int(int* p, int v, size_t n, hipStream_t st) {
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_fill_int, dim3((int)g), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}
hipError_t fill_u64(unsigned long long* p, unsigned long long v, int n,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, v, n);
  return hipGetLastError();
}
hipError_t fill_f64(double* p, double v, size_t n, hipStream_t st) {
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_fill_f64, dim3((int)g), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// A batch of same-size matrices for the blocked Gauss-Jordan inversion.
template <typename T> struct Batch {
  int cap = 0, n = 0, ld = 0;
  size_t stride = 0;
  cplx<T>* x = nullptr;
  cplx<T>* bbuf = nullptr;     // gathered pivot rows, kBRows x ld per matrix
  int* piv = nullptr;
  int* rowcol = nullptr;
  int* status = nullptr;
  MatDesc* descs = nullptr;
  TileItem* items = nullptr;
  // per outer step S and update phase q (kPhases): tile items, matrix-major
  // so that a prefix serves fewer matrices (uniform batches: cnt items and
  // flp algorithmic flops per matrix; uneven: tot items, flp flops in all)
  std::vector<int> off[kPhases], cnt[kPhases], tot[kPhases];
  std::vector<double> flp[kPhases];
  int nouter = 0;
  int nmax = 0;       // largest matrix (selects the panel shape)
  // uneven batches (matrices of different sizes packed back to back): total
  // pivot ints and capacities of the buffers
  bool uniform = true;
  size_t nints = 0;
  size_t x_cap = 0, b_cap = 0, i_cap = 0, it_cap = 0;
  int d_cap = 0;
  bool owns = true;   // false: x/bbuf/piv/rowcol are borrowed shared storage
  int variant = 0;    // trailing-update tile shape (see gje_update)
};

template <typename T> void batch_free(Batch<T>& b) {
  if (b.owns) {
    if (b.x) (void)hipFree(b.x);
    if (b.bbuf) (void)hipFree(b.bbuf);
    if (b.piv) (void)hipFree(b.piv);
    if (b.rowcol) (void)hipFree(b.rowcol);
  }
  if (b.status) (void)hipFree(b.status);
  if (b.descs) (void)hipFree(b.descs);
  if (b.items) (void)hipFree(b.items);
  b = Batch<T>();
}

// Update work items of matrix m (n rows, tiles of tr_rows rows) for outer
// step S and phase q, and their algorithmic flops (8 per complex multiply-add:
// rows x columns x K per tile).  With block S at position p of the group that
// starts at block g0 = S - p (block_pos), the phases of step S:
//   q = 0  p = 0: the next block's columns, K = block S;  p > 0: the columns
//          of the group's earlier blocks g0 .. S-1, M = block S (side rows
//          p kNBO ..), bringing them up to date
//   q = 1  p > 0: the next block's columns, the transforms of blocks g0 .. S
//   q = 2  last block of its group: the trailing update of every column
//          outside blocks g0 .. S+1 with the group's transforms (K up to
//          kBRows); nothing for the other blocks (delayed)
// Items are ordered in bands of kSwz column tiles, rows outer within a band,
// so the workgroups in flight on one XCD (consecutive items) share both their
// pivot-block rows and their B columns in its L2.
constexpr int kSwz = 8;
// The transform and the column blocks of phase q of step S (see above):
// M = columns [jb kNBO, jb kNBO + kw), B = side-buffer rows [b0, b0 + kw); for
// q < 2 the column blocks lo .. hi (none if hi < lo), for q = 2 every block
// outside lo .. hi (none if kw = 0).
struct PhasePlan {
  int jb, kw, b0, lo, hi;
};
inline PhasePlan phase_plan(int n, int S, int q) {
  const int nout = (n + kNBO - 1) / kNBO;
  PhasePlan pl{S, 0, 0, 0, -1};
  if (S >= nout) return pl;
  const int p = block_pos(n, S), g0 = S - p;
  auto width = [&](int blk) { return std::min(kNBO, n - blk * kNBO); };
  int group_w = 0;               // columns of blocks g0 .. S
  for (int blk = g0; blk <= S; ++blk) group_w += width(blk);
  const bool next = S + 1 < nout;
  pl.kw = width(S);
  if (q == 0) {
    if (p > 0) {
      pl.lo = g0;
      pl.hi = S - 1;
      pl.b0 = p * kNBO;
    } else if (next) {
      pl.lo = pl.hi = S + 1;
    }
  } else if (q == 1) {
    if (p > 0 && next) {
      pl.lo = pl.hi = S + 1;
      pl.jb = g0;
      pl.kw = group_w;
    }
  } else {
    if (!block_last(n, S)) {
      pl.kw = 0;
      return pl;
    }
    pl.jb = g0;
    pl.kw = group_w;
    pl.lo = g0;
    pl.hi = S + 1;
  }
  return pl;
}
inline double push_tiles(std::vector<TileItem>& it, int m, int n, int tr_rows, int S,
                         int q) {
  const int nout = (n + kNBO - 1) / kNBO;
  if (S >= nout) return 0.0;
  const PhasePlan pl = phase_plan(n, S, q);
  if (q == 2 && pl.kw == 0) return 0.0;
  const int jb = pl.jb, kw = pl.kw, b0 = pl.b0;
  const int lo = pl.lo, hi = pl.hi, x0 = pl.lo, x1 = pl.hi;
  const int nt = (n + kTile - 1) / kTile, ntr = (n + tr_rows - 1) / tr_rows;
  std::vector<int> cols;
  for (int tc = 0; tc < nt; ++tc) {
    const int blk = tc / (kNBO / kTile);
    const bool take = q < 2 ? (blk >= lo && blk <= hi) : (blk < x0 || blk > x1);
    if (take) cols.push_back(tc);
  }
  double flops = 0.0;
  for (size_t c0 = 0; c0 < cols.size(); c0 += kSwz) {
    const size_t c1 = std::min(cols.size(), c0 + kSwz);
    for (int tr = 0; tr < ntr; ++tr)
      for (size_t c = c0; c < c1; ++c) {
        it.push_back(TileItem{m, (short)tr, (short)cols[c], (short)jb, (short)kw,
                              (short)b0, 0});
        flops += 8.0 * std::min(tr_rows, n - tr * tr_rows) *
                 std::min(kTile, n - cols[c] * kTile) * (double)kw;
      }
  }
  return flops;
}

// Allocate a uniform batch of cap n x n matrices.  On any failure every buffer
// is released and the batch is left empty (cap 0, x null), so a caller that
// checks x and cap reallocates instead of launching on a partial batch.
template <typename T>
hipError_t batch_alloc_parts(Batch<T>& b, int cap, int n, int variant);
template <typename T>
hipError_t batch_alloc(Batch<T>& b, int cap, int n, int variant = 0) {
  const hipError_t e = batch_alloc_parts(b, cap, n, variant);
  if (e != hipSuccess) batch_free(b);
  return e;
}

template <typename T>
hipError_t batch_alloc_parts(Batch<T>& b, int cap, int n, int variant) {
  batch_free(b);
  b.variant = variant;
  b.n = n;
  b.nmax = n;
  b.ld = n;
  b.stride = (size_t)n * n;
  b.nouter = (n + kNBO - 1) / kNBO;
  hipError_t e;
  if ((e = hipMalloc(&b.x, sizeof(cplx<T>) * b.stride * cap)) != hipSuccess) return e;
  if ((e = hipMalloc(&b.bbuf, sizeof(cplx<T>) * (size_t)kBRows * b.ld * cap)) != hipSuccess)
    return e;
  if ((e = hipMalloc(&b.piv, sizeof(int) * (size_t)n * cap)) != hipSuccess) return e;
  if ((e = hipMalloc(&b.rowcol, sizeof(int) * (size_t)n * cap)) != hipSuccess) return e;
  if ((e = hipMalloc(&b.status, sizeof(int) * cap)) != hipSuccess) return e;
  std::vector<MatDesc> d(cap);
  for (int m = 0; m < cap; ++m) {
    d[m].xoff = (long long)b.stride * m;
    d[m].boff = (long long)kBRows * b.ld * m;
    d[m].n = n;
    d[m].ld = b.ld;
    d[m].ioff = n * m;
    d[m].status_idx = m;
  }
  if ((e = hipMalloc(&b.descs, sizeof(MatDesc) * cap)) != hipSuccess) return e;
  if ((e = hipMemcpy(b.descs, d.data(), sizeof(MatDesc) * cap,
                     hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  std::vector<TileItem> it;
  for (int q = 0; q < kPhases; ++q) {
    b.off[q].assign(b.nouter, 0);
    b.cnt[q].assign(b.nouter, 0);
    b.flp[q].assign(b.nouter, 0.0);
  }
  for (int S = 0; S < b.nouter; ++S) {
    for (int q = 0; q < kPhases; ++q) {
      b.off[q][S] = (int)it.size();
      for (int m = 0; m < cap; ++m) {
        const size_t before = it.size();
        b.flp[q][S] = push_tiles(it, m, n, tile_rows(variant), S, q);
        b.cnt[q][S] = (int)(it.size() - before);
      }
    }
  }
  if ((e = hipMalloc(&b.items, sizeof(TileItem) * std::max<size_t>(it.size(), 1))) !=
      hipSuccess)
    return e;
  if (!it.empty() && (e = hipMemcpy(b.items, it.data(), sizeof(TileItem) * it.size(),
                                    hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  b.cap = cap;   // complete: only now does the batch count as allocated
  return hipSuccess;
}

template <typename P> hipError_t grow(P** ptr, size_t* cap, size_t want) {
  if (*ptr && *cap >= want) return hipSuccess;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(ptr, sizeof(P) * std::max<size_t>(want, 1));
  if (e == hipSuccess) *cap = want;
  return e;
}

// Configure the batch for matrices of sizes n[m] (ld = n[m]) packed back to
// back.  status_idx[m] is the slot of matrix m in the status array passed to
// batch_invert (the caller zeroes it).  Buffers grow as needed and are kept.
template <typename T>
hipError_t batch_setup_uneven(Batch<T>& b, const std::vector<int>& n,
                              const std::vector<int>& status_idx) {
  const int nm = (int)n.size();
  b.uniform = false;
  b.cap = nm;
  b.n = 0;
  b.ld = 0;
  b.stride = 0;
  std::vector<MatDesc> d(nm);
  size_t xo = 0, bo = 0, io = 0;
  int nouter = 0;
  for (int m = 0; m < nm; ++m) {
    d[m].xoff = (long long)xo;
    d[m].boff = (long long)bo;
    d[m].n = n[m];
    d[m].ld = n[m];
    d[m].ioff = (int)io;
    d[m].status_idx = status_idx[m];
    xo += (size_t)n[m] * n[m];
    bo += (size_t)kBRows * n[m];
    io += (size_t)n[m];
    nouter = std::max(nouter, (n[m] + kNBO - 1) / kNBO);
  }
  b.nouter = nouter;
  b.nmax = 0;
  for (int m = 0; m < nm; ++m) b.nmax = std::max(b.nmax, n[m]);
  b.nints = io;
  hipError_t e;
  if ((e = grow(&b.x, &b.x_cap, xo)) != hipSuccess) return e;
  if ((e = grow(&b.bbuf, &b.b_cap, bo)) != hipSuccess) return e;
  size_t ic = b.i_cap;
  if ((e = grow(&b.piv, &ic, io)) != hipSuccess) return e;
  ic = b.i_cap;
  if ((e = grow(&b.rowcol, &ic, io)) != hipSuccess) return e;
  b.i_cap = std::max(b.i_cap, io);
  size_t dc = (size_t)b.d_cap;
  if ((e = grow(&b.descs, &dc, (size_t)nm)) != hipSuccess) return e;
  b.d_cap = (int)dc;
  if ((e = hipMemcpy(b.descs, d.data(), sizeof(MatDesc) * nm,
                     hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  std::vector<TileItem> it;
  for (int q = 0; q < kPhases; ++q) {
    b.off[q].assign(nouter, 0);
    b.tot[q].assign(nouter, 0);
    b.flp[q].assign(nouter, 0.0);
  }
  for (int S = 0; S < nouter; ++S) {
    for (int q = 0; q < kPhases; ++q) {
      b.off[q][S] = (int)it.size();
      for (int m = 0; m < nm; ++m)
        b.flp[q][S] += push_tiles(it, m, n[m], tile_rows(b.variant), S, q);
      b.tot[q][S] = (int)it.size() - b.off[q][S];
    }
  }
  if ((e = grow(&b.items, &b.it_cap, it.size())) != hipSuccess) return e;
  if (it.empty()) return hipSuccess;
  return hipMemcpy(b.items, it.data(), sizeof(TileItem) * it.size(),
                   hipMemcpyHostToDevice);
}

// Optional timing of the dominant kernel, the trailing update (phase 2
// launch): an event pair around every such launch of a uniform batch, with the
// launch's algorithmic flops, 8 per complex multiply-add (rows x columns x K
// summed over its tiles).
struct KernelClock {
  bool on = false;
  std::vector<hipEvent_t> ev;   // event pairs
  std::vector<double> flops;    // per recorded pair
  int used = 0;                 // events in use
  double ms = 0.0, flop = 0.0;
  long long launches = 0;
};

inline void clock_collect(KernelClock& k) {
  for (int i = 0; i + 1 < k.used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, k.ev[i], k.ev[i + 1]) == hipSuccess) {
      k.ms += ms;
      k.flop += k.flops[i / 2];
      k.launches++;
    }
  }
  k.used = 0;
  k.flops.clear();
}

// Side stream and events of the look-ahead (default priority).
struct Aux {
  hipStream_t st2 = nullptr;
  hipEvent_t evN = nullptr, evP = nullptr;
  bool lookahead = false;  // factor the next block on st2 (else in order on st)
  KernelClock* clk = nullptr;
};

// Invert matrices 0..nmat-1 of the batch in place (permuted storage).  With
// the look-ahead schedule the next outer block is factored on the side stream
// while the trailing update of the current group runs on st.  ev_steps (nullable) brackets the kernels.
// For an uneven batch nmat must be b.cap and status is the caller's array
// (indexed by the descriptors' status_idx, not cleared here).
template <typename T>
hipError_t batch_invert(Batch<T>& b, int nmat, hipStream_t st, const Aux& ax,
                        int* launches, hipEvent_t* ev_steps = nullptr,
                        int* status = nullptr) {
  hipError_t e;
  int* stat = status ? status : b.status;
  const size_t nints = b.uniform ? (size_t)b.n * nmat : b.nints;
  if ((e = fill_int(b.rowcol, -1, nints, st)) != hipSuccess) return e;
  if (!status && (e = fill_int(b.status, 0, (size_t)nmat, st)) != hipSuccess) return e;
  if (ev_steps && (e = hipEventRecord(ev_steps[0], st)) != hipSuccess) return e;
  int nl = 0;
  if ((e = gje_panel<T>(b.x, b.piv, b.rowcol, b.descs, nmat, b.nmax, 0, stat, st)) !=
      hipSuccess)
    return e;
  ++nl;
  auto items_of = [&](int q, int S, int* count) {
    *count = b.uniform ? nmat * b.cnt[q][S] : b.tot[q][S];
    return b.items + b.off[q][S];
  };
  for (int S = 0; S < b.nouter; ++S) {
    const bool next = S + 1 < b.nouter;
    if ((e = gje_gather<T>(b.x, b.bbuf, b.piv, b.descs, nmat, S, st)) != hipSuccess)
      return e;
    ++nl;
    if (S > 0) {
      if ((e = gje_fix<T>(b.x, b.bbuf, b.piv, b.descs, nmat, S, st)) != hipSuccess)
        return e;
      ++nl;
    }
    // the group's earlier blocks' columns and the next block's columns, so
    // that the next panel can start
    for (int q = 0; q < 2; ++q) {
      int cnt = 0;
      const TileItem* it = items_of(q, S, &cnt);
      if (cnt > 0) {
        if ((e = gje_update<T>(b.x, b.bbuf, b.rowcol, b.descs, it, cnt, b.variant, st)) !=
            hipSuccess)
          return e;
        ++nl;
      }
    }
    if (next) {
      hipStream_t ps = ax.lookahead ? ax.st2 : st;
      if (ax.lookahead) {
        if ((e = hipEventRecord(ax.evN, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ax.st2, ax.evN, 0)) != hipSuccess) return e;
      }
      if ((e = gje_panel<T>(b.x, b.piv, b.rowcol, b.descs, nmat, b.nmax, S + 1, stat,
                            ps)) != hipSuccess)
        return e;
      ++nl;
      if (ax.lookahead && (e = hipEventRecord(ax.evP, ax.st2)) != hipSuccess) return e;
    }
    int nB = 0;
    const TileItem* itB = items_of(2, S, &nB);
    if (nB > 0) {
      KernelClock* ck = (ax.clk && b.uniform &&
                         ax.clk->used + 2 <= (int)ax.clk->ev.size()) ? ax.clk : nullptr;
      if (ck && (e = hipEventRecord(ck->ev[ck->used], st)) != hipSuccess) return e;
      if ((e = gje_update<T>(b.x, b.bbuf, b.rowcol, b.descs, itB, nB, b.variant, st)) !=
          hipSuccess)
        return e;
      ++nl;
      if (ck) {
        if ((e = hipEventRecord(ck->ev[ck->used + 1], st)) != hipSuccess) return e;
        ck->flops.push_back(b.flp[2][S] * nmat);
        ck->used += 2;
      }
    }
    if (next && ax.lookahead && (e = hipStreamWaitEvent(st, ax.evP, 0)) != hipSuccess)
      return e;
  }
  if (ev_steps && (e = hipEventRecord(ev_steps[1], st)) != hipSuccess) return e;
  if (launches) *launches += nl;
  return hipSuccess;
}


}  // namespace
}  // namespace fk
