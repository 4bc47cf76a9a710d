// Multi-instance sweep: several DMFT problems (different contours, U, E) run
// their self-consistency loops together.  Every lattice step of a sweep puts
// the point matrices of all active instances into uneven batches, so each
// Gauss-Jordan step is one launch over (instance, point, tile) work items;
// the impurity updates of all instances share one batched inversion (the
// one-inversion form of the single-instance update).  The
// sweep is recorded once into a hipGraph and replayed; it is re-recorded when
// an instance converges and retires.
#include "fk_ctx.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <chrono>
#include <limits>
#include <string>
#include <vector>

using namespace fk;

namespace fk {

// Per-instance device view for the convergence norm.
struct InstDev {
  c64* gloc;
  c64* gprev;
  int n;
  int key;           // slot of this instance in the key array (2 per instance)
};

// delta = max |G_loc - G_prev| into keys[key], then G_prev <- G_loc
__global__ void k_delta(const InstDev* __restrict__ inst,
                        unsigned long long* __restrict__ keys) {
  const InstDev d = inst[blockIdx.y];
  const size_t total = (size_t)d.n * d.n;
  double mx = 0.0;
  bool bad = false;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const c64 g = d.gloc[e], p = d.gprev[e];
    const double dr = g.re - p.re, di = g.im - p.im;
    const double a = sqrt(dr * dr + di * di);
    if (!(a <= 1.79769313486231570815e308)) bad = true;
    else if (a > mx) mx = a;
    d.gprev[e] = g;
  }
  unsigned long long k = bad ? 0x7ff8000000000000ULL
                             : (unsigned long long)__double_as_longlong(mx);
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(k, off);
    k = o > k ? o : k;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(&keys[d.key], k);
}

}  // namespace fk

// ======================================================================= batch
struct Segment {
  int inst, k0, cnt;
  size_t xoff, ioff;
};
struct Chunk {
  fk::Batch<double> b;   // descriptors and tile lists; storage borrowed
  std::vector<Segment> segs;
};

struct fk_batch {
  hipStream_t st = nullptr;
  std::vector<fk_ctx*> inst;
  std::vector<int> active;
  std::vector<int> iters;
  std::vector<double> delta;
  std::vector<Chunk> chunks;
  fk::Batch<double> impA;   // the impurity slot of every active instance
  // shared storage of the lattice chunks and of the impurity slots
  c64* x = nullptr;
  c64* bbuf = nullptr;
  int* piv = nullptr;
  int* rowcol = nullptr;
  size_t x_cap = 0, b_cap = 0, i_cap = 0, i2_cap = 0;
  c64* xi = nullptr;
  c64* bi = nullptr;
  std::vector<size_t> imp_s0, imp_i0;   // per active instance: slot offsets
  std::vector<int> status_inst, status_point;   // per status slot (point -1: impurity)
  int* pivi = nullptr;
  int* rci = nullptr;
  size_t xi_cap = 0, bi_cap = 0, ii_cap = 0, ii2_cap = 0;
  int* d_status = nullptr;
  size_t status_cap = 0;
  int n_status = 0;
  unsigned long long* d_keys = nullptr;
  InstDev* d_inst = nullptr;
  size_t inst_cap = 0;
  int n_active_dev = 0;
  double chunk_bytes = 24.0 * (1 << 30);
  fk::Aux aux;
  bool dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_for_plan = false;
  int captures = 0;
  double capture_ms = 0.0, last_sweep_ms = 0.0, total_ms = 0.0;
  int max_nc = 0;
  int variant = 0;
  // per N_c class schedule from fk_batch_autotune (empty: one schedule for
  // all, chunk_bytes and variant above)
  std::vector<int> class_nc;
  std::vector<fk_tuning> class_tuning;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
};

namespace {

fk_status berr(fk_batch* b, fk_status s, const char* fmt, ...) {
  if (b) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
  }
  return s;
}

#define BCHK(bt, expr)                                                      \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return berr((bt), e_ == hipErrorOutOfMemory ? FK_ENOMEM : FK_EDEVICE, \
                  "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,  \
                  __LINE__);                                                \
  } while (0)

void drop_graph(fk_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_for_plan = false;
}

// Point the borrowed storage of a chunk batch at the shared buffers.
void borrow(fk::Batch<double>& cb, c64* x, size_t xc, c64* bb, size_t bc,
            int* pv, int* rc, size_t ic) {
  cb.owns = false;
  cb.x = x;
  cb.x_cap = xc;
  cb.bbuf = bb;
  cb.b_cap = bc;
  cb.piv = pv;
  cb.rowcol = rc;
  cb.i_cap = ic;
}

// Chunk plan for the active instances: point matrices ordered by instance,
// cut into chunks that fit chunk_bytes; impurity slots after them.  With a
// per-class schedule (fk_batch_autotune) the instances are ordered by contour
// size, a chunk holds one size class only, at most that class's tuned number
// of matrices, and runs that class's tile shape.
int class_of(const fk_batch* b, int n_c) {
  for (size_t q = 0; q < b->class_nc.size(); ++q)
    if (b->class_nc[q] == n_c) return (int)q;
  return -1;
}

fk_status build_plan(fk_batch* b) {
  drop_graph(b);
  for (Chunk& c : b->chunks) batch_free(c.b);
  b->chunks.clear();
  struct Job { int inst, k; };
  std::vector<int> order = b->active;
  const bool per_class = !b->class_nc.empty();
  if (per_class)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return b->inst[x]->ci.n_c < b->inst[y]->ci.n_c;
    });
  std::vector<std::vector<Job>> groups(1);
  std::vector<int> group_variant(1, b->variant);
  double used = 0.0;
  int used_mats = 0, cur_class = -2;
  for (int id : order) {
    const fk_ctx* c = b->inst[id];
    const double n = c->ci.n_c;
    const double per = 16.0 * (n * n + kBRows * n) + 8.0 * n;
    const int cls = per_class ? class_of(b, c->ci.n_c) : -1;
    double cap_bytes = b->chunk_bytes;
    int cap_mats = 1 << 30, variant = b->variant;
    if (cls >= 0) {
      cap_bytes = std::numeric_limits<double>::max();   // the tuned count was sized in bytes
      cap_mats = std::max(1, b->class_tuning[cls].batch);
      variant = b->class_tuning[cls].tile_rows == 128 ? 1 : 0;
    }
    for (int k = 0; k < c->npts; ++k) {
      const bool full = used + per > cap_bytes || used_mats >= cap_mats;
      if (!groups.back().empty() && (full || (per_class && cls != cur_class))) {
        groups.emplace_back();
        group_variant.push_back(variant);
        used = 0.0;
        used_mats = 0;
      }
      if (groups.back().empty()) group_variant.back() = variant;
      cur_class = cls;
      groups.back().push_back(Job{id, k});
      used += per;
      ++used_mats;
    }
  }
  if (groups.back().empty()) {
    groups.pop_back();
    group_variant.pop_back();
  }
  // storage needs
  size_t xmax = 0, bmax = 0, imax = 0;
  int status = 0;
  std::vector<std::vector<int>> sizes(groups.size()), sidx(groups.size());
  b->status_inst.clear();
  b->status_point.clear();
  for (size_t g = 0; g < groups.size(); ++g) {
    size_t xs = 0, bs = 0, is = 0;
    for (const Job& j : groups[g]) {
      const int n = b->inst[j.inst]->ci.n_c;
      sizes[g].push_back(n);
      sidx[g].push_back(status++);
      b->status_inst.push_back(j.inst);
      b->status_point.push_back(j.k);
      xs += (size_t)n * n;
      bs += (size_t)kBRows * n;
      is += n;
    }
    xmax = std::max(xmax, xs);
    bmax = std::max(bmax, bs);
    imax = std::max(imax, is);
  }
  BCHK(b, grow(&b->x, &b->x_cap, xmax));
  BCHK(b, grow(&b->bbuf, &b->b_cap, bmax));
  BCHK(b, grow(&b->piv, &b->i_cap, imax));
  BCHK(b, grow(&b->rowcol, &b->i2_cap, imax));
  b->chunks.resize(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) {
    Chunk& ch = b->chunks[g];
    borrow(ch.b, b->x, b->x_cap, b->bbuf, b->b_cap, b->piv, b->rowcol, b->i_cap);
    ch.b.variant = group_variant[g];
    BCHK(b, batch_setup_uneven(ch.b, sizes[g], sidx[g]));
    size_t xo = 0, io = 0;
    for (const Job& j : groups[g]) {
      const int n = b->inst[j.inst]->ci.n_c;
      if (ch.segs.empty() || ch.segs.back().inst != j.inst)
        ch.segs.push_back(Segment{j.inst, j.k, 0, xo, io});
      ch.segs.back().cnt++;
      xo += (size_t)n * n;
      io += n;
    }
  }
  // impurity slots: one per active instance
  const int na = (int)b->active.size();
  std::vector<int> isz(na), isx(na);
  size_t xs = 0, bs = 0, is = 0;
  for (int a = 0; a < na; ++a) {
    const int n = b->inst[b->active[a]]->ci.n_c;
    isz[a] = n;
    isx[a] = status++;
    b->status_inst.push_back(b->active[a]);
    b->status_point.push_back(-1);
    xs += (size_t)n * n;
    bs += (size_t)kBRows * n;
    is += n;
  }
  BCHK(b, grow(&b->xi, &b->xi_cap, xs));
  BCHK(b, grow(&b->bi, &b->bi_cap, bs));
  BCHK(b, grow(&b->pivi, &b->ii_cap, is));
  BCHK(b, grow(&b->rci, &b->ii2_cap, is));
  batch_free(b->impA);
  borrow(b->impA, b->xi, b->xi_cap, b->bi, b->bi_cap, b->pivi, b->rci, b->ii_cap);
  BCHK(b, batch_setup_uneven(b->impA, isz, isx));
  b->n_status = status;
  BCHK(b, grow(&b->d_status, &b->status_cap, (size_t)status));
  // instance views
  std::vector<InstDev> iv(na);
  b->imp_s0.assign(na, 0);
  b->imp_i0.assign(na, 0);
  size_t so = 0, ioff = 0;
  for (int a = 0; a < na; ++a) {
    fk_ctx* c = b->inst[b->active[a]];
    const int n = c->ci.n_c;
    b->imp_s0[a] = so;
    b->imp_i0[a] = ioff;
    so += (size_t)n * n;
    ioff += n;
    InstDev& d = iv[a];
    d.gloc = c->d_gloc;
    d.gprev = c->d_gprev;
    d.n = n;
    d.key = 2 * b->active[a];
  }
  BCHK(b, grow(&b->d_inst, &b->inst_cap, (size_t)std::max(na, 1)));
  if (na) BCHK(b, hipMemcpy(b->d_inst, iv.data(), sizeof(InstDev) * na, hipMemcpyHostToDevice));
  b->n_active_dev = na;
  b->dirty = false;
  return FK_OK;
}

// Shifts of the Falicov-Kimball update of one instance (model convention):
// d0, d1 for the empty and occupied f site, d_c = (1 - w1) d1 + w1 d0, h =
// (1 - w1) d0 + w1 d1, gam = w1 (1 - w1) (d0 - d1)^2.
void imp_shifts(const fk_ctx* c, double* dc, double* h, double* gam) {
  const double d0 = c->m.convention == 0 ? 0.5 * c->m.U : 0.0;
  const double d1 = c->m.convention == 0 ? -0.5 * c->m.U : -c->m.U;
  const double w1 = c->m.w1;
  *dc = (1.0 - w1) * d1 + w1 * d0;
  *h = (1.0 - w1) * d0 + w1 * d1;
  *gam = w1 * (1.0 - w1) * (d0 - d1) * (d0 - d1);
}

// Enqueue one sweep (lattice steps of all active instances, convergence norm,
// impurity updates) on b->st.  Stream work only: capturable into a graph.
hipError_t record_sweep(fk_batch* b) {
  hipError_t e;
  if ((e = fill_int(b->d_status, 0, (size_t)b->n_status, b->st)) != hipSuccess) return e;
  for (int id : b->active) {
    fk_ctx* c = b->inst[id];
    const int n = c->ci.n_c;
    if ((e = launch_sigma_weight(c->d_sigma, c->d_w, c->d_sigt, n, b->st)) != hipSuccess)
      return e;
    if ((e = fill_f64(reinterpret_cast<double*>(c->d_gloc), 0.0, 2 * (size_t)n * n, b->st)) !=
        hipSuccess)
      return e;
    if ((e = fill_f64(c->d_cur, 0.0, (size_t)c->ci.n_t, b->st)) != hipSuccess) return e;
  }
  for (Chunk& ch : b->chunks) {
    for (const Segment& sg : ch.segs) {
      fk_ctx* c = b->inst[sg.inst];
      const int n = c->ci.n_c;
      if ((e = launch_build<double>(c->d_sigt, c->tab, sg.k0, sg.cnt, b->x + sg.xoff,
                                    (size_t)n * n, n, n, b->st)) != hipSuccess)
        return e;
    }
    if ((e = batch_invert<double>(ch.b, ch.b.cap, b->st, b->aux, nullptr, nullptr,
                                  b->d_status)) != hipSuccess)
      return e;
    for (const Segment& sg : ch.segs) {
      fk_ctx* c = b->inst[sg.inst];
      const int n = c->ci.n_c;
      if ((e = launch_reduce<double>(b->x + sg.xoff, (size_t)n * n, n, b->piv + sg.ioff,
                                     b->rowcol + sg.ioff, n, c->d_rho + sg.k0, sg.cnt,
                                     n, c->d_gloc, 1, b->st)) != hipSuccess)
        return e;
      if ((e = launch_current<double>(b->x + sg.xoff, (size_t)n * n, n,
                                      b->piv + sg.ioff, b->rowcol + sg.ioff, n, c->tab,
                                      sg.k0, sg.cnt, c->ci.n_t, n, c->d_cur, b->st)) !=
          hipSuccess)
        return e;
    }
  }
  if ((e = fill_u64(b->d_keys, 0ULL, 2 * (int)b->inst.size(), b->st)) != hipSuccess)
    return e;
  if (b->n_active_dev == 0) return hipSuccess;
  int nmax = 0;
  for (int id : b->active) nmax = std::max(nmax, b->inst[id]->ci.n_c);
  const int gx = (int)std::min<size_t>(((size_t)nmax * nmax + 255) / 256, 1024);
  hipLaunchKernelGGL(k_delta, dim3(gx, b->n_active_dev), dim3(256), 0, b->st,
                     b->d_inst, b->d_keys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // impurity updates, the single-instance form: with X = G_loc W and
  // Y = Sigma W + d_c S, Sigma_new W = -h S + gam S X (I + Y X)^-1 S; the
  // matrices I + Y X of all instances share one batched inversion
  const int na = b->n_active_dev;
  for (int a = 0; a < na; ++a) {
    fk_ctx* c = b->inst[b->active[a]];
    const int n = c->ci.n_c;
    double dc, h, gam;
    imp_shifts(c, &dc, &h, &gam);
    c64* slot = b->xi + b->imp_s0[a];
    if ((e = launch_right_weight(c->d_gloc, c->d_w, c->d_g0inv, n, n, b->st)) != hipSuccess)
      return e;
    if ((e = launch_right_weight(c->d_sigma, c->d_w, c->d_tmp, n, n, b->st)) != hipSuccess)
      return e;
    if ((e = launch_bgemm(slot, nullptr, 0.0, c->d_tmp, 0, c->d_g0inv, n, 1, b->st)) !=
        hipSuccess)
      return e;
    if ((e = launch_add_identity_shift(slot, n, c->d_g0inv, dc, n, b->st)) != hipSuccess)
      return e;
  }
  if ((e = batch_invert<double>(b->impA, na, b->st, b->aux, nullptr, nullptr,
                                b->d_status)) != hipSuccess)
    return e;
  for (int a = 0; a < na; ++a) {
    const int id = b->active[a];
    fk_ctx* c = b->inst[id];
    const int n = c->ci.n_c;
    double dc, h, gam;
    imp_shifts(c, &dc, &h, &gam);
    c64* slot = b->xi + b->imp_s0[a];
    // (I + Y X)^-1 in natural order, then C^-1 = X (I + Y X)^-1 into the slot
    if ((e = launch_unpermute<double>(slot, (size_t)n * n, n, b->pivi + b->imp_i0[a],
                                      b->rci + b->imp_i0[a], n, 1, c->d_tmp, b->st)) !=
        hipSuccess)
      return e;
    if ((e = launch_bgemm(slot, nullptr, 0.0, c->d_g0inv, 0, c->d_tmp, n, 1, b->st)) !=
        hipSuccess)
      return e;
    if ((e = launch_sigma_fk(slot, c->d_w, c->d_sigma, n, h, gam, b->d_keys + 2 * id + 1,
                             b->st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

}  // namespace

// ===================================================================== C ABI
extern "C" fk_status fk_batch_create(int n_inst, const fk_contour* contours,
                                     const fk_model* models, fk_batch** out) {
  if (n_inst < 1 || !contours || !models || !out) return FK_EINVAL;
  *out = nullptr;
  fk_batch* b = new (std::nothrow) fk_batch();
  if (!b) return FK_ENOMEM;
  hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return FK_EDEVICE;
  }
  for (int i = 0; i < n_inst; ++i) {
    fk_ctx* c = nullptr;
    const fk_status s = fk_create(&contours[i], &models[i], b->st, &c);
    if (s != FK_OK) {
      fk_batch_destroy(b);
      return s;
    }
    b->inst.push_back(c);
    b->active.push_back(i);
    b->max_nc = std::max(b->max_nc, c->ci.n_c);
  }
  b->iters.assign(n_inst, 0);
  b->delta.assign(n_inst, std::numeric_limits<double>::infinity());
  if (const char* s = getenv("FKDMFT_BATCH_BYTES")) {
    const double v = atof(s);
    if (v > 0) b->chunk_bytes = v;
  }
  e = hipMalloc(&b->d_keys, sizeof(unsigned long long) * 2 * n_inst);
  if (e == hipSuccess) e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->aux.st2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->aux.evN, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->aux.evP, hipEventDisableTiming);
  // set the kernels' LDS attribute outside any capture
  if (e == hipSuccess) e = gje_panel<double>(nullptr, nullptr, nullptr, nullptr, 0, 0, 0, nullptr, b->st);
  if (e != hipSuccess) {
    fk_batch_destroy(b);
    return FK_EDEVICE;
  }
  *out = b;
  return FK_OK;
}

extern "C" fk_status fk_batch_destroy(fk_batch* b) {
  if (!b) return FK_OK;
  if (b->st) (void)hipStreamSynchronize(b->st);
  drop_graph(b);
  for (Chunk& c : b->chunks) batch_free(c.b);
  batch_free(b->impA);
  void* ps[] = {b->x, b->bbuf, b->piv, b->rowcol, b->xi, b->bi, b->pivi, b->rci,
                b->d_status, b->d_keys, b->d_inst};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  for (fk_ctx* c : b->inst) fk_destroy(c);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->aux.evN) (void)hipEventDestroy(b->aux.evN);
  if (b->aux.evP) (void)hipEventDestroy(b->aux.evP);
  if (b->aux.st2) (void)hipStreamDestroy(b->aux.st2);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
  return FK_OK;
}

extern "C" const char* fk_batch_last_error(const fk_batch* b) {
  return b ? b->err.c_str() : "NULL batch";
}

extern "C" fk_status fk_batch_instance(const fk_batch* b, int i, fk_ctx** ctx) {
  if (!b || !ctx || i < 0 || i >= (int)b->inst.size()) return FK_EINVAL;
  *ctx = b->inst[i];
  return FK_OK;
}

extern "C" fk_status fk_batch_set_chunk_bytes(fk_batch* b, double bytes) {
  if (!b || !(bytes > 0)) return FK_EINVAL;
  b->chunk_bytes = bytes;
  b->dirty = true;
  return FK_OK;
}

extern "C" fk_status fk_batch_reset(fk_batch* b) {
  if (!b) return FK_EINVAL;
  b->active.clear();
  for (int i = 0; i < (int)b->inst.size(); ++i) {
    b->active.push_back(i);
    b->iters[i] = 0;
    b->delta[i] = std::numeric_limits<double>::infinity();
  }
  b->dirty = true;
  return FK_OK;
}

extern "C" fk_status fk_batch_iterate(fk_batch* b, int max_sweeps, double tol,
                                      int use_graph, int* sweeps_out, int* iters,
                                      double* deltas) {
  if (!b || max_sweeps < 1) return FK_EINVAL;
  int sweep = 0;
  const int ninst = (int)b->inst.size();
  std::vector<int> st;
  std::vector<unsigned long long> keys(2 * ninst);
  for (sweep = 0; sweep < max_sweeps && !b->active.empty(); ++sweep) {
    if (b->dirty) {
      const fk_status s = build_plan(b);
      if (s != FK_OK) return s;
    }
    // the active instances' G_loc are rewritten by this sweep: valid again
    // only once it has succeeded
    for (int id : b->active) b->inst[id]->have_gloc = false;
    if (use_graph && !b->graph_for_plan) {
      drop_graph(b);
      const auto t0 = std::chrono::steady_clock::now();
      BCHK(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
      hipError_t e = record_sweep(b);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(b->st, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return berr(b, FK_EDEVICE, "graph capture failed: %s / %s",
                    hipGetErrorString(e), hipGetErrorString(e2));
      }
      b->graph = g;
      BCHK(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
      b->graph_for_plan = true;
      b->captures++;
      b->capture_ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t0).count();
    }
    BCHK(b, hipEventRecord(b->ev0, b->st));
    if (use_graph) {
      BCHK(b, hipGraphLaunch(b->gexec, b->st));
    } else {
      BCHK(b, record_sweep(b));
    }
    BCHK(b, hipEventRecord(b->ev1, b->st));
    st.assign(b->n_status, 0);
    BCHK(b, hipMemcpyAsync(st.data(), b->d_status, sizeof(int) * b->n_status,
                           hipMemcpyDeviceToHost, b->st));
    BCHK(b, hipMemcpyAsync(keys.data(), b->d_keys, sizeof(unsigned long long) * 2 * ninst,
                           hipMemcpyDeviceToHost, b->st));
    BCHK(b, hipStreamSynchronize(b->st));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
    b->last_sweep_ms = ms;
    b->total_ms += ms;
    for (int q = 0; q < b->n_status; ++q)
      if (st[q] != 0) {
        const char* what = st[q] > 0 ? "zero pivot" : "non-finite pivot";
        const int col = (st[q] > 0 ? st[q] : -st[q]) - 1;
        if (b->status_point[q] >= 0)
          return berr(b, st[q] > 0 ? FK_ESINGULAR : FK_ENONFINITE,
                      "sweep %d: instance %d: %s at column %d of matrix %d", sweep + 1,
                      b->status_inst[q], what, col, b->status_point[q]);
        return berr(b, st[q] > 0 ? FK_ESINGULAR : FK_ENONFINITE,
                    "sweep %d: instance %d: impurity update: %s at column %d",
                    sweep + 1, b->status_inst[q], what, col);
      }
    std::vector<int> still;
    for (int id : b->active) {
      b->iters[id]++;
      b->inst[id]->have_gloc = true;
      double dg, ds;
      std::memcpy(&dg, &keys[2 * id], sizeof dg);
      std::memcpy(&ds, &keys[2 * id + 1], sizeof ds);
      if (!(ds <= std::numeric_limits<double>::max()))
        return berr(b, FK_ENONFINITE, "instance %d: non-finite Sigma", id);
      b->delta[id] = (b->iters[id] == 1) ? std::numeric_limits<double>::infinity() : dg;
      if (!(b->delta[id] < tol)) still.push_back(id);
    }
    if (still.size() != b->active.size()) {
      b->active = still;
      b->dirty = true;
    }
  }
  if (sweeps_out) *sweeps_out = sweep;
  for (int i = 0; i < ninst; ++i) {
    if (iters) iters[i] = b->iters[i];
    if (deltas) deltas[i] = b->delta[i];
  }
  return FK_OK;
}

extern "C" fk_status fk_batch_timings(const fk_batch* b, double* out4) {
  if (!b || !out4) return FK_EINVAL;
  out4[0] = b->last_sweep_ms;
  out4[1] = b->total_ms;
  out4[2] = b->captures;
  out4[3] = b->capture_ms;
  return FK_OK;
}

extern "C" fk_status fk_batch_set_tuning(fk_batch* b, const fk_tuning* t) {
  if (!b || !t || (t->tile_rows != 64 && t->tile_rows != 128)) return FK_EINVAL;
  b->variant = t->tile_rows == 128 ? 1 : 0;
  b->aux.lookahead = t->lookahead != 0;
  if (t->chunk_bytes > 0) b->chunk_bytes = t->chunk_bytes;
  b->class_nc.clear();          // one schedule for every size class
  b->class_tuning.clear();
  b->dirty = true;
  return FK_OK;
}

extern "C" fk_status fk_batch_autotune(fk_batch* b, double max_bytes, int only_nc,
                                       int max_out, int* n_classes, int* class_nc,
                                       fk_tuning* class_tuning) {
  if (!b || !(max_bytes > 0) || max_out < 0 || only_nc < 0) return FK_EINVAL;
  // one representative instance per contour size (the first of each)
  std::vector<int> ncs, rep_inst;
  for (int i = 0; i < (int)b->inst.size(); ++i) {
    const int nc = b->inst[i]->ci.n_c;
    if (only_nc > 0 && nc != only_nc) continue;
    if (std::find(ncs.begin(), ncs.end(), nc) == ncs.end()) {
      ncs.push_back(nc);
      rep_inst.push_back(i);
    }
  }
  if (ncs.empty())
    return berr(b, FK_EINVAL, "no instance with N_c = %d", only_nc);
  std::vector<fk_tuning> tun(ncs.size());
  // the shared chunk storage is released first so the trials have the memory
  drop_graph(b);
  for (Chunk& c : b->chunks) batch_free(c.b);
  b->chunks.clear();
  void* shared[] = {b->x, b->bbuf, b->piv, b->rowcol};
  for (void* p : shared)
    if (p) (void)hipFree(p);
  b->x = nullptr;
  b->bbuf = nullptr;
  b->piv = b->rowcol = nullptr;
  b->x_cap = b->b_cap = b->i_cap = b->i2_cap = 0;
  for (size_t q = 0; q < ncs.size(); ++q) {
    fk_ctx* c = b->inst[rep_inst[q]];
    const fk_status s = fk_autotune(c, max_bytes, 0, &tun[q]);
    if (s != FK_OK)
      return berr(b, s, "autotune of N_c = %d (instance %d): %s", ncs[q], rep_inst[q],
                  fk_last_error(c));
  }
  // merge into the per-class table (a single class replaces its own entry)
  if (only_nc == 0) {
    b->class_nc.clear();
    b->class_tuning.clear();
  }
  for (size_t q = 0; q < ncs.size(); ++q) {
    const int at = class_of(b, ncs[q]);
    if (at >= 0) {
      b->class_tuning[at] = tun[q];
    } else {
      b->class_nc.push_back(ncs[q]);
      b->class_tuning.push_back(tun[q]);
    }
  }
  b->dirty = true;
  if (n_classes) *n_classes = (int)b->class_nc.size();
  for (int q = 0; q < (int)b->class_nc.size() && q < max_out; ++q) {
    if (class_nc) class_nc[q] = b->class_nc[q];
    if (class_tuning) class_tuning[q] = b->class_tuning[q];
  }
  return FK_OK;
}
