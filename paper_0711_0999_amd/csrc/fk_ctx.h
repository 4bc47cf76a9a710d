// The single-instance context (opaque fk_ctx of the C ABI), shared by the
// context API and the multi-instance sweep.
#pragma once

#include <string>
#include <vector>

#include "../../include/fkdmft.h"
#include "fk_driver.h"

namespace fk {
struct ContourInfo {
  int n_t = 0, n_tau = 0, n_c = 0;
  std::vector<double> zr, zi, wr, wi;
};
}  // namespace fk

// ======================================================================= ctx ==
struct fk_ctx {
  fk_contour c;
  fk_model m;
  fk::ContourInfo ci;
  int npts = 0;
  std::vector<double> eps, ebar, rho;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int dev = 0;                     // HIP device of the context
  std::string err;

  // device
  fk::c64* d_w = nullptr;          // weights W (N_c)
  fk::c64* d_sigma = nullptr;      // Sigma values
  fk::c64* d_sigt = nullptr;       // W Sigma W
  fk::c64* d_gloc = nullptr;
  fk::c64* d_gprev = nullptr;
  fk::c64* d_g0inv = nullptr;      // impurity scratch
  fk::c64* d_tmp = nullptr;        // impurity scratch
  double* d_cur = nullptr;     // j(t), N_t
  double* d_eps = nullptr;
  double* d_ebar = nullptr;
  double* d_rho = nullptr;
  fk::c64* d_da = nullptr;
  fk::c64* d_dg = nullptr;
  fk::c64* d_dz = nullptr;
  double* d_cos = nullptr;
  double* d_sin = nullptr;
  int* d_tpos = nullptr;
  double* d_coef = nullptr;    // {1, 1 - w1, w1}
  unsigned long long* d_key = nullptr;
  fk::PointTables tab;

  fk::Batch<double> b64;           // lattice batch (complex128)
  fk::Batch<float> b32;            // lattice batch (complex64), lazily
  fk::Batch<double> imp;           // the impurity update's inversion (1 slot)
  fk::Aux aux;                     // look-ahead stream and events
  fk::KernelClock clk;             // optional timing of the trailing update
  // FP64 refinement buffers of the mixed path (ir_cap matrices)
  int ir_cap = 0;
  fk::c64* ir_x = nullptr;
  fk::c64* ir_p = nullptr;
  fk::c64* ir_y = nullptr;
  fk::c64* ir_tsub = nullptr;
  fk::c64* ir_tcor = nullptr;
  int* d_iota = nullptr;
  size_t batch_bytes = 0;
  int want_batch = 0;
  int variant = 0;             // trailing-update tile shape
  fk_tuning tuned{64, 0, 0, 0.0, 0.0, 0};

  bool have_gloc = false;
  bool have_prev = false;
  int ir_steps = 1;
  double switch_tol = 3e-5;
  int low_iters = 0;               // complex64 iterations of the last loop
  int last_k0 = 0, last_nmat = 0;  // points left in the lattice batch
  int last_prec = -1;              // their precision (0 FP64, 1 mixed)
  double times[7] = {0, 0, 0, 0, 0, 0, 0};
  hipEvent_t ev[8];
};
