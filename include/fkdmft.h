/*
 * fkdmft.h -- C ABI of the MI355X (gfx950) lattice step of nonequilibrium DMFT
 * for the spinless Falicov-Kimball model on the infinite-dimensional hypercubic
 * lattice in a uniform electric field (J. K. Freericks, "Quenching Bloch
 * oscillations in a strongly correlated material", arXiv:0711.0999, Sec. II).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Contour (Sec. II, eqs. time_discrete and integration_weights), 0-based:
 *      upper real branch  j in [0, N_t):        z_j = t_min + j dt,          W_j = +dt
 *      lower real branch  j in [N_t, 2N_t):     z_j = t_max - (j - N_t) dt,  W_j = -dt
 *      imaginary branch   j in [2N_t, N_c):     z_j = t_min - i dtau (j-2N_t), W_j = -i dtau
 *    N_t = (t_max - t_min)/dt, N_tau = beta/dtau, N_c = 2 N_t + N_tau.
 *  - Every two-time function (Sigma, G_loc) crosses the boundary as its VALUES
 *    on the contour points: N_c x N_c complex128, row-major, interleaved
 *    (re, im) doubles, element (i, j) at offset 2 (i N_c + j).
 *  - Host buffers are owned by the caller and copied synchronously; the library
 *    never keeps a caller pointer.  With on_device = 1 a pointer is a device
 *    address on the context's device (e.g. a torch tensor's data_ptr()); the
 *    library finishes its stream before returning.
 *  - The context owns all of its device memory.  One context per host thread;
 *    distinct contexts are independent.
 *  - Every call returns an fk_status; no call aborts or exits.  After an error
 *    fk_last_error(ctx) holds a human-readable detail (failing point index,
 *    pivot column, HIP error string).
 */
#ifndef FKDMFT_H
#define FKDMFT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fk_ctx fk_ctx;
typedef int fk_status;

enum {
  FK_OK = 0,
  FK_EINVAL = -1,      /* bad argument (sizes, NULL, non-integral contour)      */
  FK_ENOMEM = -2,      /* device or host allocation failed                      */
  FK_EDEVICE = -3,     /* HIP runtime error or no usable gfx950 device          */
  FK_ESINGULAR = -4,   /* zero pivot in an inversion (point index in detail)    */
  FK_ENONFINITE = -5,  /* NaN/Inf in G_loc, Sigma or a pivot                    */
  FK_ENOTCONV = -6,    /* fk_iterate reached max_iter without delta < tol       */
  FK_ESTATE = -7       /* call order violated (e.g. current before a step)      */
};

/* Arithmetic of the lattice step up to its FP64 reduction. */
typedef enum {
  FK_FP64 = 0,   /* complex128 Gauss-Jordan inversion of every point matrix      */
  FK_MIXED = 1   /* complex64 inversion + FP64 iterative refinement (see below)  */
} fk_precision;

/* Contour of Sec. II.  (t_max - t_min)/dt and beta/dtau must be integers to
 * 1e-9 relative, t_min < t_max, dt > 0, dtau > 0, beta > 0; else FK_EINVAL. */
typedef struct {
  double t_min, t_max, dt, dtau, beta;
} fk_contour;

/* Model: interaction U, field E (turned on at t = 0 along the lattice diagonal,
 * eq. vector_potential), chemical potential mu, f-site filling w1 = <w_1>,
 * Gauss-Hermite orders of the (eps, ebar) product rule (eq. joint_dos), and the
 * half-filling convention of the impurity shifts:
 *   convention 0 (symmetric): U (w - 1/2) n, shifts mu0 - mu = +U/2, mu1 - mu = -U/2
 *   convention 1 (paper):     U w n,         shifts mu0 - mu = 0,    mu1 - mu = -U
 * gh_average 0: one n_eps x n_ebar product rule; 1: the average of the
 * n_eps x n_ebar and (n_eps + 1) x (n_ebar + 1) rules (the paper's N and N + 1
 * points, Sec. II quadrature paragraph), points of the first rule first, every
 * weight halved (n_eps, n_ebar <= 149). */
typedef struct {
  double U, E, mu, w1;
  int n_eps, n_ebar;
  int convention;
  int gh_average;
} fk_model;

/* ---- host-only helpers (no device needed) -------------------------------- */

/* Gauss-Hermite rule for the normalized Gaussian weight exp(-x^2)/sqrt(pi)
 * (eq. joint_dos, Sec. II quadrature paragraph): n nodes x[n] (ascending) and
 * weights w[n] summing to 1.  Nodes by Sturm-sequence bisection on the Jacobi
 * matrix, weights by the Christoffel formula.  1 <= n <= 150, else FK_EINVAL. */
fk_status fk_gauss_hermite(int n, double* x, double* w);

/* Contour sizes and points without a context: dims[3] = {N_t, N_tau, N_c};
 * z and W (each 2*N_c doubles, interleaved) may be NULL to query sizes. */
fk_status fk_contour_build(const fk_contour* c, int* dims, double* z, double* W);

/* The schedule of the batched Gauss-Jordan inversion of the point matrices
 * (the integrand of eq. g_loc, Sec. II), host logic only, for checking it
 * against a plain inversion: outer blocks of 128 columns in groups of up to
 * four counted from the last block; step S of an n x n matrix runs phases
 * q = 0, 1, 2, each the update C <- mask(C) + M B with M the columns
 * [128 jb, 128 jb + kw), B the side-buffer rows [b0, b0 + kw) (the gathered
 * pivot rows of the group's blocks) and mask zeroing the rows pivoted in M's
 * columns.  out6 = {jb, kw, b0, lo, hi, brow}: for q < 2 the column blocks
 * lo .. hi (none if hi < lo), for q = 2 every column block outside lo .. hi
 * (none if kw = 0); brow = first side-buffer row of block S's pivot rows.
 * FK_EINVAL for n outside 1 .. 5120, S < 0 or q outside 0 .. 2. */
fk_status fk_update_plan(int n, int S, int q, int* out6);

/* Extrapolation to zero time step (Sec. II, the accuracy discussion of the
 * results: Lagrange polynomials in dt through results at several steps):
 * out[e] = sum_k w_k values[k * len + e], w_k = prod_{m != k} h_m / (h_m - h_k),
 * the value at h = 0 of the polynomial of degree n_steps - 1 through
 * (steps[k], values[k][e]).  values: n_steps rows of len doubles (complex data
 * as interleaved (re, im), len doubling); host arrays.  FK_EINVAL for
 * n_steps < 1, a step that is not finite and positive, or two equal steps. */
fk_status fk_extrapolate_to_zero(int n_steps, const double* steps, int len,
                                 const double* values, double* out);

/* Status code name, e.g. "FK_ESINGULAR". */
const char* fk_status_string(fk_status s);

/* ---- context ------------------------------------------------------------- */

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * (NULL: the library creates its own default-priority stream).  The contour
 * size N_c = 2 N_t + N_tau must lie in [3, 5120] (the largest matrix the
 * inversion takes), else FK_EINVAL before any device call.  Sigma starts
 * at zero.  Device memory for the batched inversion is sized by
 * FKDMFT_BATCH_BYTES (environment, bytes; default 24 GiB) or fk_set_batch. */
fk_status fk_create(const fk_contour* c, const fk_model* m, void* hip_stream,
                    fk_ctx** out);
fk_status fk_destroy(fk_ctx* ctx);                       /* NULL-safe */
const char* fk_last_error(const fk_ctx* ctx);            /* never NULL */

fk_status fk_dims(const fk_ctx* ctx, int* n_t, int* n_tau, int* n_c);
/* z, W: 2*N_c doubles each (interleaved), host. */
fk_status fk_contour_points(const fk_ctx* ctx, double* z, double* W);
/* Number of (eps, ebar) points and their nodes/weights (host, may be NULL). */
fk_status fk_points(const fk_ctx* ctx, int* n_points, double* eps, double* ebar,
                    double* rho);

/* Number of point matrices inverted per batch (>= 1); returns the value used.
 * Reallocates the batch buffer. */
fk_status fk_set_batch(fk_ctx* ctx, int batch, int* used);

/* ---- state --------------------------------------------------------------- */

fk_status fk_set_sigma(fk_ctx* ctx, const double* sigma, int on_device);
fk_status fk_get_sigma(const fk_ctx* ctx, double* sigma, int on_device);
fk_status fk_get_gloc(const fk_ctx* ctx, double* gloc, int on_device);

/* ---- the hot path -------------------------------------------------------- */

/* Lattice step (eqs. dyson and g_loc, Sec. II): for every Gauss-Hermite point
 * k = a*n_ebar + b (eps = x_a, ebar = x_b, rho_k = w_a w_b)
 *     G_k = (G0_k^-1 - W Sigma W)^-1
 * where G0_k is eq. (g_contour_non_final2) sampled with theta_c(t,t) = 1, whose
 * inverse is the exact bidiagonal-plus-corner matrix
 *     G0_k^-1 = i D (I - P + e^{-beta(eps-mu)} e_0 e_{N-1}^T) D^-1,
 *     D = diag(exp(-i phi_k(z) + i mu z)),
 * then G_loc = sum_k rho_k G_k (fixed order, deterministic) and the current
 *     j(t_i) = Re[ i sum_k rho_k ebar_k(t_i) G_k[i, 2N_t - i] ],  i < N_t
 * (eq. current_def, velocity at the Peierls-shifted momentum, e = t* = 1).
 * FK_FP64: complex128 throughout.  FK_MIXED: complex64 inversion, then
 * ir_steps (fk_set_refinement, default 1) FP64 refinement steps
 * X <- X + X (I - A X) with the residual I - A X in FP64; the rho-weighted sum
 * is FP64.  ir_resid_out (nullable) receives a bound on max_k max|I - A_k X_k|
 * of the returned inverses: with r the largest residual entry entering the last
 * refinement step, the returned X has the residual R^2 (Newton's step), whose
 * entries are at most N_c r^2 (FK_FP64: 0).  A failed step leaves no G_loc
 * (fk_get_gloc, fk_get_current and fk_impurity_update return FK_ESTATE until a
 * step succeeds).  Errors: FK_ESINGULAR ("zero pivot at column c of matrix k",
 * k the point index), FK_ENONFINITE. */
fk_status fk_compute_gloc(fk_ctx* ctx, fk_precision prec, double* ir_resid_out);

/* Refinement steps used by FK_MIXED (0..4). */
fk_status fk_set_refinement(fk_ctx* ctx, int ir_steps);

/* j(t_i), the time t_i = t_min + i dt and (nullable) n(t_i) = Re[-i G^<_loc(t_i,t_i)]
 * from the last lattice step; N_t doubles each.  FK_ESTATE before any step. */
fk_status fk_get_current(const fk_ctx* ctx, double* t, double* j, double* n_t);
/* Zeroth spectral moment m0(t_i) = G^>_loc(t_i, t_i) - G^<_loc(t_i, t_i) =
 * G_loc[2 N_t - i][i] - G_loc[i][2 N_t - i] for i < N_t (the sum rule of the
 * moments paragraph of Sec. II: -i in the continuum, O(dt) off on the
 * discrete contour).  m0: 2 N_t doubles (re, im interleaved). */
fk_status fk_get_zeroth_moment(const fk_ctx* ctx, double* m0);

/* Nonequilibrium density of states of the last lattice step's G_loc (Sec. II,
 * eqs. gr_omega and dos_def): rho(T, w) = -Im G^R(T, w) / pi at the average
 * times T = t_min + i dt for the n_T indices t_index[r] (0 <= i < N_t) and the
 * n_w frequencies omega[q]; dos[r * n_w + q] (host arrays, caller-owned).
 * G^R(t_a, t_b) = G_loc[2N_t - a][b] - G_loc[a][2N_t - b] for a >= b (G^> - G^<
 * from the two real branches); the relative time runs over t_rel = 2 d dt,
 * d = 0..D, D = min(i, N_t - 1 - i), by the trapezoid rule (weight 1/2 at d = 0
 * and d = D), with no window function.  The integral of rho over one period of
 * w (pi / dt) is exactly -Im m0(T).  FK_EINVAL for NULL arrays, n_T or n_w < 1,
 * an index outside [0, N_t) or a non-finite frequency; FK_ESTATE before a
 * lattice step. */
fk_status fk_wigner_dos(const fk_ctx* ctx, int n_T, const int* t_index, int n_w,
                        const double* omega, double* dos);
/* fk_wigner_dos for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, result and errors, but the time indices, frequencies and
 * result are staged through a 4 MiB static device array of the library (one
 * per GPU, set up by fk_create, held until the process ends) instead of a
 * per-call allocation; no hipMalloc, hipFree or allocating library call.
 * 256-byte-aligned segments of 4 n_T + 8 n_w + 8 n_T n_w bytes must fit in
 * 4 MiB, else FK_EINVAL (e.g. 100 times x 5000 frequencies fit).  All calls on
 * one GPU share the array: calls that overlap in time on the same GPU (other
 * threads or streams) race; serialize them. */
fk_status fk_wigner_dos_noalloc(const fk_ctx* ctx, int n_T, const int* t_index,
                                int n_w, const double* omega, double* dos);
/* Equal-time spectral moments of the local retarded function (Sec. II, moments
 * paragraph) at T = t_min + i dt, i = t_index[r] (3 <= i <= N_t - 4): with
 * f(s) = G^R(T + s/2, T - s/2), mu0 = i f(0), mu1 = -f'(0), mu2 = -i f''(0)
 * (exact values 1, 0 and 1/2 + U^2/4 at half filling in the symmetric
 * convention), the derivatives by one-sided second-order differences over
 * s = 0, h, 2h, 3h with h = 2 dt.  mu: 6 n_T doubles, (re, im) of mu0, mu1, mu2
 * for each index in turn.  Errors as for fk_wigner_dos. */
fk_status fk_equal_time_moments(const fk_ctx* ctx, int n_T, const int* t_index,
                                double* mu);

/* Falicov-Kimball impurity update (eqs. effective_medium, dynamical_mean_field,
 * g_imp_solve and Dyson again), in right-weighted form A -> A W:
 *   g0inv = (G_loc W)^-1 + Sigma W
 *   G_imp = (1-w1) (g0inv + d0 S)^-1 + w1 (g0inv + d1 S)^-1
 *   Sigma <- (g0inv - G_imp^-1) W^-1
 * with S the point-split delta (S[j,j-1] = 1, S[0,N_c-1] = -1) and (d0, d1)
 * from the model's convention.  The same value is reached with one complex128
 * Gauss-Jordan inversion on the device: with X = G_loc W, Y = Sigma W + d_c S,
 * d_c = (1-w1) d1 + w1 d0 and h = (1-w1) d0 + w1 d1,
 *   Sigma W <- -h S + w1 (1-w1) (d0-d1)^2 S X (I + Y X)^-1 S.
 * max_dsigma_out (nullable) = max |Sigma_new - Sigma_old|.
 * FK_ESTATE before any lattice step. */
fk_status fk_impurity_update(fk_ctx* ctx, double* max_dsigma_out);

/* Self-consistency loop (Sec. II summary): iteration n = lattice step from
 * Sigma(n-1), delta(n) = max|G_loc(n) - G_loc(n-1)| (delta(1) = +inf), impurity
 * update -> Sigma(n); stops after the iteration with delta < tol (converged,
 * FK_OK) or after max_iter iterations (FK_ENOTCONV unless tol <= 0, in which
 * case exactly max_iter iterations run and FK_OK is returned).
 * With FK_MIXED the loop runs complex64 (+ refinement) steps until delta <
 * switch_tol (fk_set_switch, default 3e-5, above the complex64 noise floor of
 * G_loc) or stops contracting close to that floor (delta(n) > 0.95 delta(n-1)
 * with delta(n) < 100 switch_tol), FK_FP64 afterwards.
 * delta_history (nullable, max_iter doubles) receives delta(n). */
fk_status fk_iterate(fk_ctx* ctx, int max_iter, double tol, fk_precision prec,
                     int* iters_out, double* delta_out, double* delta_history);
fk_status fk_set_switch(fk_ctx* ctx, double switch_tol);
/* G_k of one quadrature point k (N_c x N_c complex128 values, row-major) as the
 * last FP64 fk_compute_gloc computed it: available for the points of the last
 * batch of that step, which stay in the batch buffers (fk_points gives their
 * (eps, ebar, rho)); otherwise FK_ESTATE: after a mixed step, a failed step,
 * fk_set_batch, fk_set_tuning or fk_autotune (each may free or overwrite the
 * batch buffers).  For parity checks of single points at full size. */
fk_status fk_get_point_green(const fk_ctx* ctx, int k, double* g, int on_device);
/* Number of complex64 iterations in the last fk_iterate / fk_iterate_judged. */
fk_status fk_low_iterations(const fk_ctx* ctx, int* n);

/* Per-phase device time of the last fk_compute_gloc / fk_impurity_update in
 * milliseconds (HIP events on the context stream): out[0] build, out[1]
 * inversion, out[2] refinement, out[3] reduction, out[4] impurity, out[5]
 * inversion kernel launches, out[6] summed duration of the step kernels. */
fk_status fk_timings(const fk_ctx* ctx, double* out7);

/* Timing of the dominant kernel, the trailing update of each group of
 * 128-column outer blocks of the batched Gauss-Jordan inversion in
 * fk_compute_gloc (FP64 or complex64): with the clock on
 * (fk_set_kernel_clock(ctx, 1), which also zeroes it) every such launch is
 * bracketed by HIP events on the context stream.  out3: summed launch duration
 * in ms, number of launches, summed algorithmic flops of those launches
 * (8 n * cols * K per matrix: n rows, cols outside the group's blocks and the
 * next block, K the group's width, up to 512). */
fk_status fk_set_kernel_clock(fk_ctx* ctx, int on);
fk_status fk_kernel_clock(const fk_ctx* ctx, double* out3);

/* ---- schedule autotuner --------------------------------------------------- */

/* A schedule of the batched inversion: the trailing-update tile height
 * (64: 64 x 64 tiles, 4 waves, two workgroups per CU; 128: 128 x 64 tiles,
 * 8 waves sharing each B chunk), the number of point matrices per batch, and
 * whether the next 128-column block is factored on a second stream. */
typedef struct {
  int tile_rows;        /* 64 or 128 */
  int batch;            /* matrices per batch (>= 1) */
  int lookahead;        /* 0 or 1 */
  double chunk_bytes;   /* device bytes of one batch at this context's N_c */
  double est_step_ms;   /* autotune: estimated inversion time of all points */
  int trials;           /* autotune: schedules timed */
} fk_tuning;

/* Time candidate schedules on this context's own point matrices (current
 * Sigma): every tile height x batch sizes within max_bytes of device memory
 * (the points split evenly into k batches for the smallest k the budget allows
 * and the next three, the budget's quarter, and one to three times the
 * device's compute unit count) x look-ahead on/off.  Each candidate inverts one
 * batch once for warm-up and once timed; the estimate is that time times the
 * number of batches.  The three fastest are timed again afterwards (the first
 * trials on a cold device run fast) and the choice uses those times only.
 * Applies and returns the fastest.  keep = 0 frees the inversion buffers
 * afterwards. */
fk_status fk_autotune(fk_ctx* ctx, double max_bytes, int keep, fk_tuning* best);
fk_status fk_set_tuning(fk_ctx* ctx, const fk_tuning* t);
fk_status fk_get_tuning(const fk_ctx* ctx, fk_tuning* t);

/* ---- many instances in one sweep ----------------------------------------- */

/* A set of independent DMFT problems (contours and models may differ: uneven
 * N_c, Gauss-Hermite orders, U, E) iterated together.  In every sweep the
 * lattice steps of all active instances share uneven batched inversions (one
 * launch per Gauss-Jordan step over all (instance, point, tile) work items),
 * the impurity updates share batched inversions as well, and each instance
 * retires after the iteration whose delta falls below tol.  Same semantics per
 * instance as fk_iterate with FK_FP64.  The batch owns its stream and device
 * memory; instance i's state is reachable as an fk_ctx through
 * fk_batch_instance (owned by the batch: do not destroy it), so fk_get_gloc,
 * fk_get_sigma, fk_set_sigma and fk_get_current apply to it. */
typedef struct fk_batch fk_batch;
fk_status fk_batch_create(int n_inst, const fk_contour* contours,
                          const fk_model* models, fk_batch** out);
fk_status fk_batch_destroy(fk_batch* b);                 /* NULL-safe */
const char* fk_batch_last_error(const fk_batch* b);
fk_status fk_batch_instance(const fk_batch* b, int i, fk_ctx** ctx);
/* Device memory for the lattice inversions of one chunk of a sweep (bytes,
 * default FKDMFT_BATCH_BYTES or 24 GiB): larger chunks, fewer launches. */
fk_status fk_batch_set_chunk_bytes(fk_batch* b, double bytes);
/* Mark every instance active again with its iteration count at zero (Sigma kept). */
fk_status fk_batch_reset(fk_batch* b);
/* Run up to max_sweeps sweeps or until every instance has converged.
 * use_graph = 1 records the sweep into a hipGraph (re-recorded when the set of
 * active instances changes) and replays it; 0 launches eagerly.
 * iters[n_inst] and deltas[n_inst] (nullable) receive each instance's
 * iteration count and last delta (+inf after its first iteration). */
fk_status fk_batch_iterate(fk_batch* b, int max_sweeps, double tol,
                           int use_graph, int* sweeps_out, int* iters,
                           double* deltas);
/* Tile height, look-ahead and chunk_bytes of t apply to every sweep. */
fk_status fk_batch_set_tuning(fk_batch* b, const fk_tuning* t);
/* Autotuner of the sweep's schedule per contour size: for every distinct N_c
 * among the instances (only_nc = 0), or for the instances of size only_nc
 * alone (merged into the table), fk_autotune on the first instance of that
 * size (its own point matrices and current Sigma, candidate tile heights x
 * matrices per chunk within max_bytes); the sweep's plan then orders the
 * instances by size, cuts chunks within one size class of at most that
 * class's tuned number of matrices and runs them with its tile height.
 * Returns the number of classes in the table and (up to max_out, nullable)
 * their sizes and schedules.  The chunk storage is released first (the trials
 * need the memory); fk_batch_set_tuning returns to one schedule for all.
 * FK_EINVAL when no instance has size only_nc. */
fk_status fk_batch_autotune(fk_batch* b, double max_bytes, int only_nc, int max_out,
                            int* n_classes, int* class_nc, fk_tuning* class_tuning);
/* out4: last sweep ms, total sweep ms, graph recordings, last recording ms. */
fk_status fk_batch_timings(const fk_batch* b, double* out4);

/* ---- learned warm start ------------------------------------------------- */

/* A fully connected network of `depth` layers (depth - 1 hidden tanh layers of
 * `width`, linear output) that predicts, pointwise on contour pairs (t_i, t_j),
 * the change of Sigma from the previous field to the current one.  Parameters
 * are float32, packed layer by layer as W_l (out x in, row-major) then b_l.
 * Training: mean squared error, Adam (b1 0.9, b2 0.999, eps 1e-8) on FP32
 * matrix cores; inference in FP32 or BF16 (bf16 matrix cores, FP32
 * accumulation).  Row-major device arrays: x [rows x d_in], y, t [rows x d_out]. */
typedef struct fk_mlp fk_mlp;
fk_status fk_mlp_create(int d_in, int width, int depth, int d_out,
                        const float* params_host, fk_mlp** out);
fk_status fk_mlp_destroy(fk_mlp* a);                     /* NULL-safe */
const char* fk_mlp_last_error(const fk_mlp* a);
fk_status fk_mlp_n_params(const fk_mlp* a, long long* n);
fk_status fk_mlp_get_params(const fk_mlp* a, float* params_host);
/* Replaces the parameters and clears the Adam state. */
fk_status fk_mlp_set_params(fk_mlp* a, const float* params_host);
fk_status fk_mlp_forward(fk_mlp* a, const float* x_dev, int rows, float* y_dev,
                         int bf16);
/* Loss of one batch and its gradient (host array of n_params, nullable). */
fk_status fk_mlp_loss_grad(fk_mlp* a, const float* x_dev, const float* t_dev,
                           int rows, double* loss, float* grad_host);
/* `steps` Adam steps, each on `batch` rows drawn uniformly with replacement
 * from the `rows` rows of (x, t) by a counter-based hash of (seed, step, slot)
 * (SplitMix64), gathered on the device; loss_hist[steps] nullable receives the
 * loss of each minibatch before its step. */
fk_status fk_mlp_train(fk_mlp* a, const float* x_dev, const float* t_dev,
                       int rows, int batch, int steps, float lr,
                       unsigned long long seed, double* loss_hist);

/* Rank-r randomized SVD (basic range finder of Halko, Martinsson & Tropp 2011)
 * of D Sigma D, D = diag(sqrt|W_j|), for an N_c x N_c complex128 device matrix
 * Sigma (values Sigma(z_i, z_j) on this context's contour): Y = D Sigma D Omega
 * with the caller's real N_c x rank host matrix Omega (row-major), Q an
 * orthonormal basis of range(Y) (modified Gram-Schmidt, twice), and sv_out the
 * rank singular values (descending) of Q^H D Sigma D.  The weighting makes them
 * approximate the singular values of the contour integral operator, independent
 * of the step sizes.  rank <= 256; the small eigen-solve runs on the host. */
fk_status fk_ws_sketch(fk_ctx* ctx, const double* sigma_dev, int rank,
                       const double* omega_host, double* sv_out);
/* Feature rows for pairs p = i*N_c + j (idx_dev: rows int64 pair indices, or
 * NULL for all N_c^2 pairs in order) of this context's contour and field E
 * (T = t_max - t_min; t+ = max(t, 0) on the real branches, 0 on the imaginary):
 *   glob[n_glob] | branch one-hot of i (3), of j (3) | t_i/T, tau_i/beta,
 *   t_j/T, tau_j/beta | [i >= j] | [i - j >= 2] | (t_i - t_j)/T |
 *   max(t_i,t_j,0)/T | sin E t_i+, cos E t_i+, sin E t_j+, cos E t_j+ |
 *   scale*Re, scale*Im of Sigma_prev(i,j) |
 *   sin(pi k t_i/T), cos(pi k t_i/T) for k = 1..8 | the same for t_j |
 *   sin(pi k tau_i/beta), cos(pi k tau_i/beta) for k = 1, 2 | the same for
 *   tau_j | zero padding to d_in   (t = 0 on the imaginary branch, tau = 0 on
 *   the real ones).
 * d_in >= n_glob + FK_WS_FEATURES, else FK_EINVAL.  A pair index outside
 * [0, N_c^2) yields a row of NaN (fk_ws_targets: a NaN target). */
#define FK_WS_FEATURES 60
fk_status fk_ws_features(fk_ctx* ctx, const double* sigma_prev_dev,
                         const float* glob_host, int n_glob,
                         const long long* idx_dev, long long rows, double scale,
                         float* x_dev, int d_in);
/* t = scale * (Sigma_new - Sigma_prev) at the pairs (2 floats per row). */
fk_status fk_ws_targets(fk_ctx* ctx, const double* sigma_prev_dev,
                        const double* sigma_new_dev, const long long* idx_dev,
                        long long rows, double scale, float* t_dev);
/* Sets the context's Sigma to Sigma_prev + y / scale (y: N_c^2 rows of 2;
 * sigma_prev_dev may be the context's own Sigma buffer).  keep_pre_field != 0:
 * the pairs whose two contour points both lie before the field is switched on
 * (real time <= 0 on the real branches; every imaginary-branch point) keep
 * Sigma_prev (causality: there the solution does not depend on E). */
fk_status fk_ws_apply(fk_ctx* ctx, const double* sigma_prev_dev,
                      const float* y_dev, double scale, int keep_pre_field);
/* The self-consistency loop of fk_iterate started from the context's current
 * Sigma (a proposed start, e.g. from fk_ws_apply) and judged by the plain
 * iteration: the start is kept if its first iteration changes Sigma by at most
 * `accept` times max|Sigma_start - Sigma_fallback| (a start equal to the
 * fallback is simply iterated); otherwise, or if a later
 * FP64 iteration grows delta three times in a row, or a step meets a singular
 * or non-finite matrix, the loop restarts from fallback_dev (an N_c x N_c
 * device matrix, e.g. the previous field's Sigma; NULL: Sigma = 0).  iters_out
 * counts every iteration run, the abandoned ones included (max_iter >= 2);
 * delta_history as for fk_iterate, with +inf again at a restart.  outcome
 * (nullable): 0 start kept, 1 rejected after its first iteration, 2 abandoned
 * later. */
fk_status fk_iterate_judged(fk_ctx* ctx, const double* fallback_dev,
                            double accept, int max_iter, double tol,
                            fk_precision prec, int* iters_out, double* delta_out,
                            double* delta_history, int* outcome);

#ifdef __cplusplus
}
#endif
#endif /* FKDMFT_H */
