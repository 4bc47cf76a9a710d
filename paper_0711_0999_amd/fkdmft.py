"""ctypes binding of libfkdmft.so (C ABI in include/fkdmft.h).

Argument marshalling only: every step of the lattice step, the impurity update
and the loop runs in the HIP library.  Loading fails loudly when the library has
not been built; there is no fallback.

Host matrices are numpy complex128 arrays (N_c x N_c, C order).  Device
matrices may be passed as torch tensors (complex128, on the context's device,
contiguous): their data_ptr() is handed to the library with on_device = 1.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfkdmft.so")

FK_OK, FK_EINVAL, FK_ENOMEM, FK_EDEVICE = 0, -1, -2, -3
FK_ESINGULAR, FK_ENONFINITE, FK_ENOTCONV, FK_ESTATE = -4, -5, -6, -7
FK_FP64, FK_MIXED = 0, 1
CONVENTION = {"symmetric": 0, "paper": 1}


class FkError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        super().__init__(f"{status_string(status)}: {detail}")


class Contour(ctypes.Structure):
    _fields_ = [("t_min", ctypes.c_double), ("t_max", ctypes.c_double),
                ("dt", ctypes.c_double), ("dtau", ctypes.c_double),
                ("beta", ctypes.c_double)]


class Model(ctypes.Structure):
    _fields_ = [("U", ctypes.c_double), ("E", ctypes.c_double),
                ("mu", ctypes.c_double), ("w1", ctypes.c_double),
                ("n_eps", ctypes.c_int), ("n_ebar", ctypes.c_int),
                ("convention", ctypes.c_int), ("gh_average", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int), ("batch", ctypes.c_int),
                ("lookahead", ctypes.c_int), ("chunk_bytes", ctypes.c_double),
                ("est_step_ms", ctypes.c_double), ("trials", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p

# name: (restype, argtypes) for every entry point of include/fkdmft.h
SIGNATURES = {
    "fk_gauss_hermite": (ctypes.c_int, [ctypes.c_int, _dp, _dp]),
    "fk_contour_build": (ctypes.c_int, [ctypes.POINTER(Contour), _ip, _dp, _dp]),
    "fk_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fk_extrapolate_to_zero": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]),
    "fk_create": (ctypes.c_int, [ctypes.POINTER(Contour), ctypes.POINTER(Model),
                                 _vp, ctypes.POINTER(_vp)]),
    "fk_destroy": (ctypes.c_int, [_vp]),
    "fk_last_error": (ctypes.c_char_p, [_vp]),
    "fk_dims": (ctypes.c_int, [_vp, _ip, _ip, _ip]),
    "fk_contour_points": (ctypes.c_int, [_vp, _dp, _dp]),
    "fk_points": (ctypes.c_int, [_vp, _ip, _dp, _dp, _dp]),
    "fk_set_batch": (ctypes.c_int, [_vp, ctypes.c_int, _ip]),
    "fk_set_sigma": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "fk_get_sigma": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "fk_get_gloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "fk_compute_gloc": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "fk_set_refinement": (ctypes.c_int, [_vp, ctypes.c_int]),
    "fk_get_current": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "fk_impurity_update": (ctypes.c_int, [_vp, _dp]),
    "fk_iterate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                  _ip, _dp, _dp]),
    "fk_set_switch": (ctypes.c_int, [_vp, ctypes.c_double]),
    "fk_timings": (ctypes.c_int, [_vp, _dp]),
    "fk_autotune": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(Tuning)]),
    "fk_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "fk_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "fk_batch_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "fk_low_iterations": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "fk_get_zeroth_moment": (ctypes.c_int, [_vp, _dp]),
    "fk_wigner_dos": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _dp, _dp]),
    "fk_equal_time_moments": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _dp]),
    "fk_wigner_dos_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _dp, _dp]),
    "fk_get_point_green": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int]),
    "fk_set_kernel_clock": (ctypes.c_int, [_vp, ctypes.c_int]),
    "fk_kernel_clock": (ctypes.c_int, [_vp, _dp]),
    "fk_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "fk_mlp_destroy": (ctypes.c_int, [_vp]),
    "fk_mlp_last_error": (ctypes.c_char_p, [_vp]),
    "fk_mlp_n_params": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_longlong)]),
    "fk_mlp_get_params": (ctypes.c_int, [_vp, _vp]),
    "fk_mlp_set_params": (ctypes.c_int, [_vp, _vp]),
    "fk_mlp_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int]),
    "fk_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _dp, _vp]),
    "fk_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_float, ctypes.c_ulonglong,
                                    _dp]),
    "fk_iterate_judged": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double), _dp,
                                         ctypes.POINTER(ctypes.c_int)]),
    "fk_ws_sketch": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _dp]),
    "fk_ws_features": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp,
                                      ctypes.c_longlong, ctypes.c_double, _vp,
                                      ctypes.c_int]),
    "fk_ws_targets": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_longlong,
                                     ctypes.c_double, _vp]),
    "fk_update_plan": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "fk_ws_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int]),
    "fk_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Contour),
                                       ctypes.POINTER(Model), ctypes.POINTER(_vp)]),
    "fk_batch_destroy": (ctypes.c_int, [_vp]),
    "fk_batch_last_error": (ctypes.c_char_p, [_vp]),
    "fk_batch_instance": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    "fk_batch_set_chunk_bytes": (ctypes.c_int, [_vp, ctypes.c_double]),
    "fk_batch_reset": (ctypes.c_int, [_vp]),
    "fk_batch_iterate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        _ip, _ip, _dp]),
    "fk_batch_timings": (ctypes.c_int, [_vp, _dp]),
    "fk_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         _ip, _ip, ctypes.POINTER(Tuning)]),
}

_lib = None


def library():
    """Load libfkdmft.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing; build the HIP library "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def status_string(s):
    return library().fk_status_string(s).decode()


def _dptr(a):
    return a.ctypes.data_as(_dp)


def gauss_hermite(n):
    x = np.zeros(max(n, 1))
    w = np.zeros(max(n, 1))
    s = library().fk_gauss_hermite(n, _dptr(x), _dptr(w))
    if s != FK_OK:
        raise FkError(s, f"gauss_hermite({n})")
    return x, w


def extrapolate_to_zero(steps, values):
    """fk_extrapolate_to_zero: values[k] (arrays of one shape, real or complex)
    at the steps[k]; returns their extrapolation to step 0."""
    hs = np.ascontiguousarray(steps, dtype=np.float64)
    arrs = [np.asarray(v) for v in values]
    cplx = any(np.iscomplexobj(a) for a in arrs)
    shape = arrs[0].shape
    rows = [np.ascontiguousarray(a, dtype=np.complex128 if cplx else np.float64).view(np.float64)
            .ravel() for a in arrs]
    data = np.ascontiguousarray(np.stack(rows))
    out = np.zeros(data.shape[1])
    s = library().fk_extrapolate_to_zero(len(hs), _dptr(hs), data.shape[1], _dptr(data),
                                         _dptr(out))
    if s != FK_OK:
        raise FkError(s, "extrapolate_to_zero")
    return (out.view(np.complex128) if cplx else out).reshape(shape)


def update_plan(n, S, q):
    """fk_update_plan: the transform and column blocks of phase q of outer step
    S of the batched inversion of an n x n matrix."""
    out = (ctypes.c_int * 6)()
    s = library().fk_update_plan(int(n), int(S), int(q), out)
    if s != FK_OK:
        raise FkError(s, "update_plan")
    return dict(jb=out[0], kw=out[1], b0=out[2], lo=out[3], hi=out[4], brow=out[5])


def contour_build(t_min, t_max, dt, dtau, beta):
    c = Contour(t_min, t_max, dt, dtau, beta)
    dims = (ctypes.c_int * 3)()
    s = library().fk_contour_build(ctypes.byref(c), dims, None, None)
    if s != FK_OK:
        raise FkError(s, "contour")
    n = dims[2]
    z = np.zeros(2 * n)
    w = np.zeros(2 * n)
    library().fk_contour_build(ctypes.byref(c), dims, _dptr(z), _dptr(w))
    return (dims[0], dims[1], dims[2]), z.view(np.complex128), w.view(np.complex128)


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class Context:
    """One fk_ctx.  stream: a torch.cuda.Stream, an int hipStream_t, or None."""

    def __init__(self, t_min, t_max, dt, dtau, beta, U, E, mu=0.0, w1=0.5,
                 n_eps=10, n_ebar=10, convention="symmetric", stream=None,
                 gh_average=False):
        lib = library()
        self._lib = lib
        c = Contour(t_min, t_max, dt, dtau, beta)
        m = Model(U, E, mu, w1, n_eps, n_ebar, CONVENTION[convention], int(gh_average))
        if stream is None:
            sp = None
        elif isinstance(stream, int):
            sp = stream
        else:
            sp = stream.cuda_stream
        h = _vp()
        s = lib.fk_create(ctypes.byref(c), ctypes.byref(m), sp, ctypes.byref(h))
        if s != FK_OK:
            raise FkError(s, "fk_create")
        self._h = h
        nt, ntau, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lib.fk_dims(h, ctypes.byref(nt), ctypes.byref(ntau), ctypes.byref(nc))
        self.n_t, self.n_tau, self.n_c = nt.value, ntau.value, nc.value

    # -- plumbing
    def _check(self, s, what):
        if s != FK_OK:
            raise FkError(s, f"{what}: {self._lib.fk_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- queries
    def contour_points(self):
        z = np.zeros(2 * self.n_c)
        w = np.zeros(2 * self.n_c)
        self._check(self._lib.fk_contour_points(self._h, _dptr(z), _dptr(w)),
                    "fk_contour_points")
        return z.view(np.complex128), w.view(np.complex128)

    def points(self):
        n = ctypes.c_int()
        self._check(self._lib.fk_points(self._h, ctypes.byref(n), None, None, None),
                    "fk_points")
        e, eb, r = np.zeros(n.value), np.zeros(n.value), np.zeros(n.value)
        self._check(self._lib.fk_points(self._h, ctypes.byref(n), _dptr(e),
                                        _dptr(eb), _dptr(r)), "fk_points")
        return e, eb, r

    def set_batch(self, batch):
        used = ctypes.c_int()
        self._check(self._lib.fk_set_batch(self._h, batch, ctypes.byref(used)),
                    "fk_set_batch")
        return used.value

    # -- state
    def _matrix_arg(self, a, write):
        if _is_torch(a):
            assert a.is_contiguous() and tuple(a.shape) == (self.n_c, self.n_c)
            return a.data_ptr(), 1, None
        if write:
            arr = a
            assert arr.dtype == np.complex128 and arr.flags.c_contiguous
            assert arr.shape == (self.n_c, self.n_c)
        else:
            arr = np.ascontiguousarray(a, dtype=np.complex128)
            assert arr.shape == (self.n_c, self.n_c)
        return arr.ctypes.data, 0, arr

    def set_sigma(self, sigma):
        p, dev, keep = self._matrix_arg(sigma, False)
        self._check(self._lib.fk_set_sigma(self._h, p, dev), "fk_set_sigma")

    def get_sigma(self, out=None):
        out = np.zeros((self.n_c, self.n_c), np.complex128) if out is None else out
        p, dev, _ = self._matrix_arg(out, True)
        self._check(self._lib.fk_get_sigma(self._h, p, dev), "fk_get_sigma")
        return out

    def get_gloc(self, out=None):
        out = np.zeros((self.n_c, self.n_c), np.complex128) if out is None else out
        p, dev, _ = self._matrix_arg(out, True)
        self._check(self._lib.fk_get_gloc(self._h, p, dev), "fk_get_gloc")
        return out

    # -- hot path
    def compute_gloc(self, precision=FK_FP64):
        r = ctypes.c_double()
        self._check(self._lib.fk_compute_gloc(self._h, precision, ctypes.byref(r)),
                    "fk_compute_gloc")
        return r.value

    def set_refinement(self, steps):
        self._check(self._lib.fk_set_refinement(self._h, steps), "fk_set_refinement")

    def set_switch(self, tol):
        self._check(self._lib.fk_set_switch(self._h, tol), "fk_set_switch")

    def get_current(self):
        t, j, n = np.zeros(self.n_t), np.zeros(self.n_t), np.zeros(self.n_t)
        self._check(self._lib.fk_get_current(self._h, _dptr(t), _dptr(j), _dptr(n)),
                    "fk_get_current")
        return t, j, n

    def get_zeroth_moment(self):
        m = np.zeros(2 * self.n_t)
        self._check(self._lib.fk_get_zeroth_moment(self._h, _dptr(m)), "fk_get_zeroth_moment")
        return m.view(np.complex128)

    def wigner_dos(self, t_index, omega):
        """rho(T_i, w) at T_i = t_min + i dt for the time indices and the
        frequencies; array [len(t_index), len(omega)]."""
        ti = np.ascontiguousarray(t_index, dtype=np.int32)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        out = np.zeros((len(ti), len(om)))
        self._check(self._lib.fk_wigner_dos(self._h, len(ti), ti.ctypes.data, len(om),
                                            _dptr(om), _dptr(out)), "fk_wigner_dos")
        return out

    def wigner_dos_noalloc(self, t_index, omega):
        """wigner_dos staged through the library's static device array (no
        device allocation in the call)."""
        ti = np.ascontiguousarray(t_index, dtype=np.int32)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        out = np.zeros((len(ti), len(om)))
        self._check(self._lib.fk_wigner_dos_noalloc(self._h, len(ti), ti.ctypes.data,
                                                    len(om), _dptr(om), _dptr(out)),
                    "fk_wigner_dos_noalloc")
        return out

    def moments(self, t_index):
        """(mu0, mu1, mu2) at the time indices: complex array [3, len(t_index)]."""
        ti = np.ascontiguousarray(t_index, dtype=np.int32)
        out = np.zeros(6 * len(ti))
        self._check(self._lib.fk_equal_time_moments(self._h, len(ti), ti.ctypes.data,
                                                    _dptr(out)), "fk_equal_time_moments")
        return out.view(np.complex128).reshape(len(ti), 3).T.copy()

    def impurity_update(self):
        d = ctypes.c_double()
        self._check(self._lib.fk_impurity_update(self._h, ctypes.byref(d)),
                    "fk_impurity_update")
        return d.value

    def iterate(self, max_iter, tol=0.0, precision=FK_FP64):
        it = ctypes.c_int()
        d = ctypes.c_double()
        hist = np.zeros(max_iter)
        s = self._lib.fk_iterate(self._h, max_iter, tol, precision, ctypes.byref(it),
                                 ctypes.byref(d), _dptr(hist))
        if s not in (FK_OK, FK_ENOTCONV):
            self._check(s, "fk_iterate")
        return dict(iters=it.value, delta=d.value, history=hist[:it.value],
                    converged=(s == FK_OK))

    def autotune(self, max_bytes=24 * 2 ** 30, keep=True):
        t = Tuning()
        self._check(self._lib.fk_autotune(self._h, float(max_bytes), int(keep),
                                          ctypes.byref(t)), "fk_autotune")
        return t.as_dict()

    def set_tuning(self, tile_rows=64, batch=0, lookahead=0):
        t = Tuning(tile_rows, batch, lookahead, 0.0, 0.0, 0)
        self._check(self._lib.fk_set_tuning(self._h, ctypes.byref(t)), "fk_set_tuning")

    def get_tuning(self):
        t = Tuning()
        self._check(self._lib.fk_get_tuning(self._h, ctypes.byref(t)), "fk_get_tuning")
        return t.as_dict()

    def get_point_green(self, k, out=None):
        out = np.zeros((self.n_c, self.n_c), np.complex128) if out is None else out
        p, dev, _ = self._matrix_arg(out, True)
        self._check(self._lib.fk_get_point_green(self._h, int(k), p, dev),
                    "fk_get_point_green")
        return out

    def low_iterations(self):
        n = ctypes.c_int()
        self._check(self._lib.fk_low_iterations(self._h, ctypes.byref(n)), "fk_low_iterations")
        return n.value

    def set_kernel_clock(self, on=True):
        self._check(self._lib.fk_set_kernel_clock(self._h, int(on)), "fk_set_kernel_clock")

    def kernel_clock(self):
        out = np.zeros(3)
        self._check(self._lib.fk_kernel_clock(self._h, _dptr(out)), "fk_kernel_clock")
        return dict(ms=out[0], launches=int(out[1]), flop=out[2])

    def iterate_judged(self, fallback, max_iter, tol=0.0, accept=0.5,
                       precision=FK_FP64):
        """fk_iterate_judged from the current Sigma; fallback: torch device
        matrix or None (Sigma = 0)."""
        it = ctypes.c_int()
        d = ctypes.c_double()
        oc = ctypes.c_int()
        hist = np.zeros(max_iter)
        fp = None if fallback is None else self._matrix_arg(fallback, False)
        if fp is not None and fp[1] != 1:
            raise ValueError("fallback must be a device tensor")
        s = self._lib.fk_iterate_judged(self._h, None if fp is None else fp[0],
                                        float(accept), max_iter, tol, precision,
                                        ctypes.byref(it), ctypes.byref(d), _dptr(hist),
                                        ctypes.byref(oc))
        if s not in (FK_OK, FK_ENOTCONV):
            self._check(s, "fk_iterate_judged")
        return dict(iters=it.value, delta=d.value, history=hist[:it.value],
                    converged=(s == FK_OK and tol > 0), outcome=oc.value)

    # -- learned warm start (device tensors: torch, contiguous)
    def ws_sketch(self, sigma_dev, omega):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        sv = np.zeros(om.shape[1])
        self._check(self._lib.fk_ws_sketch(self._h, sigma_dev.data_ptr(), om.shape[1],
                                           om.ctypes.data, _dptr(sv)), "fk_ws_sketch")
        return sv

    def ws_features(self, sigma_prev_dev, glob, idx_dev, rows, scale, x_dev, d_in):
        g = np.ascontiguousarray(glob, dtype=np.float32)
        self._check(self._lib.fk_ws_features(
            self._h, sigma_prev_dev.data_ptr(), g.ctypes.data, len(g),
            None if idx_dev is None else idx_dev.data_ptr(), rows, float(scale),
            x_dev.data_ptr(), d_in), "fk_ws_features")

    def ws_targets(self, sigma_prev_dev, sigma_new_dev, idx_dev, rows, scale, t_dev):
        self._check(self._lib.fk_ws_targets(
            self._h, sigma_prev_dev.data_ptr(), sigma_new_dev.data_ptr(),
            None if idx_dev is None else idx_dev.data_ptr(), rows, float(scale),
            t_dev.data_ptr()), "fk_ws_targets")

    def ws_apply(self, sigma_prev_dev, y_dev, scale, keep_pre_field=False):
        self._check(self._lib.fk_ws_apply(self._h, sigma_prev_dev.data_ptr(),
                                          y_dev.data_ptr(), float(scale),
                                          int(bool(keep_pre_field))), "fk_ws_apply")

    def timings(self):
        out = np.zeros(7)
        self._check(self._lib.fk_timings(self._h, _dptr(out)), "fk_timings")
        return dict(build_ms=out[0], invert_ms=out[1], refine_ms=out[2],
                    reduce_ms=out[3], impurity_ms=out[4], launches=int(out[5]),
                    step_kernels_ms=out[6])


class _Instance(Context):
    """View of one instance of a Batch (owned by the batch)."""

    def __init__(self, lib, handle, owner):
        self._lib = lib
        self._h = handle
        self._owner = owner
        nt, ntau, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lib.fk_dims(handle, ctypes.byref(nt), ctypes.byref(ntau), ctypes.byref(nc))
        self.n_t, self.n_tau, self.n_c = nt.value, ntau.value, nc.value

    def close(self):
        self._h = None


class Batch:
    """fk_batch: instances = list of dicts with the keyword arguments of
    Context (contour, model); instance(i) gives a Context-like view."""

    def __init__(self, instances):
        lib = library()
        self._lib = lib
        n = len(instances)
        cs = (Contour * n)()
        ms = (Model * n)()
        for i, kw in enumerate(instances):
            cs[i] = Contour(kw["t_min"], kw["t_max"], kw["dt"], kw["dtau"], kw["beta"])
            ms[i] = Model(kw["U"], kw["E"], kw.get("mu", 0.0), kw.get("w1", 0.5),
                          kw.get("n_eps", 10), kw.get("n_ebar", 10),
                          CONVENTION[kw.get("convention", "symmetric")],
                          int(kw.get("gh_average", False)))
        h = _vp()
        s = lib.fk_batch_create(n, cs, ms, ctypes.byref(h))
        if s != FK_OK:
            raise FkError(s, "fk_batch_create")
        self._h = h
        self.n = n
        self._views = []
        for i in range(n):
            c = _vp()
            self._check(lib.fk_batch_instance(h, i, ctypes.byref(c)), "fk_batch_instance")
            self._views.append(_Instance(lib, c, self))

    def _check(self, s, what):
        if s != FK_OK:
            raise FkError(s, f"{what}: {self._lib.fk_batch_last_error(self._h).decode()}")

    def instance(self, i):
        return self._views[i]

    def set_chunk_bytes(self, b):
        self._check(self._lib.fk_batch_set_chunk_bytes(self._h, float(b)), "chunk")

    def reset(self):
        self._check(self._lib.fk_batch_reset(self._h), "fk_batch_reset")

    def iterate(self, max_sweeps, tol=0.0, use_graph=True):
        sw = ctypes.c_int()
        it = (ctypes.c_int * self.n)()
        dl = np.zeros(self.n)
        self._check(self._lib.fk_batch_iterate(self._h, max_sweeps, tol, int(use_graph),
                                               ctypes.byref(sw), it, _dptr(dl)),
                    "fk_batch_iterate")
        return dict(sweeps=sw.value, iters=np.array(list(it)), deltas=dl)

    def set_tuning(self, tile_rows=64, lookahead=0, chunk_bytes=0.0):
        t = Tuning(tile_rows, 0, lookahead, float(chunk_bytes), 0.0, 0)
        self._check(self._lib.fk_batch_set_tuning(self._h, ctypes.byref(t)),
                    "fk_batch_set_tuning")

    def autotune(self, max_bytes=24 * 2 ** 30, only_nc=0):
        """Schedule per contour size (fk_batch_autotune; only_nc > 0: that size
        alone, merged into the table): list of dicts with n_c and the tuning
        fields of every class in the table."""
        cap = self.n
        ncls = ctypes.c_int()
        ncs = (ctypes.c_int * cap)()
        tun = (Tuning * cap)()
        self._check(self._lib.fk_batch_autotune(self._h, float(max_bytes), int(only_nc),
                                                cap, ctypes.byref(ncls), ncs, tun),
                    "fk_batch_autotune")
        return [dict(n_c=ncs[q], **tun[q].as_dict()) for q in range(ncls.value)]

    def timings(self):
        out = np.zeros(4)
        self._check(self._lib.fk_batch_timings(self._h, _dptr(out)), "fk_batch_timings")
        return dict(last_sweep_ms=out[0], total_ms=out[1], captures=int(out[2]),
                    capture_ms=out[3])

    def close(self):
        if getattr(self, "_h", None):
            for v in self._views:
                v._h = None
            self._lib.fk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class MLP:
    """fk_mlp: depth linear layers (tanh between), float32 parameters packed as
    W_l (out x in) then b_l.  Tensors passed in are torch float32 on the GPU."""

    def __init__(self, d_in, width, depth, d_out, params=None, seed=0):
        lib = library()
        self._lib = lib
        self.d_in, self.width, self.depth, self.d_out = d_in, width, depth, d_out
        dims = [d_in] + [width] * (depth - 1) + [d_out]
        self.shapes = [(dims[i + 1], dims[i]) for i in range(depth)]
        if params is None:
            rng = np.random.default_rng(seed)
            parts = []
            for o, i in self.shapes:
                parts.append((rng.standard_normal((o, i)) * np.sqrt(1.0 / i)).ravel())
                parts.append(np.zeros(o))
            params = np.concatenate(parts)
        p = np.ascontiguousarray(params, dtype=np.float32)
        h = _vp()
        st = lib.fk_mlp_create(d_in, width, depth, d_out, p.ctypes.data, ctypes.byref(h))
        if st != FK_OK:
            raise FkError(st, "fk_mlp_create")
        self._h = h
        n = ctypes.c_longlong()
        lib.fk_mlp_n_params(h, ctypes.byref(n))
        self.n_params = n.value

    def _check(self, s, what):
        if s != FK_OK:
            raise FkError(s, f"{what}: {self._lib.fk_mlp_last_error(self._h).decode()}")

    def get_params(self):
        p = np.zeros(self.n_params, np.float32)
        self._check(self._lib.fk_mlp_get_params(self._h, p.ctypes.data), "get_params")
        return p

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        self._check(self._lib.fk_mlp_set_params(self._h, p.ctypes.data), "set_params")

    def forward(self, x, bf16=False):
        import torch
        assert x.is_contiguous() and x.dtype == torch.float32 and x.shape[1] == self.d_in
        y = torch.empty((x.shape[0], self.d_out), dtype=torch.float32, device=x.device)
        self._check(self._lib.fk_mlp_forward(self._h, x.data_ptr(), x.shape[0],
                                             y.data_ptr(), int(bf16)), "fk_mlp_forward")
        return y

    def loss_grad(self, x, t):
        loss = ctypes.c_double()
        g = np.zeros(self.n_params, np.float32)
        self._check(self._lib.fk_mlp_loss_grad(self._h, x.data_ptr(), t.data_ptr(),
                                               x.shape[0], ctypes.byref(loss),
                                               g.ctypes.data), "fk_mlp_loss_grad")
        return loss.value, g

    def train(self, x, t, batch, steps, lr, seed=0):
        hist = np.zeros(steps)
        self._check(self._lib.fk_mlp_train(self._h, x.data_ptr(), t.data_ptr(),
                                           x.shape[0], batch, steps, float(lr),
                                           int(seed), _dptr(hist)), "fk_mlp_train")
        return hist

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fk_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
