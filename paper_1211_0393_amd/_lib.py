"""ctypes binding of libardeblur.so (argument marshalling only).

Every function mirrors one C entry point of ``include/ardeblur.h`` under the
same name.  Image arguments are torch tensors on the plan's device (their
data pointers are passed through); streams default to torch's current
stream.  Nothing here computes any step of the method: if the library is
missing the import fails loudly.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libardeblur.so")

AR_F32, AR_F64, AR_F32_ACC64, AR_F32_BF16X3 = 0, 1, 2, 3
DTYPES = {"f32": AR_F32, "f64": AR_F64, "f32x": AR_F32_ACC64, "bf16x3": AR_F32_BF16X3}
AR_REBLUR, AR_ADJOINT = 0, 1
AR_BC_ANTIREFLECTIVE, AR_BC_REFLECTIVE, AR_BC_PERIODIC = 0, 1, 2
BCS = {"antireflective": AR_BC_ANTIREFLECTIVE, "reflective": AR_BC_REFLECTIVE,
       "periodic": AR_BC_PERIODIC}
AR_FILTER_TIKHONOV, AR_FILTER_THRESHOLD, AR_FILTER_GAINS, AR_FILTER_IDENTITY = 0, 1, 2, 3
AR_FNET_BINS, AR_FNET_IN, AR_FNET_HIDDEN, AR_FNET_NPARAM = 64, 65, 128, 33216
AR_TUNE_ROW_WAVES, AR_TUNE_COL_WAVES, AR_TUNE_ROW_EXCL, AR_TUNE_COL_EXCL = 0, 1, 2, 3
AR_TUNE_ROW_ALGO, AR_TUNE_COL_ALGO, AR_TUNE_ROW_LANES, AR_TUNE_COL_LANES = 4, 5, 6, 7
AR_TUNE_BLUR = 8
AR_TUNE_FUSE = 9

STATUS = {
    0: "AR_OK", -1: "AR_EINVAL", -2: "AR_ESHAPE", -3: "AR_EPSF", -4: "AR_EALIAS",
    -5: "AR_EDEVICE", -6: "AR_ENOMEM", -7: "AR_ENONFINITE", -8: "AR_EUNSUPPORTED",
}

# (name, restype, argtypes) of every exported entry point
_VP, _I, _D = C.c_void_p, C.c_int, C.c_double
SIGNATURES = [
    ("ar_plan_create", _I, [C.POINTER(_VP), _I, _I, C.POINTER(_D), _I, _I, _I, _I]),
    ("ar_plan_create_bc", _I, [C.POINTER(_VP), _I, _I, C.POINTER(_D), _I, _I, _I, _I, _I]),
    ("ar_plan_destroy", _I, [_VP]),
    ("ar_blur_apply", _I, [_VP, _VP, _VP, _VP]),
    ("ar_blur_apply_T", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ar_transform", _I, [_VP, _VP, _VP, _VP]),
    ("ar_transform_inv", _I, [_VP, _VP, _VP, _VP]),
    ("ar_precond_set", _I, [_VP, _I, _D, _VP, _VP]),
    ("ar_psf_normalize", _I, [C.POINTER(_D), _I, _I]),
    ("ar_eigenvalues", _I, [_VP, _VP, _VP]),
    ("ar_filter_values", _I, [_VP, _VP, _VP]),
    ("ar_precond_solve", _I, [_VP, _VP, _VP, _VP]),
    ("ar_tikhonov_solve", _I, [_VP, _VP, _VP, _D, _VP]),
    ("ar_deblur_iterate", _I, [_VP, _VP, _VP, _I, _D, _I, _I, _VP,
                               C.POINTER(_D), C.POINTER(_D), C.POINTER(_I), _VP]),
    ("ar_deblur_iterate_noalloc", _I, [_VP, _VP, _VP, _I, _D, _I, _I, _VP,
                                       C.POINTER(_D), C.POINTER(_D), C.POINTER(_I), _VP]),
    ("ar_plan_tune", _I, [_VP, _I, _I]),
    ("ar_plan_get_tune", _I, [_VP, _I, C.POINTER(_I)]),
    ("ar_plan_autotune", _I, [_VP, C.POINTER(_D), _VP]),
    ("ar_iterate_profile", _I, [_VP, _VP, _VP, _I, _I, _I, C.POINTER(_D), _VP]),
    ("ar_batch_create", _I, [C.POINTER(_VP), _I, C.POINTER(_VP), _VP]),
    ("ar_batch_autotune", _I, [_VP, C.POINTER(_D), _VP]),
    ("ar_batch_iterate", _I, [_VP, C.POINTER(_VP), C.POINTER(_VP), _I, _D, _I, _I,
                              C.POINTER(_VP), C.POINTER(_D), C.POINTER(_D), C.POINTER(_I), _VP]),
    ("ar_batch_destroy", _I, [_VP]),
    ("ar_plan_set_psf", _I, [_VP, C.POINTER(_D), _I, _I, _VP]),
    ("ar_features", _I, [_VP, _VP, _VP, _VP]),
    ("ar_precond_set_gains", _I, [_VP, _VP, _VP]),
    ("ar_gains_label", _I, [_VP, _VP, _VP]),
    ("ar_fnet_create", _I, [C.POINTER(_VP), C.POINTER(C.c_float), _I]),
    ("ar_fnet_load", _I, [C.POINTER(_VP), C.c_char_p, _I]),
    ("ar_fnet_destroy", _I, [_VP]),
    ("ar_fnet_get_params", _I, [_VP, C.POINTER(C.c_float)]),
    ("ar_fnet_infer", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ar_fnet_grad", _I, [_VP, _VP, _VP, _I, _VP, _VP, _VP]),
    ("ar_fnet_train_step", _I, [_VP, _VP, _VP, _I, C.c_float, _VP, _VP]),
    ("ar_last_error", C.c_char_p, []),
    ("ar_version", C.c_char_p, []),
]

_lib = None


def load(path: str | None = None):
    """Load the shared library (raises if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # load torch's HIP runtime first so that the library binds to the same
    # runtime instance as the tensors and streams it is handed
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise ImportError(f"{p} is not built; run `python -m paper_1211_0393_amd.build`")
    lib = C.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class ArError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(rc):
    if rc != 0:
        raise ArError(rc, load().ar_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Plan:
    """Owns an ``ar_plan_t``; methods are the C entry points."""

    def __init__(self, n1, n2, psf, dtype="f32", device=0, bc="antireflective"):
        psf = np.ascontiguousarray(psf, dtype=np.float64)
        if psf.ndim != 2:
            raise ValueError("psf must be 2-D")
        self.n1, self.n2 = int(n1), int(n2)
        self.q1, self.q2 = (psf.shape[0] - 1) // 2, (psf.shape[1] - 1) // 2
        self.dtype = DTYPES[dtype]
        self.bc = BCS[bc]
        self.device = int(device)
        self._h = C.c_void_p()
        lib = load()
        _check(lib.ar_plan_create_bc(C.byref(self._h), self.n1, self.n2,
                                     psf.ctypes.data_as(C.POINTER(C.c_double)),
                                     self.q1, self.q2, self.dtype, self.bc, self.device))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load().ar_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- entry points -------------------------------------------------
    def ar_plan_tune(self, key, value):
        _check(load().ar_plan_tune(self._h, int(key), int(value)))

    def ar_plan_get_tune(self, key):
        v = C.c_int(0)
        _check(load().ar_plan_get_tune(self._h, int(key), C.byref(v)))
        return v.value

    def ar_plan_autotune(self, stream=None):
        """Pick the fastest launch tunables; returns the best time in us."""
        us = C.c_double(0.0)
        _check(load().ar_plan_autotune(self._h, C.byref(us), _stream(stream)))
        return us.value

    def ar_iterate_profile(self, g, x, tmode=AR_REBLUR, precondition=True, reps=20, stream=None):
        """Average microseconds of the five kernels of one iteration."""
        us = (C.c_double * 5)()
        _check(load().ar_iterate_profile(self._h, _ptr(g), _ptr(x), int(tmode),
                                         int(bool(precondition)), int(reps),
                                         C.cast(us, C.POINTER(C.c_double)), _stream(stream)))
        return list(us)

    def ar_blur_apply(self, x, y, stream=None):
        _check(load().ar_blur_apply(self._h, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def ar_blur_apply_T(self, r, y, tmode=AR_REBLUR, stream=None):
        _check(load().ar_blur_apply_T(self._h, _ptr(r), _ptr(y), int(tmode), _stream(stream)))
        return y

    def ar_transform(self, x, c, stream=None):
        _check(load().ar_transform(self._h, _ptr(x), _ptr(c), _stream(stream)))
        return c

    def ar_transform_inv(self, c, x, stream=None):
        _check(load().ar_transform_inv(self._h, _ptr(c), _ptr(x), _stream(stream)))
        return x

    def ar_precond_set(self, filt=AR_FILTER_TIKHONOV, param=1e-2, gains=None, stream=None):
        _check(load().ar_precond_set(self._h, int(filt), float(param), _ptr(gains),
                                     _stream(stream)))

    def ar_eigenvalues(self, lam, stream=None):
        _check(load().ar_eigenvalues(self._h, _ptr(lam), _stream(stream)))
        return lam

    def ar_filter_values(self, d, stream=None):
        _check(load().ar_filter_values(self._h, _ptr(d), _stream(stream)))
        return d

    def ar_precond_solve(self, y, z, stream=None):
        _check(load().ar_precond_solve(self._h, _ptr(y), _ptr(z), _stream(stream)))
        return z

    def ar_tikhonov_solve(self, g, x, alpha, stream=None):
        _check(load().ar_tikhonov_solve(self._h, _ptr(g), _ptr(x), float(alpha),
                                        _stream(stream)))
        return x

    def ar_plan_set_psf(self, psf, stream=None):
        psf = np.ascontiguousarray(psf, dtype=np.float64)
        q1, q2 = (psf.shape[0] - 1) // 2, (psf.shape[1] - 1) // 2
        _check(load().ar_plan_set_psf(self._h, psf.ctypes.data_as(C.POINTER(C.c_double)),
                                      q1, q2, _stream(stream)))
        self.q1, self.q2 = q1, q2

    def ar_features(self, g, feat, stream=None):
        _check(load().ar_features(self._h, _ptr(g), _ptr(feat), _stream(stream)))
        return feat

    def ar_precond_set_gains(self, gains, stream=None):
        _check(load().ar_precond_set_gains(self._h, _ptr(gains), _stream(stream)))

    def ar_gains_label(self, label, stream=None):
        _check(load().ar_gains_label(self._h, _ptr(label), _stream(stream)))
        return label

    def ar_deblur_iterate(self, g, x, iters, tau=1.0, tmode=AR_REBLUR, precondition=True,
                          f_true=None, want_resnorm=False, want_rre=False, stream=None):
        """Returns (status, resnorm or None, rre or None, best_it or None)."""
        res = (C.c_double * iters)() if want_resnorm and iters > 0 else None
        rre = (C.c_double * iters)() if want_rre and iters > 0 else None
        best = C.c_int(0) if want_rre else None
        rc = load().ar_deblur_iterate(
            self._h, _ptr(g), _ptr(x), int(iters), float(tau), int(tmode), int(bool(precondition)),
            _ptr(f_true),
            C.cast(res, C.POINTER(C.c_double)) if res is not None else None,
            C.cast(rre, C.POINTER(C.c_double)) if rre is not None else None,
            C.byref(best) if best is not None else None,
            _stream(stream))
        if rc not in (0, -7):
            _check(rc)
        return (rc,
                np.array(res[:]) if res is not None else None,
                np.array(rre[:]) if rre is not None else None,
                best.value if best is not None else None)


def _ptr_array(ts):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


class Batch:
    """Owns an ``ar_batch_t`` over a list of :class:`Plan` (kept alive here)."""

    def __init__(self, plans, stream=None):
        self.plans = list(plans)
        self.count = len(self.plans)
        handles = (C.c_void_p * self.count)(*[p.handle.value for p in self.plans])
        self._h = C.c_void_p()
        _check(load().ar_batch_create(C.byref(self._h), self.count, handles, _stream(stream)))

    def close(self):
        if self._h:
            load().ar_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def ar_batch_autotune(self, stream=None):
        us = C.c_double(0.0)
        _check(load().ar_batch_autotune(self._h, C.byref(us), _stream(stream)))
        return us.value

    def ar_batch_iterate(self, g, x, iters, tau=1.0, tmode=AR_REBLUR, precondition=True,
                         f_true=None, want_resnorm=False, want_rre=False, stream=None):
        """g, x, f_true: lists of tensors.  Returns (status, resnorm[count, iters] or None,
        rre[count, iters] or None, best_it[count] or None)."""
        n = self.count
        if len(g) != n or len(x) != n or (f_true is not None and len(f_true) != n):
            raise ValueError("one tensor per problem expected")
        gp, xp = _ptr_array(g), _ptr_array(x)
        fp = _ptr_array(f_true) if f_true is not None else None
        res = (C.c_double * (n * iters))() if want_resnorm and iters > 0 else None
        rre = (C.c_double * (n * iters))() if want_rre and iters > 0 else None
        best = (C.c_int * n)() if want_rre else None
        rc = load().ar_batch_iterate(
            self._h, gp, xp, int(iters), float(tau), int(tmode), int(bool(precondition)), fp,
            C.cast(res, C.POINTER(C.c_double)) if res is not None else None,
            C.cast(rre, C.POINTER(C.c_double)) if rre is not None else None,
            C.cast(best, C.POINTER(C.c_int)) if best is not None else None,
            _stream(stream))
        if rc not in (0, -7):
            _check(rc)
        return (rc,
                np.array(res[:]).reshape(n, iters) if res is not None else None,
                np.array(rre[:]).reshape(n, iters) if rre is not None else None,
                np.array(best[:]) if best is not None else None)


def ar_psf_normalize(psf):
    """Divide a host PSF (2-D float64 array) by its sum in place."""
    if not (isinstance(psf, np.ndarray) and psf.dtype == np.float64 and psf.ndim == 2
            and psf.flags.c_contiguous):
        raise ValueError("psf must be a C-contiguous 2-D float64 array")
    q1, q2 = (psf.shape[0] - 1) // 2, (psf.shape[1] - 1) // 2
    _check(load().ar_psf_normalize(psf.ctypes.data_as(C.POINTER(C.c_double)), q1, q2))
    return psf


class FNet:
    """Owns an ``ar_fnet_t`` (the filter network) on one device: created
    from a host parameter vector, or from a weights file (``path``)."""

    def __init__(self, params=None, device=0, path=None):
        self.device = int(device)
        self._h = C.c_void_p()
        if path is not None:
            _check(load().ar_fnet_load(C.byref(self._h), os.fsencode(path), self.device))
            return
        params = np.ascontiguousarray(params, dtype=np.float32)
        if params.size != AR_FNET_NPARAM:
            raise ValueError(f"expected {AR_FNET_NPARAM} parameters")
        _check(load().ar_fnet_create(C.byref(self._h),
                                     params.ctypes.data_as(C.POINTER(C.c_float)), self.device))

    def close(self):
        if self._h:
            load().ar_fnet_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def ar_fnet_get_params(self):
        out = np.empty(AR_FNET_NPARAM, dtype=np.float32)
        _check(load().ar_fnet_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def ar_fnet_infer(self, x, y, stream=None):
        _check(load().ar_fnet_infer(self._h, _ptr(x), _ptr(y), int(x.shape[0]), _stream(stream)))
        return y

    def ar_fnet_grad(self, x, t, grad, loss=None, stream=None):
        _check(load().ar_fnet_grad(self._h, _ptr(x), _ptr(t), int(x.shape[0]), _ptr(grad),
                                   _ptr(loss), _stream(stream)))
        return grad

    def ar_fnet_train_step(self, x, t, lr, loss=None, stream=None):
        _check(load().ar_fnet_train_step(self._h, _ptr(x), _ptr(t), int(x.shape[0]),
                                         float(lr), _ptr(loss), _stream(stream)))


def version():
    return load().ar_version().decode()
