"""C-ABI library: loads, exports every declared symbol, validates arguments
on the host (no GPU needed for these paths)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1211_0393_amd as P
from paper_1211_0393_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ardeblur.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ar_[A-Za-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.load()
    names = declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == bound


def test_version_string():
    assert "gfx950" in P.version()


def _create(n1, n2, psf, dtype=0, device=0):
    lib = P.load()
    h = C.c_void_p()
    psf = np.ascontiguousarray(psf, dtype=np.float64)
    q1, q2 = (psf.shape[0] - 1) // 2, (psf.shape[1] - 1) // 2
    rc = lib.ar_plan_create(C.byref(h), n1, n2, psf.ctypes.data_as(C.POINTER(C.c_double)),
                            q1, q2, dtype, device)
    return rc, h, lib.ar_last_error().decode()


@pytest.mark.parametrize("n1,n2,q", [(2, 8, 0), (8, 2, 0), (5, 5, 3), (4, 9, 2), (0, 0, 0)])
def test_shape_errors(n1, n2, q):
    psf = np.zeros((2 * q + 1, 2 * q + 1))
    psf[q, q] = 1.0
    rc, h, msg = _create(n1, n2, psf)
    assert rc == -2, msg
    assert not h.value


def test_axis_too_long_for_lds_transform():
    psf = np.ones((1, 1))
    assert _create(9597, 16, psf)[0] == -2
    assert _create(16, 4799, psf, dtype=1)[0] == -2
    assert _create(4799, 16, psf, dtype=2)[0] == -2


@pytest.mark.parametrize("bad", ["neg", "nan", "inf", "sum"])
def test_psf_errors(bad):
    psf = np.full((3, 3), 1.0 / 9)
    if bad == "neg":
        psf[0, 0] = -1e-3
        psf[1, 1] += 1e-3
    elif bad == "nan":
        psf[0, 0] = np.nan
    elif bad == "inf":
        psf[0, 0] = np.inf
    else:
        psf *= 1.001
    rc, h, msg = _create(16, 16, psf)
    assert rc == -3, msg


def test_psf_sum_tolerance_scales_with_taps():
    psf = np.full((3, 3), 1.0 / 9)
    psf[1, 1] += 5e-12          # 5e-12 <= 1e-12 * 9: accepted by validation
    rc, h, msg = _create(16, 16, psf)
    assert rc != -3, msg


def test_bad_dtype_and_null_arguments():
    lib = P.load()
    psf = np.ones((1, 1))
    assert _create(8, 8, psf, dtype=7)[0] == -1
    h = C.c_void_p()
    assert lib.ar_plan_create(None, 8, 8, psf.ctypes.data_as(C.POINTER(C.c_double)), 0, 0, 0, 0) == -1
    assert lib.ar_plan_create(C.byref(h), 8, 8, None, 0, 0, 0, 0) == -1
    # every entry point rejects a NULL plan without touching the device
    assert lib.ar_blur_apply(None, None, None, None) == -1
    assert lib.ar_blur_apply_T(None, None, None, 0, None) == -1
    assert lib.ar_transform(None, None, None, None) == -1
    assert lib.ar_transform_inv(None, None, None, None) == -1
    assert lib.ar_precond_solve(None, None, None, None) == -1
    assert lib.ar_tikhonov_solve(None, None, None, 0.1, None) == -1
    assert lib.ar_precond_set(None, 0, 1.0, None, None) == -1
    assert lib.ar_eigenvalues(None, None, None) == -1
    assert lib.ar_filter_values(None, None, None) == -1
    assert lib.ar_deblur_iterate(None, None, None, 1, 1.0, 0, 1, None, None, None, None, None) == -1
    assert lib.ar_plan_tune(None, 0, 1) == -1
    assert lib.ar_plan_get_tune(None, 0, None) == -1
    assert lib.ar_plan_autotune(None, None, None) == -1
    assert lib.ar_iterate_profile(None, None, None, 0, 1, 1, None, None) == -1
    assert lib.ar_plan_destroy(None) == 0
    assert "null" in lib.ar_last_error().decode().lower()


def test_binding_is_marshalling_only():
    """The Python package never imports the oracle and has no numerics of
    the method: its only numpy use is argument marshalling."""
    pkg = os.path.join(ROOT, "paper_1211_0393_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src.replace("oracle/", ""), fn
            assert "scipy" not in src, fn


def _prototypes():
    """name -> list of parameter types (names dropped, spaces normalised)
    of every function declared in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"(?:int\s+|const char\s*\*\s*)(ar_[a-z_0-9A-Z]+)\s*\(([^;]*?)\)\s*;", text):
        params = []
        for a in m.group(2).split(","):
            a = " ".join(a.split())
            if a in ("void", ""):
                continue
            a = re.sub(r"\s*\*\s*", " *", a)
            a = re.sub(r"\s+[A-Za-z_][A-Za-z_0-9]*$", "", a) if not a.endswith("*") else a
            a = re.sub(r"\*[A-Za-z_][A-Za-z_0-9]*$", "*", a)
            params.append(a.strip())
        out[m.group(1)] = params
    return out


# The boundary the hot path exposes, with its argument types in order.
# Where the library differs from the plain list of calls (a stream argument
# on every call that enqueues device work, the richer batched iterate, the
# network made from parameters or from a weights file), the difference is
# the second entry.
SPEC = {
    "ar_plan_create": ["ar_plan_t *", "int", "int", "const double *", "int", "int", "int", "int"],
    "ar_plan_destroy": ["ar_plan_t"],
    "ar_blur_apply": ["ar_plan_t", "const void *", "void *", "void *"],
    "ar_blur_apply_T": ["ar_plan_t", "const void *", "void *", "int", "void *"],
    "ar_transform": ["ar_plan_t", "const void *", "void *", "void *"],
    "ar_transform_inv": ["ar_plan_t", "const void *", "void *", "void *"],
    "ar_precond_set": ["ar_plan_t", "int", "double", "const float *", "void *"],
    "ar_eigenvalues": ["ar_plan_t", "double *", "void *"],
    "ar_precond_solve": ["ar_plan_t", "const void *", "void *", "void *"],
    "ar_deblur_iterate": ["ar_plan_t", "const void *", "void *", "int", "double", "int", "int",
                          "const void *", "double *", "double *", "int *", "void *"],
    "ar_batch_create": ["ar_batch_t *", "int", "const ar_plan_t *", "void *"],
    "ar_batch_iterate": ["ar_batch_t", "const void *const *", "void *const *", "int", "double",
                         "int", "int", "const void *const *", "double *", "double *", "int *",
                         "void *"],
    "ar_batch_destroy": ["ar_batch_t"],
    "ar_fnet_create": ["ar_fnet_t *", "const float *", "int"],
    "ar_fnet_load": ["ar_fnet_t *", "const char *", "int"],
    "ar_psf_normalize": ["double *", "int", "int"],
    "ar_last_error": [],
}


def test_boundary_signatures():
    protos = _prototypes()
    for name, params in SPEC.items():
        assert name in protos, name
        assert protos[name] == params, (name, protos[name])


def test_psf_normalize_host_helper():
    psf = np.array([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]])
    P.ar_psf_normalize(psf)
    assert abs(psf.sum() - 1.0) < 1e-15
    assert psf[1, 1] == 0.25
    lib = P.load()
    for bad in (np.array([[1.0, -1.0, 1.0]]), np.array([[np.nan]]), np.zeros((3, 3))):
        keep = bad.copy()
        rc = lib.ar_psf_normalize(bad.ctypes.data_as(C.POINTER(C.c_double)),
                                  (bad.shape[0] - 1) // 2, (bad.shape[1] - 1) // 2)
        assert rc == -3
        np.testing.assert_array_equal(bad, keep)
    assert lib.ar_psf_normalize(None, 0, 0) == -1
    assert lib.ar_psf_normalize(psf.ctypes.data_as(C.POINTER(C.c_double)), -1, 0) == -2


def test_fnet_load_rejects_bad_files(tmp_path):
    lib = P.load()
    h = C.c_void_p()
    assert lib.ar_fnet_load(C.byref(h), os.fsencode(str(tmp_path / "missing.npy")), 0) == -1
    wrong = tmp_path / "wrong.npy"
    np.save(wrong, np.zeros(10, dtype=np.float32))
    assert lib.ar_fnet_load(C.byref(h), os.fsencode(str(wrong)), 0) == -1
    f64 = tmp_path / "f64.npy"
    np.save(f64, np.zeros(P.AR_FNET_NPARAM, dtype=np.float64))
    assert lib.ar_fnet_load(C.byref(h), os.fsencode(str(f64)), 0) == -1
    assert "ar_fnet_load" in lib.ar_last_error().decode()
    assert not h.value
