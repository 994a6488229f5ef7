"""The allocation-free iterate entry point, called through the C ABI, against
ar_deblur_iterate on the same inputs: two calls in a row (the second on a
smaller problem with fewer iterations), bitwise equal iterates and scalars;
sizes beyond its static buffer are refused before any device work."""

import ctypes as C
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1211_0393_amd as P  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(fn, plan, g, x, iters, f):
    res = (C.c_double * iters)()
    rre = (C.c_double * iters)()
    best = C.c_int(-1)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(plan.handle, C.c_void_p(g.data_ptr()), C.c_void_p(x.data_ptr()), iters, 1.0,
            P.AR_REBLUR, 1, C.c_void_p(f.data_ptr()), C.cast(res, C.POINTER(C.c_double)),
            C.cast(rre, C.POINTER(C.c_double)), C.byref(best), stream)
    torch.cuda.synchronize()
    return rc, np.array(res[:]), np.array(rre[:]), best.value


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_matches_allocating_entry_point(dt):
    lib = P.load()
    tdt = torch.float32 if dt == "f32" else torch.float64
    cases = [(256, 7, 20), (64, 4, 5)]          # second call: smaller image, fewer iterations
    for n, q, iters in cases:
        H = synth.psf_gauss_shifted(q, q, 2.0, 1.0, shift=(0.7, -0.4))
        F = synth.phantom(n, n, 5, 3, seed=n)
        f = torch.from_numpy(F).to(DEV, tdt)
        with P.Plan(n, n, H, dtype=dt) as plan:
            plan.ar_precond_set(P.AR_FILTER_TIKHONOV, 0.2)
            g = torch.empty_like(f)
            plan.ar_blur_apply(f, g)
            xa, xb = torch.zeros_like(g), torch.zeros_like(g)
            ra = _call(lib.ar_deblur_iterate, plan, g, xa, iters, f)
            rb = _call(lib.ar_deblur_iterate_noalloc, plan, g, xb, iters, f)
            say(f"  {dt} {n}x{n} {iters} its: rc {ra[0]} / {rb[0]}, best {ra[3]} / {rb[3]}")
            assert ra[0] == 0 and rb[0] == 0
            assert torch.equal(xa, xb)
            np.testing.assert_array_equal(ra[1], rb[1])
            np.testing.assert_array_equal(ra[2], rb[2])
            assert ra[3] == rb[3] >= 1


def test_noalloc_refuses_runs_beyond_its_buffer():
    lib = P.load()
    n = 1024
    H = synth.psf_motion(7)
    with P.Plan(n, n, H, dtype="f32") as plan:
        g = torch.zeros((n, n), device=DEV, dtype=torch.float32)
        x = torch.zeros_like(g)
        f = torch.ones_like(g)
        iters = 5000
        res = (C.c_double * iters)()
        rc = lib.ar_deblur_iterate_noalloc(plan.handle, C.c_void_p(g.data_ptr()),
                                           C.c_void_p(x.data_ptr()), iters, 1.0, 0, 1, None,
                                           C.cast(res, C.POINTER(C.c_double)), None, None, None)
        assert rc == -1
        assert "static buffer" in lib.ar_last_error().decode()
        # best_it without an rre array is refused too
        best = C.c_int(0)
        rc = lib.ar_deblur_iterate_noalloc(plan.handle, C.c_void_p(g.data_ptr()),
                                           C.c_void_p(x.data_ptr()), 3, 1.0, 0, 1,
                                           C.c_void_p(f.data_ptr()), None, None, C.byref(best),
                                           None)
        assert rc == -1
        # without scalars any length runs (nothing goes to the buffer)
        rc = lib.ar_deblur_iterate_noalloc(plan.handle, C.c_void_p(g.data_ptr()),
                                           C.c_void_p(x.data_ptr()), 2, 1.0, 0, 1, None, None,
                                           None, None, None)
        torch.cuda.synchronize()
        assert rc == 0
