"""Reflective (DCT-III algebra) and Periodic (two-level circulant) boundary
conditions through the C ABI against the FP64 oracle of those BCs, whose own
pins tie it to brute-force matrices, the printed Toeplitz-plus-Hankel form
and library routines (Sec. 2.1, Sec. 4, Tables 1-2's comparators).

Tolerances (Frobenius-relative): FP64 1e-12 (1e-13 for the blur and the
eigenvalues); FP32 images with FP64 arithmetic: 2e-7 blur, 1e-6 transforms
and solve, 1e-5 one-step; FP32: 1e-6 blur, 5e-6 transforms, 2e-5 solve,
1e-5 one-step at a stable alpha (d <= 1/alpha)."""

import sys

import numpy as np
import pytest

import oracle as O
import oracle.bc_oracle as B
import synth
from tests.regions import region_errors

torch = pytest.importorskip("torch")
import paper_1211_0393_amd as P  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TDT = {"f32": torch.float32, "f32x": torch.float32, "f64": torch.float64}
NDT = {"f32": np.float32, "f32x": np.float32, "f64": np.float64}
TOL_BLUR = {"f32": 1e-6, "f32x": 2e-7, "f64": 1e-13}
TOL_T = {"f32": 5e-6, "f32x": 1e-6, "f64": 1e-12}
TOL_D = {"f32": 2e-5, "f32x": 1e-6, "f64": 1e-12}
TOL_IT = {"f32": 1e-5, "f32x": 1e-5, "f64": 1e-12}
DTS = ["f32", "f32x", "f64"]
BCS = ["reflective", "periodic"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, TDT[dt])


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def image(n1, n2, seed, dt):
    return synth.phantom(n1, n2, 5, 3, seed=seed).astype(NDT[dt]).astype(np.float64)


SHAPES = [(3, 3, 0, 0), (5, 4, 1, 1), (17, 33, 4, 7), (64, 64, 4, 4), (97, 130, 7, 5),
          (128, 96, 15, 15), (200, 157, 16, 20)]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n1,n2,q1,q2", SHAPES)
def test_blur_and_reblur(n1, n2, q1, q2, dt, bc):
    H = synth.psf_random(q1, q2, seed=7 * n1 + q2)
    X = image(n1, n2, n1 + n2, dt)
    with P.Plan(n1, n2, H, dtype=dt, bc=bc) as plan:
        x = dev(X, dt)
        y = torch.empty_like(x)
        plan.ar_blur_apply(x, y)
        e1 = rel(host(y), B.blur_bc(X, H, bc))
        plan.ar_blur_apply_T(x, y)
        e2 = rel(host(y), B.reblur_bc(X, H, bc))
    say(f"  {bc} {dt} {n1}x{n2} q=({q1},{q2}): A {e1:.2e}, A' {e2:.2e}")
    assert e1 <= TOL_BLUR[dt] and e2 <= TOL_BLUR[dt]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n1,n2,q1,q2", [(9, 10, 2, 3), (64, 64, 4, 4), (97, 130, 7, 5)])
def test_eigenvalues_and_filter(n1, n2, q1, q2, bc):
    H = synth.psf_random(q1, q2, seed=3 * n1)
    lam_ref = B.eigenvalues_bc(H, n1, n2, bc)
    if bc == "periodic":
        lam_ref = np.abs(lam_ref)
    with P.Plan(n1, n2, H, dtype="f64", bc=bc) as plan:
        lam = torch.empty((n1, n2), device=DEV, dtype=torch.float64)
        plan.ar_eigenvalues(lam)
        e = np.max(np.abs(host(lam) - lam_ref))
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, 0.05)
        d = torch.empty_like(lam)
        plan.ar_filter_values(d)
        ed = rel(host(d), B.tikhonov_bc(B.eigenvalues_bc(H, n1, n2, bc), 0.05))
    say(f"  {bc} {n1}x{n2}: lambda max abs {e:.2e}, d {ed:.2e}")
    assert e <= 1e-13 and ed <= 1e-13


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n1,n2", [(3, 3), (4, 7), (31, 64), (127, 100), (256, 255)])
def test_reflective_transform_pair(n1, n2, dt):
    X = image(n1, n2, 11, dt)
    with P.Plan(n1, n2, np.ones((1, 1)), dtype=dt, bc="reflective") as plan:
        x = dev(X, dt)
        c = torch.empty_like(x)
        plan.ar_transform(x, c)
        C = host(c)
        e1 = rel(C, B.dct_fwd(X))
        Cr = C.astype(NDT[dt]).astype(np.float64)
        y = torch.empty_like(x)
        plan.ar_transform_inv(dev(Cr, dt), y)
        e2 = rel(host(y), B.dct_inv(Cr))
    say(f"  reflective {dt} {n1}x{n2}: R^T {e1:.2e}, R {e2:.2e}")
    assert e1 <= TOL_T[dt] and e2 <= TOL_T[dt]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n1,n2,q1,q2,alpha", [(9, 10, 2, 3, 0.05), (64, 64, 4, 4, 0.1),
                                               (97, 130, 7, 5, 0.2), (255, 256, 7, 7, 0.2)])
def test_precond_solve(n1, n2, q1, q2, alpha, dt, bc):
    H = synth.psf_random(q1, q2, seed=5 * n2)
    Y = image(n1, n2, 2 * n1, dt)
    d = B.tikhonov_bc(B.eigenvalues_bc(H, n1, n2, bc), alpha)
    with P.Plan(n1, n2, H, dtype=dt, bc=bc) as plan:
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, alpha)
        y = dev(Y, dt)
        z = torch.empty_like(y)
        plan.ar_precond_solve(y, z)
        e = rel(host(z), B.precond_apply_bc(Y, d, bc))
        plan.ar_precond_solve(y, y)                        # in place
        e2 = rel(host(y), B.precond_apply_bc(Y, d, bc))
    say(f"  {bc} {dt} {n1}x{n2} alpha={alpha}: D y {e:.2e} (in place {e2:.2e})")
    assert e <= TOL_D[dt] and e2 <= TOL_D[dt]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("precondition", [True, False])
def test_iterate_one_step(dt, bc, precondition):
    n1, n2, alpha = 96, 80, 0.2
    H = synth.psf_gauss_shifted(4, 3, 2.0, 1.2, shift=(0.6, -0.4))
    F = image(n1, n2, 5, dt)
    E = synth.noise_field(n1, n2, seed=6)
    G = B.observe_bc(F, H, E, 0.01, bc).astype(NDT[dt]).astype(np.float64)
    d = B.tikhonov_bc(B.eigenvalues_bc(H, n1, n2, bc), alpha) if precondition else None
    with P.Plan(n1, n2, H, dtype=dt, bc=bc) as plan:
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, alpha)
        g = dev(G, dt)
        x = torch.zeros_like(g)
        X = np.zeros((n1, n2))
        for k in range(4):
            rc, res, _, _ = plan.ar_deblur_iterate(g, x, 1, precondition=precondition,
                                                   want_resnorm=True)
            assert rc == 0
            Xo, rn = B.landweber_step_bc(X, G, H, bc, d=d)
            Xg = host(x)
            e = rel(Xg, Xo)
            say(f"  {bc} {dt} D={'T' if precondition else 'I'} k={k}: {e:.2e}")
            assert e <= TOL_IT[dt]
            assert abs(res[0] - rn) <= (1e-12 if dt == "f64" else 1e-5) * rn
            X = Xg.astype(NDT[dt]).astype(np.float64)


@pytest.mark.parametrize("bc", BCS)
def test_trajectory_f64_and_scalars(bc):
    n1, n2, K, alpha = 64, 72, 15, 0.3
    H = synth.psf_gauss_shifted(4, 4, 2.0, 1.0, shift=(1.0, 1.0))
    F = synth.phantom(n1, n2, 6, 4, seed=101)
    E = synth.noise_field(n1, n2, seed=102)
    G = B.observe_bc(F, H, E, 0.01, bc)
    ref = B.iterate_bc(G, H, K, bc, alpha=alpha, F_true=F)
    with P.Plan(n1, n2, H, dtype="f64", bc=bc) as plan:
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, alpha)
        g, f = dev(G, "f64"), dev(F, "f64")
        x = torch.zeros_like(g)
        rc, res, rre, best = plan.ar_deblur_iterate(g, x, K, f_true=f, want_resnorm=True,
                                                    want_rre=True)
    assert rc == 0
    e = rel(host(x), ref["x"])
    say(f"  {bc} FP64 {K}-step trajectory: {e:.2e}, best it {best} (oracle {ref['best_it']})")
    assert e <= 1e-12
    assert np.max(np.abs(res - ref["resnorm"]) / ref["resnorm"]) <= 1e-12
    assert np.max(np.abs(rre - ref["rre"]) / ref["rre"]) <= 1e-12
    assert best == ref["best_it"]


@pytest.mark.parametrize("bc,dt", [("reflective", "f32"), ("periodic", "f32"),
                                   ("reflective", "f32x"), ("periodic", "f32x")])
def test_iterate_full_size_1024(bc, dt):
    """The 1024^2 motion-PSF workload under Reflective / Periodic BCs at the
    stable alpha 0.2: one-step parity at k = 0 and 5, whole image and per
    border region (Frobenius at the bar, largest pixel error within twice
    it)."""
    F, H, E, p = synth.workload("ar1024_f32_motion15")
    alpha = 0.2
    G = B.observe_bc(F, H, E, p["nu"], bc).astype(np.float32).astype(np.float64)
    d = B.tikhonov_bc(B.eigenvalues_bc(H, 1024, 1024, bc), alpha)
    with P.Plan(1024, 1024, H, dtype=dt, bc=bc) as plan:
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, alpha)
        g = dev(G, "f32")
        x = torch.zeros_like(g)
        done = 0
        for k in (0, 5):
            if k > done:
                plan.ar_deblur_iterate(g, x, k - done)
                done = k
            X = host(x)
            plan.ar_deblur_iterate(g, x, 1)
            done += 1
            Xo, _ = B.landweber_step_bc(X, G, H, bc, d=d)
            Xg = host(x)
            e = rel(Xg, Xo)
            say(f"  1024 {bc} {dt} k={k}: {e:.2e}")
            assert e <= 1e-5
            for name, (fr, mx) in region_errors(Xg, Xo).items():
                say(f"    {name}: frobenius {fr:.2e}, max-abs {mx:.2e}")
                assert fr <= 1e-5 and mx <= 2e-5, name


@pytest.mark.parametrize("dt", DTS)
def test_reflective_tikhonov_solve(dt):
    n1, n2, alpha = 130, 97, 5e-3
    S = O.symmetrize(synth.psf_random(5, 4, seed=9))
    G = image(n1, n2, 12, dt)
    ref = B.tikhonov_solve(G, S, alpha, bc="reflective")
    with P.Plan(n1, n2, S, dtype=dt, bc="reflective") as plan:
        g = dev(G, dt)
        x = torch.empty_like(g)
        plan.ar_tikhonov_solve(g, x, alpha)
        e = rel(host(x), ref)
    say(f"  reflective direct solve {dt}: {e:.2e}")
    assert e <= {"f64": 1e-12, "f32x": 1e-6, "f32": 1e-5}[dt]


def test_unsupported_requests_are_refused():
    H = synth.psf_random(2, 2, seed=1)
    with P.Plan(32, 32, H, dtype="f32", bc="periodic") as plan:
        x = torch.zeros((32, 32), device=DEV, dtype=torch.float32)
        y = torch.empty_like(x)
        for call in (lambda: plan.ar_transform(x, y), lambda: plan.ar_transform_inv(x, y),
                     lambda: plan.ar_blur_apply_T(x, y, tmode=P.AR_ADJOINT),
                     lambda: plan.ar_tikhonov_solve(x, y, 0.1),
                     lambda: plan.ar_deblur_iterate(x, y, 1, tmode=P.AR_ADJOINT),
                     lambda: plan.ar_plan_autotune(),
                     lambda: P.Batch([plan])):
            with pytest.raises(P.ArError) as ei:
                call()
            assert ei.value.status == -8
    with pytest.raises(P.ArError) as ei:
        P.Plan(32, 32, H, dtype="bf16x3", bc="reflective")
    assert ei.value.status == -8
