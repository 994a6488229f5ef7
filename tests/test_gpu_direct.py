"""Direct Tikhonov restoration for strongly symmetric PSFs through the C ABI
(x = T diag(lambda / (lambda^2 + alpha)) T~ g, Theorems 1-2 with eq.
(TikFilter)) against the FP64 oracle's solve, which its own pins tie to
numpy's dense solver on the brute-force AR matrix."""

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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def sym_psf(q1, q2, seed):
    return O.symmetrize(synth.psf_random(q1, q2, seed))


# FP64: 1e-12; FP32 images with FP64 arithmetic: 1e-6 (two FP32 roundings of
# the coefficients between the passes; the filter is <= 1/(2 sqrt(alpha)));
# FP32: 1e-5.
TOL = {"f64": 1e-12, "f32x": 1e-6, "f32": 1e-5}


@pytest.mark.parametrize("dt", ["f64", "f32x", "f32"])
@pytest.mark.parametrize("n1,n2,q1,q2,alpha", [(3, 3, 0, 0, 0.1), (9, 10, 2, 3, 1e-2),
                                               (64, 64, 4, 4, 1e-2), (130, 97, 7, 5, 1e-3),
                                               (256, 200, 10, 3, 5e-3)])
def test_tikhonov_solve_matches_oracle(n1, n2, q1, q2, alpha, dt):
    S = sym_psf(q1, q2, 10 * n1 + n2)
    G = synth.phantom(n1, n2, 5, 3, seed=n1).astype(NDT[dt]).astype(np.float64)
    ref = B.tikhonov_solve(G, S, alpha)
    with P.Plan(n1, n2, S, dtype=dt) as plan:
        g = torch.from_numpy(G).to(DEV, TDT[dt])
        x = torch.empty_like(g)
        plan.ar_tikhonov_solve(g, x, alpha)
        e = rel(host(x), ref)
        plan.ar_tikhonov_solve(g, g, alpha)               # in place
        e2 = rel(host(g), ref)
    say(f"  {n1}x{n2} q=({q1},{q2}) alpha={alpha} {dt}: {e:.2e} (in place {e2:.2e})")
    assert e <= TOL[dt] and e2 <= TOL[dt]


@pytest.mark.parametrize("dt", ["f32x", "f32"])
def test_tikhonov_solve_1024(dt):
    """1024^2 phantom blurred by a strongly symmetric 15x15 PSF (the
    4-fold symmetrization of the motion PSF) with 0.5% noise: the solve
    against the oracle over the whole image and per border region."""
    F, H, E, p = synth.workload("ar1024_f32_motion15")
    S = O.symmetrize(H)
    G = O.observe(F, S, E, p["nu"]).astype(np.float32).astype(np.float64)
    alpha = 5e-3
    ref = B.tikhonov_solve(G, S, alpha)
    with P.Plan(1024, 1024, S, dtype=dt) as plan:
        g = torch.from_numpy(G).to(DEV, torch.float32)
        x = torch.empty_like(g)
        plan.ar_tikhonov_solve(g, x, alpha)
        X = host(x)
    e = rel(X, ref)
    say(f"  1024 {dt}: {e:.2e}, RRE {rel(X, F):.4f} (oracle {rel(ref, F):.4f})")
    assert e <= 1e-5
    for name, (fr, mx) in region_errors(X, ref).items():
        say(f"    {name}: frobenius {fr:.2e}, max-abs {mx:.2e}")
        assert fr <= 1e-5 and mx <= 1e-5, name


def test_tikhonov_solve_rejects_nonsymmetric_and_bad_alpha():
    H = synth.psf_motion(3)
    with P.Plan(32, 32, H, dtype="f64") as plan:
        g = torch.zeros((32, 32), device=DEV, dtype=torch.float64)
        with pytest.raises(P.ArError) as ei:
            plan.ar_tikhonov_solve(g, g, 0.1)
        assert ei.value.status == -3
        # a strongly symmetric PSF set later is accepted
        plan.ar_plan_set_psf(O.symmetrize(H))
        plan.ar_tikhonov_solve(g, g, 0.1)
        for bad in (0.0, -1.0, float("nan")):
            with pytest.raises(P.ArError) as ei:
                plan.ar_tikhonov_solve(g, g, bad)
            assert ei.value.status == -1
