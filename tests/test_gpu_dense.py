"""The BF16x3 dense-transform precision variant (AR_F32_BF16X3) against the
FP64 oracle.

Each transform pass is one GEMM with operands split into two BF16 terms
and the lo*lo product dropped: ~2^-17 relative error per product, FP32
accumulation over m terms; measured errors are printed and held to
2e-5 per 2-D transform (forward or inverse) and 1e-4 for the
preconditioner solve; one D-Landweber step at the 2048^2 workload is
reported against the FP32 and FP64-arithmetic plans (see that test).
"""

import sys

import numpy as np
import pytest

import oracle as O
import synth
from tests.regions import region_errors

torch = pytest.importorskip("torch")
import paper_1211_0393_amd as P  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=torch.float32)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n1,n2", [(3, 3), (16, 16), (64, 64), (130, 97), (129, 300),
                                   (500, 260), (1024, 1024), (2048, 2048)])
def test_dense_transform_pair(n1, n2):
    say(f"dense transform n=({n1},{n2})")
    rng = np.random.default_rng(n1 + 5 * n2)
    X = rng.standard_normal((n1, n2)).astype(np.float32).astype(np.float64)
    with P.Plan(n1, n2, np.ones((1, 1)), dtype="bf16x3") as plan:
        x = dev(X)
        c = torch.empty_like(x)
        plan.ar_transform(x, c)
        Cg = host(c)
        e = rel(Cg, O.ar_fwd(X))
        say(f"  fwd rel err {e:.2e}")
        assert e <= 2e-5
        Cq = Cg.astype(np.float32).astype(np.float64)
        xr = torch.empty_like(x)
        plan.ar_transform_inv(dev(Cq), xr)
        e = rel(host(xr), O.ar_inv(Cq))
        say(f"  inv rel err {e:.2e}")
        assert e <= 2e-5
        # in place equals out of place
        y = dev(X)
        plan.ar_transform(y, y)
        assert np.array_equal(host(y), Cg)


@pytest.mark.parametrize("n,q,alpha", [(64, 4, 1e-2), (300, 7, 5e-3), (2048, 15, 5e-3)])
def test_dense_precond_solve(n, q, alpha):
    H = synth.psf_tail(q, 4.0, 2.0)
    Y = np.random.default_rng(n).standard_normal((n, n)).astype(np.float32).astype(np.float64)
    d = O.tikhonov(O.eigenvalues(H, n, n), alpha)
    with P.Plan(n, n, H, dtype="bf16x3") as plan:
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, alpha)
        y = dev(Y)
        z = torch.empty_like(y)
        plan.ar_precond_solve(y, z)
        e = rel(host(z), O.precond_apply(Y, d))
    say(f"  solve n={n} rel err {e:.2e}")
    assert e <= 1e-4


def test_dense_iterate_small_trajectory():
    """64^2, 10 iterations: per-iterate drift against the oracle."""
    F, H, E, p = synth.workload("ar64_f64_gauss9")
    F = F.astype(np.float32).astype(np.float64)
    G = O.observe(F, H, E, p["nu"]).astype(np.float32).astype(np.float64)
    K = 10
    with P.Plan(64, 64, H, dtype="bf16x3") as plan:
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, 0.1)
        ref = O.iterate(G, H, K, alpha=0.1, F_true=F)
        g, f = dev(G), dev(F)
        x = torch.zeros_like(g)
        rc, res, rre, best = plan.ar_deblur_iterate(g, x, K, f_true=f, want_resnorm=True,
                                                    want_rre=True)
        assert rc == 0
        e = rel(host(x), ref["x"])
        say(f"  drift after {K}: {e:.2e}")
        assert e <= 2e-4
        assert np.max(np.abs(rre - ref["rre"]) / ref["rre"]) <= 2e-4
        assert best == ref["best_it"]


@pytest.mark.timeout(600)
def test_dense_one_step_2048_tail31():
    """The 2048^2 precision workload (31x31 one-sided exponential tail,
    alpha 5e-3, 1% noise): one D-Landweber step from 0 against the oracle's
    step, for the BF16x3 dense transforms and for the FP32 and
    FP64-arithmetic FFT plans on the same FP32 data.  d reaches 1/alpha =
    200 on the many near-zero eigenvalues of this PSF, so every rounding in
    front of D is amplified, most of all the forward transform's: measured
    4.5e-6 (FP64 arithmetic), 6.2e-5 (FP32 FFT, ~1e-6 per pass) and
    6.7e-4 (BF16x3 GEMM, ~1e-5 per pass: the dropped lo*lo term and the
    BF16 rounding of lo, ~2^-17 per product).  Held to 1e-5, 1e-4 and
    2e-3."""
    F, H, E, p = synth.workload("ar2048_f32_tail31")
    say("  2048 oracle: observation")
    G = O.observe(F, H, E, p["nu"]).astype(np.float32).astype(np.float64)
    d = O.tikhonov(O.eigenvalues(H, 2048, 2048), p["alpha"])
    # the oracle's step from x_0 = 0 (tau = 1): g - A 0 = g, so x_1 = D A' g
    say("  2048 oracle: x_1 = D A' g")
    X1o = O.precond_apply(O.reblur(G, H), d)
    errs = {}
    tol = {"f32x": 1e-5, "f32": 1e-4, "bf16x3": 2e-3}
    for dt in ("f32x", "f32", "bf16x3"):
        with P.Plan(2048, 2048, H, dtype=dt) as plan:
            plan.ar_precond_set(P.AR_FILTER_TIKHONOV, p["alpha"])
            g = dev(G)
            x = torch.zeros_like(g)
            plan.ar_deblur_iterate(g, x, 1)
            Xg = host(x)
            errs[dt] = rel(Xg, X1o)
        say(f"  2048 one-step rel err at k=0, {dt}: {errs[dt]:.2e}")
        # per region: Frobenius within the bound; the largest single-pixel
        # error (over max |x|) within four times it (over 4 * 10^6 pixels the
        # maximum of the rounding field sits ~3x above its Frobenius mean,
        # measured); an error confined to the border would show as a border
        # region above the interior
        for name, (fr, mx) in region_errors(Xg, X1o).items():
            say(f"    {name}: frobenius {fr:.2e}, max-abs {mx:.2e}")
            assert fr <= tol[dt] and mx <= 4 * tol[dt], (dt, name)
    for dt, t in tol.items():
        assert errs[dt] <= t, dt
