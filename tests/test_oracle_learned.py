"""Pins of the learned-filter oracle (CPU only).

Each definition of oracle.learned is checked against something other than
itself: brute-force loops over small grids, closed forms, statistical laws
with known constants, and central finite differences for the gradient."""

import numpy as np
import pytest

import oracle as O
import synth

L = O.learned


def test_radial_rho_bruteforce():
    """rho(k1, k2) written out point by point from the grid of Theorem 2."""
    n1, n2 = 7, 10
    rho = L.radial_rho(n1, n2)
    for k1 in range(n1):
        x1 = 0.0 if k1 in (0, n1 - 1) else k1 / (n1 - 1)
        for k2 in range(n2):
            x2 = 0.0 if k2 in (0, n2 - 1) else k2 / (n2 - 1)
            assert abs(rho[k1, k2] - ((x1 * x1 + x2 * x2) / 2.0) ** 0.5) < 1e-15
    assert rho.max() < 1.0 and rho.min() == 0.0


def test_radial_bins_exact_at_edges():
    """Bins from exact rational arithmetic (Fraction) on a grid that hits
    bin edges exactly (n - 1 = 128: x / pi = k / 64 on the diagonal)."""
    from fractions import Fraction
    from math import isqrt
    n = 129
    b = L.radial_bins(n, n)
    for k1 in list(range(0, n, 7)) + [2, 4, 64, 126, 127, 128]:
        for k2 in list(range(0, n, 5)) + [2, 4, 64, 127, 128]:
            r1 = 0 if k1 in (0, n - 1) else k1
            r2 = 0 if k2 in (0, n - 1) else k2
            v = 2048 * (Fraction(r1, n - 1) ** 2 + Fraction(r2, n - 1) ** 2)
            want = min(isqrt(v.numerator // v.denominator), 63)
            assert b[k1, k2] == want, (k1, k2)
    assert b[2, 2] == 1 and b[64, 64] == 32
    # away from edges the exact rule agrees with floor(64 rho) in floating point
    rho = L.radial_rho(57, 91)
    fl = np.minimum(np.floor(64 * rho), 63).astype(int)
    assert np.mean(fl == L.radial_bins(57, 91)) > 0.999


def test_radial_profile_bruteforce_and_constants():
    rng = np.random.default_rng(3)
    n1, n2 = 40, 33
    V = rng.standard_normal((n1, n2))
    prof = L.radial_profile(V)
    bins = L.radial_bins(n1, n2)
    for b in range(L.NB):
        vals = [V[i, j] for i in range(n1) for j in range(n2) if bins[i, j] == b]
        want = sum(vals) / len(vals) if vals else 0.0
        assert abs(prof[b] - want) <= 1e-14 * (1 + abs(want))
    # a constant field gives that constant in every non-empty bin
    prof = L.radial_profile(np.full((300, 300), 2.5))
    assert np.all(prof == 2.5)
    # a tiny grid leaves empty bins at 0
    prof = L.radial_profile(np.ones((4, 4)))
    assert prof[0] == 1.0 and np.any(prof == 0.0)


def test_eigenvalue_profile_starts_at_one():
    """lambda(0, 0) = sum h = 1 and the four corner coefficients share x = 0,
    so bin 0 averages 1 with the smallest interior frequencies."""
    H = synth.psf_gauss_shifted(3, 3, 1.0, 1.0, shift=(0, 0))
    lam = O.eigenvalues(H, 256, 256)
    prof = L.radial_profile(lam)
    assert 0.98 < prof[0] <= 1.0
    assert prof[-1] < prof[0]


def test_lower_median_bruteforce():
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 10, 11, 100):
        v = rng.standard_normal(n)
        assert L.lower_median(v) == sorted(v)[(n - 1) // 2]


def test_laplacian_of_quadratic():
    """The 5-point Laplacian is exact on quadratics: 2a + 2c for
    a i^2 + b i j + c j^2 + linear terms."""
    i, j = np.meshgrid(np.arange(20.0), np.arange(17.0), indexing="ij")
    G = 0.5 * i * i - 0.3 * i * j + 1.25 * j * j + 2 * i - j + 4
    Lg = L.laplacian(G)
    assert Lg.shape == (18, 15)
    assert np.allclose(Lg, 2 * 0.5 + 2 * 1.25, atol=1e-10)


def test_noise_estimate_on_white_noise():
    """For g = c + sigma e (e iid N(0,1)) the Laplacian is a sum of 5 noise
    samples with variance 20 sigma^2, MAD / 0.6745 estimates its standard
    deviation, and nu_hat = sigma sqrt(N) / ||g|| (law of large numbers,
    a few percent at 512^2)."""
    rng = np.random.default_rng(11)
    n = 512
    for sigma in (0.01, 0.05):
        G = 1.0 + sigma * rng.standard_normal((n, n))
        want = sigma * n / np.linalg.norm(G)
        got = L.noise_estimate(G)
        assert abs(got / want - 1.0) < 0.03, (got, want)


def test_noise_estimate_tracks_observation_level():
    """On a blurred phantom with the repository's observation model the
    estimate grows with nu (a monotone, roughly proportional response)."""
    F = synth.phantom(256, 256, 10, 5, seed=1)
    H = synth.psf_gauss_shifted(4, 4, 1.5, 1.5, shift=(0, 0))
    E = synth.noise_field(256, 256, seed=2)
    est = [L.noise_estimate(O.observe(F, H, E, nu)) for nu in (0.005, 0.01, 0.02)]
    assert est[0] < est[1] < est[2]
    assert 1.5 < est[2] / est[1] < 2.5


def test_ebins_and_edges():
    e = L.ebin_edges()
    assert e.size == 63 and np.all(np.diff(e) > 0)
    assert abs(e[15] - 1e-3) < 1e-18 and abs(e[47] - 0.1) < 1e-16
    lam = np.array([0.0, 5e-5, 1e-4, 1.0001e-4 * 10 ** (1 / 16), 1e-3, -0.5, 1.0])
    b = L.ebins(lam)
    assert list(b[:3]) == [0, 0, 0] and b[3] == 1 and b[4] == 16
    assert b[5] == int(np.floor(16 * (4 + np.log10(0.5)))) and b[6] == 63
    c = L.ebin_centres()
    assert np.all(L.ebins(c) == np.arange(64))


def test_gains_filter_reproduces_plain_filters():
    """Constant gains give eq. (TikFilter) exactly; the labels of the plain
    filters reproduce them at every bin centre (within the clip range)."""
    H = synth.psf_gauss_shifted(2, 3, 1.2, 0.8, shift=(0.2, 0.1))
    lam = O.eigenvalues(H, 30, 40)
    for alpha in (1e-4, 3e-3, 0.1):
        g = np.full(L.NB, (np.log10(alpha) + 6) / 6)
        assert np.allclose(L.gains_filter(lam, g), O.tikhonov(lam, alpha), rtol=1e-12)
        assert np.allclose(L.gains_label("tikhonov", alpha), g, rtol=1e-14)
    c = L.ebin_centres()
    for t in (1e-3, 0.05, 0.3):
        g = L.gains_label("threshold", t)
        d = L.gains_filter(c, g)
        want = O.threshold_filter(c, t)
        big = c >= t
        # above t: a = 0 clipped to 1e-6, d = 1 / (c^2 + 1e-6)
        assert np.allclose(d[big], 1.0 / (c[big] ** 2 + 1e-6), rtol=1e-12)
        assert np.allclose(d[~big], want[~big], rtol=1e-12)
        assert np.all((g >= 0) & (g <= 1))


def test_bf16_round():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159265, 0.0])
    r = L.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie, to even
    assert r[2] == 1.0 + 2 ** -7             # above the tie
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12
    assert r[5] == 0.0


def _theta(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for (o, i) in L.SIZES:
        parts.append(rng.standard_normal(o * i) * np.sqrt(2.0 / i))
        parts.append(rng.standard_normal(o) * 0.1)
    return np.concatenate(parts)


def test_mlp_shapes_and_param_count():
    assert L.NPARAM == 33216
    th = _theta(0)
    Y, _ = L.mlp_forward(th, np.random.default_rng(1).standard_normal((5, 65)))
    assert Y.shape == (5, 64) and np.all((Y > 0) & (Y < 1))


def test_mlp_gradient_finite_differences():
    """Backpropagation against central differences on 60 random coordinates
    spread over every layer (relative error <= 1e-6)."""
    rng = np.random.default_rng(2)
    th = _theta(1)
    X = rng.standard_normal((7, 65))
    T = rng.uniform(0, 1, (7, 64))
    loss, g = L.mlp_loss_grad(th, X, T)
    h = 1e-6
    idx = rng.choice(L.NPARAM, 60, replace=False)
    for k in idx:
        e = np.zeros(L.NPARAM)
        e[k] = h
        fd = (L.mlp_loss_grad(th + e, X, T)[0] - L.mlp_loss_grad(th - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-11, (k, fd, g[k])


def test_mlp_loss_value():
    """Loss is the mean of squared errors: zero at the network's own output."""
    th = _theta(3)
    X = np.random.default_rng(4).standard_normal((3, 65))
    Y, _ = L.mlp_forward(th, X)
    loss, g = L.mlp_loss_grad(th, X, Y)
    assert loss == 0.0 and np.all(g == 0.0)


def test_adam_first_step_is_sign_step():
    """With zero moments the bias-corrected first Adam step is
    -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = L.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _set(theta, layer, kind, idx, value):
    """Write one weight (kind "W", idx (out, in)) or bias (kind "b", idx out)
    of a layer into the flat parameter vector at the offsets the stated
    layout gives: W1 (128 x 65), b1, W2 (128 x 128), b2, W3 (64 x 128), b3,
    each W (out, in) row-major."""
    off = 0
    for li, (no, ni) in enumerate(L.SIZES):
        if li == layer:
            if kind == "W":
                o, i = idx
                theta[off + o * ni + i] = value
            else:
                theta[off + no * ni + idx] = value
            return
        off += no * ni + no
    raise IndexError(layer)


def _forward_loops(theta, x):
    """The network written out with scalar loops over the (out, in) layout
    (ReLU, ReLU, logistic sigmoid), independent of the oracle's matrix code."""
    out = list(x)
    off = 0
    for li, (no, ni) in enumerate(L.SIZES):
        nxt = []
        for o in range(no):
            acc = theta[off + no * ni + o]
            for i in range(ni):
                acc += theta[off + o * ni + i] * out[i]
            if li < 2:
                nxt.append(acc if acc > 0.0 else 0.0)
            else:
                nxt.append(1.0 / (1.0 + np.exp(-acc)))
        off += no * ni + no
        out = nxt
    return np.array(out)


def test_mlp_forward_hand_network_literal_values():
    """A network with a handful of nonzero parameters, evaluated by hand:
    z1_0 = 2*1 - 0.25 + 0.5 = 2.25, z1_1 = 2 - 1 = 1, z1_2 = -1 (ReLU 0);
    z2_0 = 1.5*2.25 + 0.5*1 = 3.875, z2_1 = -2.25 + 0.25 = -2 (ReLU 0);
    z3_0 = 3.875 - 0.5 = 3.375, z3_3 = -0.5*3.875 = -1.9375, z3_5 = 1, all
    other z3 = 0.  A transposed weight matrix, a dropped bias or a missing
    ReLU changes at least one of these outputs."""
    th = np.zeros(L.NPARAM)
    _set(th, 0, "W", (0, 0), 2.0)
    _set(th, 0, "W", (0, 1), -1.0)
    _set(th, 0, "b", 0, 0.5)
    _set(th, 0, "W", (1, 2), 1.0)
    _set(th, 0, "b", 1, -1.0)
    _set(th, 0, "W", (2, 0), -1.0)
    _set(th, 1, "W", (0, 0), 1.5)
    _set(th, 1, "W", (0, 1), 0.5)
    _set(th, 1, "W", (1, 0), -1.0)
    _set(th, 1, "b", 1, 0.25)
    _set(th, 2, "W", (0, 0), 1.0)
    _set(th, 2, "W", (0, 1), -2.0)
    _set(th, 2, "b", 0, -0.5)
    _set(th, 2, "W", (3, 0), -0.5)
    _set(th, 2, "b", 5, 1.0)
    x = np.zeros(65)
    x[0], x[1], x[2] = 1.0, 0.25, 2.0
    Y, (_, Z1, H1, Z2, H2, Z3) = L.mlp_forward(th, x[None, :])
    assert Z1[0, 0] == 2.25 and Z1[0, 1] == 1.0 and Z1[0, 2] == -1.0 and H1[0, 2] == 0.0
    assert Z2[0, 0] == 3.875 and Z2[0, 1] == -2.0 and H2[0, 1] == 0.0
    expect = np.full(64, 0.5)
    expect[0] = 1.0 / (1.0 + np.exp(-3.375))       # 0.96691402...
    expect[3] = 1.0 / (1.0 + np.exp(1.9375))       # 0.125923...
    expect[5] = 1.0 / (1.0 + np.exp(-1.0))         # 0.731058...
    assert abs(expect[0] - 0.9669140216) < 1e-9
    assert abs(expect[3] - 0.1259228) < 1e-6
    assert abs(expect[5] - 0.7310585786) < 1e-9
    assert np.allclose(Y[0], expect, rtol=0, atol=1e-15)


def test_mlp_forward_matches_scalar_loops():
    """Random sparse network: the oracle's forward pass equals a scalar-loop
    evaluation over the stated (out, in) layout."""
    rng = np.random.default_rng(11)
    th = _theta(5) * (rng.uniform(size=L.NPARAM) < 0.2)
    X = rng.standard_normal((3, 65))
    Y, _ = L.mlp_forward(th, X)
    for b in range(3):
        ref = _forward_loops(th, X[b])
        assert np.max(np.abs(Y[b] - ref)) < 1e-12


def test_adam_three_steps_hand_computed():
    """Three Adam steps on one parameter with gradients 1, -2, 0.5 (lr 0.1,
    beta1 0.9, beta2 0.999, eps 1e-8), moments worked out by hand:
    m = 0.1, -0.11, -0.049 and v = 0.001, 0.004999, 0.005244001; the
    bias-corrected step divides m by 1 - 0.9^t and v by 1 - 0.999^t.  A
    moment that is not carried across steps, or a bias correction with the
    wrong power, fails."""
    grads = [1.0, -2.0, 0.5]
    m_hand = [0.1, -0.11, -0.049]
    v_hand = [0.001, 0.004999, 0.005244001]
    th = np.array([0.7])
    m = np.zeros(1)
    v = np.zeros(1)
    th_hand = 0.7
    for t, (g, mh, vh) in enumerate(zip(grads, m_hand, v_hand), start=1):
        th, m, v = L.adam_step(th, m, v, np.array([g]), t, 0.1)
        assert abs(m[0] - mh) < 1e-15 and abs(v[0] - vh) < 1e-15, (t, m, v)
        th_hand -= 0.1 * (mh / (1.0 - 0.9 ** t)) / (np.sqrt(vh / (1.0 - 0.999 ** t)) + 1e-8)
        assert abs(th[0] - th_hand) < 1e-14, (t, th, th_hand)
    # step 1 moves by lr (sign step); step 2's bias-corrected m is -0.11/0.19
    assert abs(th_hand - (0.7 - 0.1 / (1 + 1e-8)
                          + 0.1 * (0.11 / 0.19) / (np.sqrt(0.004999 / 0.001999) + 1e-8)
                          + 0.1 * (0.049 / 0.271) / (np.sqrt(0.005244001 / 0.002997001) + 1e-8))) < 1e-14


def test_sweep_label_prefers_best_run():
    """The sweep returns the candidate whose own run has the smallest RRE,
    checked against running each candidate separately, and that candidate's
    label."""
    n = 24
    F = synth.phantom(n, n, 3, 2, seed=9)
    H = synth.psf_gauss_shifted(2, 2, 1.0, 1.0, shift=(0.3, 0.0))
    E = synth.noise_field(n, n, seed=10)
    G = O.observe(F, H, E, 0.01)
    alphas, ts = [1e-2, 1e-1], [0.05, 0.2]
    kind, prm, e, lab = L.sweep_label(G, H, F, alphas, ts, 8)
    lam = O.eigenvalues(H, n, n)
    runs = {("tikhonov", a): O.tikhonov(lam, a) for a in alphas}
    runs.update({("threshold", t): O.threshold_filter(lam, t) for t in ts})
    errs = {k: O.iterate(G, H, 8, d=d, F_true=F)["rre"].min() for k, d in runs.items()}
    assert e == min(errs.values()) and errs[(kind, prm)] == e
    assert np.array_equal(lab, L.gains_label(kind, prm))
