"""Pins of the FP64 oracle against brute force, the paper's closed forms,
its worked example, its theorems and library routines (CPU only)."""

import os

import numpy as np
import pytest
from scipy import fft as sfft

import oracle as O
import synth
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def dense_of(op, n1, n2):
    """Matrix of a linear image map, column by column."""
    A = np.zeros((n1 * n2, n1 * n2))
    for j in range(n1 * n2):
        e = np.zeros(n1 * n2)
        e[j] = 1.0
        A[:, j] = op(e.reshape(n1, n2)).ravel()
    return A


def strongly_symmetric(q1, q2, seed):
    return O.symmetrize(synth.psf_random(q1, q2, seed))


SHAPES = [(3, 3, 0, 0), (5, 4, 1, 1), (6, 7, 2, 3), (8, 8, 3, 2), (9, 10, 4, 4), (7, 11, 4, 0), (12, 5, 0, 2)]


# ---------------------------------------------------------------- the blur A_n

@pytest.mark.parametrize("n1,n2,q1,q2", SHAPES)
def test_blur_matches_pixelwise_ghost_formulas(n1, n2, q1, q2):
    """A_n from the tensor extension == A_n built entry by entry from the
    edge and corner formulas of Sec. 2.2 (brute force)."""
    H = synth.psf_random(q1, q2, seed=n1 * 100 + n2)
    A_b = brute.dense_blur(H, n1, n2)
    A_o = dense_of(lambda X: O.blur(X, H), n1, n2)
    assert np.max(np.abs(A_o - A_b)) < 1e-15


@pytest.mark.parametrize("n,q", [(3, 0), (4, 1), (7, 3), (9, 2), (12, 6), (16, 13)])
def test_blur_1d_closed_form(n, q):
    """Rows blurred by a one-row PSF follow eq. (ARnosym1D) exactly."""
    rng = np.random.default_rng(n + 7 * q)
    hv = rng.uniform(0, 1, 2 * q + 1)
    hv /= hv.sum()
    A1 = brute.ar1d_closed(hv, n)
    X = rng.standard_normal((3, n))
    Y = O.blur(X, hv.reshape(1, -1))
    assert np.max(np.abs(Y - X @ A1.T)) < 1e-14
    # the column direction uses the same closed form
    Yc = O.blur(X.T, hv.reshape(-1, 1))
    assert np.max(np.abs(Yc - A1 @ X.T)) < 1e-14


def _golden_pattern():
    rows = []
    with open(os.path.join(GOLDEN, "ar1d_pattern_q3_n7.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_blur_1d_worked_example_q3():
    """The 7x7 symbolic pattern printed in the proof of Theorem 3 (q = 3),
    evaluated at a random mask, equals the oracle's 1-D AR matrix."""
    rng = np.random.default_rng(3)
    hv = rng.uniform(0, 1, 7)
    hv /= hv.sum()
    h = lambda k: hv[3 + k]  # noqa: E731
    pts = {}
    for i in range(4):
        pts[f"t{i}x"], pts[f"t{i}y"] = h(-i), h(i)
        pts[f"w{i}x"] = h(-i) + 2 * sum(h(-j) for j in range(i + 1, 4))
        pts[f"w{i}y"] = h(i) + 2 * sum(h(j) for j in range(i + 1, 4))
        pts[f"v{i}x"], pts[f"v{i}y"] = h(-i) - h(i), h(i) - h(-i)
    pts["t0"] = h(0)
    pts["z0x"], pts["z0y"] = h(0) - h(-2), h(0) - h(2)
    pts["z1x"], pts["z1y"] = h(-1) - h(-3), h(1) - h(3)
    pts["z2x"], pts["z2y"] = h(-1) - h(3), h(1) - h(-3)
    pts["."] = 0.0
    P = np.array([[pts[t] for t in row] for row in _golden_pattern()])
    assert P.shape == (7, 7)
    X = np.eye(7)
    A_o = O.blur(X, hv.reshape(1, -1)).T      # row i of X = e_i, so column i of A
    assert np.max(np.abs(A_o - P)) < 1e-15


@pytest.mark.parametrize("n1,n2,q1,q2", [(5, 6, 1, 2), (8, 7, 3, 2), (9, 9, 2, 4), (6, 10, 3, 0)])
def test_blur_2d_block_form(n1, n2, q1, q2):
    """Eqs. (2d_form)/(2d_form_block): block structure with 1-D AR blocks
    of the PSF rows equals the oracle's A_n."""
    H = synth.psf_random(q1, q2, seed=q1 * 10 + q2)
    A_c = brute.ar2d_closed(H, n1, n2)
    A_o = dense_of(lambda X: O.blur(X, H), n1, n2)
    assert np.max(np.abs(A_c - A_o)) < 1e-14


def test_blur_separable_kronecker():
    """For h = a (x) b the 2-D AR matrix is A(a) (x) A(b) (tensor BCs)."""
    rng = np.random.default_rng(11)
    a = rng.uniform(0, 1, 5)
    b = rng.uniform(0, 1, 7)
    a /= a.sum()
    b /= b.sum()
    n1, n2 = 8, 9
    A = dense_of(lambda X: O.blur(X, np.outer(a, b)), n1, n2)
    K = np.kron(brute.ar1d_closed(a, n1), brute.ar1d_closed(b, n2))
    assert np.max(np.abs(A - K)) < 1e-15


def test_blur_is_not_correlation():
    """eq. (modello_discreto) is a convolution: a mask with all weight at
    h_{+1,0} copies the pixel above (f_{i-s}, s = (1, 0))."""
    H = np.zeros((3, 3))
    H[2, 1] = 1.0                       # h_{1,0}
    X = np.arange(30.0).reshape(5, 6)
    Y = O.blur(X, H)
    assert np.array_equal(Y[1:], X[:-1])
    assert np.array_equal(Y[0], 2 * X[0] - X[1])    # f_0 = 2 f_1 - f_2


# ---------------------------------------------------------------- transposes

@pytest.mark.parametrize("n1,n2,q1,q2", SHAPES)
def test_adjoint_is_brute_transpose(n1, n2, q1, q2):
    H = synth.psf_random(q1, q2, seed=5 + n1)
    A_b = brute.dense_blur(H, n1, n2)
    AT = dense_of(lambda R: O.blur_adjoint(R, H), n1, n2)
    assert np.max(np.abs(AT - A_b.T)) < 1e-14


def test_adjoint_dot_product_large():
    rng = np.random.default_rng(9)
    H = synth.psf_motion(7)
    X = rng.standard_normal((70, 83))
    R = rng.standard_normal((70, 83))
    lhs = np.sum(O.blur(X, H) * R)
    rhs = np.sum(X * O.blur_adjoint(R, H))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(X) * np.linalg.norm(R)


def test_reblur_is_rot180_blur_and_differs_from_transpose():
    """A' = A(rot180 h) (Sec. 4); A' != A^T for AR BCs even when h is
    strongly symmetric, A' = A in that case."""
    n1, n2 = 8, 9
    H = synth.psf_random(2, 3, seed=4)
    A_rot = brute.dense_blur(H[::-1, ::-1], n1, n2)
    Ap = dense_of(lambda R: O.reblur(R, H), n1, n2)
    assert np.max(np.abs(Ap - A_rot)) < 1e-15
    S = strongly_symmetric(2, 3, 4)
    A_s = brute.dense_blur(S, n1, n2)
    assert np.max(np.abs(dense_of(lambda R: O.reblur(R, S), n1, n2) - A_s)) < 1e-15
    assert np.max(np.abs(A_s.T - A_s)) > 1e-3


# ---------------------------------------------------------------- Theorem 4

@pytest.mark.parametrize("n1,n2,q1,q2", [(7, 8, 2, 1), (9, 9, 3, 3), (8, 10, 1, 4)])
def test_symmetrization_is_least_squares_optimal(n1, n2, q1, q2):
    """Theorem 4: over all strongly symmetric masks s, ||A(h) - P(s)||_F is
    minimised by the 4-fold average; solved here by brute-force least
    squares over a basis of strongly symmetric masks."""
    H = synth.psf_random(q1, q2, seed=77 + n1)
    A = brute.dense_blur(H, n1, n2).ravel()
    cols, keys = [], []
    for a in range(q1 + 1):
        for b in range(q2 + 1):
            B = np.zeros_like(H)
            for sa in {a, -a}:
                for sb in {b, -b}:
                    B[q1 + sa, q2 + sb] = 1.0
            cols.append(brute.dense_blur(B, n1, n2).ravel())
            keys.append((a, b))
    coef, *_ = np.linalg.lstsq(np.stack(cols, 1), A, rcond=None)
    S = O.symmetrize(H)
    for (a, b), c in zip(keys, coef):
        assert abs(S[q1 + a, q2 + b] - c) < 1e-13


def test_symmetrization_1d_special_case():
    """Theorem 3 / eq. (simmetrizzata1d-bis): s_i = (h_{-i} + h_i)/2."""
    hv = np.array([0.1, 0.3, 0.2, 0.15, 0.25])
    S = O.symmetrize(hv.reshape(1, -1))
    assert np.allclose(S[0], (hv + hv[::-1]) / 2, atol=0, rtol=1e-15)


# ---------------------------------------------------------------- Theorem 1

@pytest.mark.parametrize("m", [3, 4, 5, 9, 16, 17, 64, 65])
def test_transform_matches_theorem1_matrices(m):
    T, Tt, alpha = brute.T_matrices(m)
    # alpha closed form from summing p_j^2
    assert abs(alpha - np.sqrt(m * (2 * m - 1) / (6.0 * (m - 1)))) < 1e-14
    assert abs(O.ar_alpha(m) - alpha) < 1e-14
    assert np.allclose(np.linalg.norm(T[:, 0]), 1.0, atol=1e-15)
    assert np.allclose(np.linalg.norm(T[:, -1]), 1.0, atol=1e-15)
    Imat = np.eye(m)
    assert np.max(np.abs(O.ar_fwd_1d(Imat, axis=0) - Tt)) < 1e-13
    assert np.max(np.abs(O.ar_inv_1d(Imat, axis=0) - T)) < 1e-13
    assert np.max(np.abs(Tt @ T - Imat)) < 1e-13


def test_alpha_value_at_9():
    assert abs(O.ar_alpha(9) - 1.7853571071357126) < 1e-15


@pytest.mark.parametrize("m", [1, 2, 5, 62, 127, 1022])
def test_dst_matches_Q_matrix_and_is_involution(m):
    rng = np.random.default_rng(m)
    x = rng.standard_normal(m)
    Q = brute.Q_matrix(m)
    assert rel(sfft.dst(x, type=1, norm="ortho"), Q @ x) < 1e-13
    if m <= 127:
        assert np.max(np.abs(Q @ Q - np.eye(m))) < 1e-13
        assert np.max(np.abs(Q - Q.T)) == 0


def test_transform_2d_kronecker_and_roundtrip():
    rng = np.random.default_rng(2)
    n1, n2 = 7, 10
    X = rng.standard_normal((n1, n2))
    _, Tt1, _ = brute.T_matrices(n1)
    _, Tt2, _ = brute.T_matrices(n2)
    assert rel(O.ar_fwd(X).ravel(), np.kron(Tt1, Tt2) @ X.ravel()) < 1e-14
    Y = rng.standard_normal((300, 257))
    assert rel(O.ar_inv(O.ar_fwd(Y)), Y) < 1e-13


# ---------------------------------------------------------------- Theorem 2

@pytest.mark.parametrize("n1,n2,q1,q2", [(5, 5, 1, 1), (6, 8, 2, 1), (10, 11, 3, 4), (9, 12, 4, 2)])
def test_factorisation_T_A_T(n1, n2, q1, q2):
    """T~ A(s) T = diag(lambda) (Theorems 1-2) for strongly symmetric s,
    with A(s) built by brute force and lambda on the extended grid."""
    S = strongly_symmetric(q1, q2, seed=n1 * n2)
    A = brute.dense_blur(S, n1, n2)
    T1, Tt1, _ = brute.T_matrices(n1)
    T2, Tt2, _ = brute.T_matrices(n2)
    D = np.kron(Tt1, Tt2) @ A @ np.kron(T1, T2)
    lam = O.eigenvalues(S, n1, n2)
    assert np.max(np.abs(D - np.diag(lam.ravel()))) < 1e-12
    ev = np.sort(np.linalg.eigvals(A).real)
    assert np.max(np.abs(ev - np.sort(lam.ravel()))) < 1e-12


def test_eigenvalues_of_nonsymmetric_use_symmetrized_psf():
    H = synth.psf_random(3, 2, seed=8)
    assert np.max(np.abs(O.eigenvalues(H, 9, 10) - O.eigenvalues(O.symmetrize(H), 9, 10))) < 1e-15


def test_eigenvalue_multiplicities_theorem2():
    """1 (x4 corners); tau_{n2-2}(h^r) eigenvalues on the first/last
    coefficient row; tau_{n1-2}(h^c) on the first/last column; the
    two-level tau eigenvalues inside."""
    n1, n2, q1, q2 = 9, 11, 3, 2
    S = strongly_symmetric(q1, q2, seed=21)
    lam = O.eigenvalues(S, n1, n2)
    for v in (lam[0, 0], lam[0, -1], lam[-1, 0], lam[-1, -1]):
        assert abs(v - 1.0) < 1e-15
    hr = S.sum(axis=0)      # h^{r}: column sums, a 1-D PSF along i2
    hc = S.sum(axis=1)      # h^{c}: row sums, a 1-D PSF along i1
    er = np.sort(np.linalg.eigvalsh(brute.tau_matrix(hr, n2 - 2)))
    ec = np.sort(np.linalg.eigvalsh(brute.tau_matrix(hc, n1 - 2)))
    for row in (lam[0, 1:-1], lam[-1, 1:-1]):
        assert np.max(np.abs(np.sort(row) - er)) < 1e-13
    for col in (lam[1:-1, 0], lam[1:-1, -1]):
        assert np.max(np.abs(np.sort(col) - ec)) < 1e-13
    # interior: two-level tau = Kronecker-structured tau of S's rows
    A = brute.dense_blur(S, n1, n2)
    inner = []
    for i1 in range(1, n1 - 1):
        for i2 in range(1, n2 - 1):
            inner.append(i1 * n2 + i2)
    Tin = A[np.ix_(inner, inner)]
    assert np.max(np.abs(np.sort(np.linalg.eigvals(Tin).real) - np.sort(lam[1:-1, 1:-1].ravel()))) < 1e-12


def test_symbol_direct_sum():
    """eq. (funzione_generatrice) equals sum_{a,b} s_ab cos(a x1) cos(b x2)
    over the full mask for a strongly symmetric s."""
    S = strongly_symmetric(4, 3, seed=2)
    x1 = np.linspace(0, np.pi, 13)
    x2 = np.linspace(0, np.pi, 7)
    direct = np.zeros((13, 7))
    for a in range(-4, 5):
        for b in range(-3, 4):
            direct += S[4 + a, 3 + b] * np.outer(np.cos(a * x1), np.cos(b * x2))
    assert np.max(np.abs(O.symbol(S, x1, x2) - direct)) < 1e-15


# ---------------------------------------------------------------- invariant

def test_symmetric_psf_preserves_bilinear_images():
    """A symmetric PSF summing to 1 maps a + b i1 + c i2 + d i1 i2 to itself
    under AR BCs; a non-symmetric one does not."""
    n1, n2 = 40, 33
    i1 = np.arange(n1, dtype=float).reshape(-1, 1)
    i2 = np.arange(n2, dtype=float).reshape(1, -1)
    X = 0.3 + 0.02 * i1 - 0.05 * i2 + 0.001 * i1 * i2
    S = strongly_symmetric(6, 5, seed=1)
    assert rel(O.blur(X, S), X) < 1e-14
    H = synth.psf_gauss_shifted(4, 4)
    assert rel(O.blur(X, H), X) > 1e-3


# ---------------------------------------------------------------- D

def test_preconditioner_is_regularised_inverse():
    """D = T diag(1/(lambda^2+alpha)) T~ = (P(s)^2 + alpha I)^{-1}."""
    n1, n2, alpha = 8, 9, 5e-3
    H = synth.psf_random(2, 3, seed=3)
    S = O.symmetrize(H)
    P = brute.dense_blur(S, n1, n2)
    d = O.tikhonov(O.eigenvalues(H, n1, n2), alpha)
    Y = np.random.default_rng(0).standard_normal((n1, n2))
    Z = O.precond_apply(Y, d)
    assert rel((P @ P + alpha * np.eye(n1 * n2)) @ Z.ravel(), Y.ravel()) < 1e-12


def test_threshold_filter_definition():
    lam = np.array([0.0, 0.05, 0.1, -0.5, 1.0])
    d = O.threshold_filter(lam, 0.1)
    assert np.allclose(d, np.array([1.0, 1.0, 100.0, 4.0, 1.0]), rtol=1e-15, atol=0)


# ---------------------------------------------------------------- iteration

@pytest.mark.parametrize("precondition", [True, False])
def test_iterate_closed_form_symmetric(precondition):
    """For strongly symmetric h, A' = A = T Lambda T~, so from x_0 = 0 the
    k-th iterate is T diag(phi_k(lambda)) T~ g with
    phi_k = (1 - (alpha/(lambda^2+alpha))^k)/lambda (D-Landweber) or
    (1 - (1 - lambda^2)^k)/lambda (Landweber)."""
    n1, n2, alpha, K = 24, 19, 1e-2, 7
    S = strongly_symmetric(3, 2, seed=6)
    G = synth.phantom(n1, n2, 3, 2, seed=1)
    lam = O.eigenvalues(S, n1, n2)
    out = O.iterate(G, S, K, alpha=alpha, precondition=precondition)
    rho = alpha / (lam ** 2 + alpha) if precondition else 1.0 - lam ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(lam != 0, (1.0 - rho ** K) / lam, 0.0)
    Xc = O.ar_inv(phi * O.ar_fwd(G))
    assert rel(out["x"], Xc) < 1e-12


def test_iterate_bookkeeping():
    n, K = 20, 6
    F = synth.phantom(n, n, 3, 2, seed=4)
    H = synth.psf_gauss_shifted(2, 2)
    G = O.blur(F, H)
    out = O.iterate(G, H, K, alpha=1e-2, F_true=F)
    X = np.zeros((n, n))
    d = O.tikhonov(O.eigenvalues(H, n, n), 1e-2)
    for k in range(K):
        R = G - O.blur(X, H)
        assert abs(out["resnorm"][k] - np.linalg.norm(R)) < 1e-12
        X = X + O.precond_apply(O.reblur(R, H), d)
        assert abs(out["rre"][k] - np.linalg.norm(X - F) / np.linalg.norm(F)) < 1e-12
    assert out["best_it"] == int(np.argmin(out["rre"])) + 1
    assert rel(out["x"], X) < 1e-14


def test_observe_noise_level():
    F = synth.phantom(32, 32, 3, 2, seed=1)
    H = synth.psf_gauss_shifted(2, 2)
    E = synth.noise_field(32, 32, seed=2)
    G = O.observe(F, H, E, 0.01)
    B = O.blur(F, H)
    assert abs(np.linalg.norm(G - B) / np.linalg.norm(B) - 0.01) < 1e-14


def test_preconditioning_reaches_same_error_in_fewer_steps():
    """Qualitative shape of the paper's tables (Sec. 4): with a stable
    alpha, D-Landweber reaches within 2% of the plain method's RRE in 10x
    fewer iterations (100 preconditioned vs 1000 plain steps), and
    beats 100 plain steps after 20."""
    F, H, E, p = synth.workload("ar64_f64_gauss9")
    G = O.observe(F, H, E, 0.001)
    pre = O.iterate(G, H, 100, alpha=0.1, F_true=F)
    plain = O.iterate(G, H, 1000, precondition=False, F_true=F)
    assert pre["rre"].min() < 1.02 * plain["rre"].min()
    assert pre["rre"][19] < plain["rre"][99]


def test_small_alpha_diverges_for_shifted_psf():
    """For the shifted Gaussian of the 64x64 workload the symmetrized
    symbol vanishes where |h^| does not, so alpha = 1e-2 makes
    I - D A' A expanding: the error grows from the first step."""
    F, H, E, p = synth.workload("ar64_f64_gauss9")
    G = O.observe(F, H, E, p["nu"])
    out = O.iterate(G, H, 12, alpha=p["alpha"], F_true=F)
    assert out["best_it"] == 1
    assert out["rre"][-1] > 100 * out["rre"][0]
