"""Pins of the Reflective / Periodic oracle and of the direct Tikhonov solve
(CPU only): brute-force matrices written from the pixelwise boundary rules,
the printed Toeplitz-plus-Hankel form of Sec. 2.1, the DCT-III
factorisation of eq. (Rn), library routines (scipy.ndimage wrap
convolution, numpy FFT) and closed forms of the iterations."""

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
import synth
from tests import brute

B = O.bc


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def dense_of(op, n1, n2):
    A = np.zeros((n1 * n2, n1 * n2))
    for j in range(n1 * n2):
        e = np.zeros(n1 * n2)
        e[j] = 1.0
        A[:, j] = op(e.reshape(n1, n2)).ravel()
    return A


def sym_psf(q1, q2, seed):
    """A strongly symmetric mask: the 4-fold average of a random one."""
    return O.symmetrize(synth.psf_random(q1, q2, seed))


@pytest.mark.parametrize("bc", ["reflective", "periodic"])
@pytest.mark.parametrize("n1,n2,q1,q2", [(7, 9, 2, 3), (10, 8, 3, 1), (6, 6, 0, 2), (9, 11, 4, 4)])
def test_blur_matches_pixelwise_rules(bc, n1, n2, q1, q2):
    H = synth.psf_random(q1, q2, 3 + q1 + 7 * q2)
    A = dense_of(lambda X: B.blur_bc(X, H, bc), n1, n2)
    assert np.max(np.abs(A - brute.dense_blur_bc(H, n1, n2, bc))) < 1e-15


@pytest.mark.parametrize("n,q", [(9, 3), (12, 4), (7, 2), (10, 0)])
def test_reflective_1d_printed_toeplitz_plus_hankel(n, q):
    """Sec. 2.1: for a symmetric PSF the Reflective blur is
    Toeplitz(v) + Hankel(sigma(v), J sigma(v))."""
    h = synth.psf_random(0, q, 40 + n)[0]
    h = 0.5 * (h + h[::-1])
    A = dense_of(lambda X: B.blur_bc(X, h.reshape(1, -1), "reflective"), 1, n)
    assert np.max(np.abs(A - brute.reflective_1d_printed(h, n))) < 1e-15


def test_periodic_blur_matches_library_wrap_convolution():
    """scipy.ndimage.convolve (a true convolution, kernel centred) with wrap
    boundaries is the periodic blur."""
    F = synth.phantom(40, 33, 4, 2, seed=5)
    H = synth.psf_random(4, 6, 9)
    G = B.blur_bc(F, H, "periodic")
    ref = ndimage.convolve(F, H, mode="wrap")
    assert np.max(np.abs(G - ref)) < 1e-14


def test_reflective_blur_matches_library_symmetric_convolution():
    """ndimage's 'reflect' mode (d c b a | a b c d) is the Reflective rule."""
    F = synth.phantom(37, 41, 4, 2, seed=6)
    H = synth.psf_random(3, 5, 10)
    G = B.blur_bc(F, H, "reflective")
    ref = ndimage.convolve(F, H, mode="reflect")
    assert np.max(np.abs(G - ref)) < 1e-14


def test_identity_psf_is_identity_under_every_bc():
    F = synth.phantom(12, 15, 3, 2, seed=1)
    H = np.ones((1, 1))
    for bc in B.BCS:
        assert np.array_equal(B.blur_bc(F, H, bc), F)


@pytest.mark.parametrize("m", [1, 2, 5, 8, 13])
def test_R_matrix_reading(m):
    """The printed eq. (Rn) is not orthogonal; its reading is, and the
    oracle's DCT pair applies R^T and R."""
    R = brute.R_matrix(m)
    assert np.max(np.abs(R.T @ R - np.eye(m))) < 1e-14
    if m >= 2:
        P = brute.R_matrix_printed(m)
        assert np.max(np.abs(P.T @ P - np.eye(m))) > 1e-3
    Y = np.random.default_rng(m).standard_normal((m, 3))
    C = np.stack([B.dct_fwd(Y[:, j].reshape(m, 1)).ravel() for j in range(3)], axis=1)
    assert np.max(np.abs(C - R.T @ Y)) < 1e-14
    assert np.max(np.abs(B.dct_inv(C[:, :1].reshape(m, 1)).ravel() - R @ C[:, 0])) < 1e-14


def test_dct_2d_is_kronecker_and_roundtrips():
    n1, n2 = 6, 9
    Y = np.random.default_rng(2).standard_normal((n1, n2))
    K = np.kron(brute.R_matrix(n1), brute.R_matrix(n2))
    assert np.max(np.abs(B.dct_fwd(Y).ravel() - K.T @ Y.ravel())) < 1e-13
    assert np.max(np.abs(B.dct_inv(B.dct_fwd(Y)) - Y)) < 1e-14


@pytest.mark.parametrize("n1,n2,q1,q2", [(8, 8, 2, 2), (9, 12, 3, 4), (11, 7, 4, 2)])
def test_reflective_factorisation_R_A_R(n1, n2, q1, q2):
    """Sec. 2.1: a strongly symmetric PSF's Reflective blur is
    R diag(f(x_r)) R^T with x_r = (r - 1) pi / m (eigenvalue grid)."""
    S = sym_psf(q1, q2, 11 + n1)
    A = brute.dense_blur_bc(S, n1, n2, "reflective")
    K = np.kron(brute.R_matrix(n1), brute.R_matrix(n2))
    lam = B.reflective_eigenvalues(S, n1, n2)
    assert np.max(np.abs(K.T @ A @ K - np.diag(lam.ravel()))) < 1e-13
    ev = np.sort(np.linalg.eigvals(A).real)
    assert np.max(np.abs(ev - np.sort(lam.ravel()))) < 1e-12
    assert abs(lam[0, 0] - 1.0) < 1e-14                  # f(0, 0) = sum h = 1


def test_reflective_eigenvalues_use_symmetrized_psf():
    H = synth.psf_random(2, 3, 17)
    a = B.reflective_eigenvalues(H, 10, 12)
    assert np.max(np.abs(a - B.reflective_eigenvalues(O.symmetrize(H), 10, 12))) < 1e-15
    # and not those of the PSF itself read as if it were symmetric
    assert np.max(np.abs(a - O.symbol(H, B.reflective_grid(10), B.reflective_grid(12)))) > 1e-3


@pytest.mark.parametrize("n1,n2,q1,q2", [(8, 6, 2, 1), (7, 9, 3, 4), (5, 5, 2, 2)])
def test_periodic_eigenvalues(n1, n2, q1, q2):
    """The periodic blur is F^{-1} diag(lambda) F with lambda the DFT of the
    PSF wrapped onto the n1 x n2 grid (numpy FFT as the library pin)."""
    H = synth.psf_random(q1, q2, 21 + n1)
    lam = B.periodic_eigenvalues(H, n1, n2)
    wrapped = np.zeros((n1, n2))
    for s1 in range(-q1, q1 + 1):
        for s2 in range(-q2, q2 + 1):
            wrapped[s1 % n1, s2 % n2] += H[q1 + s1, q2 + s2]
    assert np.max(np.abs(lam - np.fft.fft2(wrapped))) < 1e-14
    A = brute.dense_blur_bc(H, n1, n2, "periodic")
    F2 = np.kron(brute.dft_matrix(n1), brute.dft_matrix(n2))
    assert np.max(np.abs(F2 @ A @ F2.conj().T - np.diag(lam.ravel()))) < 1e-13


def test_periodic_reblur_is_transpose():
    """Sec. 4: A' and A^H coincide for periodic BCs (not for Reflective)."""
    H = synth.psf_random(2, 3, 30)
    n1, n2 = 8, 9
    A = brute.dense_blur_bc(H, n1, n2, "periodic")
    Ap = dense_of(lambda X: B.reblur_bc(X, H, "periodic"), n1, n2)
    assert np.max(np.abs(Ap - A.T)) < 1e-15
    Ar = brute.dense_blur_bc(H, n1, n2, "reflective")
    Arp = dense_of(lambda X: B.reblur_bc(X, H, "reflective"), n1, n2)
    assert np.max(np.abs(Arp - Ar.T)) > 1e-3


@pytest.mark.parametrize("bc", ["reflective", "periodic"])
def test_preconditioner_is_regularised_inverse(bc):
    """D = V diag(1/(|lambda|^2 + alpha)) V^{-1} equals (P^H P + alpha I)^{-1}
    with P the blur of the BC's algebra (symmetrized PSF for Reflective,
    the PSF itself for Periodic), brute force."""
    n1, n2, alpha = 7, 8, 0.03
    H = synth.psf_random(2, 2, 44)
    Pm = brute.dense_blur_bc(O.symmetrize(H) if bc == "reflective" else H, n1, n2, bc)
    d = B.tikhonov_bc(B.eigenvalues_bc(H, n1, n2, bc), alpha)
    Dm = dense_of(lambda Y: B.precond_apply_bc(Y, d, bc), n1, n2)
    assert np.max(np.abs(Dm @ (Pm.T @ Pm + alpha * np.eye(n1 * n2)) - np.eye(n1 * n2))) < 1e-12


def test_reflective_iterate_closed_form():
    """Strongly symmetric PSF, Reflective BCs (A' = A symmetric), x_0 = 0:
    x_k = R diag((1 - (alpha / (lambda^2 + alpha))^k) / lambda) R^T g."""
    n1, n2, k, alpha = 12, 10, 6, 0.05
    S = sym_psf(2, 3, 50)
    G = synth.phantom(n1, n2, 3, 2, seed=51)
    lam = B.reflective_eigenvalues(S, n1, n2)
    out = B.iterate_bc(G, S, k, "reflective", alpha=alpha)
    ok = np.abs(lam) > 1e-12
    coef = np.where(ok, (1 - (alpha / (lam * lam + alpha)) ** k) / np.where(ok, lam, 1), k * 0.0)
    ref = B.dct_inv(coef * B.dct_fwd(G))
    assert rel(out["x"], ref) < 1e-12


def test_periodic_iterate_closed_form():
    """Periodic BCs, any PSF, x_0 = 0: every Fourier mode follows
    x^_k = (1 - (alpha / (|lambda|^2 + alpha))^k) g^ / lambda; and the plain
    method (D = I) follows 1 - (1 - |lambda|^2)^k."""
    n1, n2, k, alpha = 10, 12, 5, 0.02
    H = synth.psf_random(2, 3, 60)
    G = synth.phantom(n1, n2, 3, 2, seed=61)
    lam = B.periodic_eigenvalues(H, n1, n2)
    Gh = np.fft.fft2(G)
    out = B.iterate_bc(G, H, k, "periodic", alpha=alpha)
    ref = np.real(np.fft.ifft2((1 - (alpha / (np.abs(lam) ** 2 + alpha)) ** k) * Gh / lam))
    assert rel(out["x"], ref) < 1e-11
    out = B.iterate_bc(G, H, k, "periodic", precondition=False)
    ref = np.real(np.fft.ifft2((1 - (1 - np.abs(lam) ** 2) ** k) * Gh / lam))
    assert rel(out["x"], ref) < 1e-11


def test_antireflective_matches_ar_oracle():
    n = 14
    H = synth.psf_gauss_shifted(2, 3, 1.2, 0.8, shift=(0.5, -0.4))
    G = synth.phantom(n, n, 3, 2, seed=70)
    a = B.iterate_bc(G, H, 4, "antireflective", alpha=0.1)["x"]
    b = O.iterate(G, H, 4, alpha=0.1)["x"]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n1,n2,q1,q2", [(9, 11, 2, 3), (12, 8, 4, 2)])
def test_tikhonov_solve_antireflective_brute(n1, n2, q1, q2):
    """Direct solve: (A'A + alpha I) x = A' g with A' = A for a strongly
    symmetric PSF, against numpy's dense solver on the brute-force AR
    matrix (pixelwise ghost formulas)."""
    S = sym_psf(q1, q2, 80 + n1)
    G = synth.phantom(n1, n2, 3, 2, seed=81)
    A = brute.dense_blur(S, n1, n2)
    alpha = 0.02
    ref = np.linalg.solve(A @ A + alpha * np.eye(n1 * n2), A @ G.ravel())
    x = B.tikhonov_solve(G, S, alpha)
    assert rel(x.ravel(), ref) < 1e-11


def test_tikhonov_solve_reflective_brute():
    n1, n2, alpha = 10, 9, 0.05
    S = sym_psf(3, 2, 90)
    G = synth.phantom(n1, n2, 3, 2, seed=91)
    A = brute.dense_blur_bc(S, n1, n2, "reflective")
    ref = np.linalg.solve(A.T @ A + alpha * np.eye(n1 * n2), A.T @ G.ravel())
    assert rel(B.tikhonov_solve(G, S, alpha, bc="reflective").ravel(), ref) < 1e-11


def test_tikhonov_solve_rejects_nonsymmetric_psf():
    with pytest.raises(ValueError):
        B.tikhonov_solve(np.zeros((9, 9)), synth.psf_random(2, 2, 3), 0.1)
    assert B.is_strongly_symmetric(sym_psf(2, 3, 4))
    assert not B.is_strongly_symmetric(synth.psf_motion(3))


def test_tikhonov_solve_is_iteration_limit():
    """The D-Landweber closed form tends to the direct solve: with
    d = 1/(lambda^2 + alpha) the factor (alpha/(lambda^2+alpha))^k -> 0, so
    x_k -> T diag(1/lambda) T~ g, while the Tikhonov solve is that with
    lambda^2/(lambda^2 + alpha) damping; for tiny alpha both agree with the
    inverse on a well-conditioned PSF."""
    n = 12
    S = O.symmetrize(synth.psf_gauss_shifted(1, 1, 0.4, 0.4, shift=(0.0, 0.0)))
    F = synth.phantom(n, n, 3, 2, seed=7)
    G = O.blur(F, S)
    x = B.tikhonov_solve(G, S, 1e-12)
    assert rel(x, F) < 1e-8
