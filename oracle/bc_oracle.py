"""FP64 CPU oracle for the boundary-condition variants the paper compares
against (Reflective and Periodic BCs) and for the direct Tikhonov solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this module: only the test-suite and the benchmark's CPU-baseline leg
use it.  It shares no code, tables or constants with the HIP library.

Source: Dell'Acqua, Serra-Capizzano, Tablino-Possio, "Optimal
preconditioning for image deblurring with Anti-Reflective boundary
conditions" (arXiv 1211.0393):
  * Reflective BCs (Sec. 2.1): the scene outside the field of view is the
    mirror image of the scene inside, f_{1-i} = f_i, f_{n+i} = f_{n+1-i},
    and a double reflection at the corners; for a strongly symmetric PSF the
    blur lies in the DCT-III algebra, A = R Lambda R^T with R of eq. (Rn),
    and its eigenvalues are the generating function
    (eq. (funzione_generatrice)) at x_r = (r - 1) pi / m;
  * Periodic BCs (Sec. 2 and Sec. 4): the blur is a two-level circulant
    matrix diagonalised by the DFT, whose eigenvalues come from the PSF
    itself (not symmetrised) "via FFT";
  * D-Landweber for every BC (Sec. 4, eqs. (DLandweberMeth), (TikFilter)):
    d = 1 / (|lambda|^2 + alpha) with the eigenvalues of the BC's algebra,
    D applied through the inverse transform; the transpose step is the
    reblurring A' (the PSF rotated by 180 degrees), which for Periodic BCs
    equals A^H (Sec. 4);
  * the direct Tikhonov solve x = (A'A + alpha I)^{-1} A' g for a strongly
    symmetric PSF, diagonal in the BC's transform: x = V diag(lambda /
    (lambda^2 + alpha)) V^{-1} g (Theorems 1-2 with eq. (TikFilter);
    Sec. 2.1 for the DCT-III algebra).

Readings (each also listed in the design notes of the repository):
  * eq. (Rn) prints R_m = [sqrt((2 - delta_{t,1}) / m) cos((s - 1)(t - 1/2)
    pi / m)]; read literally it is not orthogonal.  Read here as the
    orthogonal matrix whose column t is the normalised eigenvector
    sqrt((2 - delta_{t,1}) / m) cos((t - 1)(s - 1/2) pi / m), s = 1..m, so
    that R^T is the orthonormal DCT-II and column t carries the eigenvalue
    f((t - 1) pi / m) (pinned by R^T A(s) R = diag(lambda) on brute force);
  * Periodic extension f_{1-i} = f_{n+1-i}, f_{n+i} = f_i (the classical
    periodic BCs the paper names but does not write out); the DFT
    convention is F_k = sum_t f_t e^{-2 pi i k t / n}, so the blur's
    eigenvalues are lambda_k = sum_s h_s e^{-2 pi i (k1 s1 / n1 + k2 s2 / n2)}.
"""

from __future__ import annotations

import numpy as np
from scipy import fft as _sfft

from . import ar_oracle as _ar

__all__ = [
    "BCS",
    "reflect_extend",
    "periodic_extend",
    "extend",
    "blur_bc",
    "reblur_bc",
    "dct_fwd",
    "dct_inv",
    "reflective_grid",
    "reflective_eigenvalues",
    "periodic_eigenvalues",
    "eigenvalues_bc",
    "tikhonov_bc",
    "precond_apply_bc",
    "landweber_step_bc",
    "iterate_bc",
    "observe_bc",
    "is_strongly_symmetric",
    "tikhonov_solve",
]

BCS = ("antireflective", "reflective", "periodic")


# --------------------------------------------------------------------------
# Extensions (Sec. 2.1 for Reflective; classical periodic BCs, Sec. 2)
# --------------------------------------------------------------------------

def _reflect_axis0(F, q):
    """f_{1-i} = f_i and f_{n+i} = f_{n+1-i}, i = 1..q (Sec. 2.1)."""
    n = F.shape[0]
    E = np.empty((n + 2 * q,) + F.shape[1:], dtype=np.float64)
    E[q:q + n] = F
    for i in range(1, q + 1):
        E[q - i] = F[i - 1]                   # paper index 1 - i  <- f_i
        E[q + n - 1 + i] = F[n - i]           # paper index n + i  <- f_{n+1-i}
    return E


def reflect_extend(F, q1, q2):
    """Extended image on [1-q1, n1+q1] x [1-q2, n2+q2] under Reflective BCs:
    reflection along i1, then along i2 on the extended array (the double
    reflection the paper gives at the corners, order immaterial)."""
    F = np.asarray(F, dtype=np.float64)
    E = _reflect_axis0(F, q1)
    return _reflect_axis0(E.T, q2).T


def _periodic_axis0(F, q):
    """f_{1-i} = f_{n+1-i} and f_{n+i} = f_i, i = 1..q."""
    n = F.shape[0]
    E = np.empty((n + 2 * q,) + F.shape[1:], dtype=np.float64)
    E[q:q + n] = F
    for i in range(1, q + 1):
        E[q - i] = F[n - i]
        E[q + n - 1 + i] = F[i - 1]
    return E


def periodic_extend(F, q1, q2):
    """Extended image under periodic BCs (wrap-around along each axis)."""
    F = np.asarray(F, dtype=np.float64)
    E = _periodic_axis0(F, q1)
    return _periodic_axis0(E.T, q2).T


def extend(F, q1, q2, bc):
    if bc == "antireflective":
        return _ar.ar_extend(F, q1, q2)
    if bc == "reflective":
        return reflect_extend(F, q1, q2)
    if bc == "periodic":
        return periodic_extend(F, q1, q2)
    raise ValueError(bc)


def blur_bc(F, H, bc):
    """A_n f under the given BCs: eq. (modello_discreto) on the extended
    image, g_i = sum_s h_s f_{i-s} for i in the field of view."""
    F = np.asarray(F, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    q1, q2 = _ar.psf_halfwidths(H)
    n1, n2 = F.shape
    E = extend(F, q1, q2, bc)
    G = np.zeros((n1, n2))
    for s1 in range(-q1, q1 + 1):
        for s2 in range(-q2, q2 + 1):
            G += H[q1 + s1, q2 + s2] * E[q1 - s1:q1 - s1 + n1, q2 - s2:q2 - s2 + n2]
    return G


def reblur_bc(R, H, bc):
    """A' r: the same BCs with the PSF rotated by 180 degrees (Sec. 4)."""
    H = np.asarray(H, dtype=np.float64)
    return blur_bc(R, H[::-1, ::-1], bc)


# --------------------------------------------------------------------------
# DCT-III algebra (Sec. 2.1, eq. (Rn))
# --------------------------------------------------------------------------

def dct_fwd(Y):
    """c = (R_{n1} (x) R_{n2})^T y: the orthonormal DCT-II along both axes
    (R^T of eq. (Rn) under the reading in the module docstring)."""
    Y = np.asarray(Y, dtype=np.float64)
    return _sfft.dct(_sfft.dct(Y, type=2, axis=1, norm="ortho"), type=2, axis=0, norm="ortho")


def dct_inv(C):
    """y = (R_{n1} (x) R_{n2}) c: the orthonormal DCT-III along both axes."""
    C = np.asarray(C, dtype=np.float64)
    return _sfft.dct(_sfft.dct(C, type=3, axis=1, norm="ortho"), type=3, axis=0, norm="ortho")


def reflective_grid(m):
    """x_r = (r - 1) pi / m, r = 1..m (the eigenvalue grid of Sec. 2.1)."""
    return np.arange(m, dtype=np.float64) * np.pi / m


def reflective_eigenvalues(H, n1, n2):
    """lambda[k1, k2] = f(x_{k1}, x_{k2}) of the symmetrized PSF (Sec. 4:
    symmetrized PSF and Reflective BCs), in the column order of R."""
    S = _ar.symmetrize(H)
    return _ar.symbol(S, reflective_grid(n1), reflective_grid(n2))


def periodic_eigenvalues(H, n1, n2):
    """Complex eigenvalues of the periodic blur of the PSF itself (Sec. 4:
    the PSF and periodic BCs, via FFT), written as their defining sum
    lambda[k1, k2] = sum_s h_s exp(-2 pi i (k1 s1 / n1 + k2 s2 / n2))."""
    H = np.asarray(H, dtype=np.float64)
    q1, q2 = _ar.psf_halfwidths(H)
    s1 = np.arange(-q1, q1 + 1)
    s2 = np.arange(-q2, q2 + 1)
    E1 = np.exp(-2j * np.pi * np.outer(np.arange(n1), s1) / n1)
    E2 = np.exp(-2j * np.pi * np.outer(np.arange(n2), s2) / n2)
    return E1 @ H @ E2.T


def eigenvalues_bc(H, n1, n2, bc):
    if bc == "antireflective":
        return _ar.eigenvalues(H, n1, n2)
    if bc == "reflective":
        return reflective_eigenvalues(H, n1, n2)
    if bc == "periodic":
        return periodic_eigenvalues(H, n1, n2)
    raise ValueError(bc)


def tikhonov_bc(lam, alpha):
    """d = 1 / (|lambda|^2 + alpha), eq. (TikFilter) (complex lambda allowed)."""
    lam = np.asarray(lam)
    return 1.0 / (np.abs(lam) ** 2 + alpha)


def precond_apply_bc(Y, d, bc):
    """z = D y with D = V diag(d) V^{-1} in the BC's algebra (Sec. 4)."""
    d = np.asarray(d, dtype=np.float64)
    if bc == "antireflective":
        return _ar.precond_apply(Y, d)
    if bc == "reflective":
        return dct_inv(d * dct_fwd(Y))
    if bc == "periodic":
        return np.real(np.fft.ifft2(d * np.fft.fft2(np.asarray(Y, dtype=np.float64))))
    raise ValueError(bc)


# --------------------------------------------------------------------------
# D-Landweber under any of the three BCs (Sec. 4)
# --------------------------------------------------------------------------

def landweber_step_bc(X, G, H, bc, d=None, tau=1.0):
    """x_{k+1} = x_k + tau D A'(g - A x_k) (D = I when ``d`` is None), A
    and A' under BCs ``bc``.  Returns (x_{k+1}, ||g - A x_k||_F)."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(G, dtype=np.float64) - blur_bc(X, H, bc)
    Y = reblur_bc(R, H, bc)
    Z = Y if d is None else precond_apply_bc(Y, d, bc)
    return X + tau * Z, float(np.linalg.norm(R))


def iterate_bc(G, H, iters, bc, alpha=None, d=None, X0=None, tau=1.0, precondition=True,
               F_true=None):
    """``iters`` (D-)Landweber steps under BCs ``bc``; the same outputs as
    the Anti-Reflective oracle's ``iterate`` (x, resnorm, rre, best_it)."""
    G = np.asarray(G, dtype=np.float64)
    n1, n2 = G.shape
    if precondition and d is None:
        d = tikhonov_bc(eigenvalues_bc(H, n1, n2, bc), alpha)
    if not precondition:
        d = None
    X = np.zeros((n1, n2)) if X0 is None else np.array(X0, dtype=np.float64)
    res, errs = [], []
    for _ in range(iters):
        X, rn = landweber_step_bc(X, G, H, bc, d=d, tau=tau)
        res.append(rn)
        if F_true is not None:
            errs.append(_ar.rre(X, F_true))
    out = {"x": X, "resnorm": np.array(res)}
    if F_true is not None:
        errs = np.array(errs)
        out["rre"] = errs
        out["best_it"] = int(np.argmin(errs)) + 1 if iters else 0
    return out


def observe_bc(F, H, E, nu, bc):
    """g = A f + eta, eta = nu ||A f|| e / ||e|| under BCs ``bc`` (Sec. 4)."""
    B = blur_bc(F, H, bc)
    E = np.asarray(E, dtype=np.float64)
    return B + nu * np.linalg.norm(B) / np.linalg.norm(E) * E


# --------------------------------------------------------------------------
# Direct Tikhonov solve for strongly symmetric PSFs
# --------------------------------------------------------------------------

def is_strongly_symmetric(H, tol=1e-14):
    """h_{|i|} = h_i per axis (eq. (strong_simmetry_condition)), within
    ``tol`` times the largest entry (the default admits the last-bit
    differences that a symmetrization in floating point leaves)."""
    H = np.asarray(H, dtype=np.float64)
    scale = tol * float(np.max(np.abs(H))) if H.size else 0.0
    return (np.max(np.abs(H - H[::-1, :])) <= scale) and (np.max(np.abs(H - H[:, ::-1])) <= scale)


def tikhonov_solve(G, H, alpha, bc="antireflective"):
    """x = V diag(lambda / (lambda^2 + alpha)) V^{-1} g for a strongly
    symmetric PSF, i.e. (A'A + alpha I)^{-1} A' g with A' = A (Theorems 1-2
    and eq. (TikFilter); V = T for Anti-Reflective BCs, R for Reflective)."""
    if not is_strongly_symmetric(H):
        raise ValueError("the direct solve needs a strongly symmetric PSF")
    G = np.asarray(G, dtype=np.float64)
    n1, n2 = G.shape
    lam = eigenvalues_bc(H, n1, n2, bc)
    filt = lam / (lam * lam + alpha)
    if bc == "antireflective":
        return _ar.ar_inv(filt * _ar.ar_fwd(G))
    if bc == "reflective":
        return dct_inv(filt * dct_fwd(G))
    raise ValueError("direct solve defined for antireflective and reflective BCs")
