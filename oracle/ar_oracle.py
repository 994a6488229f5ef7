"""FP64 CPU oracle for preconditioned Landweber deblurring under
Anti-Reflective (AR) boundary conditions.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this module: only the test-suite, the smoke check of the graft entry
point and the CPU-baseline leg of the benchmark use it.  It shares no code,
tables or constants with the HIP library.

Source: Dell'Acqua, Serra-Capizzano, Tablino-Possio, "Optimal
preconditioning for image deblurring with Anti-Reflective boundary
conditions" (arXiv 1211.0393).  Every function cites the passage it
follows.  Arithmetic is IEEE FP64 throughout; library primitives used as
single steps: numpy array arithmetic and ``scipy.fft.dst`` (DST-I).

Conventions (Sec. 1, eqs. (modello_discreto) and (coefficienti_psf)):
  * images are n1 x n2 arrays, row-major, i1 = row (slow), i2 = column
    (fast); the paper's 1-based index i maps to array index i-1;
  * a PSF is a (2 q1 + 1) x (2 q2 + 1) array ``H`` with
    ``H[q1 + s1, q2 + s2] = h_{s1, s2}``; entries are >= 0 and sum to 1;
  * the blur is a true convolution g_i = sum_s h_s f_{i-s}.

Readings of passages that are garbled or silent (each also listed in the
design notes of the repository):
  * the fourth corner formula of Sec. 2.2 prints ``2 f_{n1, n1 - i2}``;
    the tensor rule of the same section gives ``2 f_{n1, n2 - i2}``, used here;
  * the AR eigenvalue grid at the end of Sec. 2.2 ("s_j = 0..n_j,
    x_r = r pi / (m + 1)") is read with m = n_j - 2, the size of the tau
    block: the interior columns of T carry x_r = r pi / (n_j - 1),
    r = 1..n_j - 2, and both the first and the last column carry x = 0;
  * D is kept as its spectrum d and applied as T (d * (T~ y)) (Sec. 4);
  * x_0 = 0 unless given; the paper uses tau = 1 (Sec. 4).

Parity pins: every public function here is pinned by a test under
``tests/test_oracle_*.py`` against brute force, closed forms, worked
examples of the paper or library routines.  The threshold filter has a
stated definition but no passage of the paper behind it (it is not part of
the method the paper describes): parity unpinned beyond its own definition.
"""

from __future__ import annotations

import numpy as np
from scipy import fft as _sfft

__all__ = [
    "psf_halfwidths",
    "check_psf",
    "ar_extend",
    "blur",
    "blur_adjoint",
    "reblur",
    "blur_T",
    "symmetrize",
    "ar_alpha",
    "ar_fwd_1d",
    "ar_inv_1d",
    "ar_fwd",
    "ar_inv",
    "symbol",
    "ar_grid",
    "eigenvalues",
    "tikhonov",
    "threshold_filter",
    "precond_apply",
    "landweber_step",
    "iterate",
    "observe",
    "rre",
]


# --------------------------------------------------------------------------
# PSF mask (Sec. 1, eq. (coefficienti_psf))
# --------------------------------------------------------------------------

def psf_halfwidths(H):
    """Half-widths (q1, q2) of a (2q1+1) x (2q2+1) mask (eq. (coefficienti_psf))."""
    H = np.asarray(H)
    if H.ndim != 2 or H.shape[0] % 2 == 0 or H.shape[1] % 2 == 0:
        raise ValueError("PSF mask must be 2-D with odd sides")
    return (H.shape[0] - 1) // 2, (H.shape[1] - 1) // 2


def check_psf(H, n1, n2, tol=1e-12):
    """Validate the mask against eq. (coefficienti_psf) (h >= 0, sum 1) and
    the support condition of Sec. 2.2 that puts the symmetrized PSF in the
    AR algebra (h_i = 0 when |i_j| >= n_j - 2, i.e. q_j <= n_j - 3)."""
    H = np.asarray(H, dtype=np.float64)
    q1, q2 = psf_halfwidths(H)
    if not np.all(np.isfinite(H)) or np.any(H < 0):
        raise ValueError("PSF entries must be finite and nonnegative")
    if abs(H.sum() - 1.0) > tol * H.size:
        raise ValueError("PSF must sum to 1")
    if n1 < 3 or n2 < 3 or q1 > n1 - 3 or q2 > n2 - 3:
        raise ValueError("need n_j >= 3 and q_j <= n_j - 3")
    return q1, q2


# --------------------------------------------------------------------------
# AR boundary conditions and the blur A_n (Sec. 2.2; Sec. 1 eq. (modello_discreto))
# --------------------------------------------------------------------------

def _ar_extend_axis0(F, q):
    """Anti-reflect the rows of F about its first and last row (Sec. 2.2):
    f_{1-i} = 2 f_1 - f_{1+i},  f_{n+i} = 2 f_n - f_{n-i},  i = 1..q."""
    n = F.shape[0]
    E = np.empty((n + 2 * q,) + F.shape[1:], dtype=np.float64)
    E[q:q + n] = F
    for i in range(1, q + 1):
        E[q - i] = 2.0 * F[0] - F[i]                 # paper index 1 - i
        E[q + n - 1 + i] = 2.0 * F[n - 1] - F[n - 1 - i]   # paper index n + i
    return E


def ar_extend(F, q1, q2):
    """Extended image on [1-q1, n1+q1] x [1-q2, n2+q2] (Sec. 2.2).

    Anti-reflection along i1 and then along i2 on the already-extended
    array: the double anti-reflection the paper uses at the corners to keep
    the tensor structure (weights 4, -2, -2, +1)."""
    F = np.asarray(F, dtype=np.float64)
    E = _ar_extend_axis0(F, q1)
    return _ar_extend_axis0(E.T, q2).T


def blur(F, H):
    """A_n f under AR BCs: eq. (modello_discreto) applied to the extended
    image, g_i = sum_{s=-q}^{q} h_s f_{i-s} for i in the field of view."""
    F = np.asarray(F, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    q1, q2 = psf_halfwidths(H)
    n1, n2 = F.shape
    E = ar_extend(F, q1, q2)
    G = np.zeros((n1, n2))
    for s1 in range(-q1, q1 + 1):
        for s2 in range(-q2, q2 + 1):
            # f_{i-s} sits at extended-array index (i - s) + q
            G += H[q1 + s1, q2 + s2] * E[q1 - s1:q1 - s1 + n1, q2 - s2:q2 - s2 + n2]
    return G


def _fold_axis0(R, q, n):
    """Adjoint of the axis-0 anti-reflection: ghost row 1-t contributes
    +2 to row 1 and -1 to row 1+t; ghost row n+t contributes +2 to row n
    and -1 to row n-t (transpose of the rule of Sec. 2.2)."""
    Y = R[q:q + n].copy()
    for t in range(1, q + 1):
        lo = R[q - t]
        hi = R[q + n - 1 + t]
        Y[0] += 2.0 * lo
        Y[t] -= lo
        Y[n - 1] += 2.0 * hi
        Y[n - 1 - t] -= hi
    return Y


def blur_adjoint(R, H):
    """Exact transpose A_n^T r (the A^H of eq. (LandweberMeth) for real data).

    A_n = C * Ext with C the valid convolution of eq. (modello_discreto)
    and Ext the AR extension of Sec. 2.2, so A_n^T = Ext^T C^T: scatter
    h_s r_i onto extended index i - s, then fold the ghosts back."""
    R = np.asarray(R, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    q1, q2 = psf_halfwidths(H)
    n1, n2 = R.shape
    X = np.zeros((n1 + 2 * q1, n2 + 2 * q2))
    for s1 in range(-q1, q1 + 1):
        for s2 in range(-q2, q2 + 1):
            X[q1 - s1:q1 - s1 + n1, q2 - s2:q2 - s2 + n2] += H[q1 + s1, q2 + s2] * R
    Y = _fold_axis0(X, q1, n1)
    return _fold_axis0(Y.T, q2, n2).T


def reblur(R, H):
    """A' r: the AR blur with the PSF rotated by 180 degrees (the
    reblurring used instead of A^H in the paper's experiments, Sec. 4)."""
    H = np.asarray(H, dtype=np.float64)
    return blur(R, H[::-1, ::-1])


def blur_T(R, H, tmode="reblur"):
    """Transpose step of the iteration: A' (``"reblur"``) or A^T (``"adjoint"``)."""
    if tmode == "reblur":
        return reblur(R, H)
    if tmode == "adjoint":
        return blur_adjoint(R, H)
    raise ValueError(tmode)


# --------------------------------------------------------------------------
# Optimal preconditioner: symmetrized PSF (Sec. 3, Theorem 4, eq. (simmetrizzata2d-bis))
# --------------------------------------------------------------------------

def symmetrize(H):
    """s_{+-i1,+-i2} = (h_{-i1,-i2} + h_{-i1,i2} + h_{i1,-i2} + h_{i1,i2}) / 4."""
    H = np.asarray(H, dtype=np.float64)
    q1, q2 = psf_halfwidths(H)
    S = np.empty_like(H)
    for i1 in range(-q1, q1 + 1):
        for i2 in range(-q2, q2 + 1):
            S[q1 + i1, q2 + i2] = (H[q1 - i1, q2 - i2] + H[q1 - i1, q2 + i2]
                                   + H[q1 + i1, q2 - i2] + H[q1 + i1, q2 + i2]) / 4.0
    return S


# --------------------------------------------------------------------------
# AR transform (Sec. 2.2, Theorem 1; tau algebra eq. (Qn))
# --------------------------------------------------------------------------

def _ramp(m):
    """p_j = 1 - j/(m-1), j = 1..m-2 (Theorem 1), and its flip J p."""
    j = np.arange(1, m - 1, dtype=np.float64)
    p = 1.0 - j / (m - 1)
    return p, p[::-1].copy()


def ar_alpha(m):
    """alpha_m of Theorem 1: the factor making the first column
    alpha^{-1} [1, p, 0] of T_m a unit vector."""
    p, _ = _ramp(m)
    return float(np.sqrt(1.0 + np.dot(p, p)))


def _dst1(X, axis):
    """Q_{m} X along ``axis`` with Q_m = [sqrt(2/(m+1)) sin(s t pi/(m+1))]
    (eq. (Qn)); the orthonormal DST-I of scipy is exactly this matrix."""
    return _sfft.dst(X, type=1, axis=axis, norm="ortho")


def ar_fwd_1d(Y, axis=0):
    """c = T~_m y along ``axis`` (Theorem 1):
    c_1 = alpha y_1, c_m = alpha y_m,
    c_mid = Q_{m-2} (y_mid - y_1 p - y_m J p)."""
    Y = np.moveaxis(np.asarray(Y, dtype=np.float64), axis, 0)
    m = Y.shape[0]
    p, Jp = _ramp(m)
    a = ar_alpha(m)
    C = np.empty_like(Y)
    C[0] = a * Y[0]
    C[m - 1] = a * Y[m - 1]
    shp = (m - 2,) + (1,) * (Y.ndim - 1)
    mid = Y[1:m - 1] - p.reshape(shp) * Y[0] - Jp.reshape(shp) * Y[m - 1]
    C[1:m - 1] = _dst1(mid, 0)
    return np.moveaxis(C, 0, axis)


def ar_inv_1d(C, axis=0):
    """y = T_m c along ``axis`` (Theorem 1):
    y_1 = c_1/alpha, y_m = c_m/alpha, y_mid = Q_{m-2} c_mid + y_1 p + y_m J p."""
    C = np.moveaxis(np.asarray(C, dtype=np.float64), axis, 0)
    m = C.shape[0]
    p, Jp = _ramp(m)
    a = ar_alpha(m)
    Y = np.empty_like(C)
    Y[0] = C[0] / a
    Y[m - 1] = C[m - 1] / a
    shp = (m - 2,) + (1,) * (C.ndim - 1)
    Y[1:m - 1] = _dst1(C[1:m - 1], 0) + p.reshape(shp) * Y[0] + Jp.reshape(shp) * Y[m - 1]
    return np.moveaxis(Y, 0, axis)


def ar_fwd(Y):
    """c = (T~_{n1} (x) T~_{n2}) y on a row-major n1 x n2 image (Theorem 1)."""
    return ar_fwd_1d(ar_fwd_1d(Y, axis=1), axis=0)


def ar_inv(C):
    """y = (T_{n1} (x) T_{n2}) c (Theorem 1)."""
    return ar_inv_1d(ar_inv_1d(C, axis=1), axis=0)


# --------------------------------------------------------------------------
# Spectrum (eq. (funzione_generatrice); Theorem 2 and the grid that follows it)
# --------------------------------------------------------------------------

def symbol(S, x1, x2):
    """Generating function f(x1, x2) of a strongly symmetric mask S,
    eq. (funzione_generatrice): h00 + 2 sum h_{s1,0} cos(s1 x1)
    + 2 sum h_{0,s2} cos(s2 x2) + 4 sum sum h_{s1,s2} cos(s1 x1) cos(s2 x2),
    evaluated on the outer grid x1 (column) x x2 (row)."""
    S = np.asarray(S, dtype=np.float64)
    q1, q2 = psf_halfwidths(S)
    x1 = np.asarray(x1, dtype=np.float64).reshape(-1, 1)
    x2 = np.asarray(x2, dtype=np.float64).reshape(1, -1)
    F = np.full((x1.shape[0], x2.shape[1]), S[q1, q2])
    for s1 in range(1, q1 + 1):
        F = F + 2.0 * S[q1 + s1, q2] * np.cos(s1 * x1)
    for s2 in range(1, q2 + 1):
        F = F + 2.0 * S[q1, q2 + s2] * np.cos(s2 * x2)
    for s1 in range(1, q1 + 1):
        for s2 in range(1, q2 + 1):
            F = F + 4.0 * S[q1 + s1, q2 + s2] * np.cos(s1 * x1) * np.cos(s2 * x2)
    return F


def ar_grid(m):
    """Evaluation points for the m columns of T_m: 0 for the first and last
    column, r pi/(m-1) for the interior column r = 1..m-2 (the tau grid of
    size m-2, extended to 0 as stated after Theorem 2)."""
    x = np.zeros(m)
    x[1:m - 1] = np.arange(1, m - 1) * np.pi / (m - 1)
    return x


def eigenvalues(H, n1, n2):
    """lambda[k1, k2] of P(s), s the symmetrized PSF of H, in the column
    order of T_{n1} (x) T_{n2} (Theorem 2 with the extended grid)."""
    S = symmetrize(H)
    return symbol(S, ar_grid(n1), ar_grid(n2))


# --------------------------------------------------------------------------
# Filters and the preconditioner (Sec. 4, eq. (TikFilter))
# --------------------------------------------------------------------------

def tikhonov(lam, alpha):
    """d_j = 1 / (|lambda_j|^2 + alpha), eq. (TikFilter)."""
    lam = np.asarray(lam, dtype=np.float64)
    return 1.0 / (lam * lam + alpha)


def threshold_filter(lam, t):
    """Truncated-spectrum filter (not in the paper; this repository's
    definition): d = 1/lambda^2 where |lambda| >= t, else 1.  Parity
    unpinned beyond this definition."""
    lam = np.asarray(lam, dtype=np.float64)
    out = np.ones_like(lam)
    big = np.abs(lam) >= t
    out[big] = 1.0 / (lam[big] * lam[big])
    return out


def precond_apply(Y, d):
    """z = D y with D = T diag(d) T~ (Sec. 4: eigenvalues of D from the
    filter, D recovered through the inverse transform of Theorem 1)."""
    return ar_inv(np.asarray(d, dtype=np.float64) * ar_fwd(Y))


# --------------------------------------------------------------------------
# Landweber and D-Landweber (Sec. 4, eqs. (LandweberMeth), (DLandweberMeth))
# --------------------------------------------------------------------------

def landweber_step(X, G, H, d=None, tau=1.0, tmode="reblur"):
    """x_{k+1} = x_k + tau D A'(g - A x_k); D = I when ``d`` is None.

    Returns (x_{k+1}, ||g - A x_k||_F)."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(G, dtype=np.float64) - blur(X, H)
    Y = blur_T(R, H, tmode)
    Z = Y if d is None else precond_apply(Y, d)
    return X + tau * Z, float(np.linalg.norm(R))


def rre(X, F):
    """Relative restoration error ||x - f||_F / ||f||_F (Sec. 4)."""
    F = np.asarray(F, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(X, dtype=np.float64) - F) / np.linalg.norm(F))


def iterate(G, H, iters, alpha=None, d=None, X0=None, tau=1.0, tmode="reblur",
            precondition=True, F_true=None):
    """Run ``iters`` steps of (D-)Landweber from x_0 (default 0).

    The preconditioner spectrum is the Tikhonov filter of the symmetrized
    PSF's eigenvalues with parameter ``alpha`` unless ``d`` is given.
    Returns a dict with the final iterate ``x``, ``resnorm[k] =
    ||g - A x_k||`` (k = 0..iters-1), ``rre[k] = RRE(x_{k+1})`` when
    ``F_true`` is given, and ``best_it`` = the first k >= 1 minimising
    RRE(x_k) (the IT of the paper's tables)."""
    G = np.asarray(G, dtype=np.float64)
    n1, n2 = G.shape
    if precondition and d is None:
        d = tikhonov(eigenvalues(H, n1, n2), alpha)
    if not precondition:
        d = None
    X = np.zeros((n1, n2)) if X0 is None else np.array(X0, dtype=np.float64)
    res, errs = [], []
    for _ in range(iters):
        X, rn = landweber_step(X, G, H, d=d, tau=tau, tmode=tmode)
        res.append(rn)
        if F_true is not None:
            errs.append(rre(X, F_true))
    out = {"x": X, "resnorm": np.array(res)}
    if F_true is not None:
        errs = np.array(errs)
        out["rre"] = errs
        out["best_it"] = int(np.argmin(errs)) + 1 if iters else 0
    return out


def observe(F, H, E, nu):
    """Data of eq. (sistema_quadrato): g = A_n f + eta with eta = nu
    ||A_n f||_F e / ||e||_F for a given standard-normal field e (white
    Gaussian noise at relative level nu, as in the experiments of Sec. 4)."""
    B = blur(F, H)
    E = np.asarray(E, dtype=np.float64)
    return B + nu * np.linalg.norm(B) / np.linalg.norm(E) * E
