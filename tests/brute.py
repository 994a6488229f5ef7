"""Independent brute-force constructions used to pin the oracle.

None of this code is shared with the oracle: each matrix is written out
from a different passage of the paper than the one the oracle follows
(pixel-wise ghost formulas instead of the tensor extension, the printed
closed-form matrices of Sec. 3 instead of a convolution, the literal
matrices of Theorem 1 instead of a fast DST)."""

import numpy as np


def ghost_terms(a, b, n1, n2):
    """Linear form (list of (weight, i1, i2)) giving the value of the
    extended image at 0-based extended position (a, b), written case by
    case from the edge and corner formulas of Sec. 2.2 (paper index = array
    index + 1).  The fourth corner uses f_{n1, n2 - i2} (reading of the
    printed f_{n1, n1 - i2})."""
    top, bot = a < 0, a > n1 - 1
    lef, rig = b < 0, b > n2 - 1
    i1 = -a if top else (a - (n1 - 1) if bot else 0)     # paper's i1 >= 1 on a border
    i2 = -b if lef else (b - (n2 - 1) if rig else 0)
    N1, N2 = n1 - 1, n2 - 1                               # 0-based index of f_{n1}, f_{n2}
    if not (top or bot or lef or rig):
        return [(1.0, a, b)]
    if top and not (lef or rig):      # f_{1-i1,i2} = 2 f_{1,i2} - f_{i1+1,i2}
        return [(2.0, 0, b), (-1.0, i1, b)]
    if bot and not (lef or rig):      # f_{n1+i1,i2} = 2 f_{n1,i2} - f_{n1-i1,i2}
        return [(2.0, N1, b), (-1.0, N1 - i1, b)]
    if lef and not (top or bot):      # f_{i1,1-i2} = 2 f_{i1,1} - f_{i1,i2+1}
        return [(2.0, a, 0), (-1.0, a, i2)]
    if rig and not (top or bot):      # f_{i1,n2+i2} = 2 f_{i1,n2} - f_{i1,n2-i2}
        return [(2.0, a, N2), (-1.0, a, N2 - i2)]
    if top and lef:   # 4 f_{1,1} - 2 f_{1,i2+1} - 2 f_{i1+1,1} + f_{i1+1,i2+1}
        return [(4.0, 0, 0), (-2.0, 0, i2), (-2.0, i1, 0), (1.0, i1, i2)]
    if top and rig:   # 4 f_{1,n2} - 2 f_{1,n2-i2} - 2 f_{i1+1,n2} + f_{i1+1,n2-i2}
        return [(4.0, 0, N2), (-2.0, 0, N2 - i2), (-2.0, i1, N2), (1.0, i1, N2 - i2)]
    if bot and lef:   # 4 f_{n1,1} - 2 f_{n1,i2+1} - 2 f_{n1-i1,1} + f_{n1-i1,i2+1}
        return [(4.0, N1, 0), (-2.0, N1, i2), (-2.0, N1 - i1, 0), (1.0, N1 - i1, i2)]
    # bot and rig:    4 f_{n1,n2} - 2 f_{n1,n2-i2} - 2 f_{n1-i1,n2} + f_{n1-i1,n2-i2}
    return [(4.0, N1, N2), (-2.0, N1, N2 - i2), (-2.0, N1 - i1, N2), (1.0, N1 - i1, N2 - i2)]


def dense_blur(H, n1, n2):
    """Dense A_n (n1 n2 x n1 n2, row-major vec) built entry by entry from
    g_i = sum_s h_s f_{i-s} (eq. (modello_discreto)) and ``ghost_terms``."""
    q1, q2 = (H.shape[0] - 1) // 2, (H.shape[1] - 1) // 2
    A = np.zeros((n1 * n2, n1 * n2))
    for i1 in range(n1):
        for i2 in range(n2):
            row = i1 * n2 + i2
            for s1 in range(-q1, q1 + 1):
                for s2 in range(-q2, q2 + 1):
                    h = H[q1 + s1, q2 + s2]
                    for w, j1, j2 in ghost_terms(i1 - s1, i2 - s2, n1, n2):
                        A[row, j1 * n2 + j2] += h * w
    return A


def ar1d_closed(hv, n):
    """1-D AR matrix from its printed closed form (eq. (ARnosym1D)):
    first row [v_0, u^T, 0], last row [0, -(J u)^T, w_0], first column
    v_0..v_q, last column w_q..w_0, interior B = T(h) - H_TL(h_2..h_q)
    - H_BR(h_-2..h_-q).  ``hv[q + k] = h_k``."""
    q = (len(hv) - 1) // 2
    h = lambda k: hv[q + k] if -q <= k <= q else 0.0  # noqa: E731
    A = np.zeros((n, n))
    v = [h(k) + 2 * sum(h(j) for j in range(k + 1, q + 1)) for k in range(q + 1)]
    w = [h(-k) + 2 * sum(h(-j) for j in range(k + 1, q + 1)) for k in range(q + 1)]
    for k in range(q + 1):
        A[k, 0] = v[k]
        A[n - 1 - k, n - 1] = w[k]
    for j in range(1, q + 1):          # u_j = h_{-j} - h_j in column j+1 of row 1
        A[0, j] = h(-j) - h(j)
        A[n - 1, n - 1 - j] = h(j) - h(-j)   # -(J u)^T
    m = n - 2                           # B acts on rows/cols 2..n-1
    for r in range(m):
        for c in range(m):
            val = h(r - c)              # Toeplitz T([h_-q..h_q]): entry (r,c) = h_{r-c}
            if r + c + 2 <= q:          # H_TL(h_2..h_q): entry (r,c) = h_{r+c+2}
                val -= h(r + c + 2)
            rr, cc = m - 1 - r, m - 1 - c
            if rr + cc + 2 <= q:        # H_BR(h_-2..h_-q): mirrored, entry h_{-(rr+cc+2)}
                val -= h(-(rr + cc + 2))
            A[1 + r, 1 + c] = val
    return A


def ar2d_closed(H, n1, n2):
    """2-D AR matrix from its printed block form (eqs. (2d_form) and
    (2d_form_block)): the 1-D closed form at the block level, with the
    block hat-H_j the 1-D AR matrix of PSF row j."""
    q1 = (H.shape[0] - 1) // 2
    blk = {j: ar1d_closed(H[q1 + j], n2) for j in range(-q1, q1 + 1)}
    Z = np.zeros((n2, n2))
    Hb = lambda j: blk[j] if -q1 <= j <= q1 else Z  # noqa: E731
    A = np.zeros((n1 * n2, n1 * n2))

    def put(r, c, M):
        A[r * n2:(r + 1) * n2, c * n2:(c + 1) * n2] += M

    for k in range(q1 + 1):
        V = Hb(k) + 2 * sum((Hb(j) for j in range(k + 1, q1 + 1)), Z)
        W = Hb(-k) + 2 * sum((Hb(-j) for j in range(k + 1, q1 + 1)), Z)
        put(k, 0, V)
        put(n1 - 1 - k, n1 - 1, W)
    for j in range(1, q1 + 1):
        put(0, j, Hb(-j) - Hb(j))
        put(n1 - 1, n1 - 1 - j, Hb(j) - Hb(-j))
    m = n1 - 2
    for r in range(m):
        for c in range(m):
            M = Hb(r - c).copy()
            if r + c + 2 <= q1:
                M -= Hb(r + c + 2)
            rr, cc = m - 1 - r, m - 1 - c
            if rr + cc + 2 <= q1:
                M -= Hb(-(rr + cc + 2))
            put(1 + r, 1 + c, M)
    return A


def Q_matrix(m):
    """Q_m = [sqrt(2/(m+1)) sin(s t pi/(m+1))]_{s,t=1..m} (eq. (Qn))."""
    s = np.arange(1, m + 1).reshape(-1, 1)
    return np.sqrt(2.0 / (m + 1)) * np.sin(s * s.T * np.pi / (m + 1))


def T_matrices(m):
    """T_m and T~_m written out block by block from Theorem 1, with alpha
    from its defining property (unit first column of T_m)."""
    j = np.arange(1, m - 1)
    p = 1.0 - j / (m - 1)
    Jp = p[::-1]
    alpha = np.sqrt(1.0 + p @ p)
    Q = Q_matrix(m - 2)
    T = np.zeros((m, m))
    T[0, 0] = 1 / alpha
    T[m - 1, m - 1] = 1 / alpha
    T[1:m - 1, 0] = p / alpha
    T[1:m - 1, m - 1] = Jp / alpha
    T[1:m - 1, 1:m - 1] = Q
    Tt = np.zeros((m, m))
    Tt[0, 0] = alpha
    Tt[m - 1, m - 1] = alpha
    Tt[1:m - 1, 0] = -Q @ p
    Tt[1:m - 1, m - 1] = -Q @ Jp
    Tt[1:m - 1, 1:m - 1] = Q
    return T, Tt, alpha


def tau_matrix(hv, m):
    """Unilevel tau matrix of a symmetric 1-D PSF (Sec. 2.2):
    Toeplitz(v) - Hankel(sigma^2(v), J sigma^2(v)), v = [h_0..h_q, 0..]."""
    q = (len(hv) - 1) // 2
    v = np.zeros(m + 2)
    v[:q + 1] = hv[q:]
    A = np.zeros((m, m))
    for r in range(m):
        for c in range(m):
            A[r, c] = v[abs(r - c)]
            # Hankel with first column sigma^2(v) and last row J sigma^2(v)
            if r + c <= m - 1:
                A[r, c] -= v[r + c + 2]
            else:
                A[r, c] -= v[2 * m - r - c]
    return A


def bc_terms(a, b, n1, n2, bc):
    """Source pixel of 0-based extended position (a, b), written case by
    case: Reflective (Sec. 2.1) f_{1-i} = f_i, f_{n+i} = f_{n+1-i} per axis
    (corners: both reflections); Periodic f_{1-i} = f_{n+1-i},
    f_{n+i} = f_i per axis.  Returns [(1.0, i1, i2)]."""
    def one(i, n):
        if 0 <= i <= n - 1:
            return i
        if bc == "reflective":
            return -i - 1 if i < 0 else 2 * n - 1 - i      # paper 1-t -> t ; n+t -> n+1-t
        return i + n if i < 0 else i - n                  # periodic
    return [(1.0, one(a, n1), one(b, n2))]


def dense_blur_bc(H, n1, n2, bc):
    """Dense blur matrix under Reflective or Periodic BCs, entry by entry
    from g_i = sum_s h_s f_{i-s} and ``bc_terms``."""
    q1, q2 = (H.shape[0] - 1) // 2, (H.shape[1] - 1) // 2
    A = np.zeros((n1 * n2, n1 * n2))
    for i1 in range(n1):
        for i2 in range(n2):
            row = i1 * n2 + i2
            for s1 in range(-q1, q1 + 1):
                for s2 in range(-q2, q2 + 1):
                    for w, j1, j2 in bc_terms(i1 - s1, i2 - s2, n1, n2, bc):
                        A[row, j1 * n2 + j2] += H[q1 + s1, q2 + s2] * w
    return A


def reflective_1d_printed(hv, n):
    """1-D Reflective blur of a symmetric PSF in the printed form of
    Sec. 2.1: Toeplitz(v) + Hankel(sigma(v), J sigma(v)) with
    v = [h_0..h_q, 0..], sigma(v) = [h_1..h_q, 0..] the first column of the
    Hankel part and J sigma(v) its last row."""
    q = (len(hv) - 1) // 2
    v = np.zeros(n + 1)
    v[:q + 1] = hv[q:]
    sv = np.zeros(n)
    sv[:q] = hv[q + 1:]
    A = np.zeros((n, n))
    for r in range(n):
        for c in range(n):
            A[r, c] = v[abs(r - c)]
            # Hankel: entry depends on r + c; first column sv, last row J sv
            if r + c <= n - 1:
                A[r, c] += sv[r + c]
            else:
                A[r, c] += sv[::-1][r + c - (n - 1)]
    return A


def R_matrix(m):
    """The orthogonal DCT-III matrix of eq. (Rn) under this repository's
    reading: column t (0-based) is sqrt((2 - delta_{t,0}) / m)
    cos(t (s + 1/2) pi / m), s = 0..m-1."""
    s = np.arange(m).reshape(-1, 1)
    t = np.arange(m).reshape(1, -1)
    R = np.sqrt(2.0 / m) * np.cos(t * (s + 0.5) * np.pi / m)
    R[:, 0] = np.sqrt(1.0 / m)
    return R


def R_matrix_printed(m):
    """eq. (Rn) exactly as printed: [sqrt((2 - delta_{t,1}) / m)
    cos((s - 1)(t - 1/2) pi / m)]_{s,t=1..m} (not orthogonal)."""
    s = np.arange(1, m + 1).reshape(-1, 1)
    t = np.arange(1, m + 1).reshape(1, -1)
    return np.sqrt((2.0 - (t == 1)) / m) * np.cos((s - 1) * (t - 0.5) * np.pi / m)


def dft_matrix(n):
    """Unitary DFT matrix F[k, t] = exp(-2 pi i k t / n) / sqrt(n)."""
    k = np.arange(n).reshape(-1, 1)
    return np.exp(-2j * np.pi * k * k.T / n) / np.sqrt(n)
