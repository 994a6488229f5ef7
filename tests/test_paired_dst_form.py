"""The pre-weighted DST-I form that the paired FP64 row passes compute (two
rows of length m through one complex DFT of length n = m - 1), checked on
the CPU against the DST-I by definition (the oracle's Q matrix, eq. (Qn)):
with y_j = sin(pi j/n)(f_j + f_{n-j}) + (f_j - f_{n-j})/2, the DFT Y of y
gives X_{2k} = -Im Y_k and X_{2k+1} = X_{2k-1} + Re Y_k (X_{-1} = -X_1), and
the running sum over all k ends at X_n = 0.  This pins the identity the
kernel relies on, not the kernel itself (its parity is a GPU test)."""

import numpy as np
import pytest

import oracle as O


def dst_by_definition(F):
    """X_k = sum_{j=1}^{n-1} f_j sin(pi j k / n), k = 1..n-1 (rows of F hold
    f_1 .. f_{n-1}); the oracle's orthonormal DST-I times sqrt(n/2)."""
    n = F.shape[1] + 1
    return O.ar_oracle._dst1(F, 1) * np.sqrt(n / 2.0)


@pytest.mark.parametrize("n", [7, 12, 31, 1023])
def test_two_rows_through_one_complex_dft(n):
    rng = np.random.default_rng(n)
    F = rng.standard_normal((2, n - 1))
    f = np.zeros((2, n + 1))
    f[:, 1:n] = F
    j = np.arange(n)
    y = np.sin(np.pi * j / n) * (f[:, j] + f[:, n - j]) + 0.5 * (f[:, j] - f[:, n - j])
    W = np.fft.fft(y[0] + 1j * y[1])
    Wm = np.concatenate([W[:1], W[1:][::-1]])           # W_{n-k}
    half = (n - 1) // 2 + 1                             # k = 0 .. floor((n - 1) / 2)
    k = np.arange(half + (n % 2 == 0))
    k = k[k < n]
    Ya = (W[k] + np.conj(Wm[k])) / 2
    Yb = (W[k] - np.conj(Wm[k])) / 2j
    X = dst_by_definition(F)                            # X[:, k - 1] = X_k
    for row, Y in ((0, Ya), (1, Yb)):
        even = [kk for kk in k if 1 <= 2 * kk <= n - 1]
        assert np.allclose(-Y[even].imag, X[row, 2 * np.array(even) - 1], atol=1e-11)
        t = Y.real.copy()
        t[0] *= 0.5                                     # X_1 = Re Y_0 / 2
        run = np.cumsum(t)
        odd = [kk for kk in k if 2 * kk + 1 <= n - 1]
        assert np.allclose(run[odd], X[row, 2 * np.array(odd)], atol=1e-11)
        if n % 2 == 1:
            # the sum over every k <= (n - 1)/2 reaches X_n = 0
            assert abs(run[(n - 1) // 2]) < 1e-10 * np.abs(X[row]).max()
