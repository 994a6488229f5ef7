"""FP64 CPU oracle for the learned preconditioner filter.

TEST INFRASTRUCTURE ONLY (same rule as the rest of this package: only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it).

The paper regularizes the preconditioner with the Tikhonov filter of
eq. (TikFilter) applied to the eigenvalues of Theorem 2.  This module
defines the repository's learned replacement for that filter; none of it is
in the paper, so each definition below is this repository's own:

  * radial coordinate of coefficient (k1, k2):
        rho = sqrt((x1 / pi)^2 + (x2 / pi)^2) / sqrt(2)  in [0, 1),
    x_j the evaluation point of column k_j of T (the grid of Theorem 2:
    0 for the first and last column, r pi / (n - 1) inside);
    bin(k1, k2) = min(floor(64 rho), 63), decided exactly in integers;
  * features (65): the mean eigenvalue lambda per radial bin (0 for an
    empty bin), then log(nu_hat), nu_hat the noise estimate below;
  * noise estimate: L = 3x3 Laplacian (0 1 0 / 1 -4 1 / 0 1 0) of g on the
    interior pixels; sigma = MAD(L) / 0.6745 / sqrt(20) with MAD(L) =
    lmed(|L - lmed(L)|) and lmed the lower median (element of rank
    floor((N - 1) / 2) in ascending order); nu_hat = sigma sqrt(n1 n2) / ||g||_F
    (the noise of eq. (sistema_quadrato) at relative level nu has per-pixel
    standard deviation nu ||A f|| / sqrt(n1 n2));
  * network: 65 -> 128 -> 128 -> 64, ReLU, ReLU, logistic sigmoid; the flat
    parameter vector is [W1 (128 x 65), b1, W2 (128 x 128), b2, W3 (64 x 128),
    b3], each W stored (out, in) row-major; outputs are per-bin gains
    phi in [0, 1];
  * eigenvalue bins: beta_j = 10^(-4 + j / 16), j = 1..63, and
    ebin(lambda) = #{j : |lambda| >= beta_j} in [0, 63]; bin centre
    c_b = 10^(-4 + (b + 1/2) / 16);
  * gains filter: the network's outputs g_b in [0, 1] set a per-bin
    regularization a_b = 10^(-6 + 6 g_b) and d = 1 / (lambda^2 + a_ebin(lambda))
    (the Tikhonov filter with a parameter that depends on |lambda|);
  * label of a training problem: among Tikhonov (d = 1 / (lambda^2 + alpha))
    and threshold (d = 1 / lambda^2 for |lambda| >= t, else 1) filters swept
    over their parameter, the one whose run reaches the smallest RRE within
    K iterations; its label is g_b = (log10(clip(a_b, 1e-6, 1)) + 6) / 6 with
    a_b = 1 / d(c_b) - c_b^2, the regularization that reproduces the filter
    at the bin centre (Tikhonov: a_b = alpha; threshold: 0 or 1 - c_b^2);
  * loss: mean squared error over batch and bins; optimizer: Adam with bias
    correction (Kingma & Ba, 2015).
"""

from __future__ import annotations

import numpy as np

from . import ar_oracle as _ar

NB = 64
NF = NB + 1
SIZES = [(128, 65), (128, 128), (64, 128)]  # (out, in) per layer
NPARAM = sum(o * i + o for o, i in SIZES)

__all__ = [
    "NB", "NF", "NPARAM", "SIZES",
    "radial_rho", "radial_bins", "radial_profile", "laplacian", "lower_median",
    "noise_estimate", "features", "ebin_edges", "ebin_centres", "ebins", "gains_filter",
    "gains_label", "unpack",
    "bf16_round", "mlp_forward", "mlp_loss_grad", "adam_step", "sweep_label",
]


def radial_rho(n1, n2):
    """rho(k1, k2) on the coefficient grid (this repository's definition)."""
    x1 = _ar.ar_grid(n1) / np.pi
    x2 = _ar.ar_grid(n2) / np.pi
    return np.sqrt(x1[:, None] ** 2 + x2[None, :] ** 2) / np.sqrt(2.0)


def radial_bins(n1, n2):
    """bin = min(floor(64 rho), 63), decided exactly: with r_j = k_j inside
    and 0 on the first and last column, N_j = n_j - 1,
    (64 rho)^2 = S / D, S = 2048 (r1^2 N2^2 + r2^2 N1^2), D = N1^2 N2^2, and
    floor(sqrt(S / D)) = isqrt(S // D) (integers; no rounding at bin edges)."""
    def r(n):
        k = np.arange(n, dtype=np.int64)
        k[0] = 0
        k[n - 1] = 0
        return k
    N1, N2 = n1 - 1, n2 - 1
    r1, r2 = r(n1)[:, None], r(n2)[None, :]
    S = 2048 * (r1 * r1 * (N2 * N2) + r2 * r2 * (N1 * N1))
    q = S // ((N1 * N1) * (N2 * N2))
    k = np.floor(np.sqrt(q.astype(np.float64))).astype(np.int64)
    k = np.where(k * k > q, k - 1, k)
    k = np.where((k + 1) * (k + 1) <= q, k + 1, k)
    return np.minimum(k, NB - 1)


def radial_profile(V):
    """Mean of V over each radial bin of its grid (0 for empty bins)."""
    V = np.asarray(V, dtype=np.float64)
    b = radial_bins(*V.shape).ravel()
    s = np.zeros(NB)
    c = np.zeros(NB)
    np.add.at(s, b, V.ravel())
    np.add.at(c, b, 1.0)
    return np.where(c > 0, s / np.maximum(c, 1.0), 0.0)


def laplacian(G):
    """3x3 Laplacian on the interior pixels (n1 - 2) x (n2 - 2)."""
    G = np.asarray(G, dtype=np.float64)
    return (G[:-2, 1:-1] + G[2:, 1:-1] + G[1:-1, :-2] + G[1:-1, 2:]
            - 4.0 * G[1:-1, 1:-1])


def lower_median(v):
    """Element of rank floor((N - 1) / 2) of v in ascending order."""
    v = np.asarray(v, dtype=np.float64).ravel()
    k = (v.size - 1) // 2
    return float(np.partition(v, k)[k])


def noise_estimate(G):
    """nu_hat of the module docstring."""
    G = np.asarray(G, dtype=np.float64)
    L = laplacian(G)
    m = lower_median(L)
    mad = lower_median(np.abs(L - m))
    sigma = mad / 0.6745 / np.sqrt(20.0)
    return float(sigma * np.sqrt(G.size) / np.linalg.norm(G))


def features(H, G):
    """65 features of one problem: radial profile of the symmetrized PSF's
    eigenvalues (Theorem 2) and log of the noise estimate."""
    G = np.asarray(G, dtype=np.float64)
    lam = _ar.eigenvalues(H, *G.shape)
    return np.concatenate([radial_profile(lam), [np.log(noise_estimate(G))]])


def ebin_edges():
    """beta_j = 10^(-4 + j/16), j = 1..63."""
    return np.array([10.0 ** (-4.0 + j / 16.0) for j in range(1, NB)])


def ebin_centres():
    return np.array([10.0 ** (-4.0 + (b + 0.5) / 16.0) for b in range(NB)])


def ebins(lam):
    """ebin(lambda) = number of edges beta_j <= |lambda|."""
    a = np.abs(np.asarray(lam, dtype=np.float64))
    return (a[..., None] >= ebin_edges()).sum(axis=-1)


def gains_filter(lam, gains):
    """d = 1 / (lambda^2 + a_ebin(lambda)), a_b = 10^(-6 + 6 g_b)."""
    lam = np.asarray(lam, dtype=np.float64)
    a = 10.0 ** (-6.0 + 6.0 * np.asarray(gains, dtype=np.float64))
    return 1.0 / (lam * lam + a[ebins(lam)])


def gains_label(kind, param):
    """Label of a plain filter: g_b = (log10(clip(1/d(c_b) - c_b^2, 1e-6, 1)) + 6) / 6."""
    c = ebin_centres()
    if kind == "tikhonov":
        a = np.full(NB, float(param))
    elif kind == "threshold":
        a = np.where(c >= param, 0.0, 1.0 - c * c)
    else:
        raise ValueError(kind)
    return (np.log10(np.clip(a, 1e-6, 1.0)) + 6.0) / 6.0


def unpack(theta):
    """Views (W1, b1, W2, b2, W3, b3) of the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for (no, ni) in SIZES:
        out.append(theta[o:o + no * ni].reshape(no, ni))
        o += no * ni
        out.append(theta[o:o + no])
        o += no
    return out


def bf16_round(x):
    """Round FP32 values to the nearest BF16 value, ties to even (the
    network's weights are BF16 numbers)."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(theta, X):
    """Outputs (B x 64) and the pre-activations (Z1, Z2, Z3) of the
    network for inputs X (B x 65)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Z3 = H2 @ W3.T + b3
    Y = 1.0 / (1.0 + np.exp(-Z3))
    return Y, (X, Z1, H1, Z2, H2, Z3)


def mlp_loss_grad(theta, X, T):
    """Mean squared error over batch and bins and its exact gradient with
    respect to the flat parameter vector (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Y, (X, Z1, H1, Z2, H2, Z3) = mlp_forward(theta, X)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    E = Y - T
    loss = float(np.mean(E * E))
    dY = 2.0 * E / (B * NB)
    dZ3 = dY * Y * (1.0 - Y)
    gW3 = dZ3.T @ H2
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3) * (Z2 > 0)
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def sweep_label(G, H, F, alphas, thresholds, K):
    """Best plain filter of a problem: runs K D-Landweber iterations (Sec. 4)
    for every Tikhonov alpha and threshold t, keeps the (kind, parameter,
    d) whose RRE minimum is smallest (first on ties, Tikhonov before
    threshold, parameters in the given order) and returns
    (kind, param, best_rre, gains label)."""
    G = np.asarray(G, dtype=np.float64)
    lam = _ar.eigenvalues(H, *G.shape)
    best = None
    cands = [("tikhonov", a, _ar.tikhonov(lam, a)) for a in alphas]
    cands += [("threshold", t, _ar.threshold_filter(lam, t)) for t in thresholds]
    for kind, prm, d in cands:
        r = _ar.iterate(G, H, K, d=d, F_true=F)["rre"]
        r = r[np.isfinite(r)]
        e = float(r.min()) if r.size else np.inf
        if best is None or e < best[2]:
            best = (kind, prm, e)
    kind, prm, e = best
    return kind, prm, e, gains_label(kind, prm)
