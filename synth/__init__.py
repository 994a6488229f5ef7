"""Seeded synthetic inputs shared by the tests, the benchmark and the
oracle-side checks.

This module holds no arithmetic of the deblurring method itself (no blur,
no boundary extension, no transform, no filter): it only draws images,
point spread functions and standard-normal noise fields from
``numpy.random.default_rng(seed)`` (PCG64), in FP64.  Each side (the FP64
oracle and the HIP library) forms the blurred data g = A f + eta from these
pieces with its own code.

The paper's own test images and PSFs are not available; these generators
stand in for them with the structure the paper describes for its
experiments (Sec. 4): natural-image-like phantoms, Gaussian-portion and
motion-type PSFs, nonnegative and normalised to sum 1, white Gaussian noise
at a small relative level.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "phantom",
    "psf_gauss_shifted",
    "psf_motion",
    "psf_tail",
    "psf_random_gauss",
    "psf_random",
    "noise_field",
    "WORKLOADS",
    "workload",
    "batch_problem",
    "psf_mixture",
    "learned_problem",
]


def phantom(n1, n2=None, blobs=6, rects=4, seed=0):
    """Gaussian blobs plus axis-aligned rectangles, scaled to max 1."""
    n2 = n1 if n2 is None else n2
    rng = np.random.default_rng(seed)
    F = np.zeros((n1, n2))
    r = np.arange(n1, dtype=np.float64).reshape(-1, 1)
    c = np.arange(n2, dtype=np.float64).reshape(1, -1)
    for _ in range(blobs):
        c1 = rng.uniform(0.1 * n1, 0.9 * n1)
        c2 = rng.uniform(0.1 * n2, 0.9 * n2)
        s1 = rng.uniform(n1 / 40.0, n1 / 8.0)
        s2 = rng.uniform(n2 / 40.0, n2 / 8.0)
        a = rng.uniform(0.3, 1.0)
        F += a * np.exp(-((r - c1) ** 2) / (2 * s1 * s1) - ((c - c2) ** 2) / (2 * s2 * s2))
    for _ in range(rects):
        t = int(rng.integers(0, int(0.8 * n1) + 1))
        left = int(rng.integers(0, int(0.8 * n2) + 1))
        h = int(rng.integers(max(1, -(-n1 // 20)), max(2, n1 // 4) + 1))
        w = int(rng.integers(max(1, -(-n2 // 20)), max(2, n2 // 4) + 1))
        F[t:t + h, left:left + w] += rng.uniform(0.2, 0.8)
    m = F.max()
    return F / m if m > 0 else F


def _normalise(H):
    H = np.clip(H, 0.0, None)
    return H / H.sum()


def psf_gauss_shifted(q1=4, q2=4, sigma_row=2.0, sigma_col=1.0, shift=(1.0, 1.0)):
    """Non-symmetric Gaussian mask (centre shifted by ``shift`` pixels)."""
    s1 = np.arange(-q1, q1 + 1, dtype=np.float64).reshape(-1, 1)
    s2 = np.arange(-q2, q2 + 1, dtype=np.float64).reshape(1, -1)
    H = np.exp(-((s1 - shift[0]) ** 2) / (2 * sigma_row ** 2)
               - ((s2 - shift[1]) ** 2) / (2 * sigma_col ** 2))
    return _normalise(H)


def _gauss_kernel(sigma, r):
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-t * t / (2 * sigma * sigma))
    return np.outer(g, g)


def _full_conv(A, B):
    out = np.zeros((A.shape[0] + B.shape[0] - 1, A.shape[1] + B.shape[1] - 1))
    for i in range(B.shape[0]):
        for j in range(B.shape[1]):
            out[i:i + A.shape[0], j:j + A.shape[1]] += B[i, j] * A
    return out


def psf_motion(q=7, length=11.0, angle_deg=30.0, sigma=1.0, samples=1101):
    """Line of ``length`` pixels at ``angle_deg`` (from +i2 towards -i1),
    bilinearly splatted, blurred by an isotropic Gaussian of ``sigma``,
    cropped to (2q+1)^2 and normalised.  Centro-symmetric, not strongly
    symmetric."""
    size = 2 * q + 1
    big = max(size, int(np.ceil(length)) + 4) + 8
    big += (big - size) % 2          # keep the canvas centre on a pixel
    c = (big - 1) / 2.0
    L = np.zeros((big, big))
    th = np.deg2rad(angle_deg)
    for t in np.linspace(-length / 2, length / 2, samples):
        y = c - t * np.sin(th)
        x = c + t * np.cos(th)
        y0, x0 = int(np.floor(y)), int(np.floor(x))
        fy, fx = y - y0, x - x0
        L[y0, x0] += (1 - fy) * (1 - fx)
        L[y0, x0 + 1] += (1 - fy) * fx
        L[y0 + 1, x0] += fy * (1 - fx)
        L[y0 + 1, x0 + 1] += fy * fx
    r = int(np.ceil(3 * sigma))
    B = _full_conv(L, _gauss_kernel(sigma, r))
    cc = (B.shape[0] - 1) // 2
    return _normalise(B[cc - q:cc + q + 1, cc - q:cc + q + 1])


def psf_tail(q=15, tail=4.0, sigma=2.0):
    """One-sided exponential tail exp(-s1/tail) along +i1 (s1 >= 0) times a
    Gaussian of ``sigma`` across: highly non-symmetric."""
    s1 = np.arange(-q, q + 1, dtype=np.float64).reshape(-1, 1)
    s2 = np.arange(-q, q + 1, dtype=np.float64).reshape(1, -1)
    H = np.where(s1 >= 0, np.exp(-np.maximum(s1, 0) / tail), 0.0) * np.exp(-s2 * s2 / (2 * sigma * sigma))
    return _normalise(H)


def psf_random_gauss(rng, size_choices=(7, 9, 11, 13, 15, 17, 19, 21)):
    """Gaussian with random per-axis sigma in [1,4] and centre offsets in
    [-3,3] on a random odd square support (batched workload)."""
    S = int(rng.choice(size_choices))
    q = (S - 1) // 2
    sg1, sg2 = rng.uniform(1.0, 4.0, size=2)
    o1, o2 = rng.uniform(-3.0, 3.0, size=2)
    s1 = np.arange(-q, q + 1, dtype=np.float64).reshape(-1, 1)
    s2 = np.arange(-q, q + 1, dtype=np.float64).reshape(1, -1)
    H = np.exp(-((s1 - o1) ** 2) / (2 * sg1 * sg1) - ((s2 - o2) ** 2) / (2 * sg2 * sg2))
    return _normalise(H)


def psf_random(q1, q2, seed, nonneg=True):
    """Dense random mask (uniform entries), normalised: a generic
    non-symmetric PSF for operator tests."""
    rng = np.random.default_rng(seed)
    H = rng.uniform(0.0, 1.0, size=(2 * q1 + 1, 2 * q2 + 1))
    return _normalise(H) if nonneg else H / H.sum()


def noise_field(n1, n2=None, seed=0):
    """Standard-normal white field e (the caller scales it)."""
    n2 = n1 if n2 is None else n2
    return np.random.default_rng(seed).standard_normal((n1, n2))


# Named workloads (sizes, PSF families, noise levels, filter parameters).
WORKLOADS = {
    "ar64_f64_gauss9": dict(n=64, blobs=6, rects=4, seed=101, psf="gauss_shifted",
                            q=4, nu=0.01, alpha=1e-2, iters=50, dtype="f64"),
    "ar1024_f32_motion15": dict(n=1024, blobs=40, rects=20, seed=202, psf="motion",
                                q=7, nu=0.005, alpha=5e-3, iters=100, dtype="f32"),
    "ar2048_f32_tail31": dict(n=2048, blobs=40, rects=20, seed=303, psf="tail",
                              q=15, nu=0.01, alpha=5e-3, iters=200, dtype="f32"),
}


def workload(name):
    """(f, H, e, params) for a named workload."""
    p = dict(WORKLOADS[name])
    n = p["n"]
    F = phantom(n, n, p["blobs"], p["rects"], seed=p["seed"])
    if p["psf"] == "gauss_shifted":
        H = psf_gauss_shifted(p["q"], p["q"])
    elif p["psf"] == "motion":
        H = psf_motion(p["q"])
    elif p["psf"] == "tail":
        H = psf_tail(p["q"])
    else:
        raise KeyError(p["psf"])
    E = noise_field(n, n, seed=p["seed"] + 1)
    return F, H, E, p


def batch_problem(i, base_seed=404):
    """Problem ``i`` of the batched workload: square size from
    {128,192,256,384,512}, random Gaussian PSF (odd side 7..21), noise level
    in [0.1%, 2%]."""
    rng = np.random.default_rng(base_seed + i)
    n = int(rng.choice([128, 192, 256, 384, 512]))
    H = psf_random_gauss(rng)
    nu = float(rng.uniform(0.001, 0.02))
    blobs = max(4, int(round(40 * n / 1024)))
    rects = max(2, int(round(20 * n / 1024)))
    F = phantom(n, n, blobs, rects, seed=base_seed * 1000 + i)
    E = noise_field(n, n, seed=base_seed * 1000 + 500 + i)
    return F, H, E, dict(n=n, nu=nu, alpha=5e-3, iters=100)


def psf_mixture(rng, sizes=(15, 17, 19, 21, 23, 25, 27, 29, 31)):
    """Random non-symmetric PSF from three families with equal probability:
    line motion (length U[5,15], angle U[0,180), Gaussian sigma U[0.5,2]),
    one-sided exponential tail (scale U[2,6], random axis and direction,
    cross sigma U[1,3]) and a shifted Gaussian (sigma U[1,4] per axis,
    centre offsets U[-3,3]); odd square side drawn from ``sizes``."""
    S = int(rng.choice(sizes))
    q = (S - 1) // 2
    fam = int(rng.integers(0, 3))
    if fam == 0:
        length = rng.uniform(5.0, 15.0)
        angle = rng.uniform(0.0, 180.0)
        sigma = rng.uniform(0.5, 2.0)
        return psf_motion(q, length, angle, sigma, samples=401)
    if fam == 1:
        tail = rng.uniform(2.0, 6.0)
        sigma = rng.uniform(1.0, 3.0)
        H = psf_tail(q, tail, sigma)
        if rng.integers(0, 2):
            H = H[::-1, :]
        if rng.integers(0, 2):
            H = H.T
        return _normalise(np.ascontiguousarray(H))
    sg1, sg2 = rng.uniform(1.0, 4.0, size=2)
    o1, o2 = rng.uniform(-3.0, 3.0, size=2)
    s1 = np.arange(-q, q + 1, dtype=np.float64).reshape(-1, 1)
    s2 = np.arange(-q, q + 1, dtype=np.float64).reshape(1, -1)
    return _normalise(np.exp(-((s1 - o1) ** 2) / (2 * sg1 * sg1)
                             - ((s2 - o2) ** 2) / (2 * sg2 * sg2)))


def learned_problem(i, n=256, base_seed=5_000_000, sizes=(15, 17, 19, 21, 23, 25, 27, 29, 31)):
    """Problem ``i`` of the learned-filter sets: phantom (10 blobs, 5
    rectangles at 256^2, scaled with n), PSF from ``psf_mixture``, noise
    level log-uniform in [1e-3, 2e-2].  Training uses base seed 5,000,000,
    the 1024^2 inference set 6,000,000."""
    rng = np.random.default_rng(base_seed + i)
    H = psf_mixture(rng, sizes)
    nu = float(np.exp(rng.uniform(np.log(1e-3), np.log(2e-2))))
    blobs = max(4, int(round(10 * n / 256)))
    rects = max(2, int(round(5 * n / 256)))
    F = phantom(n, n, blobs, rects, seed=base_seed + 7919 * i + 1)
    E = noise_field(n, n, seed=base_seed + 7919 * i + 2)
    return F, H, E, dict(n=n, nu=nu)
