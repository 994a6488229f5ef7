"""Per-region error measure shared by the full-size parity tests."""

import numpy as np


def region_errors(Xg, Xo):
    """Relative errors of the regions where the AR arithmetic differs from
    the interior (Theorem 1's endpoint scaling and ramp, the ghost weights
    of Sec. 2.2): first and last two rows, first and last two columns, the
    four 2 x 2 corners, and the interior.  Per region: the Frobenius norm of
    the difference over max(||Xo[R]||, rms(Xo) sqrt(|R|)) (so a region whose
    values happen to be tiny is measured against the image's scale), and the
    largest absolute difference over max |Xo|."""
    n1, n2 = Xo.shape
    rms = np.linalg.norm(Xo) / np.sqrt(Xo.size)
    scale = np.max(np.abs(Xo))
    masks = {}
    m = np.zeros_like(Xo, dtype=bool); m[:2] = True; masks["top rows"] = m
    m = np.zeros_like(Xo, dtype=bool); m[-2:] = True; masks["bottom rows"] = m
    m = np.zeros_like(Xo, dtype=bool); m[:, :2] = True; masks["left cols"] = m
    m = np.zeros_like(Xo, dtype=bool); m[:, -2:] = True; masks["right cols"] = m
    m = np.zeros_like(Xo, dtype=bool)
    for a in (slice(0, 2), slice(n1 - 2, n1)):
        for b in (slice(0, 2), slice(n2 - 2, n2)):
            m[a, b] = True
    masks["corners"] = m
    m = np.ones_like(Xo, dtype=bool); m[:2] = m[-2:] = False; m[:, :2] = m[:, -2:] = False
    masks["interior"] = m
    out = {}
    for k, m in masks.items():
        dlt = Xg[m] - Xo[m]
        den = max(np.linalg.norm(Xo[m]), rms * np.sqrt(m.sum()))
        out[k] = (np.linalg.norm(dlt) / den, np.max(np.abs(dlt)) / scale)
    return out
