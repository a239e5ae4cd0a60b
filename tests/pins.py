"""Independent brute-force references used only to pin the oracle.

``siddon_projection`` traces every ray exactly through the pixel squares (the
piecewise-constant pixel model), with no Fourier step: it shares nothing with
the Fubini-Radon factorisation it is compared against.
"""

from __future__ import annotations

import math

import numpy as np


def ray_pixel_lengths(n: int, theta: float, t: float) -> np.ndarray:
    """Exact length of the line ``x1 cos(theta) + x2 sin(theta) = t`` inside each
    unit pixel square centred at ``(i1 - n//2, i2 - n//2)`` (slab clipping)."""
    o = n // 2
    c1 = (np.arange(n) - o)[:, None].astype(np.float64) + np.zeros((1, n))
    c2 = (np.arange(n) - o)[None, :].astype(np.float64) + np.zeros((n, 1))
    ct, st = math.cos(theta), math.sin(theta)
    # point on the line: X(s) = t (ct, st) + s (-st, ct)
    lo = np.full((n, n), -np.inf)
    hi = np.full((n, n), np.inf)
    for centre, p0, d in ((c1, t * ct, -st), (c2, t * st, ct)):
        if abs(d) < 1e-15:
            inside = (p0 >= centre - 0.5) & (p0 <= centre + 0.5)
            lo = np.where(inside, lo, np.inf)
            continue
        s_a = (centre - 0.5 - p0) / d
        s_b = (centre + 0.5 - p0) / d
        lo = np.maximum(lo, np.minimum(s_a, s_b))
        hi = np.minimum(hi, np.maximum(s_a, s_b))
    return np.maximum(hi - lo, 0.0)


def siddon_projection(u: np.ndarray, thetas, n_p: int, center: float) -> np.ndarray:
    n = u.shape[0]
    out = np.zeros((len(thetas), n_p))
    for a, th in enumerate(thetas):
        for b in range(n_p):
            out[a, b] = np.sum(u * ray_pixel_lengths(n, th, b - center))
    return out


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))
