"""Random-ellipse / Gaussian-blob phantoms, their exact line integrals, and noise.

Conventions (shared by every consumer):

* The image is ``n x n`` pixels covering the square [-1, 1)^2 that circumscribes
  the unit disk, so the pixel size is ``delta = 2 / n``.  Pixel ``(i1, i2)`` has
  its centre at ``((i1 - n//2) * delta, (i2 - n//2) * delta)``; ``i1`` is the
  first (slow) array index and the x1 axis.
* A projection at angle ``theta`` integrates along the line
  ``x1 cos(theta) + x2 sin(theta) = t`` (the X-ray transform of Sec. 2); detector
  bin ``b`` sits at ``t = (b - c) * delta`` with ``c`` the rotation-axis bin.
* Ellipse line integrals are in physical units; Gaussian blobs are specified in
  pixel units and their line integrals are in pixel units.
"""

from __future__ import annotations

import math

import numpy as np

PIXEL_UNIT_DISK = 2.0  # the image square has side 2 (unit-disk diameter)


def slice_rng(seed: int) -> np.random.Generator:
    """PCG64 generator for one slice."""
    return np.random.default_rng(int(seed))


def ellipse_params(rng: np.random.Generator, count: int = 10, contained: bool = False) -> np.ndarray:
    """Draw ``count`` ellipses as rows ``(x1c, x2c, a, b, psi, rho)``.

    Centres are uniform in the unit disk (radius ``sqrt(U)``, angle ``2 pi U``),
    semi-axes ``U(0.05, 0.4)``, rotation ``psi ~ U(0, pi)`` (angle of the
    ``a`` axis from the x1 axis), density ``rho ~ U(0.1, 1)``, additive.
    With ``contained`` the draw is repeated until ``|centre| + max(a, b) < 0.95``,
    so that the ellipse lies inside the image and every line integral is exact.
    """
    rows = []
    while len(rows) < count:
        r = math.sqrt(rng.uniform())
        phi = 2.0 * math.pi * rng.uniform()
        a = rng.uniform(0.05, 0.4)
        b = rng.uniform(0.05, 0.4)
        psi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.1, 1.0)
        if contained and r + max(a, b) >= 0.95:
            continue
        rows.append((r * math.cos(phi), r * math.sin(phi), a, b, psi, rho))
    return np.asarray(rows, dtype=np.float64)


def rasterize_ellipses(E: np.ndarray, n: int, supersample: int = 4) -> np.ndarray:
    """Pixelise ellipses by ``supersample x supersample`` point sampling per pixel."""
    delta = PIXEL_UNIT_DISK / n
    o = n // 2
    img = np.zeros((n, n), dtype=np.float64)
    offs = ((np.arange(supersample) + 0.5) / supersample - 0.5) * delta
    for x1c, x2c, a, b, psi, rho in np.asarray(E, dtype=np.float64):
        rmax = max(a, b)
        lo1 = max(0, int(math.floor((x1c - rmax) / delta + o)) - 1)
        hi1 = min(n, int(math.ceil((x1c + rmax) / delta + o)) + 2)
        lo2 = max(0, int(math.floor((x2c - rmax) / delta + o)) - 1)
        hi2 = min(n, int(math.ceil((x2c + rmax) / delta + o)) + 2)
        if lo1 >= hi1 or lo2 >= hi2:
            continue
        x1 = (np.arange(lo1, hi1) - o) * delta - x1c
        x2 = (np.arange(lo2, hi2) - o) * delta - x2c
        cs, sn = math.cos(psi), math.sin(psi)
        acc = np.zeros((hi1 - lo1, hi2 - lo2), dtype=np.float64)
        for o1 in offs:
            d1 = (x1 + o1)[:, None]
            for o2 in offs:
                d2 = (x2 + o2)[None, :]
                u = d1 * cs + d2 * sn
                v = -d1 * sn + d2 * cs
                acc += ((u / a) ** 2 + (v / b) ** 2) <= 1.0
        img[lo1:hi1, lo2:hi2] += rho * acc / (supersample * supersample)
    return img


def ellipse_sinogram(E: np.ndarray, thetas: np.ndarray, n_p: int, center: float, n: int) -> np.ndarray:
    """Exact parallel-beam line integrals of ellipses, shape ``(n_theta, n_p)``.

    For an ellipse with semi-axes ``a, b`` rotated by ``psi`` and density
    ``rho``, the projection at angle ``theta`` and offset ``t`` is
    ``2 rho a b / s^2 * sqrt(s^2 - t'^2)`` for ``|t'| <= s``, where
    ``s^2 = a^2 cos^2(theta - psi) + b^2 sin^2(theta - psi)`` and
    ``t' = t - (x1c cos theta + x2c sin theta)`` (Kak & Slaney, 1988, Ch. 3).
    """
    delta = PIXEL_UNIT_DISK / n
    th = np.asarray(thetas, dtype=np.float64)[:, None]
    t = ((np.arange(n_p) - center) * delta)[None, :]
    out = np.zeros((th.shape[0], n_p), dtype=np.float64)
    for x1c, x2c, a, b, psi, rho in np.asarray(E, dtype=np.float64):
        s2 = (a * np.cos(th - psi)) ** 2 + (b * np.sin(th - psi)) ** 2
        tp = t - (x1c * np.cos(th) + x2c * np.sin(th))
        inside = s2 - tp * tp
        out += np.where(inside > 0, 2.0 * rho * a * b / s2 * np.sqrt(np.maximum(inside, 0.0)), 0.0)
    return out


def gaussian_blobs_image(blobs, n: int) -> np.ndarray:
    """Sum of isotropic Gaussians ``w exp(-|x - x0|^2 / (2 s^2))`` sampled at pixel
    centres, with ``x = i - n//2`` in pixel units; ``blobs`` rows are ``(x1, x2, s, w)``."""
    o = n // 2
    x1 = (np.arange(n) - o)[:, None].astype(np.float64)
    x2 = (np.arange(n) - o)[None, :].astype(np.float64)
    img = np.zeros((n, n), dtype=np.float64)
    for c1, c2, s, w in blobs:
        img += w * np.exp(-((x1 - c1) ** 2 + (x2 - c2) ** 2) / (2.0 * s * s))
    return img


def gaussian_blobs_sinogram(blobs, thetas, n_p: int, center: float) -> np.ndarray:
    """Exact line integrals (pixel units) of :func:`gaussian_blobs_image`'s blobs:
    ``w sqrt(2 pi) s exp(-(t - t0)^2 / (2 s^2))`` with ``t0 = x1 cos + x2 sin``."""
    th = np.asarray(thetas, dtype=np.float64)[:, None]
    t = (np.arange(n_p) - center)[None, :].astype(np.float64)
    out = np.zeros((th.shape[0], n_p), dtype=np.float64)
    for c1, c2, s, w in blobs:
        t0 = c1 * np.cos(th) + c2 * np.sin(th)
        out += w * math.sqrt(2.0 * math.pi) * s * np.exp(-((t - t0) ** 2) / (2.0 * s * s))
    return out


def poisson_log_sinogram(rng: np.random.Generator, P: np.ndarray, I0: float = 1e4) -> np.ndarray:
    """Beer-Lambert measurement (Sec. 2): counts ``N ~ Poisson(I0 exp(-P))`` and the
    log-normalised data ``-ln(max(N, 1) / I0)``."""
    counts = rng.poisson(I0 * np.exp(-np.asarray(P, dtype=np.float64)))
    return -np.log(np.maximum(counts, 1) / I0)


def phantom_stack(n: int, count: int, seed_base: int, supersample: int = 4,
                  n_ellipses: int = 10, contained: bool = False) -> np.ndarray:
    """``count`` random-ellipse slices, slice ``s`` drawn from seed ``seed_base + s``."""
    out = np.empty((count, n, n), dtype=np.float64)
    for s in range(count):
        E = ellipse_params(slice_rng(seed_base + s), n_ellipses, contained=contained)
        out[s] = rasterize_ellipses(E, n, supersample)
    return out
