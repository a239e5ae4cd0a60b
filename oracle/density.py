"""Density-compensation filter from the interpolation matrix, in float64.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Sec. 3 offers, besides the ramp filters, a density filter: the diagonal D = Diag(D_v) whose
weights make the interpolation of the polar samples reproduce the impulse response, a constant
in Fourier space, in the least-squares sense (arg min over D_v of ||S D_v - 1||).

Readings (the paper gives no normalisation or solver):
* the constant is kappa(0)^2 = (sum_s K(s))^2, the mass of the separable gridding kernel, so that
  a unit-area weight per Cartesian cell reproduces a flat spectrum (with the kernel's K(0) = 1
  normalisation the plain "1" would shrink every weight by that factor);
* the weights keep the reflection symmetry of the polar grid, D_v(k, a) = D_v(-k, a) (the points
  k and -k at one angle are mirror images through the origin; a real image has a Hermitian
  spectrum, so only the even part of the weights acts on it, and even weights keep the filtered
  back projection real).  The frequency -L/2 of an even detector grid has no mirror sample and is
  its own partner.  The minimisation runs over such weights: CGLS on S Pi, with Pi the average of
  a vector and its mirror image, whose iterates from zero are all even;
* the least-squares problem is rank deficient (neighbouring polar samples near the origin fall
  in the same cells), so the weights are defined as CGLS from zero with a fixed iteration count;
  S D_v is unique for any exact solution and is what the pins compare;
* the filtered back projection with these weights is (L / G^2) A^T Diag(D_v): the 1D DFT of the
  sinogram (L times the adjoint's 1/L-scaled one), the weighted gridding, the inverse 2D DFT
  with its 1/G^2, and the deapodisation.
"""

from __future__ import annotations

import numpy as np

from .fubini_radon import kappa
from .solvers import cgls


def density_target(op) -> float:
    """kappa(0)^2, the mass of the separable gridding kernel."""
    return float(kappa(np.array([0.0]), op.geom)[0]) ** 2


def mirror_average(op, v: np.ndarray) -> np.ndarray:
    """Pi v: the mean of v(k, a) and v(-k, a) (oracle polar ordering a*L + k + L//2; a frequency
    whose mirror is not on the grid is left as it is)."""
    g = op.geom
    L = g.L
    w = np.asarray(v).reshape(g.n_theta, L)
    k = np.arange(L) - L // 2
    mirror = -k + L // 2
    ok = (mirror >= 0) & (mirror < L)
    out = w.copy()
    out[:, ok] = 0.5 * (w[:, ok] + w[:, mirror[ok]])
    return out.reshape(-1)


def density_weights(op, iters: int, store=None) -> np.ndarray:
    """D_v ~ arg min ||S D_v - kappa(0)^2 1|| over even weights, CGLS from zero on S Pi;
    oracle polar ordering a*L + k + L//2."""
    t = np.full(op.S.shape[0], density_target(op))
    return cgls(lambda v: op.S @ v, lambda r: mirror_average(op, op.S_dag @ r), t, iters, store=store)


def backproject_weighted(op, y: np.ndarray, w: np.ndarray) -> np.ndarray:
    """A^T with the per-polar-sample diagonal Diag(w) inserted before S."""
    g = op.geom
    Vp = op.fft1_detector_adjoint(y) * w.reshape(g.n_theta, g.L)
    return (op.kstar * op.ifft2_centered_adjoint(op.slice_adjoint(Vp))).real


def irradon_density(op, y: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Filtered back projection with the density weights: (L / G^2) A^T Diag(w) y."""
    g = op.geom
    return (g.L / float(g.G * g.G)) * backproject_weighted(op, y, w)
