"""Total-variation regulariser and the model-based objective, in float64.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Sec. 2 states the model-based reconstruction problem as a data misfit of the Radon transform
plus mu times a regularisation term, for which it names the total-variation norm.  The paper does
not fix a discretisation; the reading used here (and by the HIP library) is:

* forward differences with a zero difference past the last row / column,
      D1 u(i1, i2) = u(i1+1, i2) - u(i1, i2)   (i1 < n-1),   0 at i1 = n-1,
      D2 u(i1, i2) = u(i1, i2+1) - u(i1, i2)   (i2 < n-1),   0 at i2 = n-1;
* isotropic, smoothed magnitude summed over all pixels,
      TV_eps(u) = sum_i sqrt(D1 u(i)^2 + D2 u(i)^2 + eps);
* objective with an unweighted norm and no preconditioner,
      f(u) = ||A u - b||_2^2 + mu * TV_eps(u),   grad f = 2 A^T (A u - b) + mu * grad TV_eps.

The gradient of TV_eps is D^T p with p = D u / sqrt(|D u|^2 + eps), where D^T is the transpose
of the difference operator written out above (so the oracle never differentiates a formula it
does not also evaluate).
"""

from __future__ import annotations

import numpy as np


def differences(u: np.ndarray):
    """(D1 u, D2 u) for an image or a stack of images (last two axes)."""
    u = np.asarray(u, dtype=np.float64)
    d1 = np.zeros_like(u)
    d2 = np.zeros_like(u)
    d1[..., :-1, :] = u[..., 1:, :] - u[..., :-1, :]
    d2[..., :, :-1] = u[..., :, 1:] - u[..., :, :-1]
    return d1, d2


def differences_adjoint(p1: np.ndarray, p2: np.ndarray) -> np.ndarray:
    """D1^T p1 + D2^T p2 for the operator of `differences` (entries of p on the last row of p1
    and the last column of p2 are multiplied by zero differences and drop out)."""
    p1 = np.array(p1, dtype=np.float64)
    p2 = np.array(p2, dtype=np.float64)
    p1[..., -1, :] = 0.0
    p2[..., :, -1] = 0.0
    g = -p1 - p2
    g[..., 1:, :] += p1[..., :-1, :]
    g[..., :, 1:] += p2[..., :, :-1]
    return g


def tv_value(u: np.ndarray, eps: float) -> np.ndarray:
    """TV_eps per image (a scalar for one image, one value per image for a stack)."""
    d1, d2 = differences(u)
    return np.sqrt(d1 * d1 + d2 * d2 + eps).sum(axis=(-2, -1))


def tv_grad(u: np.ndarray, eps: float) -> np.ndarray:
    """Gradient of TV_eps with respect to every pixel."""
    d1, d2 = differences(u)
    m = np.sqrt(d1 * d1 + d2 * d2 + eps)
    return differences_adjoint(d1 / m, d2 / m)


def objective(op, u: np.ndarray, b: np.ndarray, mu: float, eps: float) -> float:
    """f(u) = ||A u - b||^2 + mu TV_eps(u) for one slice, A the oracle's Radon operator."""
    r = op.project(u) - b
    return float(np.vdot(r, r).real + mu * tv_value(u, eps))


def objective_grad(op, u: np.ndarray, b: np.ndarray, mu: float, eps: float) -> np.ndarray:
    """grad f = 2 A^T (A u - b) + mu grad TV_eps, A^T the oracle's exact adjoint."""
    r = op.project(u) - b
    return 2.0 * op.backproject(r) + mu * tv_grad(u, eps)
