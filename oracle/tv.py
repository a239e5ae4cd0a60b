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

``split_bregman`` solves the unsmoothed problem min (mu/2)||A u - f||^2 + sum_i |D u(i)| (the
paper's TV algorithm, Sec. 3.1: TV by the split-Bregman technique of Goldstein and Osher) with
the steps of that method: the splitting d = D u with a quadratic penalty lam/2 ||d - D u - b||^2,
alternating (i) a few conjugate-gradient steps on (mu A^T A + lam D^T D) u = mu A^T f +
lam D^T (d - b) from the previous u, (ii) the isotropic shrinkage d = shrink(D u + b, 1/lam),
(iii) the Bregman update b = b + D u - d.
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


def shrink(s1: np.ndarray, s2: np.ndarray, t: float):
    """Isotropic soft threshold of the vector field (s1, s2) at t: the vector is shortened by t
    (zero if its length is at most t)."""
    mag = np.sqrt(s1 * s1 + s2 * s2)
    scale = np.where(mag > t, (mag - t) / np.where(mag > 0, mag, 1.0), 0.0)
    return scale * s1, scale * s2


def split_bregman(A, AT, f: np.ndarray, mu: float, lam: float, outer: int, inner: int,
                  store=None):
    """Split-Bregman TV reconstruction of one slice (see the module docstring).  ``A`` / ``AT``
    act on one image / sinogram; ``store`` (default identity) is applied to every stored
    vector, e.g. to model float32 storage."""
    from .normal import cg_normal

    keep = store if store is not None else (lambda v: v)
    ATf = keep(AT(f))
    u = np.zeros_like(ATf)
    d1 = np.zeros_like(u)
    d2 = np.zeros_like(u)
    b1 = np.zeros_like(u)
    b2 = np.zeros_like(u)

    def M(v):
        return mu * AT(A(v)) + lam * differences_adjoint(*differences(v))

    for _ in range(outer):
        rhs = keep(mu * ATf + lam * differences_adjoint(d1 - b1, d2 - b2))
        u = cg_normal(M, rhs, inner, x0=u, store=store)
        g1, g2 = differences(u)
        s1, s2 = g1 + b1, g2 + b2
        d1, d2 = shrink(s1, s2, 1.0 / lam)
        d1, d2 = keep(d1), keep(d2)
        b1, b2 = keep(s1 - d1), keep(s2 - d2)
    return u


def chambolle_rof(f: np.ndarray, mu: float, iters: int, tau: float = 0.125):
    """Minimiser of (mu/2)||u - f||^2 + sum_i |D u(i)| by Chambolle's dual projection algorithm
    (J. Math. Imaging Vis. 20, 2004): with div = -D^T and theta = 1/mu,
    p <- (p + tau g) / (1 + tau |g|),  g = D(div p - f / theta),  u = f - theta div p.
    An algorithm independent of ``split_bregman`` for the same denoising problem."""
    theta = 1.0 / mu
    p1 = np.zeros_like(f)
    p2 = np.zeros_like(f)
    for _ in range(iters):
        div = -differences_adjoint(p1, p2)
        g1, g2 = differences(div - f / theta)
        mag = np.sqrt(g1 * g1 + g2 * g2)
        p1 = (p1 + tau * g1) / (1.0 + tau * mag)
        p2 = (p2 + tau * g2) / (1.0 + tau * mag)
    return f + theta * differences_adjoint(p1, p2)
