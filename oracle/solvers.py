"""FP64 reference solvers for one slice (Sec. 2.1 and Sec. 3.1's list: SIRT, CGLS).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every solver takes the operator as two callables ``A(x) -> y`` and
``AT(y) -> x`` so that the same code runs on the sparse Fubini-Radon operator
and on small dense matrices.
"""

from __future__ import annotations

import numpy as np


def _dot(a, b) -> float:
    return float(np.vdot(np.ravel(a), np.ravel(b)).real)


def _keep(v):
    return v


def cgls(A, AT, b, iters: int, x0=None, history: bool = False, store=None):
    """Conjugate gradients on the normal equations ``A^T A x = A^T b`` (CGLS,
    Hestenes-Stiefel / Bjorck form).  Read here as textbook CGLS; the paper
    says its CGLS is "based on" conjugate gradient squared without details.

    Per iteration: ``q = A p``; ``alpha = gamma / |q|^2``; ``x += alpha p``;
    ``r -= alpha q``; ``s = A^T r``; ``gamma' = |s|^2``; ``p = s + (gamma'/gamma) p``.
    A slice whose ``|q|^2`` or ``gamma`` is zero has converged and stops moving.
    ``store`` (default: keep float64) is applied to every vector as it is stored; tests
    pass a float32 rounding to model solvers that keep their vectors in float32.
    """
    st = store or _keep
    x = np.zeros_like(AT(b)) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    x = st(x)
    r = st(b - A(x))
    s = st(AT(r))
    p = s.copy()
    gamma = _dot(s, s)
    hist = []
    for _ in range(iters):
        q = st(A(p))
        delta = _dot(q, q)
        alpha = gamma / delta if delta > 0 else 0.0
        x = st(x + alpha * p)
        r = st(r - alpha * q)
        s = st(AT(r))
        gamma_new = _dot(s, s)
        beta = gamma_new / gamma if gamma > 0 else 0.0
        p = st(s + beta * p)
        gamma = gamma_new
        if history:
            hist.append(x.copy())
    return (x, hist) if history else x


def sirt_bb(A, ATD, b, iters: int, history: bool = False, store=None):
    """SIRT as preconditioned gradient descent with a Barzilai-Borwein step
    (Sec. 3.1: Hamming preconditioning and BB-step acceleration).

    Objective ``f(x) = 1/2 <A x - b, Dtilde (A x - b)>`` whose gradient is
    ``g = ATD(A x - b)``, ``ATD`` being the back-projection with the ramp/Hamming
    diagonal ``D`` in the polar Fourier domain.  Start at ``x = 0``; the first
    step length is the exact line search ``<g, g> / <g, ATD(A g)>``; later steps
    use BB1, ``<s, s> / <s, y>`` with ``s = x_k - x_{k-1}``, ``y = g_k - g_{k-1}``
    (kept at the previous value when ``<s, y> <= 0``).  The gradient is recomputed
    from the current iterate every iteration.  ``store`` as in :func:`cgls`.
    """
    st = store or _keep
    x = np.zeros_like(ATD(b))
    x_prev = g_prev = None
    alpha = 0.0
    hist = []
    for it in range(iters):
        g = st(ATD(st(A(x) - b)))
        if it == 0:
            den = _dot(g, ATD(A(g)))
            alpha = _dot(g, g) / den if den > 0 else 0.0
        else:
            s = x - x_prev
            y = g - g_prev
            sy = _dot(s, y)
            if sy > 0:
                alpha = _dot(s, s) / sy
        x_prev, g_prev = x, g
        x = st(x - alpha * g)
        if history:
            hist.append(x.copy())
    return (x, hist) if history else x


def refine(A_hi, A_lo, AT_lo, b, outer: int, inner: int, store=None):
    """Iterative refinement: the residual ``r = b - A_hi x`` is formed with the
    accurate operator, the correction ``d`` solves ``A_lo d = r`` by ``inner``
    CGLS iterations from zero with the low-precision operator, and ``x += d``.
    ``store`` as in :func:`cgls`."""
    st = store or _keep
    x = None
    for _ in range(outer):
        r = b if x is None else st(b - A_hi(x))
        d = cgls(A_lo, AT_lo, r, inner, store=store)
        x = d if x is None else st(x + d)
    return x
