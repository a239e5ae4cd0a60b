"""The normal operator A^T A and the interpolation product S S^dagger, in float64.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Sec. 4 proposes a Toeplitz approach that combines the transform with its adjoint in one
operation and avoids the two 1D FFTs.  For this discretisation the reduction is exact when the
detector has as many bins as polar samples per angle (n_p = L) and the rotation centre is an
integer: the crop to n_p bins is then a bijection of the L inverse-DFT outputs, the 1D inverse
transform followed by its adjoint is 1/L times the identity on the kept radial indices, and

    A^T A u = (1/L) k* . F2D^H (S S^dagger) F2D (k* . u).

W = S S^dagger connects Cartesian points that share a polar sample, so its rows hold at most
(2 k_w - 1)^2 entries at offsets |d1|, |d2| <= k_w - 1.  ``normal`` is the definition (the full
operator followed by its exact adjoint); ``normal_factored`` is the reduced form, pinned against
the definition in the tests.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def normal(op, u: np.ndarray, filt: np.ndarray | None = None) -> np.ndarray:
    """A^T A u (or A^T D A u with the polar-domain diagonal ``filt``), by definition."""
    return op.backproject(op.project(u), filt)


def interpolation_product(op) -> sp.csr_matrix:
    """W = S S^dagger (G^2 x G^2, the oracle's centred Cartesian ordering)."""
    W = (op.S @ op.S_dag).tocsr()
    W.sort_indices()
    return W


def normal_factored(op, u: np.ndarray, W: sp.csr_matrix | None = None) -> np.ndarray:
    """(1/L) k* F2D^H W F2D (k* u): equal to ``normal`` when n_p = L and the centre is an
    integer."""
    g = op.geom
    if W is None:
        W = interpolation_product(op)
    U = op.fft2_centered(op.kstar * u)
    Z = (W @ U.reshape(-1)).reshape(g.G, g.G) / g.L
    return (op.kstar * op.ifft2_centered_adjoint(Z)).real


def cg_normal(T, rhs: np.ndarray, iters: int, x0: np.ndarray | None = None, store=None):
    """Conjugate gradients on T x = rhs for a symmetric positive semi-definite T (the normal
    equations A^T A x = A^T b; in exact arithmetic the iterates equal CGLS's).  ``store`` (default
    identity) is applied to every stored vector, e.g. to model float32 storage."""
    keep = store if store is not None else (lambda v: v)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.float64)
    r = keep(rhs - T(x)) if x0 is not None else keep(np.array(rhs, dtype=np.float64))
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    for _ in range(iters):
        if rr == 0.0:
            break
        q = T(p)
        pq = float(np.vdot(p, q).real)
        if pq <= 0.0:
            break
        a = rr / pq
        x = keep(x + a * p)
        r = keep(r - a * q)
        rr_new = float(np.vdot(r, r).real)
        p = keep(r + (rr_new / rr) * p)
        rr = rr_new
    return x
