"""Pins of the density filter (Sec. 3: weights D_v with S D_v close to a constant): the gridded
weights S D_v (unique for any least-squares solution) against scipy's LSQR, an independent
solver, run on S E with E an explicit basis of even weights built here from the polar
frequencies (a column per mirror pair); the weights' mirror symmetry; a residual no worse than
the unconstrained least-squares one by more than the grid's unpaired edge allows; the
polar-coordinate Jacobian (weights grow linearly with the radial index); and the filtered back
projection with these weights reconstructing a phantom about as well as the Ram-Lak filtered
one."""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import scipy.sparse as sp

from oracle import (Geometry, Operator, density_target, density_weights, irradon_density)
from synth import ellipse_params, ellipse_sinogram, rasterize_ellipses, slice_rng


@pytest.fixture(scope="module")
def op64():
    return Operator(Geometry(64, 90, 91))


def even_basis(g) -> sp.csr_matrix:
    """Columns spanning the weights with v(k, a) = v(-k, a): one column per angle and frequency
    pair {k, -k} with -k on the grid (0 <= k), one per unpaired frequency."""
    rows, cols = [], []
    col = 0
    for a in range(g.n_theta):
        for k in range(-(g.L // 2), g.L - g.L // 2):
            if k < 0 and -k <= g.L - 1 - g.L // 2:
                continue                      # counted with its partner +|k|
            rows.append(a * g.L + k + g.L // 2)
            cols.append(col)
            if k > 0:
                rows.append(a * g.L - k + g.L // 2)
                cols.append(col)
            col += 1
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(g.n_theta * g.L, col))


def test_gridded_weights_match_lsqr(op64):
    op = op64
    g = op.geom
    t = np.full(op.S.shape[0], density_target(op))
    # the least-squares problem is ill conditioned: CGLS reaches LSQR's gridded weights to
    # ~1e-3 after 1500 iterations and ~5e-4 after 5000
    v = density_weights(op, 5000)
    E = even_basis(g)
    u = sla.lsqr(op.S @ E, t, atol=1e-15, btol=1e-15, iter_lim=20000)[0]
    v2 = E @ u
    assert np.linalg.norm(op.S @ v - op.S @ v2) <= 1e-3 * np.linalg.norm(op.S @ v2)
    r1 = np.linalg.norm(op.S @ v - t)
    r2 = np.linalg.norm(op.S @ v2 - t)
    assert abs(r1 - r2) <= 1e-5 * r2
    # evenness costs little: the unconstrained minimum (LSQR stopped at its iteration limit, so
    # to 1e-5) is at most slightly lower
    v3 = sla.lsqr(op.S, t, atol=1e-15, btol=1e-15, iter_lim=20000)[0]
    r3 = np.linalg.norm(op.S @ v3 - t)
    assert r3 <= r2 * (1 + 1e-5) and r2 <= 1.01 * r3


@pytest.mark.parametrize("geom", [(64, 90, 91), (16, 12, 16), (15, 7, 21), (12, 10, 16, 20)])
def test_weights_are_mirror_symmetric(geom):
    op = Operator(Geometry(*geom))
    g = op.geom
    v = density_weights(op, 20).reshape(g.n_theta, g.L)
    for k in range(1, g.L - g.L // 2):
        np.testing.assert_array_equal(v[:, g.L // 2 + k], v[:, g.L // 2 - k])


def _weights_wrong_mirror(op, iters):
    """A plausible mistake: the mirror taken one frequency off (k paired with -k-1)."""
    from oracle import cgls
    g = op.geom
    t = np.full(op.S.shape[0], density_target(op))

    def pi(v):
        w = v.reshape(g.n_theta, g.L).copy()
        k = np.arange(g.L) - g.L // 2
        m = -k - 1 + g.L // 2
        ok = (m >= 0) & (m < g.L)
        w[:, ok] = 0.5 * (v.reshape(g.n_theta, g.L)[:, ok] + v.reshape(g.n_theta, g.L)[:, m[ok]])
        return w.reshape(-1)
    return cgls(lambda v: op.S @ v, lambda r: pi(op.S_dag @ r), t, iters)


def test_pins_reject_a_wrong_mirror():
    op = Operator(Geometry(16, 12, 16))
    g = op.geom
    t = np.full(op.S.shape[0], density_target(op))
    E = even_basis(g)
    v2 = E @ sla.lsqr(op.S @ E, t, atol=1e-15, btol=1e-15, iter_lim=20000)[0]
    good = density_weights(op, 3000)
    bad = _weights_wrong_mirror(op, 3000)
    ref = np.linalg.norm(op.S @ v2)
    assert np.linalg.norm(op.S @ good - op.S @ v2) <= 1e-3 * ref
    assert np.linalg.norm(op.S @ bad - op.S @ v2) > 1e-2 * ref


def test_weights_grow_like_the_radius(op64):
    op = op64
    g = op.geom
    v = density_weights(op, 200).reshape(g.n_theta, g.L)
    prof = np.abs(v).mean(axis=0)
    ratios = [prof[k + g.L // 2] / k for k in (8, 12, 16, 20, 24, 28, 32)]
    assert max(ratios) / min(ratios) < 1.05


def test_density_fbp_reconstructs_like_ramlak(op64):
    op = op64
    g = op.geom
    E = ellipse_params(slice_rng(7), 10, contained=True)
    th = np.arange(g.n_theta) * math.pi / g.n_theta
    P = ellipse_sinogram(E, th, g.n_p, g.n_p // 2, g.n) / (2.0 / g.n)
    truth = rasterize_ellipses(E, g.n, 4)
    x_d = irradon_density(op, P, density_weights(op, 200))
    x_r = op.irradon(P, "ramlak")
    e_d = np.linalg.norm(x_d - truth) / np.linalg.norm(truth)
    e_r = np.linalg.norm(x_r - truth) / np.linalg.norm(truth)
    assert e_d < 1.25 * e_r and e_d < 0.15
    # without the kernel-mass target the reconstruction is off by that factor
    x_unit = x_d / density_target(op)
    assert np.linalg.norm(x_unit - truth) / np.linalg.norm(truth) > 0.4
