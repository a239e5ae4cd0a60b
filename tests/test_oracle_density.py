"""Pins of the density filter (Sec. 3: weights D_v with S D_v close to a constant): the gridded
weights S D_v (unique for any least-squares solution) against scipy's LSQR, an independent
solver; the polar-coordinate Jacobian (weights grow linearly with the radial index); and the
filtered back projection with these weights reconstructing a phantom about as well as the
Ram-Lak filtered one."""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import (Geometry, Operator, density_target, density_weights, irradon_density)
from synth import ellipse_params, ellipse_sinogram, rasterize_ellipses, slice_rng


@pytest.fixture(scope="module")
def op64():
    return Operator(Geometry(64, 90, 91))


def test_gridded_weights_match_lsqr(op64):
    op = op64
    t = np.full(op.S.shape[0], density_target(op))
    # the least-squares problem is ill conditioned: CGLS reaches LSQR's gridded weights to
    # 2e-3 after 1500 iterations and 6e-4 after 5000
    v = density_weights(op, 5000)
    v2 = sla.lsqr(op.S, t, atol=1e-15, btol=1e-15, iter_lim=20000)[0]
    assert np.linalg.norm(op.S @ v - op.S @ v2) <= 1e-3 * np.linalg.norm(op.S @ v2)
    r1 = np.linalg.norm(op.S @ v - t)
    r2 = np.linalg.norm(op.S @ v2 - t)
    assert abs(r1 - r2) <= 1e-5 * r2


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
