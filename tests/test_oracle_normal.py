"""Pins of the normal operator A^T A and the reduced (Toeplitz, Sec. 4) form that drops the 1D
FFTs: the reduced form against the definition where the reduction is exact (n_p = L, integer
centre) and not where it is not (n_p < L), symmetry and positivity of A^T A, the stencil
structure of S S^dagger (a Gram matrix: symmetric, non-negative diagonal equal to the squared
column norms of S^dagger), and CG on the normal equations against a least-squares library
routine on a small dense problem and against CGLS on the operator."""

import numpy as np
import pytest
import scipy.linalg

from oracle import (Geometry, Operator, cg_normal, cgls, interpolation_product, normal,
                    normal_factored)
from tests.pins import rel_l2


@pytest.mark.parametrize("geom", [(64, 90, 91), (32, 24, 32), (37, 30, 53), (32, 24, 45, 45, 5)])
def test_reduced_form_equals_definition(geom):
    n, nt, npb = geom[:3]
    kw = geom[4] if len(geom) > 4 else 3
    op = Operator(Geometry(n, nt, npb, kw=kw))
    u = np.random.default_rng(n).uniform(0, 1, (n, n))
    # (at sigma = G/n = 1 with k_w = 5 the deapodisation spans a wide range and rounding is
    # amplified to ~1e-8; the geometries here keep sigma >= 1.4 for k_w = 5)
    assert rel_l2(normal_factored(op, u), normal(op, u)) < 1e-12


def test_reduced_form_fails_when_the_crop_drops_bins():
    op = Operator(Geometry(32, 24, 33, grid=40))          # L = 40 > n_p = 33
    u = np.random.default_rng(5).uniform(0, 1, (32, 32))
    assert rel_l2(normal_factored(op, u), normal(op, u)) > 1e-3


def test_normal_operator_symmetric_positive():
    op = Operator(Geometry(24, 20, 35))
    rng = np.random.default_rng(6)
    u, v = rng.standard_normal((2, 24, 24))
    lhs = np.vdot(v, normal(op, u))
    rhs = np.vdot(op.project(v), op.project(u))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    assert np.vdot(u, normal(op, u)) > 0


@pytest.mark.parametrize("kw", [3, 5])
def test_interpolation_product_is_a_stencil_gram_matrix(kw):
    g = Geometry(32, 40, 45, kw=kw)
    op = Operator(g)
    W = interpolation_product(op)
    G, R = g.G, kw - 1
    r, c = W.nonzero()
    d1 = c // G - r // G
    d2 = c % G - r % G
    assert np.abs(d1).max() <= R and np.abs(d2).max() <= R
    assert np.diff(W.indptr).max() <= (2 * R + 1) ** 2
    assert abs(W - W.T).max() == 0.0
    col_norm2 = np.asarray(op.S_dag.multiply(op.S_dag.conj()).sum(axis=0)).ravel().real
    np.testing.assert_allclose(W.diagonal(), col_norm2, rtol=1e-14, atol=1e-300)


def test_cg_normal_matches_lstsq_on_dense_problem():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((30, 10))
    b = rng.standard_normal(30)
    x = cg_normal(lambda v: M.T @ (M @ v), M.T @ b, iters=10)
    np.testing.assert_allclose(x, scipy.linalg.lstsq(M, b)[0], rtol=1e-8, atol=1e-10)


def test_cg_normal_tracks_cgls_on_the_operator():
    op = Operator(Geometry(16, 12, 23))
    b = op.project(np.random.default_rng(8).uniform(0, 1, (16, 16)))
    x1 = cg_normal(lambda v: normal(op, v), op.backproject(b), iters=8)
    x2 = cgls(op.project, op.backproject, b, iters=8)
    assert rel_l2(x1, x2) < 1e-8
