"""Pins of the total-variation oracle and the model-based objective (Sec. 2: least squares plus
mu * Reg(u), Reg the total-variation norm).

The pins do not reuse the oracle's formulas: central finite differences of the value (an
O(h^2) check of the gradient), closed forms for a constant image, a step edge and a linear
ramp, invariance under transposition (both axes treated alike), and the objective's gradient
(which uses the adjoint) against finite differences of the objective (which uses only the
forward operator) on a 16 x 16 pixel subgrid.  Each pin is also shown to reject a plausible
mistake planted in a local copy of the oracle.
"""

import math

import numpy as np
import pytest

from oracle import Geometry, Operator, differences, objective, objective_grad, tv_grad, tv_value

EPS = 1e-8


def central_fd(f, u, h, idx):
    out = np.zeros(len(idx))
    for k, i in enumerate(idx):
        up = u.copy()
        um = u.copy()
        up[i] += h
        um[i] -= h
        out[k] = (f(up) - f(um)) / (2 * h)
    return out


def test_tv_gradient_matches_central_differences():
    rng = np.random.default_rng(21)
    u = rng.standard_normal((9, 11))
    eps = 1e-2                      # keeps the smoothed magnitude well away from its kink
    g = tv_grad(u, eps)
    idx = [(i, j) for i in range(9) for j in range(11)]
    fd = central_fd(lambda v: tv_value(v, eps), u, 1e-5, idx)
    np.testing.assert_allclose(g[tuple(np.array(idx).T)], fd, rtol=1e-6, atol=1e-8)


def test_constant_image_closed_form():
    u = np.full((7, 7), 3.25)
    assert tv_value(u, EPS) == pytest.approx(49 * math.sqrt(EPS), rel=1e-14)
    assert np.abs(tv_grad(u, EPS)).max() == 0.0


def test_step_edge_closed_form():
    n, k, jump = 10, 4, 2.5
    u = np.zeros((n, n))
    u[:, k:] = jump
    expect = n * math.sqrt(jump * jump + EPS) + (n * n - n) * math.sqrt(EPS)
    assert tv_value(u, EPS) == pytest.approx(expect, rel=1e-14)
    # edge length times jump height as eps -> 0
    assert tv_value(u, 0.0) == pytest.approx(n * jump, rel=1e-15)


def test_linear_ramp_closed_form():
    n, a, b = 8, 0.7, -1.3
    i1, i2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = a * i1 + b * i2
    expect = ((n - 1) ** 2 * math.sqrt(a * a + b * b + EPS)
              + (n - 1) * (math.sqrt(a * a + EPS) + math.sqrt(b * b + EPS)) + math.sqrt(EPS))
    assert tv_value(u, EPS) == pytest.approx(expect, rel=1e-13)


def test_transpose_invariance_and_stack_form():
    rng = np.random.default_rng(22)
    u = rng.standard_normal((3, 12, 12))
    v = tv_value(u, EPS)
    assert v.shape == (3,)
    np.testing.assert_allclose(v, tv_value(np.swapaxes(u, -1, -2), EPS), rtol=1e-13)
    np.testing.assert_allclose(tv_grad(np.swapaxes(u, -1, -2), EPS),
                               np.swapaxes(tv_grad(u, EPS), -1, -2), rtol=1e-12, atol=1e-14)
    for s in range(3):
        assert v[s] == pytest.approx(tv_value(u[s], EPS), rel=1e-15)


def test_objective_gradient_on_16x16_subgrid():
    g = Geometry(32, 24, 45)
    op = Operator(g)
    rng = np.random.default_rng(23)
    u = rng.uniform(0, 1, (32, 32))
    b = op.project(rng.uniform(0, 1, (32, 32)))
    mu, eps = 0.3, 1e-2
    grad = objective_grad(op, u, b, mu, eps)
    idx = [(8 + i, 8 + j) for i in range(16) for j in range(16)]
    fd = central_fd(lambda v: objective(op, v, b, mu, eps), u, 1e-4, idx)
    got = grad[tuple(np.array(idx).T)]
    assert np.abs(got - fd).max() <= 1e-6 * np.abs(fd).max()


# ---- the pins reject plausible mistakes (planted in local copies, never in the oracle) ----

def _tv_grad_missing_neighbour_terms(u, eps):
    d1, d2 = differences(u)
    m = np.sqrt(d1 * d1 + d2 * d2 + eps)
    return -(d1 + d2) / m


def _tv_value_one_axis_twice(u, eps):
    d1, _ = differences(u)
    return np.sqrt(2 * d1 * d1 + eps).sum(axis=(-2, -1))


def test_pins_reject_planted_mistakes():
    rng = np.random.default_rng(24)
    u = rng.standard_normal((9, 11))
    eps = 1e-2
    idx = [(i, j) for i in range(9) for j in range(11)]
    fd = central_fd(lambda v: tv_value(v, eps), u, 1e-5, idx)
    wrong = _tv_grad_missing_neighbour_terms(u, eps)[tuple(np.array(idx).T)]
    assert np.abs(wrong - fd).max() > 1e-2
    w = rng.standard_normal((12, 12))
    assert abs(_tv_value_one_axis_twice(w, EPS) - _tv_value_one_axis_twice(w.T, EPS)) > 1e-3


# ---- split-Bregman TV (Sec. 3.1) -------------------------------------------------------------

def _identity(v):
    return v


def test_split_bregman_denoising_matches_chambolle():
    """A = I: the split-Bregman iterates reach the minimiser that Chambolle's dual algorithm
    (an independent method) finds for the same ROF problem."""
    from oracle import chambolle_rof, split_bregman
    rng = np.random.default_rng(31)
    f = np.zeros((24, 24))
    f[6:18, 8:20] = 1.0
    f += 0.1 * rng.standard_normal(f.shape)
    mu = 8.0
    u_sb = split_bregman(_identity, _identity, f, mu=mu, lam=4.0, outer=400, inner=4)
    u_ch = chambolle_rof(f, mu=mu, iters=6000)
    assert np.abs(u_sb - u_ch).max() < 2e-3
    # the minimiser removes noise: closer to the clean image than the data
    clean = np.zeros_like(f)
    clean[6:18, 8:20] = 1.0
    assert np.linalg.norm(u_sb - clean) < 0.6 * np.linalg.norm(f - clean)


def test_split_bregman_constant_data_is_a_fixed_point():
    from oracle import split_bregman
    f = np.full((10, 10), 2.5)
    u = split_bregman(_identity, _identity, f, mu=3.0, lam=2.0, outer=5, inner=5)
    np.testing.assert_allclose(u, f, rtol=1e-12)


def test_split_bregman_small_tv_weight_gives_least_squares():
    """With the data term weighted 1e12 times the TV term the minimiser is the least-squares
    solution (here of a well-determined tomography problem; at 1e8 the TV term still moves the
    minimiser by ~2e-5 along the operator's weakest directions, condition number ~440)."""
    from oracle import split_bregman
    op = Operator(Geometry(8, 12, 13))
    rng = np.random.default_rng(32)
    x_true = rng.uniform(0, 1, (8, 8))
    f = op.project(x_true)
    u = split_bregman(op.project, op.backproject, f, mu=1e12, lam=1.0, outer=3, inner=60)
    assert np.linalg.norm(u - x_true) < 1e-6 * np.linalg.norm(x_true)


def test_shrink_closed_form():
    from oracle import shrink
    s1 = np.array([3.0, 0.0, 0.3, 0.0])
    s2 = np.array([4.0, 0.0, 0.4, -2.0])
    d1, d2 = shrink(s1, s2, 1.0)
    np.testing.assert_allclose(d1, [2.4, 0.0, 0.0, 0.0])
    np.testing.assert_allclose(d2, [3.2, 0.0, 0.0, -1.0])
