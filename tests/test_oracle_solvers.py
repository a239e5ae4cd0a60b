"""Pins of the oracle solvers: CGLS against a least-squares library routine,
SIRT-BB's first step against FBP (Sec. 2.1: FBP is the first step of
preconditioned steepest descent from zero), and refinement convergence."""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import Geometry, Operator, cgls, ramp_filter, refine, round_values, sirt_bb
from tests.pins import rel_l2


def test_P10_cgls_reaches_lstsq_on_dense_problem():
    rng = np.random.default_rng(10)
    M = rng.standard_normal((20, 8))
    b = rng.standard_normal(20)
    x = cgls(lambda v: M @ v, lambda v: M.T @ v, b, iters=8)
    x_ref = scipy.linalg.lstsq(M, b)[0]
    np.testing.assert_allclose(x, x_ref, rtol=1e-8, atol=1e-10)


def test_cgls_error_decreases_monotonically_in_normal_norm():
    g = Geometry(8, 12, 13)
    op = Operator(g)
    rng = np.random.default_rng(11)
    x_true = rng.uniform(0, 1, (8, 8))
    b = op.project(x_true)
    # this operator's condition number is about 440: CGLS converges in ~100 steps
    _, hist = cgls(op.project, op.backproject, b, iters=100, history=True)
    errs = [np.linalg.norm(op.project(h - x_true)) for h in hist]
    assert all(e1 <= e0 * (1 + 1e-9) + 1e-13 for e0, e1 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10 * np.linalg.norm(b)
    assert rel_l2(hist[-1], x_true) < 1e-9


def test_P9_first_sirt_bb_iterate_is_scaled_fbp():
    g = Geometry(16, 12, 23)
    op = Operator(g)
    D = ramp_filter(g, "hamming")
    b = np.random.default_rng(12).uniform(0, 1, (12, 23))
    x1 = sirt_bb(op.project, lambda y: op.backproject(y, D), b, iters=1)
    fbp = op.irradon(b, "hamming")
    ratio = np.vdot(x1, fbp) / np.vdot(fbp, fbp)
    assert ratio > 0
    np.testing.assert_allclose(x1, ratio * fbp, atol=1e-12 * np.abs(x1).max())


def test_sirt_bb_converges_to_least_squares_on_consistent_data():
    g = Geometry(8, 12, 13)
    op = Operator(g)
    D = ramp_filter(g, "hamming")
    x_true = np.random.default_rng(13).uniform(0, 1, (8, 8))
    b = op.project(x_true)
    # BB steps are not monotone; on this condition-440 problem the error falls
    # below 1e-4 within a few thousand iterations
    x = sirt_bb(op.project, lambda y: op.backproject(y, D), b, iters=3000)
    assert rel_l2(x, x_true) < 1e-4
    assert rel_l2(op.project(x), b) < 1e-6


def test_refinement_recovers_accurate_solution_from_bf16_inner_operator():
    g = Geometry(8, 12, 13)
    hi = Operator(g)
    lo = Operator(g, S=round_values(hi.S, "bf16"))
    x_true = np.random.default_rng(14).uniform(0, 1, (8, 8))
    b = hi.project(x_true)
    # converged inner solves (the operator's condition number is about 440):
    # each outer step multiplies the error by about cond * (bf16 value error)
    x_lo_only = cgls(lo.project, lo.backproject, b, iters=300)
    e_lo = rel_l2(x_lo_only, x_true)
    errs = [rel_l2(refine(hi.project, lo.project, lo.backproject, b, outer=o, inner=100), x_true)
            for o in (1, 2, 3)]
    assert 1e-4 < e_lo < 1e-2                                   # bf16 values cost accuracy
    assert errs[0] == pytest.approx(e_lo, rel=1e-6)             # one outer step = plain solve
    assert errs[1] < e_lo / 100
    assert errs[2] < errs[1] / 100


def test_irradon_scale_is_pi_over_n_theta():
    g = Geometry(16, 12, 23)
    op = Operator(g)
    y = np.random.default_rng(15).standard_normal((12, 23))
    D = ramp_filter(g, "hamming")
    np.testing.assert_allclose(op.irradon(y), math.pi / 12 * op.backproject(y, D), rtol=1e-14)
