"""Checks of the input generators against closed forms (areas, projection mass)."""

import math

import numpy as np

from synth import (
    ellipse_params,
    ellipse_sinogram,
    poisson_log_sinogram,
    rasterize_ellipses,
    slice_rng,
)


def test_ellipse_raster_mass_matches_area():
    E = ellipse_params(slice_rng(30), 4, contained=True)
    n = 256
    img = rasterize_ellipses(E, n, 4)
    mass = img.sum() * (2.0 / n) ** 2
    exact = float(np.sum(E[:, 5] * math.pi * E[:, 2] * E[:, 3]))
    assert abs(mass - exact) / exact < 5e-3


def test_ellipse_projection_mass_is_angle_independent():
    E = ellipse_params(slice_rng(31), 10, contained=True)
    n, n_p = 512, 725
    th = np.linspace(0, math.pi, 17, endpoint=False)
    P = ellipse_sinogram(E, th, n_p, n_p // 2, n)
    exact = float(np.sum(E[:, 5] * math.pi * E[:, 2] * E[:, 3]))
    np.testing.assert_allclose(P.sum(axis=1) * (2.0 / n), exact, rtol=2e-4)


def test_poisson_log_data_is_unbiased_at_high_counts():
    P = np.full((200, 200), 0.7)
    b = poisson_log_sinogram(np.random.default_rng(32), P, I0=1e6)
    assert abs(b.mean() - 0.7) < 1e-3
    assert abs(b.std() - math.sqrt(math.exp(0.7) / 1e6)) < 1e-4


def test_ellipse_draw_statistics():
    E = np.concatenate([ellipse_params(slice_rng(s), 10) for s in range(50)])
    assert np.all(np.hypot(E[:, 0], E[:, 1]) <= 1.0)
    assert np.all((E[:, 2] >= 0.05) & (E[:, 2] <= 0.4) & (E[:, 3] >= 0.05) & (E[:, 3] <= 0.4))
    assert np.all((E[:, 5] >= 0.1) & (E[:, 5] <= 1.0))
