"""Pins of the oracle's kernel, deapodisation and filter against library routines
and closed forms (Sec. 3)."""

import math

import numpy as np
import pytest

from oracle import Geometry, deapodization, kappa, kernel, polar_k, ramp_filter


@pytest.mark.parametrize("W,beta", [(3, 3.783), (3, 5.43), (5, 6.0), (7, 12.0)])
def test_kernel_peak_border_symmetry(W, beta):
    assert kernel(0.0, W, beta) == pytest.approx(1.0, abs=1e-15)
    for t in (W / 2.0, -W / 2.0, W / 2.0 + 0.1, -W):
        assert kernel(t, W, beta) == 0.0
    t = np.linspace(-W / 2, W / 2, 101)
    np.testing.assert_array_equal(kernel(t, W, beta), kernel(-t, W, beta))
    inner = kernel(np.linspace(0.0, W / 2 - 1e-9, 50), W, beta)
    assert np.all(np.diff(inner) < 0)                      # decreasing away from the centre


@pytest.mark.parametrize("W,beta,M", [(3, 3.783, 11), (3, 5.426, 31), (5, 8.0, 21)])
def test_kernel_matches_numpy_kaiser_window(W, beta, M):
    """numpy.kaiser(M, beta)[m] = I0(beta sqrt(1 - (2m/(M-1) - 1)^2)) / I0(beta) samples
    the same Bessel profile at t = W (m/(M-1) - 1/2); numpy's i0 is a separate routine."""
    win = np.kaiser(M, beta)
    t = W * (np.arange(M) / (M - 1) - 0.5)
    i0b = np.i0(beta)
    expected = (win * i0b - 1.0) / (i0b - 1.0)
    expected[0] = expected[-1] = 0.0                        # the border value is subtracted
    np.testing.assert_allclose(kernel(t, W, beta), expected, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("G,W", [(16, 3), (23, 3), (64, 5)])
def test_kappa_is_fft_of_taps(G, W):
    """kappa(x) equals the DFT of the kernel taps K(s), s = -h..h, placed on a
    length-G circle (numpy.fft), at every integer x."""
    g = Geometry(n=G, n_theta=4, n_p=G, kw=W, beta=4.0)
    h = (W - 1) // 2
    taps = np.zeros(G)
    for s in range(-h, h + 1):
        taps[s % G] = kernel(float(s), W, 4.0)
    F = np.fft.fft(taps)
    x = np.arange(-(G // 2), G - G // 2)
    np.testing.assert_allclose(kappa(x, g), F[x % G].real, atol=1e-14)
    np.testing.assert_allclose(F.imag, 0.0, atol=1e-14)


def test_deapodization_inverts_kappa_on_support():
    g = Geometry(n=20, n_theta=4, n_p=29)
    ks = deapodization(g)
    x = np.arange(20) - 10
    kap = kappa(x, g)
    np.testing.assert_allclose(ks * kap[:, None] * kap[None, :], 1.0, rtol=1e-14)


@pytest.mark.parametrize("L", [91, 724, 2048, 90])
def test_ramp_filter_approximates_frequency_ramp(L):
    """The circular band-limited ramp's transfer function approaches |k|/L; the
    truncated tail bounds the difference by about 1/(pi^2 (L/2 - 1))."""
    g = Geometry(n=L, n_theta=4, n_p=L)
    k = polar_k(g).astype(float)
    R = ramp_filter(g, "ramlak")
    bound = 2.0 / (math.pi ** 2 * (L / 2 - 1))
    assert np.max(np.abs(R - np.abs(k) / L)) < bound
    assert R[k == 0][0] > 0                                  # DC stays positive
    assert np.all(R > 0)
    H = ramp_filter(g, "hamming") / R
    np.testing.assert_allclose(H, 0.54 + 0.46 * np.cos(2 * math.pi * k / L), rtol=1e-12)
    S = ramp_filter(g, "shepp") / R
    np.testing.assert_allclose(S, np.sinc(k / L), rtol=1e-12)
