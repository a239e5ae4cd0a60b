"""Helpers shared by the GPU parity tests: index maps between the library's FFT-ordered
layouts and the oracle's centred ordering, seeded inputs, and error measures."""

from __future__ import annotations

import functools

import numpy as np

from oracle import Geometry, Operator


@functools.lru_cache(maxsize=8)
def oracle_op(n, n_theta, n_p, grid=0, kw=3, center=float("nan")) -> Operator:
    return Operator(Geometry(n, n_theta, n_p, grid=grid, kw=kw, center=center))


def polar_row_map(g: Geometry) -> np.ndarray:
    """Library polar row r = k_fft * nt + a  ->  oracle row a * L + k + L//2."""
    L, nt = g.L, g.n_theta
    r = np.arange(L * nt)
    kf, a = r // nt, r % nt
    k = np.where(2 * kf < L, kf, kf - L)
    return a * L + k + L // 2


def cart_map(g: Geometry) -> np.ndarray:
    """Library Cartesian index m = j1_fft * G + j2_fft  ->  oracle (j1 + G//2) * G + j2 + G//2."""
    G = g.G
    oG = G // 2
    m = np.arange(G * G)
    j1f, j2f = m // G, m % G
    j1 = np.where(j1f <= G - 1 - oG, j1f, j1f - G)
    j2 = np.where(j2f <= G - 1 - oG, j2f, j2f - G)
    return (j1 + oG) * G + (j2 + oG)


def rel_l2(a, b) -> float:
    """Relative L2 difference |a - b| / |b| over all elements (real or complex)."""
    a = np.asarray(a)
    b = np.asarray(b)
    a = a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)
    b = b.astype(np.complex128) if np.iscomplexobj(b) else b.astype(np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def complex_channels(t) -> np.ndarray:
    """float32 tensor (P, C, 2) -> complex128 array (P, C)."""
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def r32(v):
    """Round to float32 and back (models float32 storage)."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


OP_EPS = 5e-7
"""Relative error of one float32 operator application against float64 (the operator parity
tests bound it by 1e-5 and measure about 1.5e-7 per application)."""


def noisy_fp32(fn, rng, eps: float = OP_EPS):
    """float32 model of one operator: ``fn`` on a float32-rounded input, output perturbed by
    relative noise of size ``eps`` and rounded to float32."""
    def apply(v):
        out = fn(r32(v))
        return r32(out * (1.0 + eps * rng.standard_normal(np.shape(out))))
    return apply


def krylov_tolerance(run, x64, realizations: int = 6, factor: float = 2.0, floor: float = 1e-5) -> float:
    """Tolerance for a float32 Krylov solve against its float64 oracle.  These operators are
    numerically rank-deficient, so after a few iterations float32 iterates separate from
    float64 ones in the near-null space by an amount that depends on the rounding sequence.
    ``run(rng)`` repeats the oracle solve with float32 storage and float32-level operator
    noise (:func:`noisy_fp32`); the tolerance is ``factor`` times the largest deviation over
    ``realizations`` such runs, plus ``floor``."""
    devs = [rel_l2(run(np.random.default_rng(i)), x64) for i in range(realizations)]
    return factor * max(devs) + floor
