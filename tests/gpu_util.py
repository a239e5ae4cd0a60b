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


def fp32_emulated(op: Operator):
    """The oracle operator with every input and output rounded to float32: a model of what
    float32 vector storage does to a Krylov solver (used to derive solver tolerances)."""
    def r32(v):
        return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)

    return (lambda x: r32(op.project(r32(x)))), (lambda y: r32(op.backproject(r32(y))))


def solver_tolerance(x64, x32_emulated, floor: float = 1e-5, factor: float = 4.0) -> float:
    """Allowed float32-vs-float64 iterate difference: ``factor`` times the difference the
    float32-rounded oracle itself shows, plus a floor for the kernels' own rounding."""
    return factor * rel_l2(x32_emulated, x64) + floor
