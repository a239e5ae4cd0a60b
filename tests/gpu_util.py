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


U32 = 2.0 ** -24


def summation_bound_check(name, got, S_o, out_map, in_lib, in_inv, l2_tol=1e-5, value_tol=1e-12):
    """Compare an SpMM output with the oracle's CSR product element by element.

    got: library-ordered (rows, C, 2) float32 product; S_o: oracle CSR (float64 values, or values
    already rounded to the kernel's 16-bit type); in_lib: the library-ordered (rows_in, C, 2)
    float32 input, whose oracle-ordered form is in_lib[in_inv]; out_map: library row -> oracle row.
    An output element summing k products v_e x_e of float32 inputs (a float32 value is the float64
    one rounded, relative error <= u; 16-bit values convert exactly) with one rounding per product
    and k - 1 additions in any order satisfies |computed - exact| <= gamma_{k+1} sum_e |v_e||x_e|,
    gamma_j = j u / (1 - j u), u = 2^-24 (Higham, Accuracy and Stability of Numerical
    Algorithms, Sec. 3.1 and 4.2), for the real and imaginary parts separately.  The library builds
    its matrix in float64 on its own: its entries agree with the oracle's to value_tol (exact
    window ties flip entries of size ~1e-13 between the builds; the host-builder tests hold both
    CSRs to 1e-12 per entry), which adds at most value_tol (k + 1) max|x| to an element (a row
    made only of such entries has a summation bound near zero).  Asserts that bound for every
    element (the binding check) and the relative L2 below l2_tol (default: the operators' parity
    tolerance, 1e-5; sums that cancel put some fp16 products near 1e-6); returns (rel L2,
    max|d|/max|ref|, worst error / bound)."""
    Xo = in_lib[in_inv].astype(np.float64)
    ref = S_o @ (Xo[..., 0] + 1j * Xo[..., 1])
    mag = abs(S_o) @ (np.abs(Xo[..., 0]) + 1j * np.abs(Xo[..., 1]))
    k = np.diff(S_o.indptr)
    ref, mag, k = ref[out_map], mag[out_map], k[out_map]
    ku = (k + 1).astype(np.float64) * U32
    gam = (ku / (1.0 - ku))[:, None]
    d_re = np.abs(got[..., 0] - ref.real)
    d_im = np.abs(got[..., 1] - ref.imag)
    xmax = float(np.max(np.abs(Xo))) if Xo.size else 0.0
    b_ties = value_tol * (k + 1).astype(np.float64)[:, None] * xmax
    b_re, b_im = gam * mag.real + b_ties, gam * mag.imag + b_ties
    ratio = max(float(np.max(d_re / np.maximum(b_re, 1e-300), initial=0.0)),
                float(np.max(d_im / np.maximum(b_im, 1e-300), initial=0.0)))
    gc = got[..., 0].astype(np.float64) + 1j * got[..., 1]
    l2 = rel_l2(gc, ref)
    mx = float(np.max(np.abs(gc - ref)) / np.max(np.abs(ref)))
    bad = int(np.count_nonzero(d_re > b_re) + np.count_nonzero(d_im > b_im))
    print(f"{name}: {got.shape[0]} rows x {got.shape[1]} channels: rel L2 {l2:.2e}, "
          f"max|d|/max|ref| {mx:.2e}, worst error / summation bound {ratio:.3f}, violations {bad}")
    assert bad == 0, (name, ratio)
    assert l2 < l2_tol, (name, l2)
    return l2, mx, ratio
