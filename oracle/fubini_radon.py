"""FP64 CPU oracle of the sparse Fubini-Radon operator (Sec. 2.2 Eq. (1), Sec. 3 Eq. (2)).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library and must never be used as a fallback for it.

What is computed (all in float64, per slice, no pairing of slices):

    Radon(u)  = F1D^-1 . S^dagger . F2D . (k* o u)                  Eq. (2), first line
    A^T y     = k* o Re[ F2D^H . S . F1D^-H y ]                      exact transpose
    iRadon(y) = (pi / n_theta) k* o Re[ F2D^H . S . D . F1D^-H y ]   Eq. (2), second line

Notation.  Image ``u`` is ``n x n`` with pixel ``i = (i1, i2)`` at centred
position ``x = i - n//2`` (pixel units, ``i1`` = x1 = first index).  The
Cartesian Fourier grid has ``G x G`` points with centred frequency indices
``j in [-G//2, G-1-G//2]``.  The polar grid has ``n_theta`` angles and ``L``
radial samples ``k in [-L//2, L-1-L//2]`` per angle, with ``k = -L/2`` dropped
for even ``L``.  Detector bins ``b = 0..n_p-1`` sit at offset ``b - c`` from
the rotation axis ``c``.  Defaults: ``G = L = n_p``, ``c = n_p // 2``,
kernel width ``W = k_w = 3`` (the stencil of Fig. 3).

Readings of the paper taken here (each one is listed with its reason in the
design notes): Kaiser-Bessel kernel with the border value subtracted so that
it vanishes at the window border; the interpolation weight of grid point ``j``
for polar point ``q`` is ``K(j1 - q1) K(j2 - q2)``; the discrete deapodisation
``k* = 1 / (kappa(x1) kappa(x2))`` with ``kappa(x) = sum_s K(s) cos(2 pi s x / G)``;
out-of-band entries ``|j1|`` or ``|j2| > ceil(G/2) - 1`` are removed, which keeps
the operator exactly real-to-real.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.special import i0 as bessel_i0


# --------------------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Geometry:
    """Experimental parameters of the setup stage (Sec. 3.1): pixels, angles,
    detector bins, and the kernel choice."""

    n: int
    n_theta: int
    n_p: int
    grid: int = 0                 # G = L; 0 -> n_p
    kw: int = 3                   # kernel window width W (odd)
    beta: float = float("nan")    # Kaiser-Bessel shape; NaN -> Beatty et al. (2005) rule
    center: float = float("nan")  # rotation-axis bin c; NaN -> n_p // 2 (Sec. 3: c = n_p / 2)
    angles: tuple | None = None   # radians; None -> a * pi / n_theta

    # derived quantities -------------------------------------------------------------
    @property
    def G(self) -> int:
        return self.grid if self.grid else self.n_p

    @property
    def L(self) -> int:
        return self.G

    @property
    def c(self) -> float:
        return float(self.n_p // 2) if math.isnan(self.center) else float(self.center)

    @property
    def theta(self) -> np.ndarray:
        if self.angles is not None:
            return np.asarray(self.angles, dtype=np.float64)
        return np.arange(self.n_theta, dtype=np.float64) * math.pi / self.n_theta

    @property
    def kb_beta(self) -> float:
        if not math.isnan(self.beta):
            return float(self.beta)
        return beatty_beta(self.kw, self.G / self.n)

    @property
    def jmax(self) -> int:
        """Largest kept |j| on the Cartesian grid (symmetric band)."""
        return (self.G + 1) // 2 - 1

    def validate(self) -> None:
        if self.n < 1 or self.n_theta < 1 or self.n_p < 1:
            raise ValueError("n, n_theta and n_p must be positive")
        if self.kw < 1 or self.kw % 2 == 0:
            raise ValueError("kernel width must be odd")
        if self.G < max(self.n, self.n_p):
            raise ValueError("grid must be at least max(n, n_p)")
        if self.angles is not None and len(self.angles) != self.n_theta:
            raise ValueError("angles must have n_theta entries")


def beatty_beta(W: int, sigma: float) -> float:
    """Kaiser-Bessel shape for width ``W`` and oversampling ``sigma``
    (Beatty, Nishimura, Pauly, IEEE TMI 2005, Eq. 5)."""
    return math.pi * math.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def polar_k(geom: Geometry) -> np.ndarray:
    """Centred radial indices ``k = -L//2 .. L-1-L//2`` (index ``kk = k + L//2``)."""
    L = geom.L
    return np.arange(L, dtype=np.int64) - L // 2


def polar_kept(geom: Geometry) -> np.ndarray:
    """Boolean mask over ``kk``: False only for the unpaired Nyquist sample ``k = -L/2``."""
    k = polar_k(geom)
    keep = np.ones(geom.L, dtype=bool)
    if geom.L % 2 == 0:
        keep[k == -(geom.L // 2)] = False
    return keep


# --------------------------------------------------------------------------------------
# Kernel, deapodisation, filter (Sec. 3)
# --------------------------------------------------------------------------------------

def kernel(t, W: int, beta: float) -> np.ndarray:
    """Kaiser-Bessel convolution kernel ``K`` of width ``W``, zero at the border
    (Sec. 3: Kaiser-Bessel among the kernels named; set to 0 at the borders):
    ``K(t) = (I0(beta sqrt(1 - (2t/W)^2)) - 1) / (I0(beta) - 1)`` for ``|t| < W/2``."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    inside = np.abs(t) < W / 2.0
    arg = beta * np.sqrt(1.0 - (2.0 * t[inside] / W) ** 2)
    out[inside] = (bessel_i0(arg) - 1.0) / (bessel_i0(beta) - 1.0)
    return out


def kappa(x, geom: Geometry) -> np.ndarray:
    """Discrete transform of the kernel taps, ``sum_{s=-h..h} K(s) cos(2 pi s x / G)``;
    its reciprocal is the deapodisation factor (Sec. 3: k* = (F* K)^-1)."""
    x = np.asarray(x, dtype=np.float64)
    h = (geom.kw - 1) // 2
    out = np.zeros_like(x)
    for s in range(-h, h + 1):
        out += kernel(np.float64(s), geom.kw, geom.kb_beta) * np.cos(2.0 * math.pi * s * x / geom.G)
    return out


def deapodization(geom: Geometry) -> np.ndarray:
    """``k*(i1, i2) = 1 / (kappa(i1 - n//2) kappa(i2 - n//2))`` on the ``n x n`` support
    (zero outside it by construction of the embedding)."""
    x = np.arange(geom.n, dtype=np.float64) - geom.n // 2
    kap = kappa(x, geom)
    if np.any(kap <= 0):
        raise ValueError("deapodisation undefined: kernel transform not positive on the support")
    d = 1.0 / kap
    return d[:, None] * d[None, :]


def ramp_filter(geom: Geometry, window: str = "hamming") -> np.ndarray:
    """Diagonal ``D`` (Sec. 3: Ram-Lak, Shepp-Logan, Hamming), per centred ``k``.

    ``D_k = H_k * sum_m h(m) exp(-2 pi i k m / L)`` with the band-limited spatial
    ramp ``h(0) = 1/4``, ``h(m odd) = -1/(pi m)^2``, ``h(m even) = 0`` over the
    circular range ``m in [-L//2, L-1-L//2]`` (Kak & Slaney 1988, Eq. 61), and
    window ``H``: 1 (ramlak), ``sinc(k/L)`` (shepp), ``0.54 + 0.46 cos(2 pi k / L)``
    (hamming).  The sum is real because ``h`` is even apart from ``m = -L/2``,
    whose phase is ``(-1)^k``.
    """
    L = geom.L
    m = np.arange(L, dtype=np.float64) - L // 2
    h = np.zeros(L)
    h[m == 0] = 0.25
    odd = (np.abs(m) % 2) == 1
    h[odd] = -1.0 / (math.pi * m[odd]) ** 2
    k = polar_k(geom).astype(np.float64)
    R = np.array([np.sum(h * np.cos(2.0 * math.pi * kk * m / L)) for kk in k])
    if window == "ramlak":
        H = np.ones(L)
    elif window == "shepp":
        H = np.sinc(k / L)
    elif window == "hamming":
        H = 0.54 + 0.46 * np.cos(2.0 * math.pi * k / L)
    else:
        raise ValueError(window)
    return R * H


# --------------------------------------------------------------------------------------
# The gridding matrix S (Sec. 3, Fig. 3)
# --------------------------------------------------------------------------------------

def polar_points(geom: Geometry):
    """Polar sample positions on the Cartesian Fourier grid, shape ``(n_theta, L)``:
    ``q = k (G/L) (cos theta_a, sin theta_a)`` (Fig. 3's ``p_i (cos, sin)``, centred)."""
    th = geom.theta[:, None]
    k = polar_k(geom).astype(np.float64)[None, :]
    scale = geom.G / geom.L
    return k * scale * np.cos(th), k * scale * np.sin(th)


def build_S(geom: Geometry) -> sp.csr_matrix:
    """The sparse matrix ``S`` (M x N, Sec. 3): rows are Cartesian grid points
    ``map(j) = (j1 + G//2) G + (j2 + G//2)``, columns are polar samples
    ``a L + (k + L//2)``.  Each polar sample contributes the ``W x W`` window
    ``j = rint(q) + s`` with value ``K(j1 - q1) K(j2 - q2)``; zero-valued entries,
    out-of-band entries and the unpaired Nyquist sample are removed (Sec. 3.1)
    and the result is converted from COO to CSR with sorted indices."""
    geom.validate()
    G, L, W = geom.G, geom.L, geom.kw
    h = (W - 1) // 2
    oG = G // 2
    jmax = geom.jmax
    beta = geom.kb_beta
    q1, q2 = polar_points(geom)
    r1, r2 = np.rint(q1), np.rint(q2)                   # round half to even
    col = (np.arange(geom.n_theta)[:, None] * L + np.arange(L)[None, :])
    keep_k = np.broadcast_to(polar_kept(geom)[None, :], q1.shape)
    rows, cols, vals = [], [], []
    for s1 in range(-h, h + 1):
        j1 = r1 + s1
        w1 = kernel(j1 - q1, W, beta)
        for s2 in range(-h, h + 1):
            j2 = r2 + s2
            w = w1 * kernel(j2 - q2, W, beta)
            ok = keep_k & (np.abs(j1) <= jmax) & (np.abs(j2) <= jmax) & (w != 0.0)
            rows.append(((j1[ok] + oG) * G + (j2[ok] + oG)).astype(np.int64))
            cols.append(col[ok].astype(np.int64))
            vals.append(w[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    S = sp.coo_matrix((vals, (rows, cols)), shape=(G * G, geom.n_theta * L)).tocsr()
    S.sort_indices()
    return S


class Operator:
    """Holds ``S``, ``S^dagger`` and ``k*`` for one geometry (the setup stage, Sec. 3.1)."""

    def __init__(self, geom: Geometry, S: sp.csr_matrix | None = None):
        geom.validate()
        self.geom = geom
        self.S = build_S(geom) if S is None else S
        self.S_dag = self.S.conj().T.tocsr()
        self.S_dag.sort_indices()
        self.kstar = deapodization(geom)

    # ---- Fourier steps ---------------------------------------------------------------
    def fft2_centered(self, v: np.ndarray) -> np.ndarray:
        """``U(j) = sum_i v(i) exp(-2 pi i j . (i - n//2) / G)`` on the centred grid."""
        g = self.geom
        E = np.zeros((g.G, g.G), dtype=np.complex128)
        E[: g.n, : g.n] = v
        E = np.roll(E, (-(g.n // 2), -(g.n // 2)), axis=(0, 1))   # pixel i -> (i - n//2) mod G
        F = np.fft.fft2(E)
        return np.roll(F, (g.G // 2, g.G // 2), axis=(0, 1))       # frequency j -> j + G//2

    def ifft2_centered_adjoint(self, U: np.ndarray) -> np.ndarray:
        """Adjoint of :meth:`fft2_centered`: ``x(i) = sum_j U(j) exp(+2 pi i j . (i - n//2) / G)``."""
        g = self.geom
        Uf = np.roll(U, (-(g.G // 2), -(g.G // 2)), axis=(0, 1))
        w = np.fft.ifft2(Uf) * (g.G * g.G)
        w = np.roll(w, (g.n // 2, g.n // 2), axis=(0, 1))
        return w[: g.n, : g.n]

    def ifft1_detector(self, V: np.ndarray) -> np.ndarray:
        """``P(a, b) = (1/L) sum_k V(a, k) exp(+2 pi i k (b - c) / L)``, ``b < n_p``."""
        g = self.geom
        c0 = math.floor(g.c)
        frac = g.c - c0
        k = polar_k(g).astype(np.float64)
        Vp = V * np.exp(-2j * math.pi * k * frac / g.L)[None, :]
        Vf = np.roll(Vp, -(g.L // 2), axis=1)                      # k -> k mod L
        z = np.fft.ifft(Vf, axis=1)                                # includes 1/L
        m = (np.arange(g.n_p) - c0) % g.L
        return z[:, m]

    def fft1_detector_adjoint(self, y: np.ndarray) -> np.ndarray:
        """Adjoint of :meth:`ifft1_detector`: ``V'(a, k) = (1/L) sum_b y(a, b) exp(-2 pi i k (b - c) / L)``."""
        g = self.geom
        c0 = math.floor(g.c)
        frac = g.c - c0
        Y = np.zeros((g.n_theta, g.L), dtype=np.complex128)
        m = (np.arange(g.n_p) - c0) % g.L
        Y[:, m] = y
        Zf = np.fft.fft(Y, axis=1) / g.L
        Z = np.roll(Zf, g.L // 2, axis=1)                          # k mod L -> k + L//2
        k = polar_k(g).astype(np.float64)
        return Z * np.exp(2j * math.pi * k * frac / g.L)[None, :]

    # ---- Eq. (2) ---------------------------------------------------------------------
    def slice_forward(self, U: np.ndarray) -> np.ndarray:
        """``V = S^dagger U``: Cartesian grid ``(G, G)`` -> polar ``(n_theta, L)``."""
        g = self.geom
        return (self.S_dag @ U.reshape(-1)).reshape(g.n_theta, g.L)

    def slice_adjoint(self, V: np.ndarray) -> np.ndarray:
        """``U = S V``: polar ``(n_theta, L)`` -> Cartesian grid ``(G, G)``."""
        g = self.geom
        return (self.S @ V.reshape(-1)).reshape(g.G, g.G)

    def project_complex(self, u: np.ndarray) -> np.ndarray:
        """Radon(u) before discarding the imaginary part (exactly real for real ``u``)."""
        U = self.fft2_centered(self.kstar * u)
        V = self.slice_forward(U)
        return self.ifft1_detector(V)

    def project(self, u: np.ndarray) -> np.ndarray:
        """Forward projection ``A u``, shape ``(n_theta, n_p)`` (Eq. (2), first line)."""
        return self.project_complex(u).real

    def backproject_complex(self, y: np.ndarray, filt: np.ndarray | None = None) -> np.ndarray:
        Vp = self.fft1_detector_adjoint(y)
        if filt is not None:
            Vp = Vp * filt[None, :]
        U = self.slice_adjoint(Vp)
        return self.kstar * self.ifft2_centered_adjoint(U)

    def backproject(self, y: np.ndarray, filt: np.ndarray | None = None) -> np.ndarray:
        """Exact transpose ``A^T y`` (``filt=None``), or ``A^T`` with the polar-domain
        diagonal ``D`` inserted before ``S`` (``filt`` = D per centred ``k``)."""
        return self.backproject_complex(y, filt).real

    def irradon(self, y: np.ndarray, window: str = "hamming") -> np.ndarray:
        """iRadon / FBP (Eq. (2), second line) scaled as ``(pi / n_theta) A^T D``."""
        D = ramp_filter(self.geom, window)
        return (math.pi / self.geom.n_theta) * self.backproject(y, D)

    # ---- stacks ------------------------------------------------------------------------
    def project_stack(self, u: np.ndarray) -> np.ndarray:
        return np.stack([self.project(s) for s in u])

    def backproject_stack(self, y: np.ndarray, filt=None) -> np.ndarray:
        return np.stack([self.backproject(s, filt) for s in y])


# --------------------------------------------------------------------------------------
# Slow direct forms used as cross-checks (tiny sizes only)
# --------------------------------------------------------------------------------------

def dft2_centered_direct(v: np.ndarray, geom: Geometry) -> np.ndarray:
    """Direct double sum for the centred 2D DFT (no FFT), for pinning the FFT path."""
    j = np.arange(geom.G) - geom.G // 2
    x = np.arange(geom.n) - geom.n // 2
    E = np.exp(-2j * math.pi * np.outer(j, x) / geom.G)
    return E @ v @ E.T


def project_nudft(u: np.ndarray, geom: Geometry) -> np.ndarray:
    """Projection through the exact non-uniform DFT of the pixel image at the polar
    points (Eq. (1) without gridding): the value gridding approximates."""
    q1, q2 = polar_points(geom)
    x = np.arange(geom.n, dtype=np.float64) - geom.n // 2
    V = np.zeros(q1.shape, dtype=np.complex128)
    keep = polar_kept(geom)
    for a in range(geom.n_theta):
        E1 = np.exp(-2j * math.pi * np.outer(q1[a], x) / geom.G)   # (L, n)
        E2 = np.exp(-2j * math.pi * np.outer(q2[a], x) / geom.G)
        V[a] = np.einsum("ki,ij,kj->k", E1, u, E2)
    V[:, ~keep] = 0.0
    k = polar_k(geom).astype(np.float64)
    b = np.arange(geom.n_p, dtype=np.float64) - geom.c
    F = np.exp(2j * math.pi * np.outer(k, b) / geom.L) / geom.L     # (L, n_p)
    return (V @ F).real


def sdag_dense_direct(geom: Geometry) -> np.ndarray:
    """Dense ``S^dagger`` by looping over every polar sample and every Cartesian point
    and testing window membership one entry at a time (tiny sizes only)."""
    G, L, W = geom.G, geom.L, geom.kw
    h = (W - 1) // 2
    beta = geom.kb_beta
    q1, q2 = polar_points(geom)
    keep = polar_kept(geom)
    D = np.zeros((geom.n_theta * L, G * G))
    jr = range(-(G // 2), G - G // 2)
    for a in range(geom.n_theta):
        for kk in range(L):
            if not keep[kk]:
                continue
            c1, c2 = np.rint(q1[a, kk]), np.rint(q2[a, kk])
            for j1 in jr:
                for j2 in jr:
                    if abs(j1 - c1) > h or abs(j2 - c2) > h:
                        continue
                    if abs(j1) > geom.jmax or abs(j2) > geom.jmax:
                        continue
                    w = float(kernel(j1 - q1[a, kk], W, beta) * kernel(j2 - q2[a, kk], W, beta))
                    D[a * L + kk, (j1 + G // 2) * G + (j2 + G // 2)] = w
    return D


def project_folded(u: np.ndarray, geom: Geometry) -> np.ndarray:
    """The paper's folded form (Sec. 3, last paragraph) for ``G = L = n_p = n`` even:
    no FFT-shifts anywhere.  The deapodisation carries a +1/-1 checkerboard, the
    polar index is FFT-ordered, and the rotation-axis shift and the Fourier-space
    shift live in the phase ``Phi = (-1)^(j1 + j2) exp(2 pi i c k / n_p)`` of ``S``
    (so ``S^dagger`` carries its conjugate); plain ``fft2`` / ``ifft`` are used."""
    G, L, n = geom.G, geom.L, geom.n
    if not (G == L == n == geom.n_p and G % 2 == 0):
        raise ValueError("folded form needs G = L = n_p = n even")
    S = build_S(geom).tocoo()
    oG = G // 2
    j1 = S.row // G - oG
    j2 = S.row % G - oG
    a = S.col // L
    k = S.col % L - L // 2
    phi = ((-1.0) ** (j1 + j2)) * np.exp(2j * math.pi * geom.c * k / geom.n_p)
    kappa_fft = k % L
    S_fold = sp.coo_matrix((S.data * phi, (S.row, a * L + kappa_fft)), shape=S.shape).tocsr()
    S_fold_dag = S_fold.conj().T.tocsr()
    i = np.arange(n)
    checker = ((-1.0) ** (i[:, None] + i[None, :]))
    kstar_fold = checker * deapodization(geom)
    F = np.fft.fft2(kstar_fold * u)                                  # index g = j + G/2
    W_ = (S_fold_dag @ F.reshape(-1)).reshape(geom.n_theta, L)
    return np.fft.ifft(W_, axis=1)[:, : geom.n_p].real


# --------------------------------------------------------------------------------------
# Complex pairing (Sec. 3.1)
# --------------------------------------------------------------------------------------

def project_paired(op: Operator, u_even: np.ndarray, u_odd: np.ndarray):
    """Two real slices processed as one complex slice and split at the end."""
    P = op.project_complex(u_even + 1j * u_odd)
    return P.real, P.imag
