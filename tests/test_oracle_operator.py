"""Pins of the oracle's Fubini-Radon operator (Sec. 2.2 Eq. (1), Sec. 3 Eq. (2)) against
invariants, brute force, closed forms and the paper's folded form."""

import math

import numpy as np
import pytest

from oracle import (
    Geometry,
    Operator,
    build_S,
    dft2_centered_direct,
    kernel,
    polar_k,
    polar_points,
    project_folded,
    project_nudft,
    project_paired,
    sdag_dense_direct,
)
from synth import (
    ellipse_params,
    ellipse_sinogram,
    gaussian_blobs_image,
    gaussian_blobs_sinogram,
    rasterize_ellipses,
    slice_rng,
)
from tests.pins import rel_l2, siddon_projection

GEOMS = [
    Geometry(16, 12, 23),                      # odd n_p, n < n_p
    Geometry(16, 12, 16),                      # even, G = n
    Geometry(15, 7, 21),                       # odd n
    Geometry(12, 10, 16, grid=20),             # padded grid G = L > n_p
    Geometry(16, 9, 23, center=10.0),          # off-centre integer axis
    Geometry(16, 9, 23, center=11.3),          # non-integer axis
    Geometry(14, 5, 20, angles=(0.1, 0.7, 1.3, 2.0, 2.9)),
]


def _ids(g):
    return f"n{g.n}_t{g.n_theta}_p{g.n_p}_G{g.G}_c{g.c}"


@pytest.mark.parametrize("g", GEOMS, ids=_ids)
def test_P1_adjoint_dot_product(g):
    op = Operator(g)
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal((g.n, g.n))
        y = rng.standard_normal((g.n_theta, g.n_p))
        lhs = np.vdot(op.project(x), y)
        rhs = np.vdot(x, op.backproject(y))
        assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("g", GEOMS, ids=_ids)
def test_P2_real_input_gives_real_projection(g):
    op = Operator(g)
    x = np.random.default_rng(2).standard_normal((g.n, g.n))
    P = op.project_complex(x)
    assert np.abs(P.imag).max() <= 1e-13 * np.abs(P.real).max()
    y = np.random.default_rng(3).standard_normal((g.n_theta, g.n_p))
    B = op.backproject_complex(y)
    assert np.abs(B.imag).max() <= 1e-13 * np.abs(B.real).max()


@pytest.mark.parametrize("g", [g for g in GEOMS if g.G == g.n_p], ids=_ids)
def test_P3_mass_conservation_per_angle(g):
    """With L = n_p the detector sum of every projection equals the image sum."""
    op = Operator(g)
    x = np.random.default_rng(4).uniform(0, 1, (g.n, g.n))
    P = op.project(x)
    np.testing.assert_allclose(P.sum(axis=1), x.sum(), rtol=1e-13)


@pytest.mark.parametrize("g", [g for g in GEOMS if g.G == g.n_p], ids=_ids)
def test_P4_backprojection_of_ones(g):
    op = Operator(g)
    bp = op.backproject(np.ones((g.n_theta, g.n_p)))
    np.testing.assert_allclose(bp, g.n_theta, rtol=1e-13)


@pytest.mark.parametrize("n,n_p", [(16, 16), (16, 23), (21, 31)])
def test_P5_zero_angle_is_dft_of_column_sums(n, n_p):
    """At theta = 0 the polar samples are on-grid along j1, and the gridded slice
    equals the 1D DFT (along x1) of the sums over x2 wherever the whole window
    lies inside the band."""
    g = Geometry(n, 4, n_p)
    op = Operator(g)
    u = np.random.default_rng(5).standard_normal((n, n))
    V = op.slice_forward(op.fft2_centered(op.kstar * u))[0]
    k = polar_k(g)
    x1 = np.arange(n) - n // 2
    colsum = u.sum(axis=1)
    ref = np.array([np.sum(colsum * np.exp(-2j * math.pi * kk * x1 / g.G)) for kk in k])
    inner = np.abs(k) <= g.jmax - (g.kw - 1) // 2
    np.testing.assert_allclose(V[inner], ref[inner], atol=1e-12 * np.abs(ref).max())
    # the angle pi/2 sums along x1 instead
    u2 = u.T.copy()
    V90 = op.slice_forward(op.fft2_centered(op.kstar * u2))[2]
    np.testing.assert_allclose(V90[inner], ref[inner], atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("n,n_theta,c", [(16, 8, 8), (16, 11, 5), (24, 7, 13)])
def test_P6_folded_form_equals_centred_form(n, n_theta, c):
    g = Geometry(n, n_theta, n, center=float(c))
    u = np.random.default_rng(6).standard_normal((n, n))
    np.testing.assert_allclose(project_folded(u, g), Operator(g).project(u), atol=1e-12)


def test_P7_direct_dft_equals_fft_path():
    for g in (Geometry(8, 4, 11), Geometry(9, 4, 9), Geometry(6, 4, 8, grid=12)):
        op = Operator(g)
        v = np.random.default_rng(7).standard_normal((g.n, g.n))
        np.testing.assert_allclose(op.fft2_centered(v), dft2_centered_direct(v, g), atol=1e-11)


@pytest.mark.parametrize("g", [Geometry(10, 6, 13), Geometry(8, 5, 8), Geometry(9, 7, 9, kw=5)], ids=_ids)
def test_P7_dense_direct_construction_equals_csr(g):
    dense = sdag_dense_direct(g)
    np.testing.assert_array_equal(dense, Operator(g).S_dag.toarray())


def _blobs():
    return [(5.0, -7.0, 4.0, 1.0), (-10.0, 3.0, 3.0, 0.5), (0.0, 12.0, 5.0, 0.8)]


def test_P7_gridding_approaches_exact_slice_as_kernel_widens():
    """Against the exact non-uniform DFT (no gridding) the gridded projection has
    the gridding error of the kernel: about 1e-2 for W=3 and far less for wider
    kernels, so the windows and weights converge to the true slice."""
    u = gaussian_blobs_image(_blobs(), 64)
    errs = {}
    for W, beta in ((3, float("nan")), (5, 12.0), (7, 12.0)):
        g = Geometry(64, 90, 91, kw=W, beta=beta)
        errs[W] = rel_l2(Operator(g).project(u), project_nudft(u, g))
    assert errs[3] < 1.5e-2
    assert errs[5] < 1e-4
    assert errs[7] < 5e-5
    assert errs[5] < errs[3] / 50


def test_P7_nudft_matches_analytic_gaussians():
    """The exact slice itself reproduces the analytic line integrals of smooth
    blobs; this pins the geometry (axes, angle direction, centre, scale)."""
    g = Geometry(64, 90, 91)
    u = gaussian_blobs_image(_blobs(), 64)
    Pa = gaussian_blobs_sinogram(_blobs(), g.theta, g.n_p, g.c)
    assert rel_l2(project_nudft(u, g), Pa) < 1e-4


def test_P7_siddon_ray_tracing_agrees_within_discretisation():
    g = Geometry(32, 24, 45)
    E = ellipse_params(slice_rng(11), 6, contained=True)
    u = rasterize_ellipses(E, 32, 4)
    P_sid = siddon_projection(u, g.theta, g.n_p, g.c)
    assert rel_l2(Operator(g).project(u), P_sid) < 4e-2
    ub = gaussian_blobs_image([(3.0, -4.0, 3.0, 1.0), (-5.0, 2.0, 2.5, 0.6)], 32)
    assert rel_l2(Operator(g).project(ub), siddon_projection(ub, g.theta, g.n_p, g.c)) < 2e-2


def test_P8_analytic_gaussians_and_ellipses():
    g = Geometry(64, 90, 91)
    op = Operator(g)
    u = gaussian_blobs_image(_blobs(), 64)
    assert rel_l2(op.project(u), gaussian_blobs_sinogram(_blobs(), g.theta, g.n_p, g.c)) < 1.5e-2
    errs = []
    for n, n_p in ((64, 91), (128, 181)):
        gg = Geometry(n, 90, n_p)
        E = ellipse_params(slice_rng(5), 10, contained=True)
        ue = rasterize_ellipses(E, n, 4)
        Pa = ellipse_sinogram(E, gg.theta, n_p, gg.c, n) / (2.0 / n)      # physical -> pixel units
        errs.append(rel_l2(Operator(gg).project(ue), Pa))
    assert errs[0] < 3e-2
    assert errs[1] < errs[0]


def test_R7_mirrored_stencil_reading_is_wrong():
    """Read literally, S_val = K(frac + s) weights the far side of the window;
    against the exact slice that reading is an order of magnitude worse than
    K(j - q), so the literal formula is taken as a garble."""
    g = Geometry(64, 90, 91)
    u = gaussian_blobs_image(_blobs(), 64)
    op = Operator(g)
    S = build_S(g).tocoo()
    G, L = g.G, g.L
    j1 = S.row // G - G // 2
    j2 = S.row % G - G // 2
    q1, q2 = polar_points(g)
    a, kk = S.col // L, S.col % L
    f1 = q1[a, kk] - np.rint(q1[a, kk])
    f2 = q2[a, kk] - np.rint(q2[a, kk])
    s1 = j1 - np.rint(q1[a, kk])
    s2 = j2 - np.rint(q2[a, kk])
    beta = g.kb_beta
    mirrored = kernel(s1 + f1, 3, beta) * kernel(s2 + f2, 3, beta)
    import scipy.sparse as sp
    Sm = sp.csr_matrix((mirrored, (S.row, S.col)), shape=S.shape)
    err_ok = rel_l2(op.project(u), project_nudft(u, g))
    err_mirror = rel_l2(Operator(g, S=Sm).project(u), project_nudft(u, g))
    assert err_mirror > 10 * err_ok


@pytest.mark.parametrize("g", [Geometry(16, 12, 23), Geometry(16, 12, 16), Geometry(12, 10, 16, grid=20)], ids=_ids)
def test_S_structure(g):
    """At most n_theta n_p k_w^2 entries (Sec. 3), S is exactly the transpose of
    S^dagger, no stored zeros, sorted columns, and the window set is point
    symmetric: entry (a, k, j) exists iff (a, -k, -j) does, with equal value."""
    op = Operator(g)
    S = op.S
    assert S.nnz <= g.n_theta * g.L * g.kw ** 2
    assert np.all(S.data != 0)
    assert S.has_sorted_indices
    assert (abs(op.S_dag - S.T)).max() == 0
    C = S.tocoo()
    G, L = g.G, g.L
    j1 = C.row // G - G // 2
    j2 = C.row % G - G // 2
    a, k = C.col // L, C.col % L - L // 2
    key = {(int(aa), int(kk), int(x1), int(x2)): v for aa, kk, x1, x2, v in zip(a, k, j1, j2, C.data)}
    for (aa, kk, x1, x2), v in key.items():
        assert key[(aa, -kk, -x1, -x2)] == v


def test_P11_complex_pairing_is_exact():
    g = Geometry(16, 12, 23)
    op = Operator(g)
    rng = np.random.default_rng(8)
    u0, u1 = rng.standard_normal((2, 16, 16))
    p0, p1 = project_paired(op, u0, u1)
    np.testing.assert_allclose(p0, op.project(u0), atol=1e-13)
    np.testing.assert_allclose(p1, op.project(u1), atol=1e-13)


def test_integer_axis_shift_is_a_detector_shift():
    g0 = Geometry(16, 9, 23, center=11.0)
    g1 = Geometry(16, 9, 23, center=12.0)
    u = np.random.default_rng(9).standard_normal((16, 16))
    P0 = Operator(g0).project(u)
    P1 = Operator(g1).project(u)
    np.testing.assert_allclose(P1[:, 1:], P0[:, :-1], atol=1e-12)


def test_fbp_reconstructs_phantom():
    """iRadon = (pi/n_theta) A^T D of the exact sinogram recovers the phantom to
    the accuracy expected of filtered back-projection, improving with size."""
    errs = []
    for n, n_theta, n_p in ((64, 90, 91), (128, 180, 181)):
        g = Geometry(n, n_theta, n_p)
        E = ellipse_params(slice_rng(21), 10, contained=True)
        u = rasterize_ellipses(E, n, 4)
        Pa = ellipse_sinogram(E, g.theta, n_p, g.c, n) / (2.0 / n)
        errs.append(rel_l2(Operator(g).irradon(Pa), u))
    assert errs[0] < 0.2
    assert errs[1] < errs[0]
