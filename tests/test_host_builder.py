"""The C++ setup stage (host-only operator, no GPU) against the oracle: the CSR matrices,
deapodisation factors, filter diagonals and row bins, compared by value (Sec. 3, Sec. 3.1)."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2003_12677_amd as tomo
from oracle import Geometry, Operator, beatty_beta, deapodization, ramp_filter

GEOMS = [
    dict(n=16, n_angles=12, n_det=23),
    dict(n=16, n_angles=12, n_det=16),
    dict(n=15, n_angles=7, n_det=21),
    dict(n=12, n_angles=10, n_det=16, grid=20),
    dict(n=16, n_angles=9, n_det=23, center=10.0),
    dict(n=9, n_angles=7, n_det=9, kw=5),
    dict(n=64, n_angles=90, n_det=91),                    # configuration 1 shape
    dict(n=512, n_angles=360, n_det=724),                 # configuration 2 shape
]


def _oracle_geom(d):
    return Geometry(d["n"], d["n_angles"], d["n_det"], grid=d.get("grid", 0), kw=d.get("kw", 3),
                    center=d.get("center", float("nan")))


def gpu_layout_to_oracle(rp, col, val, g: Geometry) -> sp.csr_matrix:
    """Re-index the library's S^dagger (rows k_fft*nt + a, cols j1_fft*G + j2_fft) into the
    oracle's ordering (rows a*L + k + L//2, cols (j1 + G//2)*G + j2 + G//2)."""
    G, L, nt = g.G, g.L, g.n_theta
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    kf, a = rows // nt, rows % nt
    k = np.where(2 * kf < L, kf, kf - L)
    orow = a * L + k + L // 2
    j1f, j2f = col // G, col % G
    oG = G // 2
    j1 = np.where(j1f <= G - 1 - oG, j1f, j1f - G)
    j2 = np.where(j2f <= G - 1 - oG, j2f, j2f - G)
    ocol = (j1 + oG) * G + (j2 + oG)
    return sp.csr_matrix((val, (orow, ocol)), shape=(nt * L, G * G))


@pytest.mark.parametrize("d", GEOMS, ids=lambda d: "_".join(f"{k}{v}" for k, v in d.items()))
def test_csr_matches_oracle(d):
    op = tomo.Operator(device=-1, max_batch=2, **d)
    g = _oracle_geom(d)
    ref = Operator(g)
    assert op.info.beta == pytest.approx(beatty_beta(g.kw, g.G / g.n), rel=1e-14)
    rp, col, val = op.export_csr(0)
    assert np.all(np.diff(rp) >= 0) and rp[0] == 0 and rp[-1] == op.info.nnz
    for r in range(len(rp) - 1):                                   # sorted columns per row
        assert np.all(np.diff(col[rp[r]:rp[r + 1]]) > 0)
    S_dag = gpu_layout_to_oracle(rp, col, val, g)
    diff = abs(S_dag - ref.S_dag)
    assert (diff.max() if diff.nnz else 0.0) < 1e-12
    assert abs(op.info.nnz - ref.S.nnz) <= max(2, ref.S.nnz // 10 ** 6)   # near-ties only
    # the stored transpose is exact
    rpt, colt, valt = op.export_csr(1)
    St = sp.csr_matrix((valt, colt, rpt), shape=(op.info.n_cart, op.info.n_polar))
    Sd = sp.csr_matrix((val, col, rp), shape=(op.info.n_polar, op.info.n_cart))
    assert abs(St - Sd.T).max() == 0
    for r in range(0, len(rpt) - 1, max(1, (len(rpt) - 1) // 2000)):
        assert np.all(np.diff(colt[rpt[r]:rpt[r + 1]]) > 0)
    op.close()


@pytest.mark.parametrize("d", GEOMS[:6], ids=lambda d: "_".join(f"{k}{v}" for k, v in d.items()))
def test_factors_match_oracle(d):
    op = tomo.Operator(device=-1, max_batch=2, **d)
    g = _oracle_geom(d)
    kd, _ = op.export_factors("none")
    np.testing.assert_allclose(kd[:, None] * kd[None, :], deapodization(g), rtol=1e-13)
    L = g.L
    for name in ("ramlak", "shepp", "hamming"):
        _, dfft = op.export_factors(name)
        centred = ramp_filter(g, name)                      # index k + L//2
        k = np.arange(L) - L // 2
        np.testing.assert_allclose(dfft[k % L], centred, rtol=1e-10, atol=1e-14)
    op.close()


@pytest.mark.parametrize("tuning", [{}, dict(adj_sell_max=8, adj_medium_max=40, adj_chunk=16),
                                    dict(adj_sell_max=0, adj_medium_max=0, adj_chunk=64),
                                    dict(adj_sell_sigma=1)])
def test_row_bins_partition_rows(tuning):
    op = tomo.Operator(device=-1, max_batch=2, n=64, n_angles=90, n_det=91)
    t = op.set_tuning(**tuning)
    info = op.info
    rpt, _, _ = op.export_csr(1)
    lens = np.diff(rpt)
    sm, mm, ch = t["adj_sell_max"], t["adj_medium_max"], t["adj_chunk"]
    assert info.adj_sell_rows == np.sum(lens <= sm)
    assert info.adj_medium_rows == np.sum((lens > sm) & (lens <= mm))
    assert info.adj_long_rows == np.sum(lens > mm)
    long = lens[lens > mm]
    assert info.adj_long_chunks == int(np.sum(np.ceil(long / ch)))
    assert info.cols_touched == np.sum(lens > 0)
    assert info.adj_sell_padding >= 0
    op.close()


def test_tuning_rejects_out_of_range():
    op = tomo.Operator(device=-1, max_batch=2, n=16, n_angles=12, n_det=23)
    before = op.get_tuning()
    for bad in (dict(fwd_channels_per_lane=3), dict(adj_sell_max=-1), dict(adj_chunk=4),
                dict(adj_medium_max=10, adj_sell_max=20), dict(adj_sell_sigma=0),
                dict(tile_strip=-1), dict(tile_strip=4097), dict(adj_dense_mode=3),
                dict(adj_seg_chunks=0), dict(adj_seg_chunks=257), dict(adj_run=0), dict(adj_run=257),
                dict(det_fft=3), dict(det_fft=-1), dict(grid_fft=2), dict(grid_fft=-1)):
        with pytest.raises(tomo.TomoError):
            op.set_tuning(**bad)
        assert op.get_tuning() == before
    op.close()


def test_configuration_3_statistics():
    """2048^2 image, 1501 angles, 2048 bins: matrix size and adjoint row-length spread."""
    op = tomo.Operator(device=-1, max_batch=32, n=2048, n_angles=1501, n_det=2048)
    info = op.info
    assert info.beta == pytest.approx(beatty_beta(3, 1.0), rel=1e-14)
    assert info.n_polar == 1501 * 2048 and info.n_cart == 2048 * 2048
    assert info.nnz <= 1501 * 2048 * 9
    assert 27_600_000 < info.nnz < 27_700_000
    rpt, _, _ = op.export_csr(1)
    lens = np.diff(rpt)
    assert 0.20 < np.mean(lens == 0) < 0.23                 # corners outside the polar disk
    assert lens.max() > 4000                                # rows near the origin
    op.close()


@pytest.mark.parametrize("bad,status", [
    (dict(n=0), "TOMO_EINVAL"),
    (dict(kw=4), "TOMO_EINVAL"),
    (dict(grid=10), "TOMO_EINVAL"),
    (dict(max_batch=0), "TOMO_EINVAL"),
    (dict(max_batch=257), "TOMO_EINVAL"),
    (dict(center=float("inf")), "TOMO_EINVAL"),
    (dict(beta=-1.0), "TOMO_EINVAL"),
])
def test_invalid_geometry_is_rejected(bad, status):
    args = dict(n=16, n_angles=12, n_det=23, max_batch=2)
    args.update(bad)
    with pytest.raises(tomo.TomoError) as e:
        tomo.Operator(device=-1, **args)
    assert status in str(e.value)


def test_host_only_operator_rejects_apply():
    op = tomo.Operator(device=-1, n=16, n_angles=12, n_det=23, max_batch=2)
    lib = tomo.load()
    st = lib.tomo_project(op._handle, 16, 16, 1, 0, None)
    assert st == -5                                          # TOMO_ESTATE, nothing launched
    assert "without a device" in lib.tomo_last_error().decode()
    op.close()


@pytest.mark.parametrize("d", [GEOMS[0], GEOMS[3], GEOMS[5], GEOMS[6]], ids=lambda d: "_".join(f"{k}{v}" for k, v in d.items()))
@pytest.mark.parametrize("tuning", [{}, dict(tile=8, tile_points=32, adj_tile_points=32),
                                    dict(tile=16, tile_points=64, adj_tile_points=256),
                                    dict(adj_sell_max=4, adj_medium_max=20, adj_chunk=8, adj_sell_sigma=3),
                                    dict(adj_sell_tiles=1, adj_sell_max=24),
                                    dict(tile_strip=0), dict(tile_strip=3, adj_tile_points=64),
                                    dict(tile=16, tile_strip=5),
                                    dict(adj_tile_points=32, adj_dense_mode=1, adj_seg_chunks=1),
                                    dict(adj_tile_points=64, adj_dense_mode=2, adj_seg_chunks=3),
                                    dict(adj_tile_points=64, adj_dense_mode=2, adj_seg_chunks=2, adj_run=7),
                                    dict(tile=16, adj_tile_points=128, adj_dense_mode=1)])
def test_kernel_layouts_replay_the_csr_products(d, tuning):
    """Every device layout (fixed-stride forward, sliced-ELL / wave / chunked adjoint, LDS-staged
    window-form tiles, the row layout of the staged adjoint's dense cells, or those tiles in
    chunked segments with split tiles summed from partial tiles) replayed on the host equals the
    CSR products."""
    op = tomo.Operator(device=-1, max_batch=2, **d)
    op.set_tuning(**tuning)
    err = op.check_layouts()
    assert err < 1e-14                     # NaN (an unwritten row) fails too
    op.close()


NORMAL_GEOMS = [g for g in GEOMS if g["n_det"] == g.get("grid", g["n_det"])
                and g["n"] < 512 and "center" not in g]


@pytest.mark.parametrize("d", NORMAL_GEOMS, ids=lambda d: "_".join(f"{k}{v}" for k, v in d.items()))
@pytest.mark.parametrize("filt", ["none", "hamming"])
def test_normal_stencil_matches_oracle_product(d, filt):
    """W = S diag(D) S^dagger from the host builder (float64 stencil rows) against the oracle's
    sparse product, entry by entry after re-indexing to the oracle's ordering."""
    op = tomo.Operator(device=-1, max_batch=2, **d)
    g = _oracle_geom(d)
    ref = Operator(g)
    D = np.ones(g.L) if filt == "none" else ramp_filter(g, filt)      # per centred k
    dcol = np.tile(D, g.n_theta)                                          # oracle column a*L + k
    W = (ref.S @ sp.diags(dcol) @ ref.S_dag).tocoo()
    w = op.export_normal(filt)
    G, R = g.G, g.kw - 1
    S = 2 * R + 1
    oG = G // 2
    # oracle centred index -> FFT-ordered index
    def fft_index(o):
        j1, j2 = o // G - oG, o % G - oG
        return (j1 % G) * G + (j2 % G)
    r, c = fft_index(W.row), fft_index(W.col)
    d1 = c // G - r // G
    d2 = c % G - r % G
    d1 = np.where(2 * d1 >= G, d1 - G, np.where(2 * d1 < -G, d1 + G, d1))
    d2 = np.where(2 * d2 >= G, d2 - G, np.where(2 * d2 < -G, d2 + G, d2))
    assert np.abs(d1).max() <= R and np.abs(d2).max() <= R
    dense = np.zeros((G * G, S * S))
    np.add.at(dense, (r, (d1 + R) * S + (d2 + R)), W.data)
    assert np.abs(w - dense).max() <= 1e-13 * np.abs(dense).max()
    op.close()


def test_normal_operator_needs_full_detector():
    op = tomo.Operator(12, 10, 16, grid=20, device=-1, max_batch=2)
    with pytest.raises(tomo.TomoError, match="EUNSUPPORTED"):
        op.export_normal()
    op.close()
