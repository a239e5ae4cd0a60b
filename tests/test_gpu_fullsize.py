"""Full-size parity at 2048^2 pixels, 1501 angles, 2048 bins in the benchmark's launch
configuration (one batch of 32 slices = 16 complex channels): the SpMM kernels on sampled
rows (including the longest adjoint rows), and the composed operators on sampled slices,
against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import round_values
from synth import phantom_stack
from tests.gpu_util import cart_map, oracle_op, polar_row_map, rel_l2

pytestmark = pytest.mark.gpu

N, NT, NP, B = 2048, 1501, 2048, 32


@pytest.fixture(scope="module")
def big(tomo):
    op = tomo.Operator(N, NT, NP, max_batch=B, values=("f32", "bf16"), device=0)
    yield op
    op.close()


@pytest.fixture(scope="module")
def ref():
    return oracle_op(N, NT, NP)


def _sampled_rows_ref(S_o, rows_o, col_map_inv, Xlib):
    """(S_o[rows_o] @ X) with X given in library column order."""
    sub = S_o[rows_o]
    gcols = col_map_inv[sub.indices]
    prod = sub.data[:, None] * Xlib[gcols]
    out = np.zeros((len(rows_o), Xlib.shape[1]), dtype=np.complex128)
    np.add.at(out, np.repeat(np.arange(len(rows_o)), np.diff(sub.indptr)), prod)
    return out


def test_fullsize_spmm_sampled_rows(big, ref):
    g = ref.geom
    C = B // 2
    rng = np.random.default_rng(7)
    Xc = rng.standard_normal((g.G * g.G, C, 2), dtype=np.float32)
    Xg = torch.from_numpy(Xc).cuda()
    Yg = big.slice_fwd(Xg, B)
    torch.cuda.synchronize()
    cm, pm = cart_map(g), polar_row_map(g)
    cm_inv = np.empty_like(cm)
    cm_inv[cm] = np.arange(cm.size)
    pm_inv = np.empty_like(pm)
    pm_inv[pm] = np.arange(pm.size)
    Xlib = Xc[..., 0].astype(np.float64) + 1j * Xc[..., 1]
    rows = rng.choice(g.n_theta * g.L, 4000, replace=False)
    Yref = _sampled_rows_ref(ref.S_dag, pm[rows], cm_inv, Xlib)
    Y = Yg.cpu().numpy()[rows]
    assert rel_l2(Y[..., 0] + 1j * Y[..., 1], Yref) < 1e-6
    # adjoint: random rows plus every row long enough to be split into chunks
    Yc = rng.standard_normal((g.L * g.n_theta, C, 2), dtype=np.float32)
    Ylib = Yc[..., 0].astype(np.float64) + 1j * Yc[..., 1]
    Xg2 = big.slice_adj(torch.from_numpy(Yc).cuda(), B)
    torch.cuda.synchronize()
    lens = np.diff(ref.S.indptr)[cm]                               # library row order
    long_rows = np.nonzero(lens > big.get_tuning()["adj_medium_max"])[0]
    rows2 = np.unique(np.concatenate([rng.choice(g.G * g.G, 4000, replace=False), long_rows]))
    Xref = _sampled_rows_ref(ref.S, cm[rows2], pm_inv, Ylib)
    X = Xg2.cpu().numpy()[rows2]
    assert rel_l2(X[..., 0] + 1j * X[..., 1], Xref) < 1e-6
    assert torch.equal(big.slice_adj(torch.from_numpy(Yc).cuda(), B), Xg2)


def test_fullsize_bf16_spmm_sampled_rows_in_benchmark_configuration(big, ref):
    """The launch the benchmark times: batch 32 with bf16 values, i.e. the LDS-staged forward and
    the staged adjoint with the row kernels on the cells near the origin.  Sampled rows of both
    products against the oracle's matrices with bf16-rounded values, half of the adjoint's rows
    drawn from within 400 cells of the origin (where the staged adjoint leaves the dense tiles
    to the row kernels and borders them), and run-to-run identity."""
    g = ref.geom
    C = B // 2
    tun = big.get_tuning()
    assert tun["fwd_tiled"] & 2 and tun["adj_tiled"] & 2      # the staged kernels are what runs
    rng = np.random.default_rng(11)
    cm, pm = cart_map(g), polar_row_map(g)
    cm_inv = np.empty_like(cm)
    cm_inv[cm] = np.arange(cm.size)
    pm_inv = np.empty_like(pm)
    pm_inv[pm] = np.arange(pm.size)
    Xc = rng.standard_normal((g.G * g.G, C, 2), dtype=np.float32)
    Yg = big.slice_fwd(torch.from_numpy(Xc).cuda(), B, values="bf16")
    torch.cuda.synchronize()
    rows = rng.choice(g.n_theta * g.L, 4000, replace=False)
    Xlib = Xc[..., 0].astype(np.float64) + 1j * Xc[..., 1]
    Yref = _sampled_rows_ref(round_values(ref.S_dag[pm[rows]], "bf16"), np.arange(rows.size), cm_inv, Xlib)
    Y = Yg.cpu().numpy()[rows]
    assert rel_l2(Y[..., 0] + 1j * Y[..., 1], Yref) < 1e-6
    Yc = rng.standard_normal((g.L * g.n_theta, C, 2), dtype=np.float32)
    Ylib = Yc[..., 0].astype(np.float64) + 1j * Yc[..., 1]
    Xg = big.slice_adj(torch.from_numpy(Yc).cuda(), B, values="bf16")
    torch.cuda.synchronize()
    # rows near the Fourier origin (the dense tiles) and random rows elsewhere
    j = np.arange(g.G)
    jc = np.where(j <= g.G - 1 - g.G // 2, j, j - g.G)
    rad = np.hypot(jc[:, None], jc[None, :]).reshape(-1)            # library cell order
    near = np.nonzero(rad < 400)[0]
    rows2 = np.unique(np.concatenate([rng.choice(near, 3000, replace=False),
                                      rng.choice(g.G * g.G, 3000, replace=False)]))
    Xref = _sampled_rows_ref(round_values(ref.S[cm[rows2]], "bf16"), np.arange(rows2.size), pm_inv, Ylib)
    X = Xg.cpu().numpy()[rows2]
    assert rel_l2(X[..., 0] + 1j * X[..., 1], Xref) < 1e-6
    assert torch.equal(big.slice_adj(torch.from_numpy(Yc).cuda(), B, values="bf16"), Xg)


def test_fullsize_operators_sampled_slices(big, ref):
    x = phantom_stack(N, B, seed_base=3000, supersample=1)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    y = big.project(xt)
    yb = big.project(xt, values="bf16")
    torch.cuda.synchronize()
    yh = y.cpu().numpy().astype(np.float64)
    # mass conservation per angle on every slice (L = n_p)
    mass = x.astype(np.float32).astype(np.float64).sum(axis=(1, 2))
    np.testing.assert_allclose(yh.sum(axis=2), mass[:, None] * np.ones((1, NT)), rtol=1e-5)
    xb = big.backproject(y)
    torch.cuda.synchronize()
    xbh = xb.cpu().numpy().astype(np.float64)
    for s in (0, B - 1):
        xs = x[s].astype(np.float32).astype(np.float64)
        P = ref.project(xs)
        assert rel_l2(yh[s], P) < 1e-5
        assert rel_l2(xbh[s], ref.backproject(yh[s])) < 1e-5
        err_bf16 = rel_l2(yb[s].cpu().numpy(), P)
        print(f"slice {s}: bf16-value projection error vs FP64 oracle {err_bf16:.3e}")
        assert err_bf16 < 4e-3
