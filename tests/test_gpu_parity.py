"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs.  Float32 operators must agree to 1e-5 relative L2 per slice; integer structure and
run-to-run results must agree bitwise."""

import math

import numpy as np
import pytest
import torch

from oracle import round_values, Operator as OracleOperator
from synth import phantom_stack, slice_rng
from tests.gpu_util import cart_map, complex_channels, oracle_op, polar_row_map, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5           # float32 operators vs float64 oracle, relative L2 per slice

# (n, n_angles, n_det, extra) — tiny ragged shapes, the 64^2 configuration, padding, off-centre axis
SHAPES = [
    (15, 7, 21, {}),
    (16, 12, 16, {}),
    (12, 10, 16, {"grid": 20}),
    (16, 9, 23, {"center": 10.0}),
    (16, 9, 23, {"center": 11.3}),         # fractional axis (the oracle's phase-ramp reading)
    (64, 90, 91, {}),
    (9, 7, 13, {"kw": 5}),
]


def _ids(s):
    return f"n{s[0]}_t{s[1]}_p{s[2]}" + "".join(f"_{k}{v}" for k, v in s[3].items())


def _gpu_op(tomo, n, nt, npb, extra, max_batch=8, values=("f32",)):
    return tomo.Operator(n, nt, npb, max_batch=max_batch, values=values, device=0, **extra)


def _oracle(n, nt, npb, extra):
    return oracle_op(n, nt, npb, extra.get("grid", 0), extra.get("kw", 3), extra.get("center", float("nan")))


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


# ------------------------------------------------------------------------------------------
# the SpMM kernels alone
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("shape", SHAPES, ids=_ids)
@pytest.mark.parametrize("batch", [1, 2, 5, 8])
def test_slice_spmm_matches_oracle_csr(tomo, shape, batch):
    n, nt, npb, extra = shape
    op = _gpu_op(tomo, n, nt, npb, extra)
    ref = _oracle(n, nt, npb, extra)
    g = ref.geom
    C = (batch + 1) // 2
    Xc = _rand((g.G * g.G, C, 2), 100 + batch)
    Xg = _dev(Xc)
    Yg = op.slice_fwd(Xg, batch)
    Y = complex_channels(Yg)
    cm, pm = cart_map(g), polar_row_map(g)
    Xo = np.empty((g.G * g.G, C), dtype=np.complex128)
    Xo[cm] = Xc[..., 0] + 1j * Xc[..., 1]
    Yref = (ref.S_dag @ Xo)[pm]
    assert rel_l2(Y, Yref) < 1e-6
    # adjoint, with and without the filter diagonal
    Yc = _rand((g.L * nt, C, 2), 200 + batch)
    Yo = np.empty((g.L * nt, C), dtype=np.complex128)
    Yo[pm] = Yc[..., 0] + 1j * Yc[..., 1]
    Xg2 = op.slice_adj(_dev(Yc), batch)
    Xref = (ref.S @ Yo)[cm]
    assert rel_l2(complex_channels(Xg2), Xref) < 1e-6
    from oracle import ramp_filter
    D = ramp_filter(g, "hamming")                              # per centred k
    Dpolar = np.tile(D, nt)                                     # oracle column a*L + kk
    Xg3 = op.slice_adj(_dev(Yc), batch, filter="hamming")
    Xref3 = (ref.S @ (Dpolar[:, None] * Yo))[cm]
    assert rel_l2(complex_channels(Xg3), Xref3) < 1e-6
    # bitwise reproducible (no atomics)
    assert torch.equal(op.slice_adj(_dev(Yc), batch), Xg2)
    assert torch.equal(op.slice_fwd(Xg, batch), Yg)
    op.close()


# ------------------------------------------------------------------------------------------
# composed operators
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("shape", SHAPES, ids=_ids)
@pytest.mark.parametrize("batch", [1, 3, 8])
def test_project_backproject_irradon(tomo, shape, batch):
    n, nt, npb, extra = shape
    op = _gpu_op(tomo, n, nt, npb, extra)
    ref = _oracle(n, nt, npb, extra)
    x = _rand((batch, n, n), 300 + batch)
    y = _rand((batch, nt, npb), 400 + batch)
    yg = _host(op.project(_dev(x)))
    xg = _host(op.backproject(_dev(y)))
    xf = _host(op.irradon(_dev(y), filter="hamming"))
    for s in range(batch):
        xs = x[s].astype(np.float32).astype(np.float64)
        ys = y[s].astype(np.float32).astype(np.float64)
        assert rel_l2(yg[s], ref.project(xs)) < TOL, s
        assert rel_l2(xg[s], ref.backproject(ys)) < TOL, s
        assert rel_l2(xf[s], ref.irradon(ys, "hamming")) < TOL, s
    op.close()


POW2_SHAPES = [
    (16, 12, 16, {}),
    (32, 24, 64, {}),
    (24, 20, 32, {"center": 10.0}),
    (24, 20, 32, {"center": 10.3}),        # fractional axis: a phase ramp on the polar rows
    (12, 10, 16, {"grid": 32}),            # zero-padded detector: crop / pad of L to n_p
    (40, 30, 64, {"kw": 5}),
    (100, 60, 256, {}),
    (64, 6, 4096, {}),                     # two channels per block
]

# other lengths go through Bluestein's identity at the power-of-two length M >= 2N - 1: the
# 91 / 724 / 1448 / 362 / 2896 grids of the benchmark configurations (M = 256 .. 8192; 8192 holds
# one row or column per block), a prime, a padded grid and an off-centre axis
NONPOW2_SHAPES = [
    (64, 90, 91, {}),
    (17, 11, 23, {"center": 9.0}),
    (17, 11, 23, {"center": 8.4}),         # fractional axis through Bluestein transforms
    (24, 20, 33, {"grid": 40}),
    (30, 17, 45, {"kw": 5}),
    (200, 16, 283, {}),                    # prime length
]
CONFIG_LENGTHS = [(256, 24, 362, {}), (512, 36, 724, {}), (1024, 30, 1448, {}), (2048, 12, 2896, {})]


@pytest.mark.parametrize("shape", POW2_SHAPES + NONPOW2_SHAPES, ids=_ids)
@pytest.mark.parametrize("fft", [(1, 1), (2, 1), (0, 0), (1, 0), (2, 0), (0, 1)],
                         ids=lambda f: f"det{f[0]}_grid{f[1]}")
@pytest.mark.parametrize("batch", [1, 5, 19])
def test_hand_written_transform_paths(tomo, shape, fft, batch):
    """The hand-written transforms (detector rows with crop / pad, the adjoint front writing the
    SpMM's channel-fastest polar layout (1) or channel-slowest rows (2); Cartesian rows with
    embed / crop and columns) and the rocFFT paths (0) all give the oracle's operators, for
    power-of-two lengths and, through Bluestein's identity, for others; batch 19 (10 channels)
    leaves a ragged channel group of the 8-channel adjoint front."""
    n, nt, npb, extra = shape
    if batch > 8 and max(n, npb) > 512:
        pytest.skip("the ragged channel group is covered on the smaller shapes")
    op = _gpu_op(tomo, n, nt, npb, extra, max_batch=max(batch, 8))
    op.set_tuning(det_fft=fft[0], grid_fft=fft[1])
    ref = _oracle(n, nt, npb, extra)
    x = _rand((batch, n, n), 700 + batch)
    y = _rand((batch, nt, npb), 800 + batch)
    yg = _host(op.project(_dev(x)))
    xg = _host(op.backproject(_dev(y)))
    xf = _host(op.irradon(_dev(y), filter="ramlak"))
    # batch 19: the first group's edges and the ragged group (channels 8 and 9; slice 18 alone)
    for s in (range(batch) if batch <= 8 else (0, 7, 15, 16, 17, 18)):
        xs = x[s].astype(np.float32).astype(np.float64)
        ys = y[s].astype(np.float32).astype(np.float64)
        assert rel_l2(yg[s], ref.project(xs)) < TOL, s
        assert rel_l2(xg[s], ref.backproject(ys)) < TOL, s
        assert rel_l2(xf[s], ref.irradon(ys, "ramlak")) < TOL, s
    op.close()


@pytest.mark.parametrize("shape", CONFIG_LENGTHS, ids=_ids)
def test_hand_written_transforms_at_configuration_lengths(tomo, shape):
    """The default (hand-written, Bluestein) transforms at the grid / detector lengths of the
    benchmark configurations (362, 724, 1448, 2896 = 2^k * 181; few angles to keep the oracle
    cheap): project, backproject and iRadon of two slices (one complex channel) against the
    oracle, relative L2 and the largest element error against the largest reference element."""
    n, nt, npb, extra = shape
    op = _gpu_op(tomo, n, nt, npb, extra, max_batch=2)
    assert op.get_tuning()["det_fft"] == 1 and op.get_tuning()["grid_fft"] == 1
    ref = _oracle(n, nt, npb, extra)
    x = _rand((2, n, n), 710)
    y = _rand((2, nt, npb), 810)
    yg = _host(op.project(_dev(x)))
    xg = _host(op.backproject(_dev(y)))
    xf = _host(op.irradon(_dev(y), filter="ramlak"))
    for s in range(2):
        xs = x[s].astype(np.float32).astype(np.float64)
        ys = y[s].astype(np.float32).astype(np.float64)
        for got, want in ((yg[s], ref.project(xs)), (xg[s], ref.backproject(ys)),
                          (xf[s], ref.irradon(ys, "ramlak"))):
            l2 = rel_l2(got, want)
            mx = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
            print(f"{shape[:3]} slice {s}: rel L2 {l2:.2e}, max {mx:.2e}")
            assert l2 < TOL and mx < TOL, (s, l2, mx)
    op.close()


@pytest.mark.parametrize("shape", [(64, 90, 91, {}), (100, 60, 256, {}), (24, 20, 33, {"grid": 40}),
                                   (30, 17, 45, {"kw": 5})], ids=_ids)
@pytest.mark.parametrize("dense", [0, 1, 2])
@pytest.mark.parametrize("vt", ["f32", "bf16"])
def test_operators_with_each_adjoint_form(tomo, shape, dense, vt):
    """The composed operators with the staged SpMMs on the FFT-side (channel-slowest) grid: the
    forward reads its patches there, and with the dense tiles staged (forms 1 and 2) the adjoint
    writes its tiles there (form 0 keeps the row kernels and the transpose); project,
    backproject and the filtered iRadon against the oracle, odd and even batches."""
    n, nt, npb, extra = shape
    op = _gpu_op(tomo, n, nt, npb, extra, values=("f32", "bf16"))
    op.set_tuning(adj_dense_mode=dense, adj_seg_chunks=2, adj_tile_points=64)
    base = _oracle(n, nt, npb, extra)
    ref = base if vt == "f32" else OracleOperator(base.geom, S=round_values(base.S, vt))
    for batch in (3, 4):
        x = _rand((batch, n, n), 720 + batch)
        y = _rand((batch, nt, npb), 820 + batch)
        yg = _host(op.project(_dev(x), values=vt))
        xg = _host(op.backproject(_dev(y), values=vt))
        xf = _host(op.irradon(_dev(y), values=vt, filter="hamming"))
        for s in range(batch):
            xs = x[s].astype(np.float32).astype(np.float64)
            ys = y[s].astype(np.float32).astype(np.float64)
            assert rel_l2(yg[s], ref.project(xs)) < TOL, (batch, s)
            assert rel_l2(xg[s], ref.backproject(ys)) < TOL, (batch, s)
            assert rel_l2(xf[s], ref.irradon(ys, "hamming")) < TOL, (batch, s)
    op.close()


def test_odd_channel_count_above_64(tomo):
    """133 slices (67 complex channels, odd, above the row kernels' 64 lane groups) run through the
    staged kernels, which split channels over blocks (the dense tiles in segments, whatever
    adj_dense_mode selects); with the staged adjoint off, the row kernels refuse such a batch."""
    n, nt, npb, B = 16, 12, 23, 133
    op = tomo.Operator(n, nt, npb, max_batch=B, device=0)
    ref = oracle_op(n, nt, npb)
    x = _rand((B, n, n), 740)
    y = _rand((B, nt, npb), 840)
    yg = _host(op.project(_dev(x)))
    xg = _host(op.backproject(_dev(y)))
    for s in (0, 1, 64, 131, 132):
        assert rel_l2(yg[s], ref.project(x[s].astype(np.float32).astype(np.float64))) < TOL, s
        assert rel_l2(xg[s], ref.backproject(y[s].astype(np.float32).astype(np.float64))) < TOL, s
    # the channel-fastest adjoint: with adj_dense_mode 0 it falls back to the segments of mode 1
    Yc = torch.randn(op.polar_shape(B), device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    outs = {}
    for mode in (0, 1, 2):
        op.set_tuning(adj_dense_mode=mode)
        outs[mode] = op.slice_adj(Yc, B).clone()
    assert torch.equal(outs[0], outs[1])
    assert (outs[2] - outs[1]).abs().max().item() <= 1e-5 * outs[1].abs().max().item()
    op.set_tuning(adj_dense_mode=0)
    xg0 = _host(op.backproject(_dev(y)))
    assert rel_l2(xg0[132], ref.backproject(y[132].astype(np.float32).astype(np.float64))) < TOL
    op.set_tuning(adj_tiled=0)
    with pytest.raises(tomo.TomoError, match="EUNSUPPORTED"):
        op.backproject(_dev(y))
    op.close()


def test_phantom_stack_configuration_1_shape(tomo):
    """Random-ellipse phantoms at 64^2, 90 angles, 91 bins, through the paired path."""
    x = phantom_stack(64, 5, seed_base=1000)
    op = tomo.Operator(64, 90, 91, max_batch=5, device=0)
    ref = oracle_op(64, 90, 91)
    yg = _host(op.project(_dev(x)))
    for s in range(5):
        assert rel_l2(yg[s], ref.project(x[s].astype(np.float32).astype(np.float64))) < TOL
    op.close()


@pytest.mark.parametrize("vt", ["bf16", "f16"])
def test_low_precision_values_match_rounded_oracle(tomo, vt):
    """16-bit matrix values with float32 accumulation equal the oracle run with the same
    rounded values; the error against the float64 operator is stated, not bounded tightly."""
    n, nt, npb = 64, 90, 91
    op = tomo.Operator(n, nt, npb, max_batch=4, values=("f32", vt), device=0)
    ref = oracle_op(n, nt, npb)
    lo = OracleOperator(ref.geom, S=round_values(ref.S, vt))
    x = phantom_stack(n, 4, seed_base=1100)
    y = _rand((4, nt, npb), 12)
    yg = _host(op.project(_dev(x), values=vt))
    xg = _host(op.backproject(_dev(y), values=vt))
    xf = _host(op.irradon(_dev(y), values=vt, filter="hamming"))
    errs = []
    for s in range(4):
        xs = x[s].astype(np.float32).astype(np.float64)
        ys = y[s].astype(np.float32).astype(np.float64)
        assert rel_l2(yg[s], lo.project(xs)) < TOL
        assert rel_l2(xg[s], lo.backproject(ys)) < TOL
        assert rel_l2(xf[s], lo.irradon(ys, "hamming")) < TOL
        errs.append(rel_l2(yg[s], ref.project(xs)))
    # bf16 keeps 8 significant bits (relative rounding <= 2^-9), f16 11 bits
    assert max(errs) < (4e-3 if vt == "bf16" else 5e-4)
    op.close()


# ------------------------------------------------------------------------------------------
# invariants on the GPU (float32)
# ------------------------------------------------------------------------------------------
def test_gpu_adjoint_mass_conservation_and_ones(tomo):
    n, nt, npb = 64, 90, 91
    op = tomo.Operator(n, nt, npb, max_batch=8, device=0)
    x = np.random.default_rng(31).uniform(0, 1, (8, n, n))
    y = np.random.default_rng(32).standard_normal((8, nt, npb))
    Ax = _host(op.project(_dev(x)))
    ATy = _host(op.backproject(_dev(y)))
    xf = x.astype(np.float32).astype(np.float64)
    yf = y.astype(np.float32).astype(np.float64)
    for s in range(8):
        lhs, rhs = np.vdot(Ax[s], yf[s]), np.vdot(xf[s], ATy[s])
        assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Ax[s]) * np.linalg.norm(yf[s])
        np.testing.assert_allclose(Ax[s].sum(axis=1), xf[s].sum(), rtol=1e-5)
    ones = _host(op.backproject(_dev(np.ones((2, nt, npb)))))
    np.testing.assert_allclose(ones, nt, rtol=1e-5)
    op.close()


def test_gpu_determinism_and_batch_edges(tomo):
    op = tomo.Operator(16, 12, 23, max_batch=4, device=0)
    x = _dev(_rand((4, 16, 16), 41))
    a = op.project(x)
    b = op.project(x)
    assert torch.equal(a, b)
    # batch 0 is a no-op; batch above max_batch is rejected before any launch
    lib = tomo.load()
    assert lib.tomo_project(op._handle, x.data_ptr(), a.data_ptr(), 0, 0, None) == 0
    assert lib.tomo_project(op._handle, x.data_ptr(), a.data_ptr(), 5, 0, None) == -1
    assert lib.tomo_project(op._handle, None, a.data_ptr(), 1, 0, None) == -1
    assert lib.tomo_project(op._handle, x.data_ptr(), a.data_ptr(), 1, 1, None) == -5  # bf16 absent
    # slices are independent: a batch of 3 equals three batches of 1
    x3 = _dev(_rand((3, 16, 16), 42))
    y3 = _host(op.project(x3))
    for s in range(3):
        ys = _host(op.project(x3[s:s + 1].contiguous()))
        assert rel_l2(ys[0], y3[s]) < 1e-6
    op.close()


ROW = dict(fwd_tiled=0, adj_tiled=0)
TUNINGS = [
    dict(ROW, fwd_channels_per_lane=1, adj_channels_per_lane=1),
    dict(ROW, fwd_channels_per_lane=4, adj_channels_per_lane=4),
    dict(ROW, adj_sell_max=0, adj_medium_max=0, adj_chunk=8),     # every row chunked
    dict(ROW, adj_sell_max=1024, adj_medium_max=1024),            # every row in sliced ELL
    dict(ROW, adj_sell_max=4, adj_medium_max=16, adj_chunk=24, adj_sell_sigma=1),
    dict(ROW, adj_sell_tiles=1),                                   # sliced ELL in 4 x 8 cell tiles
    dict(adj_sell_tiles=1, adj_tile_points=64),
    dict(fwd_tiled=7, adj_tiled=7, tile=8, tile_points=32, adj_tile_points=32),   # many dense tiles
    dict(fwd_tiled=7, adj_tiled=7, tile=8, tile_points=64, adj_tile_points=128),
    dict(fwd_tiled=7, adj_tiled=7, tile=16, tile_points=128, adj_tile_points=256),
    dict(fwd_tiled=2, adj_tiled=1),                                  # staged for one value type
    dict(fwd_tiled=7, adj_tiled=7, tile_strip=0),                    # row-major tile order
    dict(fwd_tiled=7, adj_tiled=7, tile=8, tile_strip=3, adj_tile_points=64),   # ragged strips
    dict(fwd_tiled=0, adj_tiled=7, adj_sell_max=4, adj_medium_max=16, adj_chunk=24),
    dict(ROW, adj_sell_xcd_rows=64, adj_medium_xcd_rows=8),       # short XCD interleave runs
    dict(ROW, adj_sell_xcd_rows=0, adj_medium_xcd_rows=0),        # one contiguous range per XCD
    dict(ROW, fwd_rows_per_group=2),                              # pipelined forward
    dict(ROW, fwd_rows_per_group=4),
    # dense tiles staged in chunked segments: one chunk per segment (every dense tile split and
    # reduced from partial tiles), a few, and one launch for every tile
    dict(fwd_tiled=7, adj_tiled=7, tile=8, adj_tile_points=32, adj_dense_mode=1, adj_seg_chunks=1),
    dict(fwd_tiled=7, adj_tiled=7, tile=8, adj_tile_points=64, adj_dense_mode=1, adj_seg_chunks=8),
    dict(fwd_tiled=7, adj_tiled=7, tile=8, adj_tile_points=128, adj_dense_mode=2, adj_seg_chunks=4),
    dict(fwd_tiled=7, adj_tiled=7, tile=16, adj_tile_points=256, adj_dense_mode=2, adj_seg_chunks=2),
    # staged tiles in runs per block (odd and even run lengths: both register sets end a run)
    dict(fwd_tiled=7, adj_tiled=7, tile=8, adj_tile_points=64, adj_dense_mode=2, adj_seg_chunks=3, adj_run=5),
    dict(fwd_tiled=7, adj_tiled=7, tile=8, adj_tile_points=128, adj_dense_mode=2, adj_seg_chunks=8, adj_run=8),
]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "_".join(f"{k}{v}" for k, v in t.items()))
@pytest.mark.parametrize("batch", [5, 7, 16, 32])
def test_slice_spmm_tunings(tomo, tuning, batch):
    """Every kernel layout the tuning space allows gives the oracle's CSR products."""
    n, nt, npb = 64, 90, 91
    op = tomo.Operator(n, nt, npb, max_batch=32, values=("f32", "bf16"), device=0)
    op.set_tuning(**tuning)
    ref = oracle_op(n, nt, npb)
    g = ref.geom
    C = (batch + 1) // 2
    cm, pm = cart_map(g), polar_row_map(g)
    Xc = _rand((g.G * g.G, C, 2), 500 + batch)
    Xo = np.empty((g.G * g.G, C), dtype=np.complex128)
    Xo[cm] = Xc[..., 0] + 1j * Xc[..., 1]
    assert rel_l2(complex_channels(op.slice_fwd(_dev(Xc), batch)), (ref.S_dag @ Xo)[pm]) < 1e-6
    lo_dag = round_values(ref.S_dag, "bf16")
    assert rel_l2(complex_channels(op.slice_fwd(_dev(Xc), batch, values="bf16")), (lo_dag @ Xo)[pm]) < 1e-6
    Yc = _rand((g.L * nt, C, 2), 600 + batch)
    Yo = np.empty((g.L * nt, C), dtype=np.complex128)
    Yo[pm] = Yc[..., 0] + 1j * Yc[..., 1]
    Xa = op.slice_adj(_dev(Yc), batch)
    assert rel_l2(complex_channels(Xa), (ref.S @ Yo)[cm]) < 1e-6
    assert torch.equal(op.slice_adj(_dev(Yc), batch), Xa)
    lo = round_values(ref.S, "bf16")
    assert rel_l2(complex_channels(op.slice_adj(_dev(Yc), batch, values="bf16")), (lo @ Yo)[cm]) < 1e-6
    # the filter diagonal on the way in (scaled staging in the staged adjoint)
    from oracle import ramp_filter
    Dpolar = np.tile(ramp_filter(g, "hamming"), nt)
    for vt, S_vt in (("f32", ref.S), ("bf16", lo)):
        Xf = op.slice_adj(_dev(Yc), batch, values=vt, filter="hamming")
        assert rel_l2(complex_channels(Xf), (S_vt @ (Dpolar[:, None] * Yo))[cm]) < 1e-6, vt
    op.close()


@pytest.mark.parametrize("shape", SHAPES, ids=_ids)
@pytest.mark.parametrize("tile", [8, 16])
@pytest.mark.parametrize("dense", [0, 1, 2])
def test_staged_kernels_on_every_geometry(tomo, shape, tile, dense):
    """The LDS-staged SpMMs at ragged sizes, padded and off-centre geometries and k_w = 5
    (windows on the grid's upper edge, tiles past the grid's end), with the adjoint's dense tiles
    on the row kernels (0) or staged in segments of two chunks (1: second stream, 2: one launch)."""
    n, nt, npb, extra = shape
    op = _gpu_op(tomo, n, nt, npb, extra, max_batch=6)
    op.set_tuning(fwd_tiled=7, adj_tiled=7, tile=tile, tile_points=64, adj_tile_points=64,
                  adj_dense_mode=dense, adj_seg_chunks=2, adj_run=3)
    ref = _oracle(n, nt, npb, extra)
    g = ref.geom
    cm, pm = cart_map(g), polar_row_map(g)
    for batch in (1, 6):
        C = (batch + 1) // 2
        Xc = _rand((g.G * g.G, C, 2), 800 + batch)
        Xo = np.empty((g.G * g.G, C), dtype=np.complex128)
        Xo[cm] = Xc[..., 0] + 1j * Xc[..., 1]
        assert rel_l2(complex_channels(op.slice_fwd(_dev(Xc), batch)), (ref.S_dag @ Xo)[pm]) < 1e-6
        Yc = _rand((g.L * nt, C, 2), 900 + batch)
        Yo = np.empty((g.L * nt, C), dtype=np.complex128)
        Yo[pm] = Yc[..., 0] + 1j * Yc[..., 1]
        assert rel_l2(complex_channels(op.slice_adj(_dev(Yc), batch)), (ref.S @ Yo)[cm]) < 1e-6
    op.close()


def test_staged_adjoint_on_a_side_stream_matches_the_default_stream(tomo):
    """The staged adjoint forks its dense-cell kernels to streams of its own and joins them back
    to the caller's stream: a call on a non-default torch stream, consumed after the caller
    synchronises that stream, equals the default-stream result bit for bit."""
    n, nt, npb, batch = 64, 90, 91, 16
    op = _gpu_op(tomo, n, nt, npb, {}, max_batch=16, values=("f32", "bf16"))
    g = oracle_op(n, nt, npb).geom
    C = batch // 2
    Y = _dev(_rand((g.L * nt, C, 2), 950))
    for mode in (0, 1, 2):
        op.set_tuning(adj_dense_mode=mode, adj_seg_chunks=2)
        ref = {vt: op.slice_adj(Y, batch, values=vt).clone() for vt in ("f32", "bf16")}
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            outs = {vt: op.slice_adj(Y, batch, values=vt) for vt in ("f32", "bf16")}
            again = op.slice_adj(Y, batch, values="bf16")
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        for vt in ("f32", "bf16"):
            assert torch.equal(outs[vt], ref[vt]), (mode, vt)
        assert torch.equal(again, ref["bf16"]), mode
    op.close()


def test_tile_visiting_order_does_not_change_the_results(tomo):
    """The staged kernels' tile order (strips of tiles, or row-major) only moves work between
    blocks: every order gives the same products bit for bit, in every value type."""
    n, nt, npb, batch = 96, 120, 137, 12
    op = _gpu_op(tomo, n, nt, npb, {}, max_batch=12, values=("f32", "bf16", "f16"))
    op.set_tuning(fwd_tiled=7, adj_tiled=7, tile=8, tile_points=64, adj_tile_points=64)
    X = _dev(_rand(tuple(op.cart_shape(batch)), 960))
    Y = _dev(_rand(tuple(op.polar_shape(batch)), 961))
    ref = None
    for strip in (0, 1, 3, 5, 32):
        op.set_tuning(tile_strip=strip)
        out = [op.slice_fwd(X, batch, values=vt).clone() for vt in ("f32", "bf16", "f16")]
        out += [op.slice_adj(Y, batch, values=vt).clone() for vt in ("f32", "bf16", "f16")]
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            assert torch.equal(a, b), strip
    op.close()
