"""GPU tests of the multi-operator HIP graph and of the autotuner.

* A graph of steps over two operators of different sizes (SpMM pair, project, backproject,
  normal operator; float32 and bfloat16 values; odd and even batches) reproduces the eager
  entry points bit for bit, on every replay, with the inputs changed and eager work run on
  the same operators between replays (stream-captured graphs read the buffers' current
  contents).
* The autotuner returns a valid tuning with positive times, and the operator still matches
  the oracle's CSR products after it (to the SpMM bar, 1e-6)."""

import numpy as np
import pytest
import torch

from tests.gpu_util import (cart_map, complex_channels, oracle_op, polar_row_map, rel_l2,
                            summation_bound_check)

pytestmark = pytest.mark.gpu


def _fill(t, seed):
    g = torch.Generator(device=t.device)
    g.manual_seed(seed)
    t.copy_(torch.rand(t.shape, generator=g, device=t.device) * 2 - 1)


def test_graph_replays_match_eager(tomo):
    a = tomo.Operator(64, 90, 91, max_batch=8, values=("f32", "bf16"), device=0)
    b = tomo.Operator(37, 30, 53, max_batch=8, values=("f32", "bf16"), device=0)
    dev = "cuda"
    Xc = torch.empty(a.cart_shape(7), device=dev)
    Yp = torch.empty(a.polar_shape(7), device=dev)
    Xa = torch.empty(a.cart_shape(7), device=dev)
    xb = torch.empty((3, 37, 37), device=dev)
    yb = torch.empty((3, 30, 53), device=dev)
    ya = torch.empty((4, 90, 91), device=dev)
    xa = torch.empty((4, 64, 64), device=dev)
    xn = torch.empty((2, 37, 37), device=dev)
    nb = torch.empty((2, 37, 37), device=dev)
    steps = [dict(op=a, kind="spmm_pair", batch=7, values="bf16", inp=Xc, out=Yp, aux=Xa),
             dict(op=b, kind="project", batch=3, values="f32", inp=xb, out=yb),
             dict(op=a, kind="backproject", batch=4, values="f32", inp=ya, out=xa),
             dict(op=b, kind="normal", batch=2, values="bf16", inp=xn, out=nb)]
    for t, sd in ((Xc, 1), (xb, 2), (ya, 3), (xn, 4)):
        _fill(t, sd)
    g = tomo.Graph(steps)
    for rep in range(3):
        for t, sd in ((Xc, 10 + rep), (xb, 20 + rep), (ya, 30 + rep), (xn, 40 + rep)):
            _fill(t, sd)
        g.launch()
        torch.cuda.synchronize()
        got = [t.clone() for t in (Yp, Xa, yb, xa, nb)]
        ref = [a.slice_fwd(Xc, 7, values="bf16")]
        ref.append(a.slice_adj(ref[0], 7, values="bf16"))
        ref += [b.project(xb), a.backproject(ya), b.normal(xn, values="bf16")]
        torch.cuda.synchronize()
        for k, (x, y) in enumerate(zip(got, ref)):
            assert torch.equal(x, y), (rep, k)
    g.close()
    a.close()
    b.close()


def test_graph_rejects_bad_steps(tomo):
    a = tomo.Operator(16, 12, 23, grid=24, max_batch=2, device=0)
    x = torch.zeros((1, 16, 16), device="cuda")
    with pytest.raises(tomo.TomoError, match="EUNSUPPORTED"):
        tomo.Graph([dict(op=a, kind="normal", batch=1, inp=x, out=x.clone())])
    with pytest.raises(tomo.TomoError, match="EINVAL"):
        tomo.Graph([dict(op=a, kind="project", batch=3, inp=x, out=x.clone())])
    a.close()


def test_autotune_keeps_parity(tomo):
    n, nt, npb, batch = 64, 90, 91, 16
    op = tomo.Operator(n, nt, npb, max_batch=16, values=("f32", "bf16"), device=0)
    res = op.autotune(batch, values="bf16")
    assert res["fwd_ms"] > 0 and res["adj_ms"] > 0
    assert res["adj_sell_max"] <= res["adj_medium_max"]
    assert op.get_tuning()["adj_sell_max"] == res["adj_sell_max"]
    ref = oracle_op(n, nt, npb)
    g = ref.geom
    C = batch // 2
    rng = np.random.default_rng(5)
    Xc = rng.standard_normal((g.G * g.G, C, 2)).astype(np.float32)
    cm, pm = cart_map(g), polar_row_map(g)
    Xo = np.empty((g.G * g.G, C), dtype=np.complex128)
    Xo[cm] = Xc[..., 0] + 1j * Xc[..., 1]
    got = complex_channels(op.slice_fwd(torch.from_numpy(Xc).cuda(), batch))
    assert rel_l2(got, (ref.S_dag @ Xo)[pm]) < 1e-6
    Yc = rng.standard_normal((g.L * nt, C, 2)).astype(np.float32)
    Yo = np.empty((g.L * nt, C), dtype=np.complex128)
    Yo[pm] = Yc[..., 0] + 1j * Yc[..., 1]
    got = complex_channels(op.slice_adj(torch.from_numpy(Yc).cuda(), batch))
    assert rel_l2(got, (ref.S @ Yo)[cm]) < 1e-6
    op.close()


def test_graph_uneven_stack_shapes_match_oracle(tomo):
    """A captured graph over the uneven stack's two smallest operators (256^2 / 192 angles / 362
    bins and 512^2 / 384 / 724, fp16 values, odd uneven batches of 5 and 3 slices): project,
    backproject and the SpMM pair of each, checked on every replay against the FP64 oracle with
    the same fp16-rounded matrix values (1e-5 relative L2 per slice for the operators, 1e-6 for
    the SpMMs, and the largest element error against the largest reference element)."""
    from oracle import Operator as OracleOperator, round_values
    from synth import phantom_stack

    dev = "cuda"
    cases = []
    for (n, nt, npb, batch) in ((256, 192, 362, 5), (512, 384, 724, 3)):
        op = tomo.Operator(n, nt, npb, max_batch=batch, values=("f16",), device=0)
        ref = OracleOperator(oracle_op(n, nt, npb).geom, S=round_values(oracle_op(n, nt, npb).S, "f16"))
        bufs = dict(x=torch.empty((batch, n, n), device=dev), y=torch.empty((batch, nt, npb), device=dev),
                    yin=torch.empty((batch, nt, npb), device=dev), xb=torch.empty((batch, n, n), device=dev),
                    Xc=torch.empty(op.cart_shape(batch), device=dev), Yp=torch.empty(op.polar_shape(batch), device=dev),
                    Xa=torch.empty(op.cart_shape(batch), device=dev))
        cases.append((op, ref, batch, bufs))
    steps = []
    for op, ref, batch, t in cases:
        steps += [dict(op=op, kind="project", batch=batch, values="f16", inp=t["x"], out=t["y"]),
                  dict(op=op, kind="backproject", batch=batch, values="f16", inp=t["yin"], out=t["xb"]),
                  dict(op=op, kind="spmm_pair", batch=batch, values="f16", inp=t["Xc"], out=t["Yp"], aux=t["Xa"])]

    def errs(a, b):
        return rel_l2(a, b), float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    def fill(rep):
        for k, (op, ref, batch, t) in enumerate(cases):
            n = op.n
            t["x"].copy_(torch.from_numpy(phantom_stack(n, batch, seed_base=4000 + 100 * rep + 10 * k,
                                                        supersample=1).astype(np.float32)))
            _fill(t["yin"], 50 + 10 * rep + k)
            _fill(t["Xc"], 60 + 10 * rep + k)

    fill(0)
    g = tomo.Graph(steps)
    for rep in range(2):
        fill(rep + 1)
        g.launch()
        torch.cuda.synchronize()
        for op, ref, batch, t in cases:
            geo = ref.geom
            cm, pm = cart_map(geo), polar_row_map(geo)
            x = t["x"].cpu().numpy().astype(np.float64)
            y = t["y"].cpu().numpy().astype(np.float64)
            yin = t["yin"].cpu().numpy().astype(np.float64)
            xb = t["xb"].cpu().numpy().astype(np.float64)
            for s in range(batch):
                l2, mx = errs(y[s], ref.project(x[s]))
                assert l2 < 1e-5 and mx < 1e-5, (op.n, rep, s, "project", l2, mx)
                l2, mx = errs(xb[s], ref.backproject(yin[s]))
                assert l2 < 1e-5 and mx < 1e-5, (op.n, rep, s, "backproject", l2, mx)
            cm_inv = np.empty_like(cm)
            cm_inv[cm] = np.arange(cm.size)
            pm_inv = np.empty_like(pm)
            pm_inv[pm] = np.arange(pm.size)
            Yl = t["Yp"].cpu().numpy()
            summation_bound_check(f"{op.n}^2 replay {rep} forward", Yl, ref.S_dag, pm,
                                  t["Xc"].cpu().numpy(), cm_inv)
            summation_bound_check(f"{op.n}^2 replay {rep} adjoint", t["Xa"].cpu().numpy(), ref.S, cm,
                                  Yl, pm_inv)
            print(f"graph replay {rep}: {op.n}^2 batch {batch} fp16 matches the oracle")
    g.close()
    for op, _, _, _ in cases:
        op.close()
