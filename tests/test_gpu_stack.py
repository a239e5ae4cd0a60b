"""GPU tests of the persistent SpMM-pair launch over a stack of operators (tomo_stack_*): one
forward kernel and one adjoint kernel walk device work lists covering every (operator, batch)
item.

* Every item's products equal the FP64 oracle's CSR products with the same rounded values (every
  element within the float32 summation bound), and the item's own staged tomo_slice_fwd bit for
  bit, and its tomo_slice_adj too when that runs the same segment body on every tile
  (adj_dense_mode 2; with 1 the eager staged tiles sum in float32, the stack in float64); odd
  and even batches, f32 / bf16 / f16 values, several tile runs and segment lengths.
* At the uneven stack's two smallest shapes (256^2 / 192 / 362 and 512^2 / 384 / 724, fp16, odd
  batches) the stack, eager and captured in a HIP graph, matches the oracle on every replay.
* Operators whose adjoint keeps its dense tiles on the row kernels, and items that mix kernel
  widths, are rejected before anything is launched."""

import numpy as np
import pytest
import torch

from oracle import round_values
from tests.gpu_util import cart_map, oracle_op, polar_row_map, summation_bound_check

pytestmark = pytest.mark.gpu


def _fill(t, seed):
    g = torch.Generator(device=t.device)
    g.manual_seed(seed)
    t.copy_(torch.rand(t.shape, generator=g, device=t.device) * 2 - 1)


def _check_item(op, geom_args, batch, vt, Xc, Yp, Xa):
    """Both products of one item against the oracle's CSR (values rounded to vt when 16-bit),
    every element within the float32 summation bound."""
    ref = oracle_op(*geom_args)
    g = ref.geom
    cm, pm = cart_map(g), polar_row_map(g)
    cm_inv = np.empty_like(cm)
    cm_inv[cm] = np.arange(cm.size)
    pm_inv = np.empty_like(pm)
    pm_inv[pm] = np.arange(pm.size)
    S_dag = ref.S_dag if vt == "f32" else round_values(ref.S_dag, vt)
    S = ref.S if vt == "f32" else round_values(ref.S, vt)
    Xl, Yl = Xc.cpu().numpy(), Yp.cpu().numpy()
    summation_bound_check(f"{geom_args} b{batch} {vt} forward", Yl, S_dag, pm, Xl, cm_inv)
    summation_bound_check(f"{geom_args} b{batch} {vt} adjoint", Xa.cpu().numpy(), S, cm, Yl, pm_inv)


@pytest.mark.parametrize("vt", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("tuning", [dict(adj_dense_mode=1, adj_seg_chunks=2),
                                    dict(adj_dense_mode=2, adj_seg_chunks=1, adj_run=3,
                                         adj_tile_points=64),
                                    dict(adj_dense_mode=2, adj_seg_chunks=8, adj_run=8)],
                         ids=["mode1_k2", "mode2_k1_run3", "mode2_k8_run8"])
def test_stack_matches_oracle_and_eager(tomo, vt, tuning):
    geoms = [((64, 90, 91), [7, 4]), ((37, 30, 53), [3]), ((96, 120, 137), [5, 1])]
    dev = "cuda"
    items, keep = [], []
    for k, (ga, batches) in enumerate(geoms):
        op = tomo.Operator(*ga, max_batch=8, values=("f32", "bf16", "f16"), device=0)
        op.set_tuning(**tuning)
        keep.append(op)
        for j, b in enumerate(batches):
            Xc = torch.empty(op.cart_shape(b), device=dev)
            _fill(Xc, 100 * k + j)
            items.append(dict(op=op, geom=ga, batch=b, inp=Xc, out=torch.empty(op.polar_shape(b), device=dev),
                              aux=torch.empty(op.cart_shape(b), device=dev)))
    st = tomo.Stack([{k: it[k] for k in ("op", "batch", "inp", "out", "aux")} for it in items], values=vt)
    for rep in range(2):
        for j, it in enumerate(items):
            _fill(it["inp"], 1000 * rep + j)
        st.launch()
        torch.cuda.synchronize()
        for it in items:
            op, b = it["op"], it["batch"]
            _check_item(op, it["geom"], b, vt, it["inp"], it["out"], it["aux"])
            assert torch.equal(op.slice_fwd(it["inp"], b, values=vt), it["out"])
            if tuning["adj_dense_mode"] == 2:       # eager runs the same segment body on every tile
                assert torch.equal(op.slice_adj(it["out"], b, values=vt), it["aux"])
    st.close()
    for op in keep:
        op.close()


def test_stack_uneven_shapes_graph_replays_match_oracle(tomo):
    dev = "cuda"
    items, keep = [], []
    for k, (ga, b) in enumerate((((256, 192, 362), 5), ((512, 384, 724), 3))):
        op = tomo.Operator(*ga, max_batch=b, values=("f16",), device=0)
        op.set_tuning(adj_dense_mode=1)
        keep.append(op)
        items.append(dict(op=op, geom=ga, batch=b, inp=torch.empty(op.cart_shape(b), device=dev),
                          out=torch.empty(op.polar_shape(b), device=dev),
                          aux=torch.empty(op.cart_shape(b), device=dev)))
    st = tomo.Stack([{k: it[k] for k in ("op", "batch", "inp", "out", "aux")} for it in items], values="f16")
    for j, it in enumerate(items):
        _fill(it["inp"], 7 + j)
    st.launch()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            st.launch()
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for j, it in enumerate(items):
            _fill(it["inp"], 20 + 10 * rep + j)
        graph.replay()
        torch.cuda.synchronize()
        for it in items:
            _check_item(it["op"], it["geom"], it["batch"], "f16", it["inp"], it["out"], it["aux"])
            eager = it["op"].slice_fwd(it["inp"], it["batch"], values="f16")   # eager work between replays
            assert torch.equal(eager, it["out"])
        torch.cuda.synchronize()
        print(f"stack graph replay {rep}: matches the oracle")
    st.close()
    for op in keep:
        op.close()


def test_stack_rejects_bad_items(tomo):
    a = tomo.Operator(64, 90, 91, max_batch=2, device=0)
    b = tomo.Operator(37, 30, 53, max_batch=2, kw=5, device=0)
    dev = "cuda"

    def item(op):
        return dict(op=op, batch=2, inp=torch.zeros(op.cart_shape(2), device=dev),
                    out=torch.zeros(op.polar_shape(2), device=dev), aux=torch.zeros(op.cart_shape(2), device=dev))

    # the dense tiles' segments are built whatever adj_dense_mode selects for the eager adjoint
    a.set_tuning(adj_dense_mode=0)
    tomo.Stack([item(a)]).close()
    with pytest.raises(ValueError):
        tomo.Stack([dict(item(a), batch=0)])               # buffers not of the batch's shape
    a.set_tuning(adj_dense_mode=1)
    b.set_tuning(adj_dense_mode=1)
    with pytest.raises(tomo.TomoError, match="EINVAL"):
        tomo.Stack([item(a), item(b)])                     # different kernel widths
    with pytest.raises(tomo.TomoError, match="ESTATE"):
        tomo.Stack([item(a)], values="bf16")               # value type not built
    a.close()
    b.close()
