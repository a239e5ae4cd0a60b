"""tomo_tv_noalloc, the allocation-free variant of tomo_tv (reduction partials in the library's
file-scope scratch array), called through the C ABI: its value and gradient equal tomo_tv's bit
for bit (same kernels, same reduction order) on two calls in a row, the second with a smaller
batch, then on a smaller operator sharing the same scratch array; a host-only operator and a
batch beyond the operator's maximum are rejected before anything is launched."""

import ctypes

import numpy as np
import pytest
import torch

from synth import phantom_stack

pytestmark = pytest.mark.gpu


def _call_noalloc(tomo, op, x, value, grad, eps, weight):
    lib = tomo.load()
    st = torch.cuda.current_stream(op.device).cuda_stream
    return lib.tomo_tv_noalloc(op._handle, x.data_ptr(), x.shape[0], ctypes.c_double(eps),
                               ctypes.c_double(weight), grad.data_ptr() if grad is not None else None,
                               value.data_ptr() if value is not None else None, st)


def test_tv_noalloc_matches_tv(tomo):
    eps, weight = 1e-8, 1e-3
    big = tomo.Operator(64, 90, 91, max_batch=6, device=0)
    small = tomo.Operator(24, 20, 33, max_batch=2, device=0)
    for op, B, seed in ((big, 6, 700), (big, 3, 710), (small, 2, 720)):
        x = torch.from_numpy(phantom_stack(op.n, B, seed_base=seed, supersample=1).astype(np.float32)).cuda()
        v_ref, g_ref = op.tv(x, eps, weight)
        value = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        grad = torch.full_like(x, float("nan"))
        assert _call_noalloc(tomo, op, x, value, grad, eps, weight) == 0
        torch.cuda.synchronize()
        assert torch.equal(value, v_ref), (op.n, B)
        assert torch.equal(grad, g_ref), (op.n, B)
        # value only, and gradient only
        value2 = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        assert _call_noalloc(tomo, op, x, value2, None, eps, weight) == 0
        grad2 = torch.full_like(x, float("nan"))
        assert _call_noalloc(tomo, op, x, None, grad2, eps, weight) == 0
        torch.cuda.synchronize()
        assert torch.equal(value2, v_ref) and torch.equal(grad2, g_ref), (op.n, B)
    x = torch.zeros((7, 64, 64), device="cuda")
    value = torch.zeros(7, dtype=torch.float64, device="cuda")
    assert _call_noalloc(tomo, big, x, value, None, eps, weight) == -1          # TOMO_EINVAL
    host = tomo.Operator(16, 12, 23, device=-1)
    assert _call_noalloc(tomo, host, x[:1, :16, :16].contiguous(), value[:1], None, eps, weight) == -5
    host.close()
    small.close()
    big.close()
