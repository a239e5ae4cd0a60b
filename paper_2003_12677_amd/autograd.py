"""Differentiable reconstruction on top of the HIP operators (Sec. 2: the model-based problem,
a data misfit of the Radon transform plus mu times a total-variation regulariser).

* :func:`project` / :func:`backproject` are ``torch.autograd.Function`` pairs: the backward of
  the forward projection is the exact adjoint (``tomo_backproject``, Eq. (2) second line with
  D = I) and the backward of the back projection is the forward projection.
* :func:`tv` is the smoothed isotropic total variation per slice (``tomo_tv``: value and
  gradient in one pass over the image).
* :func:`model_loss` is ``||A x - b||^2 + mu * TV_eps(x)`` per slice, and
  :func:`reconstruct_tv` minimises it with Adam, writing a checkpoint (image, optimiser state,
  loss history) every ``checkpoint_every`` steps and resuming from the newest one.

Every operator application runs in the library's kernels; torch provides the tensors, the
element-wise residual and the optimiser.
"""

from __future__ import annotations

import os
import threading

import torch

from . import Operator


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op: Operator, values: str):
        ctx.op, ctx.values = op, values
        return op.project(x.contiguous(), values=values)

    @staticmethod
    def backward(ctx, gy):
        return ctx.op.backproject(gy.contiguous(), values=ctx.values), None, None


class _Backproject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, op: Operator, values: str):
        ctx.op, ctx.values = op, values
        return op.backproject(y.contiguous(), values=values)

    @staticmethod
    def backward(ctx, gx):
        return ctx.op.project(gx.contiguous(), values=ctx.values), None, None


class _TV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op: Operator, eps: float):
        value, grad = op.tv(x.contiguous(), eps, grad=ctx.needs_input_grad[0])
        ctx.save_for_backward(grad if grad is not None else x.new_empty(0))
        return value

    @staticmethod
    def backward(ctx, gv):
        (grad,) = ctx.saved_tensors
        return grad * gv.to(grad.dtype)[:, None, None], None, None


def project(x: torch.Tensor, op: Operator, values: str = "f32") -> torch.Tensor:
    """A x for a stack x[B][n][n]; differentiable (backward = A^T)."""
    return _Project.apply(x, op, values)


def backproject(y: torch.Tensor, op: Operator, values: str = "f32") -> torch.Tensor:
    """A^T y for a stack y[B][n_angles][n_det]; differentiable (backward = A)."""
    return _Backproject.apply(y, op, values)


def tv(x: torch.Tensor, op: Operator, eps: float = 1e-8) -> torch.Tensor:
    """TV_eps per slice as float64 [B]; differentiable."""
    return _TV.apply(x, op, eps)


def model_loss(x: torch.Tensor, b: torch.Tensor, op: Operator, mu: float = 1e-3,
               eps: float = 1e-8, values: str = "f32") -> torch.Tensor:
    """Per-slice ``||A x - b||^2 + mu * TV_eps(x)`` as float64 [B]."""
    r = project(x, op, values) - b
    return (r * r).sum(dim=(1, 2), dtype=torch.float64) + mu * tv(x, op, eps)


def _checkpoint_path(directory: str) -> str:
    return os.path.join(directory, "tv_recon.pt")


def reconstruct_tv(op: Operator, b: torch.Tensor, *, mu: float = 1e-3, eps: float = 1e-8,
                   steps: int = 200, lr: float = 1e-2, x0: torch.Tensor | None = None,
                   values: str = "f32", checkpoint_dir: str | None = None,
                   checkpoint_every: int = 10, resume: bool = True):
    """Minimise ``sum over slices of ||A x - b||^2 + mu TV_eps(x)`` with Adam.

    Returns ``(x, history)`` where history[k] is the per-slice loss (float64 [B], on the host)
    before step k.  With ``checkpoint_dir`` the state after every ``checkpoint_every`` steps is
    copied to host memory and written by a background thread (atomically, through a rename;
    the run returns only after the last write), and with ``resume`` a run restarts from the
    newest checkpoint there (same inputs and settings continue the run bit for bit)."""
    B = b.shape[0]
    x = (torch.zeros((B, op.n, op.n), dtype=torch.float32, device=b.device) if x0 is None
         else x0.detach().clone()).requires_grad_(True)
    opt = torch.optim.Adam([x], lr=lr)
    history: list = []
    start = 0
    if checkpoint_dir is not None:
        os.makedirs(checkpoint_dir, exist_ok=True)
        path = _checkpoint_path(checkpoint_dir)
        if resume and os.path.exists(path):
            state = torch.load(path, map_location="cpu", weights_only=True)
            with torch.no_grad():
                x.copy_(state["x"])
            opt.load_state_dict(state["adam"])          # moves the moments to x's device
            history = list(state["history"])
            start = int(state["step"])
    writer = None

    def write(state, path):
        tmp = path + ".tmp"
        torch.save(state, tmp)
        os.replace(tmp, path)

    def host_copy(obj):
        if isinstance(obj, torch.Tensor):
            return obj.detach().to("cpu", copy=True)
        if isinstance(obj, dict):
            return {k: host_copy(v) for k, v in obj.items()}
        if isinstance(obj, list):
            return [host_copy(v) for v in obj]
        return obj

    try:
        for k in range(start, steps):
            opt.zero_grad(set_to_none=False)
            loss = model_loss(x, b, op, mu, eps, values)
            loss.sum().backward()
            history.append(loss.detach().cpu())
            opt.step()
            if checkpoint_dir is not None and ((k + 1) % checkpoint_every == 0 or k + 1 == steps):
                # snapshot to host memory now, write to disk while the device keeps going (at most
                # one write in flight; each write is atomic through a rename)
                state = host_copy({"step": k + 1, "x": x, "adam": opt.state_dict(),
                                   "history": history})
                if writer is not None:
                    writer.join()
                writer = threading.Thread(target=write, args=(state, _checkpoint_path(checkpoint_dir)))
                writer.start()
    finally:
        if writer is not None:
            writer.join()
    return x.detach(), history
