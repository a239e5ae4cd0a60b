"""Benchmark: slices/s of the forward + adjoint gridding SpMM (S^dagger then S) at a 2048^2
image, 1501 angles over [0, pi), 2048 detector bins, one batch of 32 slices (16 complex
channels), matrix values in bfloat16 (mixed) and float32, float32 accumulation.

One step = one forward SpMM + one adjoint SpMM over the batch, inputs resident in HBM.
Besides the contract line it reports, for the same workload: per-kernel durations and the
HBM roofline fraction of the dominant kernel, the float32-value rate, the full operator
(project + backproject incl. FFTs) and a CGLS iteration, and the FP64 oracle timed on the
host cores.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
N_IMG, N_ANG, N_DET, BATCH = 2048, 1501, 2048, 32
WORKLOAD = "parallel-beam 2048x2048, 1501 angles in [0,pi), 2048 bins, batch 32 slices"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    p.add_argument("--extras", type=int, default=1, help="also time the full operator and CGLS")
    return p.parse_args()


def algorithmic_bytes(info, value_bytes: int, C: int):
    """Bytes the method must move per SpMM launch: matrix once (values + int32 columns + row
    pointers), every gathered vector row once (8*C bytes), every output row once."""
    nnz, N, M = info.nnz, info.n_polar, info.n_cart
    fwd = nnz * (value_bytes + 4) + 4 * (N + 1) + 8 * C * (info.cols_touched + N)
    adj = nnz * (value_bytes + 4) + 4 * (M + 1) + 8 * C * (info.polar_nonempty + M)
    return fwd, adj


def time_loop(torch, fn, iters: int) -> float:
    """Average milliseconds of fn() over iters launches, HIP events on the current stream."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(iters):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / iters


def cpu_baseline(budget_s: float):
    """The FP64 oracle's forward and adjoint sparse products (S^dagger U, S V') per slice on the
    host, on as many slices as fit the time budget."""
    import numpy as np

    from oracle import Geometry, Operator

    t0 = time.perf_counter()
    ref = Operator(Geometry(N_IMG, N_ANG, N_DET))
    build_s = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    U = rng.standard_normal((N_DET, N_DET)) + 1j * rng.standard_normal((N_DET, N_DET))
    V = rng.standard_normal((N_ANG, N_DET)) + 1j * rng.standard_normal((N_ANG, N_DET))
    done = 0
    t0 = time.perf_counter()
    while True:
        ref.slice_forward(U)
        ref.slice_adjoint(V)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or done >= 64:
            break
    return {"value": done / el, "unit": "slices/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} slices of S^dagger U + S V' (scipy CSR, complex128 vectors), "
                      f"{el:.1f} s; operator build {build_s:.1f} s not timed"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2003_12677_amd as tomo

    tomo.load()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    op = tomo.Operator(N_IMG, N_ANG, N_DET, max_batch=BATCH, values=("f32", "bf16"), device=0)
    build_s = time.perf_counter() - t0
    info = op.info
    C = BATCH // 2
    gen = torch.Generator(device=dev)
    gen.manual_seed(1234)
    Xc = torch.randn(op.cart_shape(BATCH), generator=gen, device=dev)
    Yp = torch.randn(op.polar_shape(BATCH), generator=gen, device=dev)
    Yo = torch.empty_like(Yp)
    Xo = torch.empty_like(Xc)

    def step(values):
        op.slice_fwd(Xc, BATCH, Yp=Yo, values=values)
        op.slice_adj(Yp, BATCH, Xc=Xo, values=values)

    # warmup, then exactly K timed steps bracketed by synchronisations
    for _ in range(args.warmup):
        step("bf16")
    torch.cuda.synchronize()
    ms_step = time_loop(torch, lambda: step("bf16"), args.steps)
    value = BATCH / (ms_step * 1e-3)

    res = {}
    for vt, vb in (("bf16", 2), ("f32", 4)):
        fwd_ms = time_loop(torch, lambda: op.slice_fwd(Xc, BATCH, Yp=Yo, values=vt), args.steps)
        adj_ms = time_loop(torch, lambda: op.slice_adj(Yp, BATCH, Xc=Xo, values=vt), args.steps)
        fb, ab = algorithmic_bytes(info, vb, C)
        res[vt] = {"fwd_ms": fwd_ms, "adj_ms": adj_ms, "fwd_GBs": fb / fwd_ms / 1e6,
                   "adj_GBs": ab / adj_ms / 1e6, "fwd_bytes": fb, "adj_bytes": ab}
    ms_f32 = time_loop(torch, lambda: step("f32"), args.steps)

    # device-to-device copy of a known size: the achievable streaming bandwidth on this GPU, and
    # the calibration kernel for HBM byte counters
    copy_bytes = 1 << 30
    src = torch.empty(copy_bytes // 4, dtype=torch.float32, device=dev).uniform_()
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms = time_loop(torch, lambda: dst.copy_(src), 20)
    copy_gbs = 2 * copy_bytes / copy_ms / 1e6
    del src, dst

    m = res["bf16"]
    dom = "adj" if m["adj_ms"] >= m["fwd_ms"] else "fwd"
    achieved = m[f"{dom}_GBs"]
    out = {
        "metric": "slices/s fwd+adj SpMM at 2048², 1501 angles; % HBM roofline; mixed vs FP32",
        "value": value,
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": N_IMG, "n_angles": N_ANG, "n_det": N_DET,
                   "batch": BATCH, "complex_channels": C, "values": "bf16", "accumulate": "f32",
                   "kernel_width": info.kw, "nnz": info.nnz, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": f"spmm_{dom}", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "frac_of_copy": achieved / copy_gbs},
        "copy_GBs": {"value": copy_gbs, "what": "torch copy_ of 1 GiB (read + write bytes / time)"},
        "kernels": res,
        "fp32_values": {"value": BATCH / (ms_f32 * 1e-3), "ms_per_step": ms_f32},
        "mixed_vs_fp32": ms_f32 / ms_step,
        "operator_build_s": build_s,
    }
    if args.extras:
        x = torch.rand((BATCH, N_IMG, N_IMG), generator=gen, device=dev)
        y = op.project(x)
        xb = torch.empty_like(x)
        ms_op = {}
        for vt in ("bf16", "f32"):
            op.project(x, y, values=vt)
            op.backproject(y, xb, values=vt)
            ms_op[vt] = time_loop(torch, lambda: (op.project(x, y, values=vt),
                                                  op.backproject(y, xb, values=vt)), 10)
        out["operator"] = {"what": "project + backproject (embed, 2D FFT, SpMM, 1D FFT, crop; and back)",
                           "slices_per_s_bf16": BATCH / (ms_op["bf16"] * 1e-3),
                           "slices_per_s_f32": BATCH / (ms_op["f32"] * 1e-3),
                           "ms_bf16": ms_op["bf16"], "ms_f32": ms_op["f32"]}
        op.solve(y, xb, iters=1)
        ms_cg = time_loop(torch, lambda: op.solve(y, xb, iters=10), 2)
        ms_cg1 = time_loop(torch, lambda: op.solve(y, xb, iters=0), 2)
        out["cgls"] = {"ms_per_iteration_f32": (ms_cg - ms_cg1) / 10, "batch": BATCH}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    op.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
