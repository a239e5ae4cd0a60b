"""Benchmark: slices/s of the forward + adjoint gridding SpMM (S^dagger then S) at a 2048^2
image, 1501 angles over [0, pi), 2048 detector bins, one batch of 32 slices (16 complex
channels), matrix values in bfloat16 (mixed) and float32, float32 accumulation.

One step = one forward SpMM + one adjoint SpMM over the batch, inputs resident in HBM.
Besides the contract line it reports, for the same workload: per-step percentiles, per-kernel
durations and the HBM roofline fraction of the dominant kernel (with the HBM bytes that the
counter summary under profiles/ measured for the same kernel source, when it matches), the
float32-value rate, the two-slice (one complex channel) form, the full operator (project +
backproject incl. FFTs) and a CGLS iteration, and the FP64 oracle timed on the host cores
(before the GPU is touched).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
N_IMG, N_ANG, N_DET, BATCH = 2048, 1501, 2048, 32
WORKLOAD = "parallel-beam 2048x2048, 1501 angles in [0,pi), 2048 bins, batch 32 slices"
COUNTERS = os.path.join(ROOT, "profiles", "spmm_2048_1501_b32_counters.json")
SPMM_SOURCES = [os.path.join(ROOT, "paper_2003_12677_amd", "csrc", f)
                for f in ("spmm.hip", "tiles.hip", "builder.cpp", "internal.h", "fft_lds.h")]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=8.0,
                   help="budget of each oracle sample (one process, then all host cores)")
    p.add_argument("--extras", type=int, default=1, help="also time the full operator and CGLS")
    p.add_argument("--uneven", action="store_true",
                   help="also time a 200-slice stack of mixed sizes (256..2048, fp16 values) as "
                        "eager launches and as one HIP graph, each operator autotuned")
    p.add_argument("--tv", action="store_true",
                   help="also time 200 Adam steps of the TV-regularised reconstruction at 1024^2, "
                        "720 angles, 1448 bins, 32 slices, with a checkpoint every 10 steps")
    p.add_argument("--accuracy", action="store_true",
                   help="also compare float32 and mixed-precision CGLS-100 with the FP64 oracle on 4 "
                        "noisy slices and time CGLS-100 on a 256-slice stack (several minutes)")
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


def step_percentiles(torch, fn, iters: int):
    """p10 / p50 / p90 of single-step durations (ms), one event pair per step."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(iters)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    d = sorted(a.elapsed_time(b) for a, b in ev)

    def q(f):
        return d[min(len(d) - 1, int(round(f * (len(d) - 1))))]

    return {"p10": q(0.1), "p50": q(0.5), "p90": q(0.9)}


def source_digest(tuning: dict) -> str:
    """Identity of the SpMM kernels a counter summary was taken from: their sources, the
    builder of their layouts and the operator's layout tuning."""
    h = hashlib.sha256()
    for f in SPMM_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(json.dumps(tuning, sort_keys=True).encode())
    return h.hexdigest()


def measured_traffic(kernel: str, tuning: dict):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by the copy-kernel calibration), or None when the summary is missing or
    was taken from different kernel sources."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != source_digest(tuning) or kernel not in c.get("kernels", {}):
        return None
    k = c["kernels"][kernel]
    return {"read_bytes": k["read_bytes"], "write_bytes": k["write_bytes"],
            "total_bytes": k["read_bytes"] + k["write_bytes"], "unit": "bytes per launch",
            "calibration": c.get("calibration")}


def _oracle_slices(budget_s: float, max_slices: int, seed: int):
    """Forward + adjoint sparse products of the FP64 oracle on as many slices as fit the budget;
    returns (slices, seconds).  Uses the operator built in the parent process (fork)."""
    import numpy as np

    ref = _ORACLE["op"]
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((N_DET, N_DET)) + 1j * rng.standard_normal((N_DET, N_DET))
    V = rng.standard_normal((N_ANG, N_DET)) + 1j * rng.standard_normal((N_ANG, N_DET))
    done = 0
    t0 = time.perf_counter()
    while True:
        ref.slice_forward(U)
        ref.slice_adjoint(V)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or done >= max_slices:
            return done, el


_ORACLE = {}


def host_cpu():
    """CPU model and physical core count of this host (lscpu), and the cores this process may use."""
    import subprocess

    model, sockets, per_socket = None, None, None
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "Model name":
                model = v
            elif k == "Socket(s)":
                sockets = int(v)
            elif k == "Core(s) per socket":
                per_socket = int(v)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    physical = sockets * per_socket if sockets and per_socket else None
    return {"cpu_model": model, "physical_cores": physical,
            "usable_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(budget_s: float):
    """The FP64 oracle's forward and adjoint sparse products (S^dagger U, S V') per slice on the
    host: one process, then one process per usable host core, each on its own slices (the
    slice decomposition of Sec. 3.1).  Runs before anything touches the GPU, so the forked
    workers hold no GPU state."""
    import multiprocessing as mp

    from oracle import Geometry, Operator

    t0 = time.perf_counter()
    _ORACLE["op"] = Operator(Geometry(N_IMG, N_ANG, N_DET))
    build_s = time.perf_counter() - t0
    one, el1 = _oracle_slices(budget_s, 64, 0)
    host = host_cpu()
    # one process per core this job may use, at most 16: the host share one GPU's job is given
    cores = min(16, host["usable_cores"])
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        parts = pool.starmap(_oracle_slices, [(budget_s, 64, 1 + i) for i in range(cores)])
    wall = time.perf_counter() - t0
    done = sum(p[0] for p in parts)
    rate = sum(p[0] / p[1] for p in parts)      # concurrent processes, each over its own loop
    _ORACLE.clear()
    return {"value": rate, "unit": "slices/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} slices of S^dagger U + S V' (scipy CSR, complex128 vectors) in "
                      f"{cores} concurrent processes, about {budget_s:.0f} s each ({wall:.1f} s "
                      f"wall); operator build {build_s:.1f} s not timed",
            "host": dict(host, note="processes are capped at 16, the host CPU share of a one-GPU job"),
            "single_process": {"value": one / el1, "cores": 1,
                               "sample": f"{one} slices in {el1:.1f} s"}}


ACC_SLICES, ACC_ITERS = 4, 100


def _accuracy_inputs():
    """Seeded noisy sinograms in pixel units: exact line integrals of 10 random ellipses per slice
    with Poisson noise at I0 = 1e4, stored as float32 (what the GPU receives); and the phantoms
    themselves rasterised with 2x2 supersampling (the ground truth)."""
    import math

    import numpy as np

    from synth import (ellipse_params, ellipse_sinogram, poisson_log_sinogram,
                       rasterize_ellipses, slice_rng)

    th = np.arange(N_ANG) * math.pi / N_ANG
    sinos, truth = [], []
    for s in range(ACC_SLICES):
        rng = slice_rng(3000 + s)
        E = ellipse_params(rng, 10, contained=True)
        P = poisson_log_sinogram(rng, ellipse_sinogram(E, th, N_DET, N_DET // 2, N_IMG), 1e4)
        sinos.append((P / (2.0 / N_IMG)).astype(np.float32))
        truth.append(rasterize_ellipses(E, N_IMG, 2))
    return np.stack(sinos), truth


def _progress(tag: str):
    calls = [0]

    def hook(v):                 # identity on the stored vectors; reports every 10 iterations
        calls[0] += 1
        if calls[0] % 50 == 0:
            print(f"oracle {tag}: ~{calls[0] // 5} iterations", file=sys.stderr, flush=True)
        return v

    return hook


def _oracle_solves(s: int):
    """FP64 CGLS-100, and the FP64 form of the mixed-precision solve (4 outer steps with
    float32-rounded values for the residual, 25 inner CGLS steps with bfloat16-rounded values)."""
    from oracle import cgls, refine

    hi, hi32, lo = _ORACLE["op"], _ORACLE["op32"], _ORACLE["op16"]
    b = _ORACLE["b"][s].astype("float64")
    x = cgls(hi.project, hi.backproject, b, ACC_ITERS, store=_progress(f"CGLS slice {s}"))
    xr = refine(hi32.project, lo.project, lo.backproject, b, 4, ACC_ITERS // 4,
                store=_progress(f"refinement slice {s}"))
    return x, xr


def accuracy_reference():
    """The oracle's solves of each accuracy slice, one forked process per slice, before the GPU
    is touched."""
    import multiprocessing as mp

    from oracle import Geometry, Operator, round_values

    b, truth = _accuracy_inputs()
    op = Operator(Geometry(N_IMG, N_ANG, N_DET))
    _ORACLE.update(op=op, op32=Operator(op.geom, S=round_values(op.S, "f32")),
                   op16=Operator(op.geom, S=round_values(op.S, "bf16")), b=b)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(ACC_SLICES) as pool:
        xs = pool.map(_oracle_solves, range(ACC_SLICES))
    el = time.perf_counter() - t0
    _ORACLE.clear()
    return b, truth, xs, el


def accuracy_leg(torch, tomo, op, ref):
    """Errors of the GPU reconstructions against the oracle's (the same algorithm in float64) and
    against the phantoms, and CGLS-100 wall time for a 256-slice stack (8 batches of 32)."""
    import numpy as np

    b_host, truth, x_ref, oracle_s = ref
    dev = torch.device("cuda:0")
    b = torch.from_numpy(b_host).to(dev)

    def rel(a, r):
        return float(np.linalg.norm(a - r) / np.linalg.norm(r))

    forms = {"cgls_f32": dict(iters=ACC_ITERS),
             "cgls_bf16": dict(iters=ACC_ITERS, values="bf16"),
             "cgls_mixed_bf16_4x25": dict(iters=ACC_ITERS // 4, refine_outer=4, values="bf16"),
             "cgnr_f32": dict(iters=ACC_ITERS, method="cgnr"),
             "cgnr_mixed_bf16_4x25": dict(iters=ACC_ITERS // 4, refine_outer=4, values="bf16",
                                          method="cgnr")}
    res = {"slices": ACC_SLICES, "iterations": ACC_ITERS, "oracle_seconds": oracle_s,
           "inputs": "exact ellipse line integrals with Poisson noise (I0 = 1e4), float32",
           "oracle_cgls_vs_phantom": [rel(x_ref[s][0], truth[s]) for s in range(ACC_SLICES)]}
    for name, kw in forms.items():
        xh = op.solve(b, **kw).cpu().numpy().astype(np.float64)
        # the oracle solve of the same algorithm (CG on the normal equations is CGLS in exact
        # arithmetic, so both inner forms are compared with the oracle's CGLS refinement)
        same = 1 if "4x25" in name else 0
        res[name] = {"rel_l2_vs_oracle_same_algorithm":
                     [rel(xh[s], x_ref[s][same]) for s in range(ACC_SLICES)],
                     "rel_l2_vs_phantom": [rel(xh[s], truth[s]) for s in range(ACC_SLICES)]}
    e32 = np.mean(res["cgls_f32"]["rel_l2_vs_phantom"])
    res["mixed_over_f32_phantom_error"] = float(np.mean(res["cgls_mixed_bf16_4x25"]["rel_l2_vs_phantom"]) / e32)
    res["bf16_over_f32_phantom_error"] = float(np.mean(res["cgls_bf16"]["rel_l2_vs_phantom"]) / e32)
    res["mixed_cgnr_over_f32_phantom_error"] = float(
        np.mean(res["cgnr_mixed_bf16_4x25"]["rel_l2_vs_phantom"]) / e32)
    # timing: 256 slices as 8 batches of 32 (inputs: projections of random images; speed does
    # not depend on the values)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    stack = op.project(torch.rand((BATCH, N_IMG, N_IMG), generator=gen, device=dev))
    xb = torch.empty((BATCH, N_IMG, N_IMG), device=dev)
    for name, kw in forms.items():
        op.solve(stack, xb, **dict(kw, iters=1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(256 // BATCH):
            op.solve(stack, xb, **kw)
        torch.cuda.synchronize()
        res[name]["stack256_seconds"] = time.perf_counter() - t0
    return res


STACK_SLICES, STACK_ITERS = 256, 100


def _stack_slice(s: int):
    """Slice s of the 2048^2 stack: exact ellipse line integrals with Poisson noise (I0 = 1e4) in
    pixel units as float32, and the phantom rasterised with 2x2 supersampling."""
    import math

    import numpy as np

    from synth import (ellipse_params, ellipse_sinogram, poisson_log_sinogram,
                       rasterize_ellipses, slice_rng)

    th = np.arange(N_ANG) * math.pi / N_ANG
    rng = slice_rng(5000 + s)
    E = ellipse_params(rng, 10, contained=True)
    P = poisson_log_sinogram(rng, ellipse_sinogram(E, th, N_DET, N_DET // 2, N_IMG), 1e4)
    return (P / (2.0 / N_IMG)).astype(np.float32), rasterize_ellipses(E, N_IMG, 2).astype(np.float32)


def stack_inputs():
    """One batch of 32 phantom slices and their noisy sinograms, made by a process pool before
    the GPU is touched."""
    import multiprocessing as mp

    import numpy as np

    procs = min(16, len(os.sched_getaffinity(0)), BATCH)
    with mp.get_context("fork").Pool(procs) as pool:
        out = pool.map(_stack_slice, range(BATCH))
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def stack_leg(torch, op, inputs):
    """The 2048^2 / 1501 / 2048 reconstruction workload: a 256-slice stack streamed through the
    GPU in batches of 32, CGLS-100 per batch, as plain float32, with bf16 values, and as float32
    iterative refinement (4 outer float32 residuals of 25 inner iterations with bf16 values, the
    inner solves as CGLS or as CG on the normal equations through the bf16 normal-operator
    stencil).  Errors: relative L2 against the phantoms of one batch (32 slices); times: the
    whole stack (8 batches; the speed does not depend on the values)."""
    import numpy as np

    sino, truth = inputs
    dev = torch.device("cuda:0")
    b = torch.from_numpy(sino).to(dev)
    t = torch.from_numpy(truth).to(dev)
    forms = {"cgls_f32": dict(iters=STACK_ITERS),
             "cgls_bf16": dict(iters=STACK_ITERS, values="bf16"),
             "cgnr_f32": dict(iters=STACK_ITERS, method="cgnr"),
             "mixed_cgls_bf16_4x25": dict(iters=STACK_ITERS // 4, refine_outer=4, values="bf16"),
             "mixed_cgnr_bf16_4x25": dict(iters=STACK_ITERS // 4, refine_outer=4, values="bf16",
                                          method="cgnr")}
    x = torch.empty((BATCH, N_IMG, N_IMG), device=dev)
    res = {"workload": f"{STACK_SLICES} slices of 2048^2, 1501 angles, 2048 bins in batches of "
                       f"{BATCH}; {STACK_ITERS} iterations per batch",
           "inputs": "exact line integrals of 10 random ellipses per slice with Poisson noise "
                     "(I0 = 1e4), float32; phantoms rasterised with 2x2 supersampling",
           "error_slices": BATCH}
    for name, kw in forms.items():
        op.solve(b, x, **kw)
        err = ((x - t).flatten(1).norm(dim=1) / t.flatten(1).norm(dim=1)).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(STACK_SLICES // BATCH):
            op.solve(b, x, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[name] = {"stack_seconds": el, "slices_per_s": STACK_SLICES / el,
                     "rel_l2_vs_phantom": {"mean": float(err.mean()), "min": float(err.min()),
                                           "max": float(err.max())}}
    ref = res["cgls_f32"]
    for name in ("mixed_cgls_bf16_4x25", "mixed_cgnr_bf16_4x25", "cgls_bf16", "cgnr_f32"):
        res[name]["time_over_cgls_f32"] = res[name]["stack_seconds"] / ref["stack_seconds"]
        res[name]["phantom_error_over_cgls_f32"] = (res[name]["rel_l2_vs_phantom"]["mean"] /
                                                     ref["rel_l2_vs_phantom"]["mean"])
    return res


def paper_comparison(torch, tomo, gen):
    """The paper's only GPU throughput figure is for iRadon (filtered back projection incl. the
    FFTs) of a 2048-slice stack with 2048 angles and 2048 bins.  The same operation here: one
    MI355X, tomo_irradon with the Hamming-windowed ramp on batches of 32 slices at (2048 angles,
    2048 bins, 2048^2 pixels), float32 values."""
    dev = torch.device("cuda:0")
    op = tomo.Operator(N_IMG, 2048, N_DET, max_batch=BATCH, device=0)
    y = torch.rand((BATCH, 2048, N_DET), generator=gen, device=dev)
    x = torch.empty((BATCH, N_IMG, N_IMG), device=dev)
    op.irradon(y, x)
    ms = time_loop(torch, lambda: op.irradon(y, x), 10)
    op.close()
    return {"ours": {"what": "tomo_irradon, 2048^2 pixels, 2048 angles, 2048 bins, batch 32, f32 values",
                     "gpus": "1 x MI355X", "slices_per_s": BATCH / (ms * 1e-3), "ms_per_batch": ms},
            "paper": [
                {"what": "iRadon of (n_z, n_theta, n_p) = (2048, 2048, 2048)", "seconds": 1.55,
                 "hardware": "16 x NVIDIA V100 16 GB (Cori GPU nodes)", "slices_per_s": 2048 / 1.55,
                 "slices_per_s_per_gpu": 2048 / 1.55 / 16, "section": "Sec. 4 (Cori GPU results)"},
                {"what": "iRadon of (2048, 2048, 2048)", "seconds": 4.11,
                 "hardware": "256 Intel Haswell cores (8 Cori nodes), MPI", "slices_per_s": 2048 / 4.11,
                 "section": "Sec. 4 (Cori CPU results)"},
                {"what": "iRadon of the bread-crumb scan (n_z, n_theta, n_p) = (128, 1313, 3620)",
                 "seconds": 4.0, "hardware": "8 GPUs of 4 x NVIDIA K80 (CAM)", "slices_per_s": 128 / 4.0,
                 "section": "Sec. 4 (experimental data)"}],
            "note": "context, not a target: other hardware, and the paper states no precision"}


def uneven_leg(torch, tomo):
    """200 slices with sizes drawn from {256, 512, 1024, 2048}^2 (seeded), 0.75 N angles,
    round(N sqrt 2) bins, fp16 matrix values: one operator per size, autotuned for batches of
    32; each operator's slices go in batches of <= 32 (the last one uneven).  One step = the
    forward + adjoint SpMM of every batch; timed as eager launches and as one HIP graph."""
    import math

    import numpy as np

    sizes = np.random.default_rng(2020).choice([256, 512, 1024, 2048], size=200)
    dev = torch.device("cuda:0")
    res = {"slices": 200, "values": "f16", "operators": []}
    steps, eager = [], []
    for n in (256, 512, 1024, 2048):
        count = int((sizes == n).sum())
        if count == 0:
            continue
        nt, npb = round(0.75 * n), round(n * math.sqrt(2))
        print(f"uneven: building and tuning the {n}^2 operator", file=sys.stderr, flush=True)
        op = tomo.Operator(n, nt, npb, max_batch=BATCH, values=("f16",), device=0)
        tune = op.autotune(BATCH, values="f16")
        gen = torch.Generator(device=dev)
        gen.manual_seed(n)
        batches = [BATCH] * (count // BATCH) + ([count % BATCH] if count % BATCH else [])
        bufs = {}
        for b in sorted(set(batches)):            # one buffer set per batch width
            Xc = torch.rand(op.cart_shape(b), generator=gen, device=dev)
            bufs[b] = (Xc, torch.empty(op.polar_shape(b), device=dev), torch.empty_like(Xc))
        for b in batches:
            Xc, Yp, Xa = bufs[b]
            steps.append(dict(op=op, kind="spmm_pair", batch=b, values="f16", inp=Xc, out=Yp, aux=Xa))
            eager.append((op, b, Xc, Yp, Xa))
        res["operators"].append({"n": n, "n_angles": nt, "n_det": npb, "slices": count,
                                 "batches": batches, "nnz": op.info.nnz,
                                 "tuned": {k: tune[k] for k in ("fwd_tiled", "adj_tiled", "tile",
                                           "tile_points", "adj_tile_points", "tile_strip",
                                           "fwd_rows_per_group",
                                           "fwd_channels_per_lane", "adj_channels_per_lane",
                                           "adj_sell_max", "adj_medium_max",
                                           "adj_sell_xcd_rows", "adj_medium_xcd_rows",
                                           "adj_dense_mode", "adj_seg_chunks", "adj_run")},
                                 "tuned_ms_b32": [tune["fwd_ms"], tune["adj_ms"]]})

    print("uneven: timing eager launches, the graph and the stack", file=sys.stderr, flush=True)

    def run_eager():
        for op, b, Xc, Yp, Xa in eager:
            op.slice_fwd(Xc, b, Yp=Yp, values="f16")
            op.slice_adj(Yp, b, Xc=Xa, values="f16")

    graph = tomo.Graph(steps)
    for _ in range(3):
        run_eager()
        graph.launch()
    ms_e = time_loop(torch, run_eager, 20)
    ms_g = time_loop(torch, graph.launch, 20)
    graph.close()
    res.update(steps=len(steps), eager_ms=ms_e, graph_ms=ms_g,
               eager_slices_per_s=200 / (ms_e * 1e-3), graph_slices_per_s=200 / (ms_g * 1e-3))
    # the same SpMM pairs as one persistent forward and one persistent adjoint launch over every
    # operator's staged work
    ops = []
    for st in steps:
        if st["op"] not in ops:
            ops.append(st["op"])
    # one kernel per operator set needs one tile side for all (8, the default)
    for op in ops:
        op.set_tuning(tile=8)
    stack = tomo.Stack([dict(op=st["op"], batch=st["batch"], inp=st["inp"], out=st["out"], aux=st["aux"])
                        for st in steps], values="f16")
    stack.launch()
    torch.cuda.synchronize()
    cg = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(cg, stream=side):
            stack.launch()
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(3):
        stack.launch()
        cg.replay()
    ms_s = time_loop(torch, stack.launch, 20)
    ms_sg = time_loop(torch, cg.replay, 20)
    stack.close()
    res.update(stack_ms=ms_s, stack_graph_ms=ms_sg, stack_slices_per_s=200 / (ms_s * 1e-3),
               stack_graph_slices_per_s=200 / (ms_sg * 1e-3),
               stack_what="one persistent forward kernel + one persistent adjoint kernel (+ split-"
                          "tile sums) over device work lists of every operator's batches (tile side "
                          "8 and staged dense tiles on every operator)")
    return res


def tv_leg(torch, tomo):
    """Differentiable reconstruction: ||A x - b||^2 + 1e-3 TV_eps(x) (eps = 1e-8) minimised by
    Adam for 200 steps at 1024^2 / 720 / 1448 with 32 slices, checkpoint every 10 steps.
    Inputs: exact ellipse line integrals of 32 seeded phantoms (pixel units)."""
    import math
    import tempfile

    import numpy as np

    from paper_2003_12677_amd.autograd import reconstruct_tv
    from synth import ellipse_params, ellipse_sinogram, rasterize_ellipses, slice_rng

    n, nt, npb, B = 1024, 720, 1448, 32
    th = np.arange(nt) * math.pi / nt
    sinos, truth = [], []
    for s in range(B):
        E = ellipse_params(slice_rng(4000 + s), 10, contained=True)
        sinos.append(ellipse_sinogram(E, th, npb, npb // 2, n) / (2.0 / n))
        if s < 4:
            truth.append(rasterize_ellipses(E, n, 2))
    dev = torch.device("cuda:0")
    b = torch.from_numpy(np.stack(sinos).astype(np.float32)).to(dev)
    op = tomo.Operator(n, nt, npb, max_batch=B, device=0)
    reconstruct_tv(op, b, mu=1e-3, eps=1e-8, steps=2, lr=2e-2)         # warm-up (plans, buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reconstruct_tv(op, b, mu=1e-3, eps=1e-8, steps=20, lr=2e-2)
    torch.cuda.synchronize()
    no_ck = (time.perf_counter() - t0) / 20
    with tempfile.TemporaryDirectory() as ck:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, hist = reconstruct_tv(op, b, mu=1e-3, eps=1e-8, steps=200, lr=2e-2,
                                 checkpoint_dir=ck, checkpoint_every=10)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    xh = x[:4].cpu().numpy().astype(np.float64)
    err = [float(np.linalg.norm(xh[s] - truth[s]) / np.linalg.norm(truth[s])) for s in range(4)]
    op.close()
    first, last = hist[0].sum().item(), hist[-1].sum().item()
    return {"workload": "1024^2, 720 angles, 1448 bins, 32 slices, 200 Adam steps (lr 2e-2), "
                        "loss ||Ax-b||^2 + 1e-3 TV_eps, eps 1e-8, checkpoint every 10 steps",
            "seconds": el, "ms_per_step": el / 200 * 1e3, "slices_per_s": B * 200 / el,
            "ms_per_step_without_checkpoints": no_ck * 1e3,
            "loss_first": first, "loss_last": last,
            "rel_l2_vs_phantom_slices_0_3": err}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds)
    acc_ref = accuracy_reference() if args.accuracy else None
    stack_in = stack_inputs() if args.extras else None
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
    pct = step_percentiles(torch, lambda: step("bf16"), args.steps)

    res = {}
    for vt, vb in (("bf16", 2), ("f32", 4)):
        fwd_ms = time_loop(torch, lambda: op.slice_fwd(Xc, BATCH, Yp=Yo, values=vt), args.steps)
        adj_ms = time_loop(torch, lambda: op.slice_adj(Yp, BATCH, Xc=Xo, values=vt), args.steps)
        fb, ab = algorithmic_bytes(info, vb, C)
        res[vt] = {"fwd_ms": fwd_ms, "adj_ms": adj_ms, "fwd_GBs": fb / fwd_ms / 1e6,
                   "adj_GBs": ab / adj_ms / 1e6, "fwd_bytes": fb, "adj_bytes": ab}
    ms_f32 = time_loop(torch, lambda: step("f32"), args.steps)

    # the paper's form: one pair of slices (a single complex channel) per product
    X2 = Xc[:, :1].contiguous()
    Y2 = Yp[:, :1].contiguous()
    Y2o = torch.empty_like(Y2)
    X2o = torch.empty_like(X2)
    pair = {}
    for vt in ("bf16", "f32"):
        ms = time_loop(torch, lambda: (op.slice_fwd(X2, 2, Yp=Y2o, values=vt),
                                       op.slice_adj(Y2, 2, Xc=X2o, values=vt)), args.steps)
        pair[vt] = {"ms_per_step": ms, "slices_per_s": 2 / (ms * 1e-3)}

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
        "step_ms_percentiles": pct,
        "roofline": {"bound": "hbm", "kernel": f"spmm_{dom}", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"spmm_{dom}_bf16", op.get_tuning()),
                     "algorithmic_bytes": m[f"{dom}_bytes"], "frac_of_copy": achieved / copy_gbs,
                     "step": {"what": "forward + adjoint SpMM step (the metric's fwd+adj)",
                              "algorithmic_bytes": m["fwd_bytes"] + m["adj_bytes"],
                              "achieved": (m["fwd_bytes"] + m["adj_bytes"]) / ms_step / 1e6,
                              "frac": (m["fwd_bytes"] + m["adj_bytes"]) / ms_step / 1e6 / HBM_PEAK_GBS}},
        "copy_GBs": {"value": copy_gbs, "what": "torch copy_ of 1 GiB (read + write bytes / time)"},
        "kernels": res,
        "fp32_values": {"value": BATCH / (ms_f32 * 1e-3), "ms_per_step": ms_f32},
        "mixed_vs_fp32": ms_f32 / ms_step,
        "pair_form_b2": pair,
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
        ms_nrm = {}
        for vt in ("bf16", "f32"):
            op.normal(x, xb, values=vt)
            ms_nrm[vt] = time_loop(torch, lambda: op.normal(x, xb, values=vt), 10)
        out["normal_operator"] = {
            "what": "A^T A in one pass (embed, 2D FFT, S S^dagger stencil, inverse 2D FFT, crop)",
            "ms_bf16": ms_nrm["bf16"], "ms_f32": ms_nrm["f32"],
            "speedup_vs_project_backproject_bf16": ms_op["bf16"] / ms_nrm["bf16"]}
        op.solve(y, xb, iters=1)
        ms_cg = time_loop(torch, lambda: op.solve(y, xb, iters=10), 2)
        ms_cg1 = time_loop(torch, lambda: op.solve(y, xb, iters=0), 2)
        op.solve(y, xb, iters=1, method="cgnr")
        ms_cn = time_loop(torch, lambda: op.solve(y, xb, iters=10, method="cgnr"), 2)
        ms_cn1 = time_loop(torch, lambda: op.solve(y, xb, iters=0, method="cgnr"), 2)
        out["cgls"] = {"ms_per_iteration_f32": (ms_cg - ms_cg1) / 10, "batch": BATCH,
                       "normal_form_ms_per_iteration_f32": (ms_cn - ms_cn1) / 10}
        sb = dict(method="tv_split_bregman", iters=5, tv_mu=0.5, tv_lambda=2.0)
        op.solve(y, xb, refine_outer=1, **sb)
        ms_sb3 = time_loop(torch, lambda: op.solve(y, xb, refine_outer=3, **sb), 2)
        ms_sb1 = time_loop(torch, lambda: op.solve(y, xb, refine_outer=1, **sb), 2)
        out["tv_split_bregman"] = {"ms_per_bregman_step_f32": (ms_sb3 - ms_sb1) / 2,
                                   "cg_steps_per_bregman_step": 5, "batch": BATCH}
        out["stack_2048"] = stack_leg(torch, op, stack_in)
        st = out["stack_2048"]
        best = min(("mixed_cgls_bf16_4x25", "mixed_cgnr_bf16_4x25"), key=lambda k: st[k]["stack_seconds"])
        out["mixed_vs_fp32_reconstruction"] = {
            "mixed_form": best, "fp32_form": "cgls_f32",
            "time_ratio": st[best]["time_over_cgls_f32"],
            "phantom_error_ratio": st[best]["phantom_error_over_cgls_f32"]}
        out["paper_comparison"] = paper_comparison(torch, tomo, gen)
    if acc_ref is not None:
        out["accuracy"] = accuracy_leg(torch, tomo, op, acc_ref)
    if args.uneven:
        out["uneven_stack"] = uneven_leg(torch, tomo)
    if args.tv:
        out["tv_reconstruction"] = tv_leg(torch, tomo)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    op.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
