"""GPU parity of the normal operator A^T D A (Sec. 4: the Toeplitz approach, the transform
combined with its adjoint without the 1D FFTs) and of the solvers built on it, against the
float64 oracle's definition (the full forward operator followed by its exact adjoint).

Float32 values: <= 1e-5 relative L2 per slice (the same bar as the operators).  bfloat16 /
float16 values: the normal operator of the forward operator with S's values rounded the same way
(float64 -> float32 -> 16 bit), i.e. the oracle's project then backproject with the rounded
matrix, <= 1e-5.  Solvers: tolerances from repeated oracle solves with float32 storage and
float32-level operator noise, as for CGLS."""

import numpy as np
import pytest
import torch

from oracle import (cg_normal, interpolation_product, normal, normal_factored, ramp_filter,
                    round_values, sirt_bb)
from tests.gpu_util import krylov_tolerance, noisy_fp32, oracle_op, r32, rel_l2

pytestmark = pytest.mark.gpu

GEOMS = [(64, 90, 91, 3), (37, 30, 53, 3), (16, 12, 16, 3), (32, 24, 45, 5)]
# a fractional rotation axis: its phase ramp is unitary on the polar rows, so A^T D A keeps the
# stencil form (the oracle applies the ramp in project and backproject)
CENTERED = [(64, 90, 91, 3, 44.6), (37, 30, 53, 3, 25.25)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("B", [1, 3, 8])
@pytest.mark.parametrize("tiled", [1, 0])
def test_normal_matches_oracle(tomo, geom, B, tiled):
    n, nt, npb, kw = geom
    op = tomo.Operator(n, nt, npb, kw=kw, max_batch=8, device=0)
    op.set_tuning(normal_tiled=tiled)
    ref = oracle_op(n, nt, npb, kw=kw)
    x = r32(np.random.default_rng(B * 100 + n).uniform(0, 1, (B, n, n)))
    got = _host(op.normal(_dev(x)))
    got_h = _host(op.normal(_dev(x), filter="hamming"))
    D = ramp_filter(ref.geom, "hamming")
    for s in range(B):
        e = rel_l2(got[s], normal(ref, x[s]))
        eh = rel_l2(got_h[s], normal(ref, x[s], D))
        print(f"{geom} B={B} slice {s}: A^T A {e:.2e}, A^T D A {eh:.2e}")
        assert e <= 1e-5 and eh <= 1e-5
    op.close()


@pytest.mark.parametrize("geom", CENTERED, ids=lambda g: "x".join(map(str, g)))
def test_normal_fractional_axis_matches_oracle(tomo, geom):
    n, nt, npb, kw, c = geom
    op = tomo.Operator(n, nt, npb, kw=kw, max_batch=3, center=c, device=0)
    ref = oracle_op(n, nt, npb, kw=kw, center=c)
    x = r32(np.random.default_rng(17).uniform(0, 1, (3, n, n)))
    got = _host(op.normal(_dev(x)))
    for s in range(3):
        e = rel_l2(got[s], normal(ref, x[s]))
        print(f"{geom} slice {s}: A^T A with a fractional axis {e:.2e}")
        assert e <= 1e-5
    op.close()


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_normal_low_precision_values(tomo, fmt):
    """A_v^T A_v for the matrix with 16-bit values: the oracle's project then backproject with the
    same rounded values (and its factored form with W built from them), and positive
    semidefinite: x . A_v^T A_v x = |A_v x|^2 >= 0 for random and for high-frequency images."""
    from oracle import Operator as OracleOperator

    n, nt, npb = 64, 90, 91
    op = tomo.Operator(n, nt, npb, max_batch=4, values=("f32", fmt), device=0)
    ref = oracle_op(n, nt, npb)
    lo = OracleOperator(ref.geom, S=round_values(ref.S, fmt))
    x = r32(np.random.default_rng(7).uniform(0, 1, (4, n, n)))
    got = _host(op.normal(_dev(x), values=fmt))
    for s in range(4):
        e = rel_l2(got[s], normal(lo, x[s]))
        ef = rel_l2(got[s], normal_factored(lo, x[s], interpolation_product(lo)))
        print(f"{fmt} slice {s}: vs the rounded matrix's A^T A {e:.2e} (factored {ef:.2e}); vs "
              f"the float64 operator {rel_l2(got[s], normal(ref, x[s])):.2e}")
        assert e <= 1e-5 and ef <= 1e-5
    # high-frequency (checkerboard-modulated) images probe the near-null space
    i = np.arange(n)
    hf = r32(np.random.default_rng(8).standard_normal((4, n, n)) * ((-1.0) ** (i[:, None] + i[None, :])))
    q = _host(op.normal(_dev(hf), values=fmt))
    for s in range(4):
        assert float(np.vdot(hf[s], q[s])) >= -1e-6 * np.linalg.norm(hf[s]) * np.linalg.norm(q[s])
    op.close()


def test_normal_full_size_sampled_slices(tomo):
    """2048^2, 1501 angles, 2048 bins, batch 32; the oracle recomputes two slices."""
    n, nt, npb, B = 2048, 1501, 2048, 32
    op = tomo.Operator(n, nt, npb, max_batch=B, values=("f32", "bf16"), device=0)
    rng = np.random.default_rng(11)
    x = np.empty((B, n, n), dtype=np.float32)
    for s in range(B):
        x[s] = rng.uniform(0, 1, (n, n))
    got = op.normal(_dev(x))
    op.set_tuning(normal_tiled=0)
    got_direct = op.normal(_dev(x))
    ref = oracle_op(n, nt, npb)
    for s in (0, B - 1):
        assert rel_l2(_host(got_direct[s]), _host(got[s])) <= 1e-6
        xs = x[s].astype(np.float64)
        e = rel_l2(_host(got[s]), normal(ref, xs))
        print(f"slice {s}: A^T A at 2048^2 vs FP64 oracle {e:.2e}")
        assert e <= 1e-5
    op.close()


def _sinos(ref, B, seed):
    from synth import phantom_stack
    xt = phantom_stack(ref.geom.n, B, seed)
    return np.stack([ref.project(v) for v in xt])


def test_cgnr_matches_oracle(tomo):
    n, nt, npb, B, iters = 64, 90, 91, 3, 20
    ref = oracle_op(n, nt, npb)
    b = _sinos(ref, B, 600)
    op = tomo.Operator(n, nt, npb, max_batch=B, device=0)
    xg = _host(op.solve(_dev(b), method="cgnr", iters=iters))
    for s in range(B):
        bs = r32(b[s])
        xr = cg_normal(lambda v: normal(ref, v), ref.backproject(bs), iters)

        def run(rng):
            T = noisy_fp32(lambda v: normal(ref, v), rng)
            return cg_normal(T, noisy_fp32(ref.backproject, rng)(bs), iters, store=r32)

        err = rel_l2(xg[s], xr)
        print(f"slice {s}: CG on normal equations ({iters}) GPU vs FP64 oracle {err:.3e}")
        assert err < krylov_tolerance(run, xr), s
        assert rel_l2(ref.project(xg[s]), ref.project(xr)) < 2e-3
    op.close()


@pytest.mark.parametrize("grid_fft,B", [(1, 2), (1, 3), (0, 3)], ids=["fused", "fused_odd_batch", "separate"])
def test_cgnr_early_iterates_match_cgls_oracle(tomo, grid_fft, B):
    """In exact arithmetic CG on the normal equations and CGLS give the same iterates; before
    float32 separation (a few iterations) the GPU's normal-form solve agrees with the oracle's
    CGLS tightly.  With the hand-written grid transform the step x += alpha p, p = r + beta p
    rides in the normal operator's first kernel and p . q in its last; with rocFFT both are
    separate passes."""
    from oracle import cgls

    n, nt, npb, iters = 64, 90, 91, 5
    ref = oracle_op(n, nt, npb)
    b = _sinos(ref, B, 610)
    op = tomo.Operator(n, nt, npb, max_batch=B, device=0)
    op.set_tuning(grid_fft=grid_fft)
    xg = _host(op.solve(_dev(b), method="cgnr", iters=iters))
    for s in range(B):
        xr = cgls(ref.project, ref.backproject, r32(b[s]), iters)
        assert rel_l2(xg[s], xr) < 1e-4, s
    op.close()


def test_cgnr_bf16_refinement_matches_cgls_refinement_oracle(tomo):
    """Refinement with float32 outer residuals and CG on the normal equations of the operator
    with bfloat16 values as the inner solve: in exact arithmetic the inner iterates equal CGLS's
    on the same rounded matrix, so before float32 separation (short inner solves) the GPU agrees
    with the oracle's CGLS refinement tightly, and the misfit decreases from one outer step to
    the next (the inner normal operator is positive semidefinite)."""
    from oracle import Operator as OracleOperator, refine

    n, nt, npb, B, R, I = 64, 90, 91, 2, 3, 4
    hi = oracle_op(n, nt, npb)
    hi32 = OracleOperator(hi.geom, S=round_values(hi.S, "f32"))
    lo = OracleOperator(hi.geom, S=round_values(hi.S, "bf16"))
    b = _sinos(hi, B, 630)
    op = tomo.Operator(n, nt, npb, max_batch=B, values=("f32", "bf16"), device=0)
    mis = []
    for r in range(1, R + 1):
        xg = _host(op.solve(_dev(b), method="cgnr", iters=I, refine_outer=r, values="bf16"))
        mis.append([np.linalg.norm(hi.project(xg[s]) - b[s]) for s in range(B)])
    for s in range(B):
        xr = refine(hi32.project, lo.project, lo.backproject, r32(b[s]), R, I)
        err = rel_l2(xg[s], xr)
        print(f"slice {s}: refinement {R}x{I} (bf16 CGNR inner) vs oracle CGLS refinement {err:.3e}; "
              f"misfits {[f'{m[s]:.4e}' for m in mis]}")
        assert err < 1e-4, s
        assert all(mis[k + 1][s] < mis[k][s] for k in range(R - 1)), s
    op.close()


def test_sirt_bb_normal_matches_oracle(tomo):
    n, nt, npb, iters = 64, 90, 91, 20
    ref = oracle_op(n, nt, npb)
    b = _sinos(ref, 2, 620)
    op = tomo.Operator(n, nt, npb, max_batch=2, device=0)
    D = ramp_filter(ref.geom, "hamming")
    xg = _host(op.solve(_dev(b), method="sirt_bb_normal", iters=iters, filter="hamming"))
    xs = _host(op.solve(_dev(b), method="sirt_bb", iters=iters, filter="hamming"))

    def atd(y):
        return ref.backproject(y, D)

    for s in range(2):
        bs = r32(b[s])
        xr = sirt_bb(ref.project, atd, bs, iters)

        def run(rng):
            return sirt_bb(noisy_fp32(ref.project, rng), noisy_fp32(atd, rng), bs, iters, store=r32)

        tol = krylov_tolerance(run, xr)
        err, err_full = rel_l2(xg[s], xr), rel_l2(xs[s], xr)
        print(f"slice {s}: SIRT-BB-{iters} normal form {err:.3e}, full operator {err_full:.3e}")
        assert err < tol, s
    op.close()


def test_normal_rejects_unsupported_geometry(tomo):
    op = tomo.Operator(12, 10, 16, grid=20, max_batch=2, device=0)
    x = torch.zeros((1, 12, 12), device="cuda")
    with pytest.raises(tomo.TomoError, match="EUNSUPPORTED"):
        op.normal(x)
    with pytest.raises(tomo.TomoError, match="EUNSUPPORTED"):
        op.solve(torch.zeros((1, 10, 16), device="cuda"), method="cgnr", iters=2)
    op.close()
