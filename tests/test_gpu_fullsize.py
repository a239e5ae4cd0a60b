"""Full-size parity at 2048^2 pixels, 1501 angles, 2048 bins in the benchmark's launch
configuration (one batch of 32 slices = 16 complex channels).

* Both SpMMs, float32 and bf16 values: EVERY output row against the FP64 oracle's CSR product
  (SciPy on the host), element by element, within the float32 summation bound.  An output
  element that sums k products v_e x_e is computed from float32 inputs (bf16 values convert to
  float32 exactly; float32 values are the float64 ones rounded, relative error <= u), with one
  rounding per product and k - 1 additions in some order, so whatever the summation tree
      |computed - exact| <= gamma_{k+1} * sum_e |v_e| |x_e|,   gamma_j = j u / (1 - j u),
  u = 2^-24 (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1 and 4.2).  The
  bound is applied to the real and imaginary parts separately (each is a real sum).  Matrix
  entries on which the library's and the oracle's float64 builds disagree (exact window ties,
  values below 1e-12) are far inside it.  A wrong
  tile, strip, bin or chunk boundary anywhere in the grid errs by O(|v| |x|) and fails it.
* The composed operators on four sampled slices (two complex channels): relative L2 and the
  largest element error against the largest reference element, both within 1e-5; with bf16
  values against the oracle's operators with the same rounded values, likewise.
* CGLS (Sec. 3.1) in the benchmark's batch: its first iterates against the oracle's float64
  CGLS on the same float32 sinograms, in every slice position of the batch; likewise the first
  steps of the mixed-precision refinement (float32 residuals, bf16-value inner CGLS)."""

import numpy as np
import pytest
import torch

from oracle import Operator as OracleOperator, cgls, refine, round_values
from synth import phantom_stack
from tests.gpu_util import cart_map, oracle_op, polar_row_map, r32, rel_l2, summation_bound_check

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


@pytest.fixture(scope="module")
def maps(ref):
    g = ref.geom
    cm, pm = cart_map(g), polar_row_map(g)
    cm_inv = np.empty_like(cm)
    cm_inv[cm] = np.arange(cm.size)
    pm_inv = np.empty_like(pm)
    pm_inv[pm] = np.arange(pm.size)
    return cm, pm, cm_inv, pm_inv


def _vals(S, values):
    """The oracle matrix the kernel's products are compared with: float32 values against the
    float64 matrix itself (their rounding is one of the k + 1 roundings the bound allows), 16-bit
    values against the matrix with the same rounded values (they convert to float32 exactly)."""
    return S if values == "f32" else round_values(S, values)


@pytest.mark.parametrize("values", ["f32", "bf16"])
def test_fullsize_forward_spmm_every_row(big, ref, maps, values):
    cm, pm, cm_inv, pm_inv = maps
    g = ref.geom
    C = B // 2
    tun = big.get_tuning()
    assert tun["fwd_tiled"] & (1 if values == "f32" else 2)        # the staged forward runs
    rng = np.random.default_rng(7)
    Xc = rng.standard_normal((g.G * g.G, C, 2), dtype=np.float32)
    Yg = big.slice_fwd(torch.from_numpy(Xc).cuda(), B, values=values)
    torch.cuda.synchronize()
    got = Yg.cpu().numpy()
    summation_bound_check(f"forward {values}", got, _vals(ref.S_dag, values), pm, Xc, cm_inv, l2_tol=1e-6)
    assert torch.equal(big.slice_fwd(torch.from_numpy(Xc).cuda(), B, values=values), Yg)


@pytest.mark.parametrize("values", ["f32", "bf16"])
def test_fullsize_adjoint_spmm_every_row(big, ref, maps, values):
    """The staged adjoint with the row kernels on the cells near the origin (every chunked long
    row included), on its three streams, as the benchmark launches it."""
    cm, pm, cm_inv, pm_inv = maps
    g = ref.geom
    C = B // 2
    tun = big.get_tuning()
    assert tun["adj_tiled"] & (1 if values == "f32" else 2)
    rng = np.random.default_rng(11)
    Yc = rng.standard_normal((g.L * g.n_theta, C, 2), dtype=np.float32)
    Xg = big.slice_adj(torch.from_numpy(Yc).cuda(), B, values=values)
    torch.cuda.synchronize()
    got = Xg.cpu().numpy()
    summation_bound_check(f"adjoint {values}", got, _vals(ref.S, values), cm, Yc, pm_inv, l2_tol=1e-6)
    assert torch.equal(big.slice_adj(torch.from_numpy(Yc).cuda(), B, values=values), Xg)


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

    def errs(a, b):
        return rel_l2(a, b), float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    for s in (0, 1, B - 2, B - 1):
        xs = x[s].astype(np.float32).astype(np.float64)
        P = ref.project(xs)
        BP = ref.backproject(yh[s])
        (l2p, mxp), (l2b, mxb) = errs(yh[s], P), errs(xbh[s], BP)
        print(f"slice {s}: project rel L2 {l2p:.2e} max {mxp:.2e}; backproject rel L2 {l2b:.2e} "
              f"max {mxb:.2e}")
        assert l2p < 1e-5 and mxp < 1e-5
        assert l2b < 1e-5 and mxb < 1e-5
        err_bf16 = rel_l2(yb[s].cpu().numpy(), P)
        print(f"slice {s}: bf16-value projection error vs FP64 oracle {err_bf16:.3e}")
        assert err_bf16 < 4e-3


def test_fullsize_bf16_operators_against_rounded_oracle(big, ref):
    """project / backproject with bf16 values (the staged forward's channel-slowest output, the
    staged adjoint and its dense-tile segments writing the FFT-side grid) against the oracle's
    operators built from the same bf16-rounded matrix values: 16-bit values convert to float32
    exactly, so the only differences are float32 arithmetic, held to the float32 operators'
    1e-5 (relative L2 and largest element error against the largest reference element) on
    slices at both ends of the batch."""
    lo = OracleOperator(ref.geom, S=round_values(ref.S, "bf16"))
    x = phantom_stack(N, B, seed_base=3300, supersample=1).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y = big.project(xt, values="bf16")
    xb = big.backproject(y, values="bf16")
    torch.cuda.synchronize()
    yh = y.cpu().numpy().astype(np.float64)
    xbh = xb.cpu().numpy().astype(np.float64)
    for s in (0, 1, B - 1):
        P = lo.project(x[s].astype(np.float64))
        BP = lo.backproject(yh[s])
        for got, want, what in ((yh[s], P, "project"), (xbh[s], BP, "backproject")):
            l2 = rel_l2(got, want)
            mx = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
            print(f"slice {s}: bf16 {what} rel L2 {l2:.2e} max {mx:.2e}")
            assert l2 < 1e-5 and mx < 1e-5


def test_fullsize_cgls_first_iterates(big, ref):
    """Four CGLS iterations on the batch of 32 with float32 values and every fused step on (norms
    from the transforms' output passes, the residual update in the adjoint front, the direction
    and solution updates in the forward transform's first kernel).  Two sinograms of the oracle's
    own projections of seeded phantoms fill the batch alternately, so every slice position (the
    real and imaginary halves of all 16 channels) is compared with the oracle's float64 CGLS on
    the same float32 data.  Before the float32 Krylov process separates in the near-null space
    (about eight iterations) an iterate differs from the float64 one by the operators' own
    errors carried through the recurrence, which does not amplify them this early: the bound is
    the project and backproject bounds added (1e-5 each) in relative L2; measured 7-8e-7."""
    iters = 4
    x = phantom_stack(N, 2, seed_base=3100, supersample=1)
    b2 = [r32(ref.project(v.astype(np.float64))) for v in x]
    b = np.stack([b2[s % 2] for s in range(B)])
    xg = big.solve(torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).cuda(), iters=iters)
    torch.cuda.synchronize()
    xg = xg.cpu().numpy().astype(np.float64)
    for k in range(2):
        xr = cgls(ref.project, ref.backproject, b2[k], iters)
        errs = [rel_l2(xg[s], xr) for s in range(k, B, 2)]
        print(f"sinogram {k}: CGLS-{iters} rel L2 against the oracle, worst over 16 slice positions "
              f"{max(errs):.2e}")
        assert max(errs) < 2e-5


def test_fullsize_bf16_refinement_first_steps(big, ref):
    """The mixed-precision solve at the benchmark's size, two outer steps of three inner CGLS
    iterations: outer residuals with float32 values, inner solves with bf16 values, against the
    oracle's float64 refinement with the same rounded values (bf16 values convert to float32
    exactly, so each GPU application differs from the oracle's only by float32 summation).

    * The first outer step is CGLS-3 with bf16 values: within 2e-5, as the CGLS iterates above.
    * The second step starts from the first one's image x1 and is far more sensitive to an error
      of x1 along the constant image (the DC coefficient, where the float32 sums of thousands of
      same-sign terms near the Fourier origin leave most of the kernels' error) than along a
      generic direction: the residual b - A x1 is a tenth of b, and a DC error of x1 moves its
      low frequencies a hundredfold more.  The oracle measures that amplification A itself, from
      a constant perturbation of its own x1 (measured ~130, against ~1 for a random one).  The
      bound is 2 A e1 + 2e-5, with e1 the first step's measured error; measured 8-10e-5."""
    R, I = 2, 3
    hi32 = OracleOperator(ref.geom, S=round_values(ref.S, "f32"))
    lo = OracleOperator(ref.geom, S=round_values(ref.S, "bf16"))
    x = phantom_stack(N, 2, seed_base=3200, supersample=1)
    b2 = [r32(ref.project(v.astype(np.float64))) for v in x]
    bd = torch.from_numpy(np.ascontiguousarray(np.stack([b2[s % 2] for s in range(B)]), dtype=np.float32)).cuda()
    xg1 = big.solve(bd, iters=I, refine_outer=1, values="bf16")
    xg2 = big.solve(bd, iters=I, refine_outer=R, values="bf16")
    torch.cuda.synchronize()
    xg1 = xg1.cpu().numpy().astype(np.float64)
    xg2 = xg2.cpu().numpy().astype(np.float64)
    for k in range(2):
        x1 = refine(hi32.project, lo.project, lo.backproject, b2[k], 1, I)
        x2 = refine(hi32.project, lo.project, lo.backproject, b2[k], R, I)
        e1 = max(rel_l2(xg1[s], x1) for s in range(k, B, 2))
        eps = 1e-6
        xp = x1 + np.full_like(x1, eps * np.linalg.norm(x1) / x1.shape[0])
        x2p = xp + cgls(lo.project, lo.backproject, b2[k] - hi32.project(xp), I)
        amp = rel_l2(x2p, x2) / eps
        e2 = max(rel_l2(xg2[s], x2) for s in range(k, B, 2))
        bound = 2.0 * amp * e1 + 2e-5
        print(f"sinogram {k}: refinement first step {e1:.2e}; {R}x{I} (bf16 inner) {e2:.2e}, bound "
              f"{bound:.2e} (oracle's DC amplification {amp:.0f})")
        assert e1 < 2e-5
        assert e2 < bound
