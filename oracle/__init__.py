"""FP64 CPU oracle for the sparse Fubini-Radon tomography operator.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test-suite, the
package's smoke check and the benchmark's CPU-baseline leg may import anything
here.  The oracle is written from the paper (Sec. 2-3), shares no code with the
HIP library, and is never a fallback for it.

Pins (the tests that tie the oracle to something other than itself) live in
``tests/test_oracle_*.py``; every oracle function is covered by at least one.
"""

from .fubini_radon import (  # noqa: F401
    Geometry,
    Operator,
    beatty_beta,
    build_S,
    deapodization,
    dft2_centered_direct,
    kappa,
    kernel,
    polar_k,
    polar_kept,
    polar_points,
    project_folded,
    project_nudft,
    project_paired,
    ramp_filter,
    sdag_dense_direct,
)
from .density import backproject_weighted, density_target, density_weights, mirror_average, irradon_density  # noqa: F401,E501
from .lowprec import round_to_bf16, round_to_f16, round_values  # noqa: F401
from .solvers import cgls, refine, sirt_bb  # noqa: F401
from .normal import cg_normal, interpolation_product, normal, normal_factored  # noqa: F401
from .tv import (chambolle_rof, differences, differences_adjoint, objective,  # noqa: F401
                 objective_grad, shrink, split_bregman, tv_grad, tv_value)
