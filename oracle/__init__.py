"""CPU oracle for the 18th-order hyperpower iteration of Pan, Soleymani and Zhao,
"Highly Efficient Computation of Generalized Inverse of a Matrix" (arXiv 1604.07893).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it. The product path (the HIP library
and its Python binding) never imports, links or calls anything here, and nothing
here imports the product path.

It is a plain, slow, obviously literal implementation: every product is a numpy
``@`` in the association the paper prints, with no blocking, fusion or reordering.
The same code runs in IEEE binary64 (numpy float64, OpenBLAS for ``@``) and in
multiple precision (numpy object arrays of mpmath numbers), the latter for the
paper's 150-digit worked example.
"""

from .hyperpower import (  # noqa: F401
    Arith,
    F64,
    MP,
    pm_constants,
    octic_constants,
    norm_1,
    norm_inf,
    norm_fro,
    adjoint,
    x0_moore_penrose,
    x0_drazin,
    x0_diag,
    chop,
    pm_step,
    stabilise,
    sm_step,
    cm_step,
    fm_step,
    hm_step,
    hyperpower_direct_step,
    solve,
    coc,
    penrose_residuals,
    drazin_residuals,
    STEP_FUNCTIONS,
    ORDER,
)
