"""MI355X (gfx950) hot path of singles-and-doubles Quantum Flow (QFlow).

The compute path lives in ``libqflow.so`` (hand-written HIP kernels behind the
C ABI of ``include/qflow.h``); this package only marshals arguments.  Importing
it does not load the library; ``lib()`` does, and raises if it was not built
(``python -m paper_2606_04186_amd.build``).  There is no CPU fallback.
"""
from .api import (  # noqa: F401
    FP64, FP32, BF16X3, UNOWNED_FROZEN, GRAPH, DIIS, SOLVER_VQE, Z_AUTO, Z_SPACE, Z_DENSE,
    SPACE_DTYPE, TRUNC_F, TRUNC_H,
    QFlowError, Context, lib,
    make_spaces, sample_spaces, build_owners, heff_size, amp_size, ci_size,
)
