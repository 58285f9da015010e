"""Python binding of libhydot, the MI355X hyperspectral DOT Born hot path.

Argument marshalling only: every step runs inside the HIP library
(``libhydot.so``, C ABI in ``include/hydot.h``).  PyTorch provides device
memory and streams.  Importing this package loads the library and fails
loudly if it has not been built (``python paper_1410_0986_amd/build.py``).
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    HydotError,
    Operator,
    SolveOptions,
    PalsOptions,
    apply_operator,
    apply_preconditioner,
    solve_workspace_bytes,
    solve_fields,
    solve_fields_batch,
    SOLVE_BATCH_MAX,
    SolveSession,
    born_apply,
    born_workspace_bytes,
    born_apply_adjoint,
    pals_shape,
    pals_shape_vjp,
    pals_shape_jacobian,
    misfit,
    BornMisfit,
    library_path,
    version,
    profile_enable,
    profile_read,
    measure_peaks,
    get_tuning,
    set_tuning,
    autotune_solve,
    autotune_born,
    C128, C64, CBF16, F64, F32,
    BORN_NATIVE, BORN_SPLIT_BF16, BORN_PAIRS_MIN_NV,
    PREC_FP64, PREC_MIXED,
    FLAG_NO_RECYCLE, FLAG_MEAN_SHIFT, FLAG_GRAPH, FLAG_PER_SYSTEM, FLAG_FULL_REORTH,
    FLAG_SHIFT_MIN, FLAG_SHIFT_MAX, FLAG_PRECOND_SEP, FLAG_PRECOND_SEP_FIXED,
    PALS_WENDLAND, PALS_GAUSSIAN,
    OK, ENOCONV, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED,
)
