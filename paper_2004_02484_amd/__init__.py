"""MI355X double-layer Jacobi NMPC solver (HIP, gfx950).

Python binding of ``libnmpc.so`` (C ABI declared in ``include/nmpc.h``).
The functions keep the C names and only marshal arguments: every step of the
solver runs in the library's HIP kernels. PyTorch is used for device memory
and streams only. The first call fails loudly (ImportError) if the library
has not been built (``python -m paper_2004_02484_amd.build``); there is no
fallback path.
"""
from ._binding import (  # noqa: F401
    NMPC_E_ARG,
    NMPC_E_DEVICE,
    NMPC_E_NOCONV,
    NMPC_E_NONFINITE,
    NMPC_E_OOM,
    NMPC_E_UNSUPPORTED,
    NMPC_FP32_SWEEP,
    NMPC_FP64,
    NMPC_OK,
    NMPC_PATH_AUTO,
    NMPC_PATH_FUSED,
    NMPC_PATH_STREAM,
    NMPC_UPPER_BGS,
    NMPC_UPPER_FGS,
    NMPC_UPPER_JACOBI,
    NMPC_UPPER_SGS,
    NMPC_RES_PAPER,
    NMPC_RES_SCALED,
    ModelSolver,
    NmpcError,
    RaggedSolver,
    Solver,
    library_path,
    nmpc_autotune,
    nmpc_create,
    nmpc_default_options,
    nmpc_destroy,
    nmpc_kernel_config,
    nmpc_last_error,
    nmpc_model_create,
    nmpc_plant_step_batch,
    nmpc_ragged_autotune,
    nmpc_ragged_config,
    nmpc_ragged_create,
    nmpc_ragged_destroy,
    nmpc_ragged_solve,
    nmpc_ragged_timing_enable,
    nmpc_ragged_timing_read,
    nmpc_residual_batch,
    nmpc_set_options,
    nmpc_shift_batch,
    nmpc_solve,
    nmpc_solve_batch,
    nmpc_strerror,
    nmpc_timing_enable,
    nmpc_timing_read,
)
