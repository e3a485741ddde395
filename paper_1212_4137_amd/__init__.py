"""MI355X-native alternating maximization (AM) for sparse PCA.

Implements the batched AM iteration (Algorithm 2 of arXiv:1212.4137 run from
many starting points at once, Section 4) for the 8 formulations of Table 1 as
HIP kernels for gfx950 behind the C-ABI of ``include/spca.h``.  This package
is the thin Python binding; see ``_lib`` for the functions.
"""
from ._lib import (  # noqa: F401
    CONVERGED, DEGENERATE, EXPORTED, WARN_ALL_DEGENERATE, WARN_ALL_ZERO, WARN_NO_CONVERGED, WARN_NONE, FLAG_AUTOTUNE, FLAG_CHECK_FINITE, FLAG_DENSE_ONLY, FLAG_GRAPH, FLAG_NO_UNION,
    FLAG_SPARSE_NO_PANELS, FLAG_SPARSE_PANELS, FLAG_TIME_SAMPLED,
    LIB_PATH, MAXIT, PREC_BF16_POLISH, PREC_FP32, ZERO, Context, Server, SpcaError, am_solve,
    am_components, am_components_sparse, am_solve_group, am_solve_simple, group_workspace_bytes,
    GROUP_MAX_P, GROUP_MAX_REQUESTS, GROUP_MAX_STARTS, am_solve_sparse, colmajor_view, default_context, generate_spiked, gemm_nt, gemm_nt_bf16, gemm_nt_shape, gemm_plan, load, request_footprint, sparse_to_device, tune_table_clear, tune_table_export,
    tune_table_import, workspace_bytes,
    x_update,
)
