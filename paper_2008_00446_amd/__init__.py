"""MI355X (gfx950) hot path of Stochastic Bundle Adjustment (arXiv 2008.00446).

The work runs in libstba.so (HIP kernels behind the C ABI of include/stba.h);
this package is its thin binding.  Import does not load the library; the first
call does, and raises if it has not been built.
"""
from .binding import (  # noqa: F401
    STBA_FP64, STBA_MIXED, STBA_MIXED_NOREFINE, STBA_NUM_PHASES, STBA_CHOL_AUTO, STBA_CHOL_TILES, STBA_CHOL_TEAM,
    STBA_CHOL_WORKGROUP, StbaError, load_library, make_problem, make_sample,
    alloc_workspace, new_state, read_state, set_lambda_min, StbaDamping, StbaDims,
    stba_version, stba_phase_name, stba_analyze_scratch_bytes, stba_analyze, stba_workspace_bytes, stba_prepare,
    stba_residual_jacobian, stba_residual_jacobian_static, stba_build_cluster_rcs, stba_solve_clusters,
    stba_solve_clusters_pcg,
    stba_sample_clusters, stba_lm_step_pcg, stba_lm_init,
    stba_lm_step, stba_lm_step_batched, new_states,
    stba_lm_step_profiled, stba_residual_vjp, stba_residual_vjp_stored, stba_autotune,
)
from .tuning import shape_class, autotune_solver  # noqa: F401
from .solver import StbaSolver, BatchSolver, ResidualPlan, residuals, hip_events, event_ms  # noqa: F401
