"""MI355X recursive-skeletonization fast direct solver (Ho & Greengard).

Python binding of the HIP library (include/rs.h).  The package imports the built
library eagerly and fails if it is missing: no part of the solver runs in Python.
"""
from .binding import (  # noqa: F401
    EXPORTED, KINDS, LAUNCH, Handle, RSError, Tree, build_tree, device_count, factor,
    rs_box_export, rs_box_skeletons, rs_build_tree, rs_device_count, rs_factor, rs_factor_ex,
    rs_free, rs_last_error, rs_query, rs_query_levels, rs_solve, rs_solve_ex, rs_solve_noalloc,
    rs_matvec, rs_factor_estimate, factor_estimate, factor_solve, rs_factor_solve_ex,
    rs_tree_export,
    rs_tree_free,
    rs_tree_info, LIB_PATH, FAMILIES, profile_enable, profile_read, profile_reset,
    rs_profile_enable, rs_profile_read, rs_profile_reset, factor_batched, solve_batched,
    rs_factor_batched, rs_solve_batched, Server, rs_server_create, rs_server_destroy,
    rs_server_poll, rs_server_query, rs_server_release, rs_server_reset_stats,
    rs_server_submit_factor, rs_server_submit_solve, Plan, autotune, tune_entries, tune_clear,
    tune_save, tune_load, rs_plan_create, rs_plan_launch, rs_plan_free, rs_autotune,
    rs_tune_entries, rs_tune_clear, rs_tune_save, rs_tune_load,
    RS_OK, RS_EINVAL, RS_ENOMEM, RS_ESINGULAR, RS_EDEVICE, RS_EBUSY, RS_ENOTSUP,
)
from . import binding  # noqa: F401


def device_available() -> bool:
    """True if the library sees at least one HIP device."""
    return device_count() > 0
