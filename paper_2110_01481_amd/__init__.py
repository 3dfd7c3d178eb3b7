"""MI355X (gfx950) AB-GMRES / BA-GMRES for CT with an unmatched back projector.

Python face of libabgmres (include/abgmres.h). Importing the package loads nothing;
the first Geometry or solver call loads the HIP library and fails loudly if it is
missing.
"""
from ._binding import (AbgError, Engine, Geometry, Problem, SolveResult, ab_gmres, ba_gmres,
                       batch_solve, fp_force_block_shape, fp_force_stage_share, gmres,
                       load_library, lsq, lsq_workspace_bytes, mgs_force_stream,
                       ncp_force_goertzel, profile_enable, profile_read, request_bytes,
                       shutdown, workspace_bytes, EXPORTS, LIB_PATH)

__all__ = ["AbgError", "Engine", "Geometry", "Problem", "SolveResult", "ab_gmres", "ba_gmres",
           "batch_solve", "fp_force_block_shape", "fp_force_stage_share", "gmres",
           "load_library", "lsq", "lsq_workspace_bytes", "mgs_force_stream",
           "ncp_force_goertzel", "profile_enable", "profile_read", "request_bytes",
           "shutdown", "workspace_bytes", "EXPORTS", "LIB_PATH"]
