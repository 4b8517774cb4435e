"""MI355X (gfx950) library for the 3D radiative-transfer formal solution and
its operator-splitting (ALI) iteration (Hauschildt & Baron, arXiv 2102.01734).

The compute lives in ``librt3d.so`` (hand-written HIP kernels behind a C ABI,
``include/rt3d.h``); this package is its ctypes binding.  Importing it loads
the library and fails if it has not been built.
"""
from .rt3d import (Grid, RtError, RtGridDesc, RtSolveOpts, RtSolveReport, RtState, lib, rt_ali_step, rt_autotune,  # noqa: F401
                   rt_set_launch_shape, rt_sphere_tracks, sphere_desc, SphereGrid, rt_set_preconditioner,
                   rt_precond_forward, rt_formal_solution_dirs, rt_shard_directions,
                   rt_box_template, rt_create_grid, rt_destroy_grid, rt_formal_solution, rt_grid_info, rt_last_error, rt_profile_enable, rt_profile_read, rt_solve,
                   rt_version)

lib()
