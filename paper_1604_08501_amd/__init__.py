"""semvol: the strong-form spectral-element volume term of the dry Euler
equations (Klöckner, Wilcox, Warburton, ARRAY'16, Sec. 2) as hand-written
HIP kernels for one MI355X (gfx950) behind a C-ABI library, ``libsem.so``.

``semvol`` holds the Python binding (argument marshalling only);
``inputs`` builds GLL nodes, differentiation matrices, meshes and seeded
states; ``build`` compiles the library.
"""
from .semvol import (  # noqa: F401
    SemError, VolumeRHS, BatchPlan, RK3Graph, axpby, lib, set_max_workgroups, tile_options,
    version, volume_rhs,
    volume_rhs_adjoint, volume_rhs_ext, volume_rhs_affine, volume_rhs_ladder, LADDER_LEVELS,
    surface_rhs, batch_rhs_static, rhs,
)
