"""dgmi: nodal interior-penalty DG right-hand side for 2D compressible
Navier-Stokes on triangles, in hand-written HIP for MI355X (gfx950).

The compute path lives in libdgmi.so (C-ABI declared in include/dgmi.h);
this package holds its ctypes binding (`_lib`, same names as the C calls)
and a small convenience wrapper (`Solver`) that keeps the state in torch
device tensors.  There is no CPU fallback: without the built library every
call raises.
"""
from ._lib import (DGError, DG_FP32_PERT, DG_FP32_PERT_BF16OPS, DG_FP64, DG_FP64_PERT, DG_PENALTY_PAPER, DG_PENALTY_STANDARD, DG_WALL_ADIABATIC, DG_WALL_PRINTED, dg_create,  # noqa: F401
                   dg_destroy, dg_force, dg_get_host_table, dg_get_nodes, dg_last_error,
                   dg_newmark_step, dg_num_elements, dg_num_face_nodes, dg_num_nodes, dg_rhs,
                   dg_rk_stage, dg_rk_step, dg_set_mesh, dg_set_physics, dg_setup, dg_setup_host,
                   load)
from .solver import Batch, Solver  # noqa: F401
