"""MI355X-native matrix-free multi-body stream-function solver.

Python face of libmfpsi.so: a body-conforming Q1 mesh from a Cartesian grid and
circles, the multi-point-constrained conjugate-gradient solve for psi, and the
derived body stream-function values, surface velocities, inter-body flow rate
and CoPFI; the velocity potential phi on the same mesh (the flow net); the
mixed-cell variant of the mesh (cut points on the grid lines, triangles and
quadrilaterals) with its element product and constrained solve; the Kutta
constraint (psi at an added fluid point equals the body's psi_b).  All
arithmetic runs in the library's HIP kernels.
"""
from .binding import (MFP_OK, MFP_W_NOCONV, MFP_W_STAGNATION, MFP_E_ARG, MFP_E_HIP,
                      MFP_E_GEOMETRY, MFP_E_TANGLED, MFP_E_BREAKDOWN, MFP_E_WORKSPACE,
                      MfpError, check_geometry, contour, cubic_fit, element_apply,
                      element_apply_noalloc, MixedMesh, mixed_element_apply, mixed_mesh,
                      mixed_psi_solve, psi_solve_kutta, mixed_mesh_bodies, body_bounds,
                      mixed_psi_solve_kutta, last_error, load,
                      mesh_conform, mesh_conform_grad, phi_solve, psi_grad, psi_solve,
                      psi_solve_batched, solve_workspace_size, EXPORTS)
from .autograd import CoPFIFunction, copfi

__all__ = ["MFP_OK", "MFP_W_NOCONV", "MFP_W_STAGNATION", "MFP_E_ARG", "MFP_E_HIP",
           "MFP_E_GEOMETRY", "MFP_E_TANGLED", "MFP_E_BREAKDOWN", "MFP_E_WORKSPACE",
           "MfpError", "check_geometry", "contour", "cubic_fit", "element_apply",
           "element_apply_noalloc", "MixedMesh", "mixed_element_apply", "mixed_mesh",
           "mixed_psi_solve", "psi_solve_kutta", "mixed_mesh_bodies", "body_bounds",
           "mixed_psi_solve_kutta", "last_error", "load",
           "mesh_conform", "mesh_conform_grad", "phi_solve", "psi_grad", "psi_solve",
           "psi_solve_batched",
           "solve_workspace_size", "EXPORTS", "CoPFIFunction", "copfi"]
