"""Plain FP64 CPU oracle for the matrix-free stream-function solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

The oracle is written for obviousness, not speed: vectorised NumPy over whole
arrays, an assembled SciPy sparse stiffness matrix and a direct sparse LU
solve.  It follows the paper (Sadasivan & Yadav, "A Computational Approach for
Multi-Body Potential-Flow Interaction Effects Using Matrix-Free FEM and
Body-Conforming Grids"):

* ``mesh``  -- body-conforming grid generation (section "Body-Conforming Grid
  Generation": projection of just-inside nodes onto the body, displacement
  d_ik = x_ik - x_gk, Laplacian propagation of d, x_new = x_old + d);
* ``fem``   -- Q1 element stiffness K_e = int (grad N)^T (grad N) dOmega
  (section "Weak formulation") and its assembly;
* ``solve`` -- the reduced constrained system whose solution Algorithm 1
  (appendix, "CG solver") iterates towards, solved directly, and the
  post-processing (surface tangential velocity, Q_54, CoPFI);
* ``grad``  -- derivatives of CoPFI with respect to body centres and the gap
  ratio by complex step, by a discrete adjoint and by finite differences;
* ``potential`` -- the velocity potential phi on the same mesh (section
  "Governing Equation": the flow net's other family of curves), solved
  directly;
* ``contour`` -- contour lines of a nodal field (flow net, stagnation
  streamlines) by marching squares on the conformed mesh;
* ``sweep`` -- the cubic fit of CoPFI over the gap ratio (section "Effect of
  Gap Ratio");
* ``cg``    -- a plain conjugate-gradient loop on the assembled matrix (CPU
  timing baseline);
* ``spectrum`` -- extreme eigenvalues of the reduced operator (condition number)
  and the Ritz extremes of the Lanczos process from a right-hand side;
* ``mixed`` -- the paper's own mesher with mixed cells (grid points moved onto the
  body along grid lines, node splitting, triangles, pentagons cut into a triangle
  and a quadrilateral) and the stream-function solve on it (P1 and Q1 elements);
* ``airfoil`` -- bodies with a sharp trailing edge (Joukowski airfoils) for the
  mixed-cell mesh: inside test, cut points along grid lines, and the exact flow
  with any circulation and with the Kutta circulation;
* ``kutta`` -- the Kutta condition as a constraint: psi at an added fluid point
  equals the body's psi_b, in place of the body's zero-circulation row (section
  "Boundary Conditions"), and the exact lifting cylinder that pins it.

Readings of passages where the paper is silent or ambiguous are listed in the
module docstrings where they are applied.
"""
from .mesh import (FLUID, SNAPPED, DEEP, GeometryError, spacing, node_coords,
                   check_geometry, classify, snap_displacement, jacobi_weights,
                   smooth, conform, active_cells, cell_nodes, Mesh)
from .fem import (element_stiffness, element_coords, assemble, apply_at_nodes,
                  rectangle_stiffness)
from .solve import (dirichlet_mask, dirichlet_values, dof_numbering,
                    reduced_system, solve, surface_samples, copfi, Solution)
from .potential import in_domain, phi_solve, cell_velocity, PhiSolution
from .sweep import cubic_fit
from .contour import contour
from .spectrum import condition_number, lanczos_extremes

__all__ = [
    "FLUID", "SNAPPED", "DEEP", "GeometryError", "spacing", "node_coords",
    "check_geometry", "classify", "snap_displacement", "jacobi_weights",
    "smooth", "conform", "active_cells", "cell_nodes", "Mesh",
    "element_stiffness", "element_coords", "assemble", "apply_at_nodes",
    "rectangle_stiffness", "dirichlet_mask", "dirichlet_values",
    "dof_numbering", "reduced_system", "solve", "surface_samples", "copfi",
    "Solution", "in_domain", "phi_solve", "cell_velocity", "PhiSolution", "cubic_fit",
    "contour", "condition_number", "lanczos_extremes",
]
