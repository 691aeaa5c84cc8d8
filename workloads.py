"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only describes *inputs*: background grids, circle lists, free-stream
and boundary-condition choices, and seeded random vectors.  It contains none of
the method's arithmetic (no classification, projection, smoothing, element
integrals or solves), so that the CPU oracle and the HIP path can both draw
their inputs from here without sharing any computation.

Geometry follows the paper's two experiments in form, since their exact
coordinates only appear in figures that are not available:

* a single circular cylinder in a large box (Validation section);
* three streamwise cylinders plus a transverse pair whose gap is varied
  (Results and Discussion, "Potential Flow Interferences in a Multiple-Body
  System" and "Effect of Gap Ratio").  Here the gap delta is the surface gap
  between the centre cylinder and each transverse cylinder, in diameters.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

# Side boundary-condition codes (same values as the C-ABI header).
BC_NATURAL = 0        # natural (zero normal derivative of psi): free nodes
BC_DIRICHLET_UY = 1   # psi = U * y
BC_DIRICHLET_CYL = 2  # psi = U (y - cy)(1 - a^2 / rho^2) about circle 0
BC_DIRICHLET_UX = 3   # phi = U * x (velocity potential of the free stream)
BC_DIRICHLET_CYLPHI = 4  # phi = U (x - cx)(1 + a^2 / rho^2) about circle 0

SIDE_L, SIDE_R, SIDE_B, SIDE_T = 0, 1, 2, 3


@dataclass(frozen=True)
class Grid:
    """Cartesian background grid of nx x ny cells on [x0,x1] x [y0,y1]."""
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float

    @property
    def nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)


@dataclass(frozen=True)
class Flow:
    """Free-stream speed and the boundary condition type of each side."""
    U: float = 1.0
    side_bc: Tuple[int, int, int, int] = (BC_DIRICHLET_UY, BC_NATURAL,
                                          BC_DIRICHLET_UY, BC_DIRICHLET_UY)


@dataclass
class Case:
    name: str
    grid: Grid
    circles: List[Tuple[float, float, float]]
    flow: Flow = field(default_factory=Flow)
    nsweeps: int = 200
    pair: Tuple[int, int] = (-1, -1)   # (lo, hi) body pair for Q and CoPFI
    delta: float = float("nan")


def single_cylinder(n: int = 64, half: float = 8.0, radius: float = 0.5,
                    exact_bc: bool = False) -> Case:
    """One cylinder of radius 0.5 at the origin in [-half, half]^2, n x n cells.

    exact_bc=False: psi = U y on inlet, bottom and top, natural outlet.
    exact_bc=True: the isolated-cylinder stream function on all four sides.
    """
    g = Grid(n, n, -half, half, -half, half)
    if exact_bc:
        bc = (BC_DIRICHLET_CYL,) * 4
    else:
        bc = (BC_DIRICHLET_UY, BC_NATURAL, BC_DIRICHLET_UY, BC_DIRICHLET_UY)
    return Case(f"cyl{n}", g, [(0.0, 0.0, radius)], Flow(1.0, bc))


def five_cylinders(nx: int, ny: int, delta: float,
                   extent=(-20.0, 20.0, -10.0, 10.0), U: float = 1.0,
                   diameter: float = 1.0) -> Case:
    """Three streamwise cylinders at x = -3, 0, 3 on y = 0 and a transverse pair
    at (0, -(D + delta)) [body index 3, "cylinder 4"] and (0, D + delta)
    [body index 4, "cylinder 5"], all of diameter D.
    """
    r = 0.5 * diameter
    yc = diameter + delta * diameter
    circles = [(-3.0, 0.0, r), (0.0, 0.0, r), (3.0, 0.0, r),
               (0.0, -yc, r), (0.0, yc, r)]
    g = Grid(nx, ny, *extent)
    return Case(f"five{nx}x{ny}_d{delta:g}", g, circles,
                Flow(U, (BC_DIRICHLET_UY, BC_NATURAL, BC_DIRICHLET_UY, BC_DIRICHLET_UY)),
                pair=(3, 4), delta=delta)


def five_cylinders_asymmetric(nx: int, ny: int, extent=(-20.0, 20.0, -10.0, 10.0)) -> Case:
    """The five-cylinder layout moved off every symmetry: the streamwise cylinders
    off the axis, the transverse pair shifted apart in x and in y (D = 1).  Used
    where the right-hand side must have weight on every eigenvector of the operator
    (condition estimates)."""
    circles = [(-3.0, 0.2, 0.5), (0.0, -0.15, 0.5), (3.0, 0.3, 0.5), (0.35, -1.3, 0.5),
               (-0.3, 1.4, 0.5)]
    g = Grid(nx, ny, *extent)
    return Case(f"five_asym{nx}x{ny}", g, circles,
                Flow(1.0, (BC_DIRICHLET_UY, BC_NATURAL, BC_DIRICHLET_UY, BC_DIRICHLET_UY)),
                pair=(3, 4))


def potential_flow(case: Case, exact_bc: bool = False) -> Case:
    """The same geometry with the boundary data of the velocity-potential problem:
    phi = U x on the inlet and outlet, natural (no flow through) on the walls;
    exact_bc=True: the isolated-cylinder potential about circle 0 on all four
    sides.  The body surfaces are natural boundaries in either case."""
    bc = (BC_DIRICHLET_CYLPHI,) * 4 if exact_bc else (BC_DIRICHLET_UX, BC_DIRICHLET_UX,
                                                       BC_NATURAL, BC_NATURAL)
    return Case("phi_" + case.name, case.grid, case.circles, Flow(case.flow.U, bc),
                case.nsweeps, case.pair, case.delta)


def validation_cylinder(n: int = 64) -> Case:
    """The 64x64 single-cylinder workload on [-8,8]^2 (psi = U y on three sides)."""
    return single_cylinder(n)


def five_cyl_1024() -> Case:
    """Five cylinders, 1024 x 512 cells on [-20,20]x[-10,10], delta = 0.25."""
    return five_cylinders(1024, 512, 0.25)


def five_cyl_4096() -> Case:
    """Five cylinders, 4096 x 2048 cells (~8.4M nodes), delta = 0.5."""
    return five_cylinders(4096, 2048, 0.5)


def five_cyl_2048_adjoint() -> Case:
    """Five cylinders, 2048 x 1024 cells, delta = 0.15 (gradient workload)."""
    return five_cylinders(2048, 1024, 0.15)


def batch_variants(count: int = 256, seed: int = 0,
                   nx_range=(256, 1024), delta_range=(0.05, 2.0)) -> List[Case]:
    """Seeded delta-sweep: delta ~ U[0.05, 2.0], nx uniform over even integers
    in [256, 1024], ny = nx / 2, five-cylinder layout."""
    rng = np.random.default_rng(seed)
    deltas = rng.uniform(delta_range[0], delta_range[1], size=count)
    nxs = 2 * rng.integers(nx_range[0] // 2, nx_range[1] // 2 + 1, size=count)
    return [five_cylinders(int(nx), int(nx) // 2, float(d))
            for nx, d in zip(nxs, deltas)]


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded N(0,1) vector."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)
