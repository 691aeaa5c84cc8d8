"""ctypes binding of libmfpsi.so (see include/mfpsi.h for the C ABI).

Argument marshalling only: tensors supply device pointers, the current HIP stream
comes from torch, every computation runs in the library's kernels.  Missing or
unloadable native code raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int8, c_int32,
                    c_int64, c_size_t, c_void_p)
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmfpsi.so")

MFP_OK, MFP_W_NOCONV, MFP_W_STAGNATION = 0, 1, 2
MFP_E_ARG, MFP_E_HIP, MFP_E_GEOMETRY, MFP_E_TANGLED, MFP_E_BREAKDOWN, MFP_E_WORKSPACE = (
    -1, -2, -3, -4, -5, -6)
MFP_FLUID, MFP_SNAPPED, MFP_DEEP = 0, 1, 2
BC_NATURAL, BC_DIRICHLET_UY, BC_DIRICHLET_CYL = 0, 1, 2
FP64, FP32, FP32_IR = 0, 1, 2
MAX_BODIES = 64
_PREC = {"fp64": FP64, "fp32": FP32, "fp32_ir": FP32_IR}

# Every symbol the header declares (checked by the CPU test-suite).
EXPORTS = [
    "mfp_last_error", "mfp_check_geometry", "mfp_conform_workspace_size",
    "mfp_mesh_conform", "mfp_solve_workspace_size", "mfp_element_apply", "mfp_psi_solve",
    "mfp_grad_workspace_size", "mfp_psi_grad", "mfp_conform_grad_workspace_size",
    "mfp_mesh_conform_grad", "mfp_batched_workspace_size", "mfp_psi_solve_batched",
    "mfp_phi_solve", "mfp_cubic_fit", "mfp_contour_workspace_size", "mfp_contour",
    "mfp_element_apply_noalloc", "mfp_solve_workspace_size_opts",
    "mfp_batched_workspace_size_opts", "mfp_mixed_workspace_size", "mfp_mixed_mesh",
    "mfp_mixed_solve_workspace_size", "mfp_mixed_element_apply", "mfp_mixed_psi_solve",
    "mfp_kutta_workspace_size", "mfp_psi_solve_kutta", "mfp_body_bounds",
    "mfp_mixed_mesh_bodies", "mfp_mixed_kutta_workspace_size", "mfp_mixed_psi_solve_kutta",
]


class MfpGrid(Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("x0", c_double), ("x1", c_double),
                ("y0", c_double), ("y1", c_double)]


class MfpCircle(Structure):
    _fields_ = [("cx", c_double), ("cy", c_double), ("r", c_double)]


class MfpFlow(Structure):
    _fields_ = [("U", c_double), ("side_bc", c_int32 * 4)]


class MfpSolverOpts(Structure):
    _fields_ = [("precision", c_int32), ("rtol", c_double), ("kmax", c_int64),
                ("check_every", c_int32), ("inner_rtol", c_double), ("max_outer", c_int32),
                ("psi0", c_void_p), ("profile_every", c_int32), ("estimate_kappa", c_int32),
                ("rtol_from_start", c_int32), ("task_rows", c_int32), ("element_mode", c_int32),
                ("store_mode", c_int32), ("launch_blocks", c_int32),
                ("batch_tasks_per_wave", c_int32)]


SCHEDULE_KEYS = ("task_rows", "element_mode", "store_mode", "launch_blocks",
                 "batch_tasks_per_wave")


def _set_schedule(o: "MfpSolverOpts", schedule: Optional[dict]) -> "MfpSolverOpts":
    """Explicit schedule fields of the iteration kernel (0 or missing = automatic)."""
    for k, v in (schedule or {}).items():
        if k not in SCHEDULE_KEYS:
            raise ValueError(f"unknown schedule field {k!r}")
        setattr(o, k, int(v))
    return o


class MfpStats(Structure):
    _fields_ = [("iters", c_int64), ("outer_iters", c_int64), ("applies", c_int64),
                ("n_dof", c_int64), ("n_free", c_int64), ("relres_true", c_double),
                ("rnorm0", c_double), ("solve_ms", c_double), ("apply_ms", c_double),
                ("apply_samples", c_int64), ("n_plain_tiles", c_int64), ("n_tiles", c_int64),
                ("inner_iters", c_int64), ("kappa_est", c_double), ("ritz_min", c_double),
                ("ritz_max", c_double), ("kappa_steps", c_int64),
                ("step_blocks", c_int64), ("step_block_waves", c_int64),
                ("step_element_mode", c_int64)]


class MfpVariant(Structure):
    _fields_ = [("grid", MfpGrid), ("disp", c_void_p), ("kind", c_void_p), ("body", c_void_p),
                ("psi", c_void_p)]


BODY_CIRCLE, BODY_JOUKOWSKI = 0, 1


class MfpBody(Structure):
    _fields_ = [("kind", c_int32), ("x", c_double), ("y", c_double), ("r", c_double),
                ("xi0", c_double), ("eta0", c_double), ("alpha", c_double)]


class MfpMixedMesh(Structure):
    _fields_ = [("disp", c_void_p), ("body", c_void_p), ("hpt", c_void_p), ("vpt", c_void_p),
                ("cell_first", c_void_p), ("pxy", c_void_p), ("pbody", c_void_p),
                ("pedge", c_void_p), ("elem", c_void_p), ("nne", c_void_p),
                ("cap_points", c_int64), ("cap_elems", c_int64), ("n_points", c_int64),
                ("n_elems", c_int64), ("n_tri", c_int64)]


class MfpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mfpsi status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libmfpsi.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run `python -m paper_2512_12232_amd.build`")
    lib = ctypes.CDLL(path)
    lib.mfp_last_error.restype = c_char_p
    lib.mfp_check_geometry.argtypes = [POINTER(MfpGrid), POINTER(MfpCircle), c_int32]
    lib.mfp_conform_workspace_size.restype = c_size_t
    lib.mfp_conform_workspace_size.argtypes = [POINTER(MfpGrid), c_int32]
    lib.mfp_mesh_conform.argtypes = [POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_int32,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.mfp_solve_workspace_size.restype = c_size_t
    lib.mfp_solve_workspace_size.argtypes = [POINTER(MfpGrid), c_int32, c_int32]
    lib.mfp_solve_workspace_size_opts.restype = c_size_t
    lib.mfp_solve_workspace_size_opts.argtypes = [POINTER(MfpGrid), c_int32,
                                                  POINTER(MfpSolverOpts)]
    lib.mfp_element_apply.argtypes = [POINTER(MfpGrid), c_void_p, c_void_p, c_int32, c_void_p,
                                      c_void_p, c_int32, POINTER(c_double), c_void_p, c_size_t,
                                      c_void_p]
    lib.mfp_element_apply_noalloc.argtypes = [POINTER(MfpGrid), c_void_p, c_void_p, c_int32,
                                              c_void_p, c_void_p, c_void_p]
    lib.mfp_psi_solve.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_void_p, c_void_p, c_void_p,
        POINTER(MfpFlow), POINTER(MfpSolverOpts), c_int32, c_int32, c_void_p,
        POINTER(c_double), POINTER(c_double), POINTER(c_double), c_void_p, c_void_p, c_int32,
        POINTER(c_int32), POINTER(MfpStats), c_void_p, c_size_t, c_void_p]
    lib.mfp_phi_solve.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_void_p, c_void_p, c_void_p,
        POINTER(MfpFlow), POINTER(MfpSolverOpts), c_void_p, POINTER(MfpStats), c_void_p,
        c_size_t, c_void_p]
    lib.mfp_cubic_fit.argtypes = [POINTER(c_double), POINTER(c_double), c_int32,
                                  POINTER(c_double), POINTER(c_double), POINTER(c_double)]
    lib.mfp_contour_workspace_size.restype = c_size_t
    lib.mfp_contour_workspace_size.argtypes = [POINTER(MfpGrid)]
    lib.mfp_contour.argtypes = [POINTER(MfpGrid), c_void_p, c_void_p, c_void_p, c_double,
                                c_void_p, c_int64, POINTER(c_int64), c_void_p, c_size_t,
                                c_void_p]
    lib.mfp_grad_workspace_size.restype = c_size_t
    lib.mfp_grad_workspace_size.argtypes = [POINTER(MfpGrid), c_int32, c_int32]
    lib.mfp_psi_grad.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_void_p, c_void_p, c_void_p,
        POINTER(MfpFlow), POINTER(MfpSolverOpts), c_void_p, POINTER(c_double), c_void_p,
        c_double, c_int32, c_int32, c_void_p, POINTER(c_double), POINTER(c_double),
        POINTER(MfpStats), c_void_p, c_size_t, c_void_p]
    lib.mfp_conform_grad_workspace_size.restype = c_size_t
    lib.mfp_conform_grad_workspace_size.argtypes = [POINTER(MfpGrid), c_int32]
    lib.mfp_mesh_conform_grad.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
        POINTER(c_double), POINTER(c_double), c_void_p, c_size_t, c_void_p]
    lib.mfp_batched_workspace_size.restype = c_size_t
    lib.mfp_batched_workspace_size.argtypes = [c_int32, POINTER(MfpVariant), c_int32, c_int32]
    lib.mfp_batched_workspace_size_opts.restype = c_size_t
    lib.mfp_batched_workspace_size_opts.argtypes = [c_int32, POINTER(MfpVariant), c_int32,
                                                    POINTER(MfpSolverOpts)]
    lib.mfp_psi_solve_batched.argtypes = [
        c_int32, POINTER(MfpVariant), POINTER(MfpCircle), c_int32, POINTER(MfpFlow),
        POINTER(MfpSolverOpts), c_int32, c_int32, c_int32, POINTER(c_double),
        POINTER(c_double), POINTER(MfpStats), c_void_p, c_size_t, c_void_p]
    lib.mfp_kutta_workspace_size.restype = c_size_t
    lib.mfp_kutta_workspace_size.argtypes = [POINTER(MfpGrid), c_int32, c_int32,
                                             POINTER(MfpSolverOpts)]
    lib.mfp_psi_solve_kutta.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_void_p, c_void_p, c_void_p,
        POINTER(MfpFlow), POINTER(MfpSolverOpts), POINTER(c_double), c_int32, c_int32,
        c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double), POINTER(c_int64),
        POINTER(MfpStats), c_void_p, c_size_t, c_void_p]
    lib.mfp_body_bounds.argtypes = [POINTER(MfpBody), c_int32, POINTER(MfpCircle)]
    lib.mfp_mixed_mesh_bodies.argtypes = [POINTER(MfpGrid), POINTER(MfpBody), c_int32, c_int32,
                                          POINTER(MfpMixedMesh), c_void_p, c_size_t, c_void_p]
    lib.mfp_mixed_kutta_workspace_size.restype = c_size_t
    lib.mfp_mixed_kutta_workspace_size.argtypes = [POINTER(MfpGrid), c_int64, c_int64, c_int32,
                                                   c_int32, POINTER(MfpSolverOpts)]
    lib.mfp_mixed_psi_solve_kutta.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, POINTER(MfpMixedMesh), POINTER(MfpFlow),
        POINTER(MfpSolverOpts), POINTER(c_double), c_int32, c_int32, c_void_p,
        POINTER(c_double), POINTER(c_double), POINTER(c_double), POINTER(c_int64),
        POINTER(MfpStats), c_void_p, c_size_t, c_void_p]
    lib.mfp_mixed_workspace_size.restype = c_size_t
    lib.mfp_mixed_workspace_size.argtypes = [POINTER(MfpGrid), c_int32]
    lib.mfp_mixed_mesh.argtypes = [POINTER(MfpGrid), POINTER(MfpCircle), c_int32, c_int32,
                                   POINTER(MfpMixedMesh), c_void_p, c_size_t, c_void_p]
    lib.mfp_mixed_solve_workspace_size.restype = c_size_t
    lib.mfp_mixed_solve_workspace_size.argtypes = [POINTER(MfpGrid), c_int64, c_int64, c_int32,
                                                   POINTER(MfpSolverOpts)]
    lib.mfp_mixed_element_apply.argtypes = [POINTER(MfpGrid), POINTER(MfpMixedMesh), c_void_p,
                                            c_void_p, c_int32, POINTER(c_double), c_void_p,
                                            c_size_t, c_void_p]
    lib.mfp_mixed_psi_solve.argtypes = [
        POINTER(MfpGrid), POINTER(MfpCircle), c_int32, POINTER(MfpMixedMesh), POINTER(MfpFlow),
        POINTER(MfpSolverOpts), c_int32, c_int32, c_void_p, POINTER(c_double),
        POINTER(c_double), POINTER(c_double), POINTER(MfpStats), c_void_p, c_size_t, c_void_p]
    _lib = lib
    return lib


def last_error() -> str:
    return load().mfp_last_error().decode()


def _check(status: int, allow_warn: bool = True) -> int:
    if status < 0 or (status > 0 and not allow_warn):
        raise MfpError(status, last_error())
    return status


def make_grid(g) -> MfpGrid:
    return MfpGrid(int(g.nx), int(g.ny), float(g.x0), float(g.x1), float(g.y0), float(g.y1))


def make_circles(circles: Sequence) -> ctypes.Array:
    arr = (MfpCircle * max(1, len(circles)))()
    for k, (cx, cy, r) in enumerate(circles):
        arr[k] = MfpCircle(float(cx), float(cy), float(r))
    return arr


def make_flow(flow) -> MfpFlow:
    f = MfpFlow()
    f.U = float(flow.U)
    for k in range(4):
        f.side_bc[k] = int(flow.side_bc[k])
    return f


def _stream() -> c_void_p:
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> c_void_p:
    return c_void_p(t.data_ptr() if t is not None else 0)


def check_geometry(grid, circles) -> int:
    """Host-only geometry check; returns the status code."""
    g = make_grid(grid)
    c = make_circles(circles)
    return load().mfp_check_geometry(byref(g), c, len(circles))


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def mesh_conform(grid, circles, nsweeps: int = 200, device="cuda"):
    """Returns (disp[2*nodes] f64, kind[nodes] i8, body[nodes] i8) device tensors."""
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    n = (g.nx + 1) * (g.ny + 1)
    disp = torch.empty(2 * n, dtype=torch.float64, device=device)
    kind = torch.empty(n, dtype=torch.int8, device=device)
    body = torch.empty(n, dtype=torch.int8, device=device)
    wsz = lib.mfp_conform_workspace_size(byref(g), len(circles))
    ws = workspace(wsz, device)
    _check(lib.mfp_mesh_conform(byref(g), c, len(circles), int(nsweeps), _ptr(disp),
                                _ptr(kind), _ptr(body), _ptr(ws), ws.numel(), _stream()))
    return disp, kind, body


def element_apply(grid, disp: torch.Tensor, body: torch.Tensor, p: torch.Tensor,
                  precision: str = "fp64", repeat: int = 1):
    """q = K p over active cells (no boundary conditions).  Returns (q, mean ms)."""
    lib = load()
    g = make_grid(grid)
    prec = _PREC[precision]
    dt = torch.float64 if prec == FP64 else torch.float32
    p = p.to(dt).contiguous()
    q = torch.empty_like(p)
    wsz = lib.mfp_solve_workspace_size(byref(g), MAX_BODIES, prec)
    ws = workspace(wsz, p.device)
    ms = c_double(0.0)
    _check(lib.mfp_element_apply(byref(g), _ptr(disp), _ptr(body), prec, _ptr(p), _ptr(q),
                                 int(repeat), byref(ms), _ptr(ws), ws.numel(), _stream()))
    return q, ms.value


def element_apply_noalloc(grid, disp: torch.Tensor, body: torch.Tensor, p: torch.Tensor,
                          precision: str = "fp64", q: Optional[torch.Tensor] = None):
    """q = K p through mfp_element_apply_noalloc (no workspace: the library's static
    scratch).  q: optional preallocated output of p's dtype and size."""
    lib = load()
    g = make_grid(grid)
    prec = _PREC[precision]
    dt = torch.float64 if prec == FP64 else torch.float32
    p = p.to(dt).contiguous()
    if q is None:
        q = torch.empty_like(p)
    _check(lib.mfp_element_apply_noalloc(byref(g), _ptr(disp), _ptr(body), prec, _ptr(p),
                                         _ptr(q), _stream()))
    return q


@dataclass
class SolveResult:
    psi: torch.Tensor
    psi_b: list
    Q: float
    copfi: float
    theta: torch.Tensor
    ut: torch.Tensor
    sample_body: torch.Tensor
    n_samples: int
    stats: dict
    status: int


def psi_solve(grid, circles, disp, kind, body, flow, *, precision="fp64", rtol=1e-12,
              kmax=10 ** 7, check_every=16, inner_rtol=0.1, max_outer=1000, pair=(-1, -1),
              sample_cap=None, ws: Optional[torch.Tensor] = None,
              allow_warn: bool = True, profile_every: int = 0,
              psi0: Optional[torch.Tensor] = None, estimate_kappa: bool = False,
              rtol_from_start: bool = False, schedule: Optional[dict] = None) -> SolveResult:
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    nb = len(circles)
    f = make_flow(flow)
    prec = _PREC[precision]
    o = MfpSolverOpts(prec, float(rtol), int(kmax), int(check_every), float(inner_rtol),
                      int(max_outer), _ptr(psi0) if psi0 is not None else None,
                      int(profile_every), int(bool(estimate_kappa)), int(bool(rtol_from_start)))
    _set_schedule(o, schedule)
    n = (g.nx + 1) * (g.ny + 1)
    dev = disp.device
    psi = torch.empty(n, dtype=torch.float64, device=dev)
    if sample_cap is None:
        sample_cap = 64 * (g.nx + g.ny) if nb else 0
    samples = torch.empty(max(2 * sample_cap, 2), dtype=torch.float64, device=dev)
    sbody = torch.empty(max(sample_cap, 1), dtype=torch.int8, device=dev)
    psib = (c_double * max(nb, 1))()
    Q = c_double(float("nan"))
    cop = c_double(float("nan"))
    ns = c_int32(0)
    st = MfpStats()
    if ws is None:
        ws = workspace(lib.mfp_solve_workspace_size_opts(byref(g), nb, byref(o)), dev)
    status = _check(lib.mfp_psi_solve(
        byref(g), c, nb, _ptr(disp), _ptr(kind), _ptr(body), byref(f), byref(o),
        int(pair[0]), int(pair[1]), _ptr(psi), psib, byref(Q), byref(cop), _ptr(samples),
        _ptr(sbody), int(sample_cap), byref(ns), byref(st), _ptr(ws), ws.numel(), _stream()),
        allow_warn)
    m = min(ns.value, sample_cap)
    stats = {k: getattr(st, k) for k, _ in MfpStats._fields_}
    return SolveResult(psi, [psib[k] for k in range(nb)], Q.value, cop.value,
                       samples[0:2 * m:2], samples[1:2 * m:2], sbody[:m], ns.value, stats,
                       status)


@dataclass
class PhiResult:
    phi: torch.Tensor    # nodal potential (NaN at nodes of no active cell)
    stats: dict
    status: int


def phi_solve(grid, circles, disp, kind, body, flow, *, precision="fp64", rtol=1e-12,
              kmax=10 ** 7, check_every=16, inner_rtol=0.1, max_outer=1000,
              ws: Optional[torch.Tensor] = None, allow_warn: bool = True,
              profile_every: int = 0, phi0: Optional[torch.Tensor] = None,
              estimate_kappa: bool = False, rtol_from_start: bool = False,
              schedule: Optional[dict] = None) -> PhiResult:
    """Velocity potential on the conformed mesh (mfp_phi_solve): ``flow`` gives the
    Dirichlet sides (e.g. phi = U x on inlet and outlet), bodies and the other sides
    are natural boundaries.  phi0: optional nodal warm start (device doubles; its
    values at the unknowns are used, NaN elsewhere is ignored)."""
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    nb = len(circles)
    f = make_flow(flow)
    prec = _PREC[precision]
    o = MfpSolverOpts(prec, float(rtol), int(kmax), int(check_every), float(inner_rtol),
                      int(max_outer), _ptr(phi0) if phi0 is not None else None,
                      int(profile_every), int(bool(estimate_kappa)), int(bool(rtol_from_start)))
    _set_schedule(o, schedule)
    n = (g.nx + 1) * (g.ny + 1)
    dev = disp.device
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    st = MfpStats()
    if ws is None:
        ws = workspace(lib.mfp_solve_workspace_size_opts(byref(g), nb, byref(o)), dev)
    status = _check(lib.mfp_phi_solve(
        byref(g), c, nb, _ptr(disp), _ptr(kind), _ptr(body), byref(f), byref(o), _ptr(phi),
        byref(st), _ptr(ws), ws.numel(), _stream()), allow_warn)
    return PhiResult(phi, {k: getattr(st, k) for k, _ in MfpStats._fields_}, status)


def cubic_fit(x: Sequence[float], y: Sequence[float]):
    """Least-squares cubic y ~ c3 x^3 + c2 x^2 + c1 x + c0 (mfp_cubic_fit), e.g. CoPFI
    over the gap ratio of a sweep.  Returns ((c3, c2, c1, c0), R^2, MSE)."""
    n = len(x)
    if len(y) != n:
        raise ValueError("x and y differ in length")
    xa = (c_double * max(n, 1))(*[float(v) for v in x])
    ya = (c_double * max(n, 1))(*[float(v) for v in y])
    c = (c_double * 4)()
    r2 = c_double(0.0)
    mse = c_double(0.0)
    _check(load().mfp_cubic_fit(xa, ya, n, c, byref(r2), byref(mse)), False)
    return (c[0], c[1], c[2], c[3]), r2.value, mse.value


def contour(grid, disp: torch.Tensor, body: torch.Tensor, field: torch.Tensor, level: float,
            cap: Optional[int] = None) -> torch.Tensor:
    """Contour line field = level (mfp_contour): (k, 4) device tensor of segments
    (x0, y0, x1, y1) in cell order.  cap None: all of them (counted first)."""
    lib = load()
    g = make_grid(grid)
    dev = field.device
    ws = workspace(lib.mfp_contour_workspace_size(byref(g)), dev)
    n = c_int64(0)
    if cap is None:
        _check(lib.mfp_contour(byref(g), _ptr(disp), _ptr(body), _ptr(field), float(level),
                               None, 0, byref(n), _ptr(ws), ws.numel(), _stream()), False)
        cap = n.value
    seg = torch.empty(max(4 * cap, 4), dtype=torch.float64, device=dev)
    _check(lib.mfp_contour(byref(g), _ptr(disp), _ptr(body), _ptr(field), float(level),
                           _ptr(seg), int(cap), byref(n), _ptr(ws), ws.numel(), _stream()),
           False)
    return seg[:4 * min(cap, n.value)].view(-1, 4)


def solve_workspace_size(grid, nbody: int, precision: str = "fp64") -> int:
    g = make_grid(grid)
    return load().mfp_solve_workspace_size(byref(g), int(nbody), _PREC[precision])


def _opts(precision, rtol, kmax, check_every, inner_rtol, max_outer, estimate_kappa=False,
          schedule=None):
    o = MfpSolverOpts(_PREC[precision], float(rtol), int(kmax), int(check_every),
                      float(inner_rtol), int(max_outer), None, 0, int(bool(estimate_kappa)), 0)
    return _set_schedule(o, schedule)


def psi_grad(grid, circles, disp, kind, body, flow, psi, psi_b, *, dL_dpsib=None,
             dL_dcopfi=0.0, pair=(-1, -1), precision="fp64", rtol=1e-12, kmax=10 ** 7,
             check_every=16, inner_rtol=0.1, max_outer=1000, allow_warn=True,
             estimate_kappa=False, schedule=None):
    """Adjoint solve + shape derivative.  Returns (dL_ddisp device tensor [2*nodes],
    explicit dL/dcentre list of (dx, dy) per body, stats, status, dL/dU)."""
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    nb = len(circles)
    f = make_flow(flow)
    o = _opts(precision, rtol, kmax, check_every, inner_rtol, max_outer, estimate_kappa,
              schedule)
    n = (g.nx + 1) * (g.ny + 1)
    dev = disp.device
    out = torch.empty(2 * n, dtype=torch.float64, device=dev)
    pb = (c_double * max(nb, 1))(*[float(v) for v in psi_b])
    dpb = None
    if dL_dpsib is not None:
        dpb = (c_double * max(nb, 1))(*[float(v) for v in dL_dpsib])
    dcen = (c_double * max(2 * nb, 1))()
    dU = c_double(0.0)
    st = MfpStats()
    # an explicit schedule can need more solver workspace than the automatic one
    extra = max(0, lib.mfp_solve_workspace_size_opts(byref(g), nb, byref(o)) -
                lib.mfp_solve_workspace_size(byref(g), nb, _PREC[precision]))
    ws = workspace(lib.mfp_grad_workspace_size(byref(g), nb, _PREC[precision]) + extra, dev)
    status = _check(lib.mfp_psi_grad(
        byref(g), c, nb, _ptr(disp), _ptr(kind), _ptr(body), byref(f), byref(o), _ptr(psi),
        pb, dpb, float(dL_dcopfi), int(pair[0]), int(pair[1]), _ptr(out), dcen, byref(dU),
        byref(st), _ptr(ws), ws.numel(), _stream()), allow_warn)
    stats = {k: getattr(st, k) for k, _ in MfpStats._fields_}
    return (out, [(dcen[2 * b], dcen[2 * b + 1]) for b in range(nb)], stats, status,
            dU.value)


def mesh_conform_grad(grid, circles, kind, body, dL_ddisp, nsweeps=200, dL_dcentre=None,
                      dL_dradius=None):
    """Adds the mesh part of the gradient; returns (dL_dcentre [(dx, dy)], dL_dradius)."""
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    nb = len(circles)
    dcen = (c_double * max(2 * nb, 1))()
    drad = (c_double * max(nb, 1))()
    if dL_dcentre is not None:
        for b, (gx, gy) in enumerate(dL_dcentre):
            dcen[2 * b], dcen[2 * b + 1] = float(gx), float(gy)
    if dL_dradius is not None:
        for b, v in enumerate(dL_dradius):
            drad[b] = float(v)
    ws = workspace(lib.mfp_conform_grad_workspace_size(byref(g), nb), dL_ddisp.device)
    _check(lib.mfp_mesh_conform_grad(byref(g), c, nb, int(nsweeps), _ptr(kind), _ptr(body),
                                     _ptr(dL_ddisp), dcen, drad, _ptr(ws), ws.numel(),
                                     _stream()))
    return [(dcen[2 * b], dcen[2 * b + 1]) for b in range(nb)], [drad[b] for b in range(nb)]


@dataclass
class BatchResult:
    psi: list            # device tensors (or None)
    psi_b: list          # per system, list of nbody values
    copfi: list
    stats: list
    status: int


def psi_solve_batched(systems, flow, *, precision="fp32_ir", rtol=1e-10, kmax=10 ** 7,
                      iters_per_launch=0, pair=(-1, -1), want_psi=False,
                      ws: Optional[torch.Tensor] = None,
                      schedule: Optional[dict] = None) -> BatchResult:
    """systems: list of (grid, circles, disp, kind, body); all with the same number of
    bodies.  One graph-replayed launch sequence for all of them."""
    lib = load()
    nvar = len(systems)
    nb = len(systems[0][1])
    vars_ = (MfpVariant * nvar)()
    circ = (MfpCircle * max(1, nvar * nb))()
    psis = []
    for i, (grid, circles, disp, kind, body) in enumerate(systems):
        assert len(circles) == nb
        g = make_grid(grid)
        psi = None
        if want_psi:
            psi = torch.empty((g.nx + 1) * (g.ny + 1), dtype=torch.float64, device=disp.device)
        psis.append(psi)
        vars_[i] = MfpVariant(g, c_void_p(disp.data_ptr()), c_void_p(kind.data_ptr()),
                              c_void_p(body.data_ptr()), _ptr(psi) if psi is not None else None)
        for b, (cx, cy, r) in enumerate(circles):
            circ[i * nb + b] = MfpCircle(float(cx), float(cy), float(r))
    f = make_flow(flow)
    o = _opts(precision, rtol, kmax, 64, 0.1, 1000, schedule=schedule)
    psib = (c_double * max(1, nvar * nb))()
    cop = (c_double * nvar)()
    st = (MfpStats * nvar)()
    if ws is None:
        ws = workspace(lib.mfp_batched_workspace_size_opts(nvar, vars_, nb, byref(o)),
                       systems[0][2].device)
    status = _check(lib.mfp_psi_solve_batched(
        nvar, vars_, circ, nb, byref(f), byref(o), int(iters_per_launch), int(pair[0]),
        int(pair[1]), psib, cop, st, _ptr(ws), ws.numel(), _stream()))
    stats = [{k: getattr(st[i], k) for k, _ in MfpStats._fields_} for i in range(nvar)]
    return BatchResult(psis, [[psib[i * nb + b] for b in range(nb)] for i in range(nvar)],
                       [cop[i] for i in range(nvar)], stats, status)


def batched_workspace_size(systems, precision="fp32_ir", schedule=None) -> int:
    lib = load()
    nvar = len(systems)
    vars_ = (MfpVariant * nvar)()
    for i, s in enumerate(systems):
        vars_[i] = MfpVariant(make_grid(s[0]), None, None, None, None)
    o = _opts(precision, 1e-10, 1, 64, 0.1, 1000, schedule=schedule)
    return lib.mfp_batched_workspace_size_opts(nvar, vars_, len(systems[0][1]), byref(o))


@dataclass
class MixedMesh:
    """Device arrays of a mixed-cell mesh (see mfp_mixed_mesh_t)."""
    grid: object
    circles: list
    disp: torch.Tensor        # 2 nodes f64 (x, then y)
    body: torch.Tensor        # nodes i8
    hpt: torch.Tensor         # (ny+1) nx i32
    vpt: torch.Tensor         # ny (nx+1) i32
    cell_first: torch.Tensor  # nx ny + 1 i32
    pxy: torch.Tensor         # (n_points, 2) f64
    pbody: torch.Tensor       # n_points i8
    pedge: torch.Tensor       # n_points i32
    elem: torch.Tensor        # (n_elems, 4) i32
    nne: torch.Tensor         # n_elems i8
    n_tri: int

    @property
    def n_points(self) -> int:
        return int(self.pbody.numel())

    @property
    def n_elems(self) -> int:
        return int(self.nne.numel())

    @property
    def n_nodes(self) -> int:
        return (self.grid.nx + 1) * (self.grid.ny + 1) + self.n_points

    def c_struct(self) -> MfpMixedMesh:
        return MfpMixedMesh(_ptr(self.disp), _ptr(self.body), _ptr(self.hpt), _ptr(self.vpt),
                            _ptr(self.cell_first), _ptr(self.pxy), _ptr(self.pbody),
                            _ptr(self.pedge), _ptr(self.elem), _ptr(self.nne), self.n_points,
                            self.n_elems, self.n_points, self.n_elems, self.n_tri)


def make_bodies(bodies: Sequence) -> ctypes.Array:
    """Bodies as ("circle", cx, cy, r) or ("joukowski", x, y, c, xi0, eta0, alpha)."""
    arr = (MfpBody * max(1, len(bodies)))()
    for k, b in enumerate(bodies):
        if b[0] == "circle":
            arr[k] = MfpBody(BODY_CIRCLE, float(b[1]), float(b[2]), float(b[3]), 0.0, 0.0, 0.0)
        elif b[0] == "joukowski":
            arr[k] = MfpBody(BODY_JOUKOWSKI, *(float(v) for v in b[1:7]))
        else:
            raise ValueError(f"unknown body kind {b[0]!r}")
    return arr


def body_bounds(bodies: Sequence) -> list:
    """The circle that mfp_body_bounds gives for each body: [(cx, cy, r), ...]."""
    arr = make_bodies(bodies)
    out = (MfpCircle * max(1, len(bodies)))()
    _check(load().mfp_body_bounds(arr, len(bodies), out))
    return [(out[k].cx, out[k].cy, out[k].r) for k in range(len(bodies))]


def mixed_mesh_bodies(grid, bodies, nsweeps: int = 200, device="cuda") -> MixedMesh:
    """Mixed-cell mesh of general bodies (see make_bodies); the mesh's circles are the
    bodies' bounding circles (mfp_body_bounds)."""
    return mixed_mesh(grid, body_bounds(bodies), nsweeps, device, _bodies=bodies)


def mixed_mesh(grid, circles, nsweeps: int = 200, device="cuda", _bodies=None) -> MixedMesh:
    """Mixed-cell mesh: a sizing call (zero capacities), then the filling call."""
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    nb = len(circles)
    if _bodies is not None:
        barr = make_bodies(_bodies)

        def build(m):
            return lib.mfp_mixed_mesh_bodies(byref(g), barr, nb, int(nsweeps), byref(m),
                                             _ptr(ws), ws.numel(), _stream())
    else:
        def build(m):
            return lib.mfp_mixed_mesh(byref(g), c, nb, int(nsweeps), byref(m), _ptr(ws),
                                      ws.numel(), _stream())
    n = (g.nx + 1) * (g.ny + 1)
    disp = torch.empty(2 * n, dtype=torch.float64, device=device)
    body = torch.empty(n, dtype=torch.int8, device=device)
    hpt = torch.empty((g.ny + 1) * g.nx, dtype=torch.int32, device=device)
    vpt = torch.empty(g.ny * (g.nx + 1), dtype=torch.int32, device=device)
    first = torch.empty(g.nx * g.ny + 1, dtype=torch.int32, device=device)
    ws = workspace(lib.mfp_mixed_workspace_size(byref(g), nb), device)
    m = MfpMixedMesh(_ptr(disp), _ptr(body), _ptr(hpt), _ptr(vpt), _ptr(first))
    _check(build(m))
    npts, nel = m.n_points, m.n_elems
    pxy = torch.empty((max(npts, 1), 2), dtype=torch.float64, device=device)
    pbody = torch.empty(max(npts, 1), dtype=torch.int8, device=device)
    pedge = torch.empty(max(npts, 1), dtype=torch.int32, device=device)
    elem = torch.empty((max(nel, 1), 4), dtype=torch.int32, device=device)
    nne = torch.empty(max(nel, 1), dtype=torch.int8, device=device)
    m.pxy, m.pbody, m.pedge = _ptr(pxy), _ptr(pbody), _ptr(pedge)
    m.elem, m.nne = _ptr(elem), _ptr(nne)
    m.cap_points, m.cap_elems = npts, nel
    _check(build(m))
    return MixedMesh(grid, list(circles), disp, body, hpt, vpt, first, pxy[:npts],
                     pbody[:npts], pedge[:npts], elem[:nel], nne[:nel], int(m.n_tri))


def mixed_element_apply(mm: MixedMesh, p: torch.Tensor, repeat: int = 1):
    """q = K p on the mixed mesh (mixed-node numbering).  Returns (q, mean ms)."""
    lib = load()
    g = make_grid(mm.grid)
    p = p.to(torch.float64).contiguous()
    if p.numel() != mm.n_nodes:
        raise ValueError(f"p has {p.numel()} values, the mesh {mm.n_nodes} nodes")
    q = torch.empty_like(p)
    m = mm.c_struct()
    ws = workspace(lib.mfp_mixed_solve_workspace_size(byref(g), mm.n_points, mm.n_elems, 0,
                                                      None), p.device)
    ms = c_double(0.0)
    _check(lib.mfp_mixed_element_apply(byref(g), byref(m), _ptr(p), _ptr(q), int(repeat),
                                       byref(ms), _ptr(ws), ws.numel(), _stream()))
    return q, ms.value


@dataclass
class MixedSolveResult:
    psi: torch.Tensor   # mixed-node values
    psi_b: list
    Q: float
    copfi: float
    stats: dict
    status: int


def mixed_psi_solve(mm: MixedMesh, flow, *, precision="fp64", rtol=1e-12, kmax=10 ** 7,
                    check_every=16, inner_rtol=0.1, max_outer=1000, pair=(-1, -1),
                    estimate_kappa: bool = False, schedule: Optional[dict] = None,
                    profile_every: int = 0, allow_warn: bool = True) -> MixedSolveResult:
    lib = load()
    g = make_grid(mm.grid)
    c = make_circles(mm.circles)
    nb = len(mm.circles)
    f = make_flow(flow)
    o = _opts(precision, rtol, kmax, check_every, inner_rtol, max_outer, estimate_kappa,
              schedule)
    o.profile_every = int(profile_every)
    dev = mm.disp.device
    psi = torch.empty(mm.n_nodes, dtype=torch.float64, device=dev)
    psib = (c_double * max(nb, 1))()
    Q = c_double(float("nan"))
    cop = c_double(float("nan"))
    st = MfpStats()
    m = mm.c_struct()
    ws = workspace(lib.mfp_mixed_solve_workspace_size(byref(g), mm.n_points, mm.n_elems, nb,
                                                      byref(o)), dev)
    status = _check(lib.mfp_mixed_psi_solve(
        byref(g), c, nb, byref(m), byref(f), byref(o), int(pair[0]), int(pair[1]), _ptr(psi),
        psib, byref(Q), byref(cop), byref(st), _ptr(ws), ws.numel(), _stream()), allow_warn)
    stats = {k: getattr(st, k) for k, _ in MfpStats._fields_}
    return MixedSolveResult(psi, [psib[k] for k in range(nb)], Q.value, cop.value, stats, status)


@dataclass
class KuttaResult:
    psi: torch.Tensor
    psi_b: list
    Q: float
    copfi: float
    kutta_nodes: list
    stats: dict
    status: int


def psi_solve_kutta(grid, circles, disp, kind, body, flow, kutta_points, *, precision="fp64",
                    rtol=1e-12, kmax=10 ** 7, check_every=16, inner_rtol=0.1, max_outer=1000,
                    pair=(-1, -1), estimate_kappa: bool = False,
                    schedule: Optional[dict] = None, allow_warn: bool = True) -> KuttaResult:
    """Solve with Kutta constraints: kutta_points holds one (x, y) or None per body."""
    lib = load()
    g = make_grid(grid)
    c = make_circles(circles)
    nb = len(circles)
    if len(kutta_points) != nb:
        raise ValueError("one Kutta point (or None) per body")
    f = make_flow(flow)
    o = _opts(precision, rtol, kmax, check_every, inner_rtol, max_outer, estimate_kappa,
              schedule)
    kxy = (c_double * max(2 * nb, 2))()
    for b, pt in enumerate(kutta_points):
        kxy[2 * b], kxy[2 * b + 1] = (float("nan"), float("nan")) if pt is None else (
            float(pt[0]), float(pt[1]))
    nk = sum(pt is not None for pt in kutta_points)
    dev = disp.device
    psi = torch.empty((g.nx + 1) * (g.ny + 1), dtype=torch.float64, device=dev)
    psib = (c_double * max(nb, 1))()
    Q = c_double(float("nan"))
    cop = c_double(float("nan"))
    kn = (c_int64 * max(nb, 1))()
    st = MfpStats()
    ws = workspace(lib.mfp_kutta_workspace_size(byref(g), nb, nk, byref(o)), dev)
    status = _check(lib.mfp_psi_solve_kutta(
        byref(g), c, nb, _ptr(disp), _ptr(kind), _ptr(body), byref(f), byref(o), kxy,
        int(pair[0]), int(pair[1]), _ptr(psi), psib, byref(Q), byref(cop), kn, byref(st),
        _ptr(ws), ws.numel(), _stream()), allow_warn)
    stats = {k: getattr(st, k) for k, _ in MfpStats._fields_}
    return KuttaResult(psi, [psib[k] for k in range(nb)], Q.value, cop.value,
                       [kn[k] for k in range(nb)], stats, status)


def mixed_psi_solve_kutta(mm: MixedMesh, flow, kutta_points, *, precision="fp64", rtol=1e-12,
                          kmax=10 ** 7, check_every=16, inner_rtol=0.1, max_outer=1000,
                          pair=(-1, -1), estimate_kappa: bool = False,
                          schedule: Optional[dict] = None,
                          allow_warn: bool = True) -> MixedSolveResult:
    """mixed_psi_solve with Kutta constraints: one (x, y) or None per body."""
    lib = load()
    g = make_grid(mm.grid)
    c = make_circles(mm.circles)
    nb = len(mm.circles)
    if len(kutta_points) != nb:
        raise ValueError("one Kutta point (or None) per body")
    f = make_flow(flow)
    o = _opts(precision, rtol, kmax, check_every, inner_rtol, max_outer, estimate_kappa,
              schedule)
    kxy = (c_double * max(2 * nb, 2))()
    for b, pt in enumerate(kutta_points):
        kxy[2 * b], kxy[2 * b + 1] = (float("nan"), float("nan")) if pt is None else (
            float(pt[0]), float(pt[1]))
    nk = sum(pt is not None for pt in kutta_points)
    dev = mm.disp.device
    psi = torch.empty(mm.n_nodes, dtype=torch.float64, device=dev)
    psib = (c_double * max(nb, 1))()
    Q = c_double(float("nan"))
    cop = c_double(float("nan"))
    kn = (c_int64 * max(nb, 1))()
    st = MfpStats()
    m = mm.c_struct()
    ws = workspace(lib.mfp_mixed_kutta_workspace_size(byref(g), mm.n_points, mm.n_elems, nb, nk,
                                                      byref(o)), dev)
    status = _check(lib.mfp_mixed_psi_solve_kutta(
        byref(g), c, nb, byref(m), byref(f), byref(o), kxy, int(pair[0]), int(pair[1]),
        _ptr(psi), psib, byref(Q), byref(cop), kn, byref(st), _ptr(ws), ws.numel(), _stream()),
        allow_warn)
    stats = {k: getattr(st, k) for k, _ in MfpStats._fields_}
    res = MixedSolveResult(psi, [psib[k] for k in range(nb)], Q.value, cop.value, stats, status)
    res.kutta_nodes = [kn[k] for k in range(nb)]
    return res
