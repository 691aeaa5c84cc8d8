"""CoPFI as a differentiable function of the body centres (torch.autograd).

forward:  centres (nbody x 2, float64, any device) -> CoPFI of the pair (lo, hi):
          mesh_conform + psi_solve on the GPU.
backward: psi_grad (adjoint solve + shape derivative + the explicit dependence of
          CoPFI on the pair's centre heights) then mesh_conform_grad (transposed
          sweeps + projection), all in the library; the result is handed back to torch
          so that any parametrisation of the centres (for example by the gap ratio)
          is differentiated by torch's own chain rule.
"""
from __future__ import annotations

import torch

from . import binding as B


def _require_converged(status: int) -> None:
    if status not in (B.MFP_OK, B.MFP_W_STAGNATION):
        raise B.MfpError(status, B.last_error())


class CoPFIFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, centres, radii, grid, flow, pair, nsweeps=200, precision="fp64",
                rtol=1e-12, device="cuda"):
        cen = centres.detach().to("cpu", torch.float64)
        circles = [(float(cen[b, 0]), float(cen[b, 1]), float(radii[b]))
                   for b in range(cen.shape[0])]
        disp, kind, body = B.mesh_conform(grid, circles, nsweeps, device=device)
        # an unconverged solve must not feed torch: warnings other than a refined
        # solve finished in FP64 (MFP_W_STAGNATION, converged) raise
        res = B.psi_solve(grid, circles, disp, kind, body, flow, precision=precision,
                          rtol=rtol, pair=pair)
        _require_converged(res.status)
        ctx.saved = (grid, flow, pair, nsweeps, precision, rtol, circles, disp, kind, body,
                     res.psi, res.psi_b)
        ctx.centres_meta = (centres.device, centres.dtype)
        return torch.tensor(res.copfi, dtype=torch.float64, device=centres.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grid, flow, pair, nsweeps, precision, rtol, circles, disp, kind, body, psi,
         psi_b) = ctx.saved
        g = float(grad_out)
        dL_ddisp, explicit, _, status, _ = B.psi_grad(grid, circles, disp, kind, body, flow,
                                                      psi, psi_b, dL_dcopfi=g, pair=pair,
                                                      precision=precision, rtol=rtol)
        _require_converged(status)
        dcen, _ = B.mesh_conform_grad(grid, circles, kind, body, dL_ddisp, nsweeps,
                                      dL_dcentre=explicit)
        dev, dt = ctx.centres_meta
        return (torch.tensor(dcen, dtype=dt, device=dev), None, None, None, None, None, None,
                None, None)


def copfi(centres, radii, grid, flow, pair, nsweeps=200, precision="fp64", rtol=1e-12,
          device="cuda"):
    """Differentiable CoPFI(centres)."""
    return CoPFIFunction.apply(centres, radii, grid, flow, pair, nsweeps, precision, rtol,
                               device)
