"""GPU: the Lanczos condition estimate against the oracle's eigenvalues, warm starts,
the free-stream derivative of the adjoint, and the error paths forced from the host.

kappa_est comes from the CG scalars of the solve (Algorithm 1's alpha and beta) and
is compared with the oracle's extreme eigenvalues of A = T^T K T on layouts without
mirror symmetry, where the right-hand side reaches every eigenvector: each Ritz
extreme within 5% of the eigenvalue (and inside the spectrum up to rounding).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle.spectrum import condition_number
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

ASYM_SMALL = W.five_cylinders_asymmetric(96, 48, extent=(-6, 6, -3, 3))


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


def _kappa_case(mfp, c, precision, rtol):
    say(f"[kappa] {c.name} {precision}")
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    res = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=rtol,
                        precision=precision, estimate_kappa=True)
    assert res.status == 0
    mesh = O.conform(c.grid, c.circles, c.nsweeps)
    ref = O.solve(mesh, c.flow)
    lmin, lmax, kappa = condition_number(ref.A)
    st = res.stats
    say(f"  kappa {st['kappa_est']:.5e} (oracle {kappa:.5e}); ritz {st['ritz_min']:.4e} "
        f"{st['ritz_max']:.4e} (oracle {lmin:.4e} {lmax:.4e}); steps {st['kappa_steps']}")
    assert st["kappa_steps"] >= min(res.stats["iters"], 16383) - 1
    assert st["ritz_min"] >= lmin * (1 - 1e-6) and st["ritz_max"] <= lmax * (1 + 1e-6)
    assert st["ritz_min"] == pytest.approx(lmin, rel=0.05)
    assert st["ritz_max"] == pytest.approx(lmax, rel=0.05)
    assert st["kappa_est"] == pytest.approx(kappa, rel=0.05)
    return res


def test_kappa_estimate_fp64_96x48(mfp):
    _kappa_case(mfp, ASYM_SMALL, "fp64", 1e-12)


def test_kappa_estimate_fp32_refined_96x48(mfp):
    """The refined solve's FP32 runs, joined across the residual replacements."""
    res = _kappa_case(mfp, ASYM_SMALL, "fp32_ir", 1e-12)
    assert res.stats["inner_iters"] > 0 and res.stats["outer_iters"] >= 2


def test_kappa_estimate_fp64_1024x512(mfp):
    """Full size (520k unknowns); the oracle's extremes by ARPACK (shift-invert about
    zero for the smallest)."""
    _kappa_case(mfp, W.five_cylinders_asymmetric(1024, 512), "fp64", 1e-12)


def test_kappa_not_requested_is_zero(mfp):
    c = ASYM_SMALL
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    res = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-10)
    assert res.stats["kappa_est"] == 0.0 and res.stats["kappa_steps"] == 0
    assert res.stats["inner_iters"] == 0


def test_warm_start_keeps_the_target_and_saves_iterations(mfp):
    """rtol is relative to ||b|| whatever the start: a warm start from a looser
    solution reaches the same target in fewer iterations than a cold start, and one
    from the converged solution needs none."""
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    loose = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-8)
    cold = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12)
    warm = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12,
                         psi0=loose.psi, allow_warn=False)
    say(f"[warm] cold {cold.stats['iters']} warm {warm.stats['iters']}")
    assert warm.stats["rnorm0"] == pytest.approx(cold.stats["rnorm0"], rel=1e-14)
    assert warm.stats["relres_true"] <= 1.5e-12
    assert warm.stats["iters"] < cold.stats["iters"]
    a, b = warm.psi.cpu().numpy(), cold.psi.cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)
    again = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-11,
                          psi0=cold.psi, allow_warn=False)
    assert again.stats["iters"] <= 1
    assert np.abs(again.psi.cpu().numpy() - b).max() <= 1e-12 * np.abs(b).max()


def test_correction_solve_tolerance_from_the_start(mfp):
    """rtol_from_start: the threshold is rtol times the warm start's own residual."""
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    loose = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-6)
    r = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-4,
                      psi0=loose.psi, rtol_from_start=True, allow_warn=False)
    cold = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-4)
    # the reference residual is that of the start, about 1e-6 ||b||
    assert r.stats["rnorm0"] < 1e-5 * cold.stats["rnorm0"]
    assert r.stats["relres_true"] <= 1.5e-4


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_non_finite_warm_start_is_a_breakdown(mfp, precision):
    """A NaN in the warm start makes the first residual non-finite: MFP_E_BREAKDOWN,
    every kernel ends normally, and the next solve in the process is unaffected."""
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    ref = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12)
    bad = ref.psi.clone()
    bad[10 * (c.grid.nx + 1) + 10] = float("nan")  # a fluid node (body nodes take psi_b)
    say(f"[nan warm start] {precision}")
    with pytest.raises(mfp.MfpError) as e:
        mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12,
                      precision=precision, psi0=bad)
    assert e.value.status == mfp.MFP_E_BREAKDOWN
    torch.cuda.synchronize()
    after = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12)
    assert torch.equal(after.psi, ref.psi)


def test_non_finite_free_stream_rejected_before_device_work(mfp):
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    for U in (float("nan"), float("inf")):
        flow = W.Flow(U, c.flow.side_bc)
        with pytest.raises(mfp.MfpError) as e:
            mfp.psi_solve(c.grid, c.circles, disp, kind, body, flow, rtol=1e-12)
        assert e.value.status == mfp.MFP_E_ARG
        with pytest.raises(mfp.MfpError) as e:
            mfp.phi_solve(c.grid, c.circles, disp, kind, body, W.potential_flow(
                W.Case("x", c.grid, c.circles, flow)).flow, rtol=1e-12)
        assert e.value.status == mfp.MFP_E_ARG


# a single circle on the unit square that the radial projection alone (no smoothing
# sweeps) folds over: the oracle finds a negative Gauss-point Jacobian
TANGLE_GRID = W.Grid(16, 16, 0.0, 1.0, 0.0, 1.0)
TANGLE_CIRCLES = [(0.7288, 0.2475, 0.1633)]


def _min_detj(mesh):
    act = np.flatnonzero(O.active_cells(mesh.grid, mesh.body))
    xe, ye = O.element_coords(mesh, act)
    _, det = O.element_stiffness(xe, ye, return_det=True)
    hx, hy = O.spacing(mesh.grid)
    return det.min() / (0.25 * hx * hy)


def test_tangled_mesh_reported(mfp):
    m0 = O.conform(TANGLE_GRID, TANGLE_CIRCLES, 0)
    m200 = O.conform(TANGLE_GRID, TANGLE_CIRCLES, 200)
    assert _min_detj(m0) < 0.0 < _min_detj(m200)
    with pytest.raises(mfp.MfpError) as e:
        mfp.mesh_conform(TANGLE_GRID, TANGLE_CIRCLES, 0, device=DEV)
    assert e.value.status == mfp.MFP_E_TANGLED
    disp, _, _ = mfp.mesh_conform(TANGLE_GRID, TANGLE_CIRCLES, 200, device=DEV)
    assert np.array_equal(disp.cpu().numpy(), m200.disp.reshape(-1))


def test_free_stream_derivative_of_the_adjoint(mfp):
    """dL/dU of L = sum_b w_b psi_b + v CoPFI against a central difference of GPU
    solves in U (psi_b is linear in U, CoPFI independent of it)."""
    c = W.five_cylinders(96, 48, 0.5, extent=(-6, 6, -3, 3))
    w = [0.3, -1.0, 0.5, 2.0, 1.0]
    v = 0.7
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)

    def loss(U):
        f = W.Flow(U, c.flow.side_bc)
        r = mfp.psi_solve(c.grid, c.circles, disp, kind, body, f, rtol=1e-13, pair=c.pair)
        return float(np.dot(w, r.psi_b)) + v * r.copfi, r

    L0, r0 = loss(c.flow.U)
    *_, status, dU = mfp.psi_grad(c.grid, c.circles, disp, kind, body, c.flow, r0.psi,
                                  r0.psi_b, dL_dpsib=w, dL_dcopfi=v, pair=c.pair,
                                  rtol=1e-13)
    assert status == 0
    h = 1e-3
    fd = (loss(c.flow.U + h)[0] - loss(c.flow.U - h)[0]) / (2 * h)
    assert dU == pytest.approx(fd, rel=1e-8)
    assert dU == pytest.approx(float(np.dot(w, r0.psi_b)) / c.flow.U, rel=1e-12)
    assert math.isfinite(L0)
