"""GPU parity of the velocity-potential solve against the oracle's direct solve.

The potential uses the psi solver's operator and iteration with the bodies as
natural boundaries and no body constraint (unknowns: every non-Dirichlet node
of an active cell; nodes of no active cell are NaN).  Bars, as for psi: FP64
CG stopped at relative residual 1e-13, nodal phi relative L2 error <= 1e-10
over the domain, the NaN pattern and the unknown count exact.  phi is O(10)
on these grids (U x on [-20, 20]).
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = {
    "cyl64": W.potential_flow(W.single_cylinder(64)),
    "cyl64_exact_bc": W.potential_flow(W.single_cylinder(64), exact_bc=True),
    "five96x48": W.potential_flow(W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))),
    "five_ragged130x67": W.potential_flow(
        W.five_cylinders(130, 67, 0.4, extent=(-6.5, 6.5, -3.35, 3.35))),
    "five_gap_lt_h_256x128": W.potential_flow(W.five_cylinders(256, 128, 0.05)),
    "channel_nobody_70x9": W.potential_flow(
        W.Case("channel", W.Grid(70, 9, 0.0, 7.0, 0.0, 0.9), [])),
}


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


def run_pair(mfp, c, rtol=1e-13, precision="fp64"):
    say(f"[phi] {c.name} {precision}")
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    res = mfp.phi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=rtol,
                        precision=precision)
    mesh = O.conform(c.grid, c.circles, c.nsweeps)
    ref = O.phi_solve(mesh, c.flow)
    return res, ref, mesh


def _compare(res, ref, bar):
    phi = res.phi.cpu().numpy()
    np.testing.assert_array_equal(np.isnan(phi), np.isnan(ref.phi))
    dom = ~np.isnan(ref.phi)
    err = np.linalg.norm(phi[dom] - ref.phi[dom]) / np.linalg.norm(ref.phi[dom])
    assert err <= bar, err
    # node by node as well (one bad node would hide in the norm)
    dmax = np.abs(phi[dom] - ref.phi[dom]).max() / np.abs(ref.phi[dom]).max()
    assert dmax <= bar, dmax
    assert res.stats["n_dof"] == ref.ndof
    return err


@pytest.mark.parametrize("name", list(CASES))
def test_phi_fp64_matches_oracle(mfp, name):
    res, ref, _ = run_pair(mfp, CASES[name])
    assert res.status == 0
    err = _compare(res, ref, 1e-10)
    say(f"  iters {res.stats['iters']} relres {res.stats['relres_true']:.2e} rel L2 {err:.2e}")
    assert res.stats["relres_true"] <= 2e-13


def test_phi_without_bodies_is_the_free_stream(mfp):
    c = CASES["channel_nobody_70x9"]
    res, _, mesh = run_pair(mfp, c)
    X, _ = mesh.coords()
    np.testing.assert_allclose(res.phi.cpu().numpy(), c.flow.U * X.ravel(), rtol=0, atol=1e-10)


@pytest.mark.parametrize("name", ["five96x48", "five_gap_lt_h_256x128"])
def test_phi_fp32_refined_matches_oracle(mfp, name):
    res, ref, _ = run_pair(mfp, CASES[name], precision="fp32_ir")
    assert res.status == 0
    _compare(res, ref, 1e-10)


def test_phi_leaves_the_psi_solve_unchanged(mfp):
    """The potential's switches (body nodes free, no body sums) are per call: a psi
    solve after a phi solve in the same process gives the same result as before."""
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    a = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12, pair=c.pair)
    cp = W.potential_flow(c)
    mfp.phi_solve(cp.grid, cp.circles, disp, kind, body, cp.flow, rtol=1e-12)
    b = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12, pair=c.pair)
    assert torch.equal(a.psi, b.psi) and a.psi_b == b.psi_b


def test_phi_bench_workload_1024x512_matches_oracle_direct_solve(mfp):
    """The potential of the benchmark's five-cylinder workload at full size
    (1024x512), FP64 to relative residual 1e-12, against the oracle's direct solve.
    Bar 2e-10 relative L2 (as for psi at this size and tolerance)."""
    c = W.potential_flow(W.five_cyl_1024())
    res, ref, _ = run_pair(mfp, c, rtol=1e-12)
    assert res.status == 0 and res.stats["relres_true"] <= 1.5e-12
    err = _compare(res, ref, 2e-10)
    say(f"  1024x512 phi: iters {res.stats['iters']} rel L2 {err:.2e} "
        f"unknowns {res.stats['n_dof']}")


def test_phi_warm_start_from_its_solution(mfp):
    """A warm start from the potential converged to 1e-13 (psi0 of the options: its
    values at the unknowns, body nodes included) already meets a 1e-12 tolerance,
    which stays relative to ||b||: the solve ends converged after at most one
    iteration, and the result stays within 1e-12."""
    c = CASES["five96x48"]
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    a = mfp.phi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-13)
    b = mfp.phi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12,
                      phi0=a.phi.clone(), kmax=50, allow_warn=False)
    assert b.status == 0 and b.stats["iters"] <= 1
    assert b.stats["rnorm0"] == pytest.approx(a.stats["rnorm0"], rel=1e-14)
    assert b.stats["relres_true"] <= 2e-13
    pa, pb = a.phi.cpu().numpy(), b.phi.cpu().numpy()
    dom = ~np.isnan(pa)
    np.testing.assert_array_equal(np.isnan(pb), ~dom)
    assert np.abs(pa[dom] - pb[dom]).max() <= 1e-12 * np.abs(pa[dom]).max()
