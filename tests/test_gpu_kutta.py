"""GPU parity of the Kutta constraint (psi at an added fluid point equals psi_b in place
of the body's zero-circulation row; section "Boundary Conditions").

The library solves it by superposition of constrained CG solves; the oracle
(oracle/kutta.py) writes the square, nonsymmetric system out and solves it by sparse
LU.  Compared: psi node by node and psi_b within 1e-9 of max|psi| on the small
meshes (each sub-solve to 1e-12 relative residual at kappa <= 1e4 leaves at most
about 1e-8, measured far less), the Kutta equation psi(K_b) = psi_b itself, the
summed body rows recomputed with the oracle's matrix (zero circulation on the
bodies without a Kutta point, the oracle's circulation on the others), two Kutta
bodies at once (the host's 2 x 2 system), FP32 with FP64 refinement, the 1024 x 512
channel at full size, and the rejected points.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import kutta as KU
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = {
    "cyl64": (W.single_cylinder(64, half=4.0), [(0.875, -0.375)]),
    "five96x48_one": (W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
                      [None, None, None, (0.75, -1.5), None]),
    "five96x48_two": (W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
                      [None, None, None, (0.75, -1.5), (0.75, 1.0)]),
    "five_asym120x60": (W.five_cylinders_asymmetric(120, 60, extent=(-6, 6, -3, 3)),
                        [(-2.2, 0.0), None, None, None, (0.5, 1.0)]),
}


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


def _compare(mfp, case, pts, precision, tol_rel):
    say(f"[kutta] {case.name} {precision}")
    disp, kind, body = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=DEV)
    res = mfp.psi_solve_kutta(case.grid, case.circles, disp, kind, body, case.flow, pts,
                              precision=precision, rtol=1e-12, pair=case.pair)
    assert res.status == mfp.MFP_OK
    mesh = O.conform(case.grid, case.circles, case.nsweeps)
    ref = KU.solve_kutta(mesh, case.flow, pts)
    assert res.kutta_nodes == ref.kutta_nodes
    psi = res.psi.cpu().numpy()
    scale = np.abs(ref.psi).max()
    err = np.abs(psi - ref.psi).max()
    assert err <= tol_rel * scale, f"max |dpsi| {err:.2e}"
    np.testing.assert_allclose(res.psi_b, ref.psi_b, rtol=0, atol=tol_rel * scale)
    for b, n in enumerate(ref.kutta_nodes):
        if n >= 0:
            assert psi[n] == pytest.approx(res.psi_b[b], abs=tol_rel * scale)
    rows = O.assemble(mesh) @ psi
    bflat = mesh.body.ravel()
    for b, n in enumerate(ref.kutta_nodes):
        rb = rows[bflat == b].sum()
        if n < 0:
            assert abs(rb) <= 1e-8 * scale
        else:
            assert rb == pytest.approx(ref.body_rows[b], rel=1e-6)
    return res, ref


@pytest.mark.parametrize("name", list(CASES))
def test_kutta_matches_oracle(mfp, name):
    case, pts = CASES[name]
    _compare(mfp, case, pts, "fp64", 1e-9)


@pytest.mark.parametrize("name", ["cyl64", "five96x48_two"])
def test_kutta_fp32_refined(mfp, name):
    case, pts = CASES[name]
    _compare(mfp, case, pts, "fp32_ir", 1e-9)


def test_no_kutta_point_is_the_plain_solve(mfp):
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=DEV)
    a = mfp.psi_solve_kutta(case.grid, case.circles, disp, kind, body, case.flow,
                            [None] * 5, rtol=1e-12, pair=case.pair)
    b = mfp.psi_solve(case.grid, case.circles, disp, kind, body, case.flow, rtol=1e-12,
                      pair=case.pair, sample_cap=0)
    assert torch.equal(a.psi, b.psi)
    assert a.psi_b == b.psi_b and a.copfi == pytest.approx(b.copfi, rel=1e-14)


def test_kutta_full_size_1024x512(mfp):
    case = W.five_cyl_1024()
    pts = [None, None, None, (0.75, -1.25), (0.75, 1.25)]
    res, ref = _compare(mfp, case, pts, "fp64", 1e-8)
    say(f"[kutta 1024x512] iters {res.stats['iters']} ms {res.stats['solve_ms']:.1f} "
        f"psi_b {res.psi_b}")


def test_rejected_points(mfp):
    case = W.single_cylinder(32, half=4.0)
    disp, kind, body = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=DEV)
    for pt in ((0.0, 0.0), (-4.0, 1.0), (9.0, 0.0)):
        with pytest.raises(mfp.MfpError) as e:
            mfp.psi_solve_kutta(case.grid, case.circles, disp, kind, body, case.flow, [pt])
        assert e.value.status == mfp.MFP_E_ARG
