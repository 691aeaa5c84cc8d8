"""Batched delta-sweep solves (one graph-replayed launch sequence for all systems):
each system against its own single solve and against the oracle.

Small systems of uneven, ragged sizes and different gaps (including a gap below one
cell); FP64 CG and FP32 CG with FP64 refinement.  Bars: every system's FP64 true
relative residual <= the requested tolerance (x1.5 for the FP32 recursion's final
block), psi relative L2 error vs the oracle <= 1e-9 at rtol 1e-12, body values vs
the single FP64 solve <= 1e-9 absolute.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

SMALL = [
    W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
    W.five_cylinders(130, 67, 0.4, extent=(-6.5, 6.5, -3.35, 3.35)),
    W.five_cylinders(160, 80, 0.1, extent=(-6, 6, -3, 3)),
    W.five_cylinders(200, 100, 1.0, extent=(-6, 6, -3, 3)),
    W.five_cylinders(256, 128, 0.05),
    W.five_cylinders(98, 49, 0.7, extent=(-6, 6, -3, 3)),
]


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


def meshes(mfp, cases):
    out = []
    for c in cases:
        disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
        out.append((c.grid, c.circles, disp, kind, body))
    return out


@pytest.mark.parametrize("rows", [4, 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batched_matches_single_and_oracle(mfp, precision, rows):
    say(f"[batched] {precision} {rows}-row tasks")
    systems = meshes(mfp, SMALL)
    res = mfp.psi_solve_batched(systems, SMALL[0].flow, precision=precision, rtol=1e-12,
                                pair=(3, 4), want_psi=True, iters_per_launch=32,
                                schedule={"task_rows": rows})
    assert res.status == 0, res.status
    for i, c in enumerate(SMALL):
        s = res.stats[i]
        assert s["relres_true"] <= 1.5e-12, (i, s["relres_true"])
        single = mfp.psi_solve(c.grid, c.circles, *systems[i][2:], c.flow, rtol=1e-13,
                               pair=c.pair)
        np.testing.assert_allclose(res.psi_b[i], single.psi_b, rtol=0, atol=1e-9)
        assert res.copfi[i] == pytest.approx(single.copfi, abs=1e-9)
        mesh = O.conform(c.grid, c.circles, c.nsweeps)
        ref = O.solve(mesh, c.flow)
        psi = res.psi[i].cpu().numpy()
        err = np.linalg.norm(psi - ref.psi) / np.linalg.norm(ref.psi)
        dmax = np.abs(psi - ref.psi).max() / np.abs(ref.psi).max()
        say(f"  system {i} {c.name}: iters {s['iters']} outer {s['outer_iters']} "
            f"relres {s['relres_true']:.2e} err {err:.2e} node max {dmax:.2e}")
        assert err <= 1e-9 and dmax <= 1e-9, (i, err, dmax)


def test_batched_sweep_sample_full_sizes(mfp):
    """Eight systems of the seeded delta-sweep (256x128 .. 1024x512), FP32 CG with FP64
    refinement to 1e-10 against single FP64 solves to 1e-12."""
    cases = W.batch_variants(count=8, seed=0)
    systems = meshes(mfp, cases)
    res = mfp.psi_solve_batched(systems, cases[0].flow, precision="fp32_ir", rtol=1e-10,
                                pair=(3, 4))
    assert res.status == 0
    for i, c in enumerate(cases):
        s = res.stats[i]
        assert s["relres_true"] <= 1.5e-10, (i, s["relres_true"])
        single = mfp.psi_solve(c.grid, c.circles, *systems[i][2:], c.flow, rtol=1e-12,
                               pair=c.pair)
        d = np.abs(np.array(res.psi_b[i]) - np.array(single.psi_b)).max()
        say(f"  system {i} {c.name}: iters {s['iters']} relres {s['relres_true']:.2e} "
            f"|dpsi_b| {d:.2e} copfi {res.copfi[i]:.9f} vs {single.copfi:.9f}")
        assert d <= 1e-6


def test_batched_full_sweep_every_system_converges(mfp):
    """The whole seeded delta-sweep (256 systems, 256x128 .. 1024x512) in one batch.
    FP64: every system's FP64 true relative residual <= 2x the tolerance (a system's
    blocks must agree on the launch that stops it; a block that ran on past it would
    corrupt its tasks' iterate).  FP32 with FP64 refinement: every system converges in
    at most 1.6x its FP64 iteration count plus one refinement block (a restart that lost
    the last direction's conjugacy would take several times more)."""
    cases = W.batch_variants(count=256, seed=0)
    systems = meshes(mfp, cases)
    r64 = mfp.psi_solve_batched(systems, cases[0].flow, precision="fp64", rtol=1e-10,
                                pair=(3, 4))
    assert r64.status == 0
    worst = max(s["relres_true"] for s in r64.stats)
    say(f"  fp64: worst relres {worst:.2e}")
    assert worst <= 2e-10, [(i, s["relres_true"]) for i, s in enumerate(r64.stats)
                            if s["relres_true"] > 2e-10]
    r32 = mfp.psi_solve_batched(systems, cases[0].flow, precision="fp32_ir", rtol=1e-10,
                                pair=(3, 4))
    assert r32.status == 0
    for i, (a, b) in enumerate(zip(r32.stats, r64.stats)):
        assert a["relres_true"] <= 1.5e-10, (i, a["relres_true"])
        assert a["iters"] <= 1.6 * b["iters"] + 64, (i, a["iters"], b["iters"])
    np.testing.assert_allclose(r32.copfi, r64.copfi, rtol=0, atol=1e-7)


def test_batched_schedule_rejects_other_task_rows(mfp):
    """The batched layouts take 4- or 5-row tasks; 8 is an argument error before any
    launch."""
    systems = meshes(mfp, SMALL[:2])
    with pytest.raises(mfp.MfpError) as e:
        mfp.psi_solve_batched(systems, SMALL[0].flow, precision="fp64", rtol=1e-10,
                              pair=(3, 4), schedule={"task_rows": 8},
                              ws=torch.empty(1 << 20, dtype=torch.uint8, device=DEV))
    assert e.value.status == mfp.MFP_E_ARG
