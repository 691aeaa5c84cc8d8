"""The allocation-free element apply (mfp_element_apply_noalloc) against the
workspace entry point mfp_element_apply on the same inputs: bit-for-bit the same
product (same kernels, same work list), and within the apply's bar of the oracle's
assembled K p.  Two calls in a row, the second on a smaller grid (the static scratch
keeps the first call's contents), in FP64 and FP32; a grid beyond the scratch is
rejected before any device work."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

BIG = W.five_cyl_1024()
SMALL = W.five_cylinders(130, 67, 0.4, extent=(-6.5, 6.5, -3.35, 3.35))


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_apply_matches_workspace_apply(mfp, precision):
    for c, seed in ((BIG, 11), (SMALL, 12)):
        say(f"[noalloc] {c.name} {precision}")
        disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
        p = torch.from_numpy(W.random_vector(c.grid.nodes, seed)).to(DEV)
        ref, _ = mfp.element_apply(c.grid, disp, body, p, precision)
        got = mfp.element_apply_noalloc(c.grid, disp, body, p, precision)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        mesh = O.conform(c.grid, c.circles, c.nsweeps)
        qref = O.assemble(mesh) @ p.cpu().numpy()
        tol = 1e-13 if precision == "fp64" else 2e-5
        err = np.abs(got.double().cpu().numpy() - qref).max() / np.abs(qref).max()
        assert err <= tol, err


def test_noalloc_apply_rejects_a_grid_beyond_its_scratch(mfp):
    c = W.five_cylinders(1400, 700, 0.25)
    g = c.grid
    n = g.nodes
    disp = torch.zeros(2 * n, dtype=torch.float64, device=DEV)
    body = torch.full((n,), -1, dtype=torch.int8, device=DEV)
    p = torch.zeros(n, dtype=torch.float64, device=DEV)
    with pytest.raises(mfp.MfpError) as e:
        mfp.element_apply_noalloc(g, disp, body, p)
    assert e.value.status == mfp.MFP_E_WORKSPACE
