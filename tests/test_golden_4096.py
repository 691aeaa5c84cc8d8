"""The two stored oracle solutions of the 4096x2048 workload agree with each other (no
GPU): the refined one (extended-precision residuals, relative residual 2.4e-18) and
the plain CG one (true relative residual 3.8e-14) hold the same 2000 seeded nodes,
their recorded differences are the ones recomputed here, and those differences are
of the size that CG's residual allows at this conditioning (1e-11 of the field).  The
layout is mirror-symmetric, so the refined solution's body values are odd in y."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    meta, nodes, vals = {}, [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                if len(parts) >= 2:
                    try:
                        meta[parts[0]] = [float(v) for v in parts[1:]]
                    except ValueError:
                        pass
                continue
            n, v = line.split()
            nodes.append(int(n))
            vals.append(float(v))
    return meta, np.array(nodes), np.array(vals)


def test_refined_and_cg_references_agree():
    rm, rn, rv = read("five_cyl_4096x2048_refined.txt")
    cm, cn, cv = read("five_cyl_4096x2048_reference.txt")
    assert np.array_equal(rn, cn)
    assert rm["final_relative_residual"][0] <= 1e-16
    assert cm["true_relative_residual"][0] <= 1e-13
    dpsi = np.abs(rv - cv).max()
    dpb = np.abs(np.array(rm["psi_b"]) - np.array(cm["psi_b"])).max()
    dcop = abs(rm["copfi"][0] - cm["copfi"][0])
    assert dpsi == pytest.approx(rm["cg_reference_max_abs_dpsi"][0], rel=1e-5)
    assert dpb == pytest.approx(rm["cg_reference_max_abs_dpsi_b"][0], rel=1e-5)
    assert dcop == pytest.approx(rm["cg_reference_abs_dcopfi"][0], rel=1e-5)
    scale = np.abs(rv).max()
    assert dpsi <= 1e-10 * scale and dpb <= 1e-10 and dcop <= 1e-10


def test_refined_reference_is_odd_in_y():
    rm, _, _ = read("five_cyl_4096x2048_refined.txt")
    pb = np.array(rm["psi_b"])
    assert np.abs(pb[:3]).max() <= 1e-10
    assert abs(pb[3] + pb[4]) <= 1e-10
