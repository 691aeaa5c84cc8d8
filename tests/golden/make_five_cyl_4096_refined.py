"""Writes five_cyl_4096x2048_refined.txt: the oracle's reduced system of the
4096x2048 five-cylinder workload (delta 0.5) solved to well below FP64 rounding of
the solution, as a cross-check of the CG reference in
five_cyl_4096x2048_reference.txt and as the more accurate of the two.

The system has 8.3M unknowns; SciPy's sparse LU cannot factor it (its 32-bit
workspace bookkeeping gives out; the 2.1M-unknown 2048x1024 system factors in
half a minute), so the solution is refined iteratively instead:

  1. the conformed mesh, the assembled K, the lifting g and the reduced system
     A = T^T K T, b = -T^T K g exactly as the oracle builds them;
  2. y_0 = 0; step k: r_k = b - A y_k evaluated in numpy.longdouble (x86 80-bit
     extended: 64-bit significand) from the FP64 entries of A and b; the
     correction e_k solves A e = r_k by the oracle's plain FP64 CG to a relative
     residual of 1e-9; y_(k+1) = y_k + e_k kept in extended precision.  Each step
     cuts the error by about 1e-9 sqrt(cond A) < 1e-5, so four steps leave the
     rounding of the extended residual, about cond(A) 1e-19 relative, far below
     FP64 rounding of y;
  3. stored: psi_b, CoPFI, every step's extended-precision residual and correction
     size, psi at the same 2000 seeded free nodes as the CG reference, and the
     largest differences to that reference.

The reduced system's entries are FP64 numbers; the refined solution is its exact
solution to far better than FP64 rounding, so what separates any FP64 solver
(the CG reference, the GPU) from it is that solver's own error.  A checkpoint
after every step lets an interrupted run resume.

Usage: python tests/golden/make_five_cyl_4096_refined.py   (about 1.5 hours on one
host core, ~8 GB of memory)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle.cg import cg  # noqa: E402

REF = os.path.join(HERE, "five_cyl_4096x2048_reference.txt")
OUT = os.path.join(HERE, "five_cyl_4096x2048_refined.txt")
STEPS = 4
INNER_RTOL = 1e-9


def read_cg_reference():
    nodes, vals, hdr = [], [], {}
    with open(REF) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                if parts and parts[0] in ("psi_b", "copfi"):
                    hdr[parts[0]] = np.array([float(v) for v in parts[1:]])
                continue
            n, v = line.split()
            nodes.append(int(n))
            vals.append(float(v))
    return np.array(nodes), np.array(vals), hdr


def main():
    case = W.five_cyl_4096()
    t0 = time.time()
    mesh = oracle.conform(case.grid, case.circles, case.nsweeps)
    K = oracle.assemble(mesh)
    g = oracle.dirichlet_values(case.grid, case.flow, case.circles)
    dmask = oracle.dirichlet_mask(case.grid, case.flow).ravel()
    g = np.where(dmask, g, 0.0)
    nb = len(case.circles)
    dof, nfree, ndof = oracle.dof_numbering(case.grid, mesh.body, case.flow, nb)
    A, b, T = oracle.reduced_system(K, dof, ndof, g)
    del K, mesh
    A = A.tocsr()
    Ald = A.astype(np.longdouble)
    bld = b.astype(np.longdouble)
    bn = float(np.linalg.norm(b))
    print(f"assembled {ndof} unknowns in {time.time() - t0:.0f} s", flush=True)
    ckpt = os.environ.get("MFP_REFINE_CHECKPOINT", "/tmp/five_cyl_4096_refine_ckpt.npz")
    y = np.zeros(ndof, dtype=np.longdouble)
    log = []  # (relative residual before the step, max |e|, max |e| at bodies, CG its)
    if os.path.exists(ckpt):
        z = np.load(ckpt)
        if z["hi"].shape == (ndof,):
            y = z["hi"].astype(np.longdouble) + z["lo"].astype(np.longdouble)
            log = [tuple(row) for row in z["log"]]
            print(f"resumed after {len(log)} steps", flush=True)
    t0 = time.time()
    while len(log) < STEPS:
        r = bld - Ald @ y
        rel = float(np.linalg.norm(r.astype(np.float64))) / bn
        e, its, _ = cg(A, r.astype(np.float64), rtol=INNER_RTOL)
        y = y + e.astype(np.longdouble)
        log.append((rel, float(np.max(np.abs(e))), float(np.max(np.abs(e[nfree:]))), its))
        hi = y.astype(np.float64)
        lo = (y - hi.astype(np.longdouble)).astype(np.float64)
        np.savez(ckpt, hi=hi, lo=lo, log=np.array(log))
        print(f"step {len(log)}: residual {rel:.3e}, correction max {log[-1][1]:.3e} "
              f"(bodies {log[-1][2]:.3e}), {its} CG iterations, {time.time() - t0:.0f} s",
              flush=True)
    rel_final = float(np.linalg.norm((bld - Ald @ y).astype(np.float64))) / bn
    y64 = y.astype(np.float64)
    psi = g + T @ y64
    psi_b = y64[nfree:]
    lo_b, hi_b = case.pair
    _, cop = oracle.copfi(psi_b, lo_b, hi_b, case.flow.U, case.circles[lo_b][1],
                          case.circles[hi_b][1])
    nodes, cg_vals, hdr = read_cg_reference()
    dpsi = np.abs(psi[nodes] - cg_vals)
    dpb = np.abs(psi_b - hdr["psi_b"])
    dcop = abs(cop - hdr["copfi"][0])
    with open(OUT, "w") as f:
        f.write("# Oracle solution of the 4096x2048 five-cylinder workload (delta 0.5, U = 1,\n")
        f.write("# 200 Jacobi sweeps): the assembled reduced system refined with residuals in\n")
        f.write("# extended precision and FP64 CG corrections.  Written by\n")
        f.write("# make_five_cyl_4096_refined.py.\n")
        f.write(f"# unknowns {ndof}\n")
        f.write("# step_relative_residual " + " ".join(f"{s[0]:.6e}" for s in log) + "\n")
        f.write("# step_correction_max " + " ".join(f"{s[1]:.6e}" for s in log) + "\n")
        f.write("# step_correction_bodies " + " ".join(f"{s[2]:.6e}" for s in log) + "\n")
        f.write("# step_cg_iterations " + " ".join(f"{int(s[3])}" for s in log) + "\n")
        f.write(f"# final_relative_residual {rel_final:.6e}\n")
        f.write("# psi_b " + " ".join(f"{v:.17e}" for v in psi_b) + "\n")
        f.write(f"# copfi {cop:.17e}\n")
        f.write(f"# cg_reference_max_abs_dpsi {dpsi.max():.6e}\n")
        f.write(f"# cg_reference_rel_l2_dpsi {np.linalg.norm(dpsi) / np.linalg.norm(cg_vals):.6e}\n")
        f.write(f"# cg_reference_max_abs_dpsi_b {dpb.max():.6e}\n")
        f.write(f"# cg_reference_abs_dcopfi {dcop:.6e}\n")
        f.write("# node psi   (node = j*(nx+1) + i, the 2000 seeded free nodes of the CG reference)\n")
        for n in nodes:
            f.write(f"{n} {psi[n]:.17e}\n")
    print("wrote", OUT, "max |dpsi| vs CG", dpsi.max(), "max |dpsi_b|", dpb.max(), flush=True)


if __name__ == "__main__":
    main()
