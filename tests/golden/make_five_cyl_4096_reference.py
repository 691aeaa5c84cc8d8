"""Writes five_cyl_4096x2048_reference.txt: the oracle's solution of the 4096x2048
five-cylinder workload (delta 0.5), for the full-size GPU parity test.

The reduced system has 8.3M unknowns, too many for a direct factorisation here, so
the oracle solves it with its plain FP64 conjugate gradients on the assembled CSR
matrix (standard form, from x0 = 0, restarted from the current iterate every 3000
iterations, so that an interrupted run can resume from a checkpoint) until the true
relative residual ||b - A y|| / ||b|| is at most 1e-13.  Stored: the body values psi_b, CoPFI of the
transverse pair, the CG iteration count, the reached true residual, and psi at 2000
free nodes drawn uniformly with a fixed seed.  Calls only the oracle; takes about an
hour on one host core.

Usage: python tests/golden/make_five_cyl_4096_reference.py
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

CHUNK = 3000


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
    A = A.tocsr()
    print(f"assembled {ndof} DOF in {time.time() - t0:.0f} s", flush=True)
    # CG in runs of CHUNK iterations, each restarted from the last iterate (its state
    # is kept in a checkpoint file so that an interrupted run resumes); the stopping
    # test is the true relative residual of the reduced system
    ckpt = os.environ.get("MFP_REF_CHECKPOINT", "/tmp/five_cyl_4096_ref_ckpt.npz")
    y, k = None, 0
    if os.path.exists(ckpt):
        z = np.load(ckpt)
        if z["y"].shape == (ndof,):
            y, k = z["y"], int(z["k"])
            print(f"resumed at {k} iterations", flush=True)
    bn = float(np.linalg.norm(b))
    true_rel = 1.0 if y is None else float(np.linalg.norm(b - A @ y)) / bn
    t0 = time.time()
    while true_rel > 1e-13:
        # the run's own relative target: the remaining reduction, a little past it
        target = min(0.5, 0.5e-13 / true_rel)
        y, kk, _ = cg(A, b, rtol=target, x0=y, max_iters=CHUNK)
        k += kk
        true_rel = float(np.linalg.norm(b - A @ y)) / bn
        np.savez(ckpt, y=y, k=k)
        print(f"CG: {k} iterations, true relative residual {true_rel:.2e}, "
              f"{time.time() - t0:.0f} s", flush=True)
    assert true_rel <= 1e-13, true_rel
    psi = g + T @ y
    psi_b = y[nfree:]
    lo, hi = case.pair
    c_lo, c_hi = case.circles[lo], case.circles[hi]
    _, cop = oracle.copfi(psi_b, lo, hi, case.flow.U, c_lo[1], c_hi[1])
    free = np.flatnonzero((dof >= 0) & (dof < nfree))
    nodes = np.sort(np.random.default_rng(20251203).choice(free, size=2000, replace=False))
    out = os.path.join(HERE, "five_cyl_4096x2048_reference.txt")
    with open(out, "w") as f:
        f.write("# Oracle solution of the 4096x2048 five-cylinder workload (delta 0.5, U = 1,\n")
        f.write("# 200 Jacobi sweeps): plain FP64 CG on the assembled reduced system to a true\n")
        f.write("# relative residual <= 1e-13.  Written by make_five_cyl_4096_reference.py.\n")
        f.write(f"# cg_iterations {k}\n# true_relative_residual {true_rel:.6e}\n")
        f.write("# psi_b " + " ".join(f"{v:.17e}" for v in psi_b) + "\n")
        f.write(f"# copfi {cop:.17e}\n")
        f.write("# node psi   (node = j*(nx+1) + i, 2000 seeded free nodes)\n")
        for n in nodes:
            f.write(f"{n} {psi[n]:.17e}\n")
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
