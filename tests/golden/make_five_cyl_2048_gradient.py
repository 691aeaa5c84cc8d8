"""Writes five_cyl_2048x1024_gradient.txt: the oracle's gradient of CoPFI for the
2048x1024 five-cylinder gradient workload (delta 0.15): dCoPFI/d(cx_b, cy_b) for
the five centres and dCoPFI/d(delta) for the symmetric motion of the transverse
pair (y_hi = D + delta, y_lo = -(D + delta)).

It calls oracle.grad.adjoint_gradient, the oracle's discrete adjoint of the
frozen-classification map (a direct sparse-LU solve of the 2.1M-unknown reduced
system, the adjoint solve A lambda = dJ/dy, the element shape derivative of
lambda^T K(X) psi by complex step per coordinate, the transposed Jacobi sweeps and
the projection Jacobian).  On small meshes that function agrees with the
complex-step derivative of the whole chain to rounding (tests/test_oracle_grad.py).

Usage: python tests/golden/make_five_cyl_2048_gradient.py   (a few minutes, ~20 GB
of host memory)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import workloads as W  # noqa: E402
from oracle.grad import adjoint_gradient  # noqa: E402

OUT = os.path.join(HERE, "five_cyl_2048x1024_gradient.txt")


def main():
    case = W.five_cyl_2048_adjoint()
    t0 = time.time()
    gc, gd, ex = adjoint_gradient(case.grid, case.circles, case.flow, case.pair, case.nsweeps)
    print(f"adjoint gradient in {time.time() - t0:.0f} s", flush=True)
    sol = ex["sol"]
    with open(OUT, "w") as f:
        f.write("# Oracle gradient of CoPFI, 2048x1024 five-cylinder workload (delta 0.15,\n")
        f.write("# U = 1, 200 Jacobi sweeps, pair (3, 4)), discrete adjoint of the\n")
        f.write("# frozen-classification map.  Written by make_five_cyl_2048_gradient.py.\n")
        f.write(f"# unknowns {sol.ndof}\n")
        f.write("# psi_b " + " ".join(f"{v:.17e}" for v in sol.psi_b) + "\n")
        f.write(f"# copfi {ex['J']:.17e}\n")
        f.write(f"# dcopfi_ddelta {gd:.17e}\n")
        f.write("# body dcopfi_dcx dcopfi_dcy\n")
        for b in range(len(case.circles)):
            f.write(f"{b} {gc[b, 0]:.17e} {gc[b, 1]:.17e}\n")
    print("wrote", OUT, gc.tolist(), gd, flush=True)


if __name__ == "__main__":
    main()
