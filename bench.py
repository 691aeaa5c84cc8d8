#!/usr/bin/env python3
"""Benchmark of the matrix-free multi-body stream-function path on one MI355X.

One step = the whole hot path on one synthetic input: body-conforming mesh
(classification, radial projection, 200 Jacobi sweeps), the multi-point
constrained conjugate-gradient solve for psi in FP64 to relative residual 1e-12,
the recomputed FP64 true residual, nodal psi, body psi_b, Q_54, CoPFI and the
surface-velocity samples.  Workload: five cylinders of diameter 1 at (-3,0),
(0,0), (3,0), (0,+-1.25) (gap 0.25 D), 1024 x 512 cells on [-20,20] x [-10,10],
U = 1, psi = U y on inlet/bottom/top, natural outlet.

Prints ONE JSON line.  value = sum over timed steps of N_dof x CG iterations,
divided by the wall time of those steps (inputs resident on the GPU).  The
roofline entry is for the dominant kernel, the fused direction-update + element
apply, timed with HIP events inside the timed steps on the solver's stream.
The CPU baseline is the oracle's plain CG on its assembled sparse matrix, timed
on a bounded number of iterations on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CG DOF·iter/s + matvec HBM GB/s (% peak); adjoint/forward time; err vs FP64"
HBM_PEAK_GBS = 8000.0


def apply_bytes(case, disp, body):
    """Algorithmic bytes of one fused apply launch: every node reads r and the old
    direction and writes the new direction and K p (4 x 8 B); every node with a
    non-zero displacement also reads it (2 x 8 B); every node that is not a free
    fluid node is identified by its one-byte tag."""
    import torch
    n = case.grid.nodes
    d = disp.view(2, n)
    moved = int(((d[0] != 0) | (d[1] != 0)).sum().item())
    nx, ny = case.grid.nx, case.grid.ny
    boundary = 2 * (nx + 1) + 2 * (ny - 1)
    bodies = int((body >= 0).sum().item())
    return 32 * n + 16 * moved + (boundary + bodies), moved


def cpu_baseline(case, iters):
    """The oracle's plain CG on the assembled reduced system, `iters` iterations,
    one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle.cg import cg
    mesh = oracle.conform(case.grid, case.circles, case.nsweeps)
    K = oracle.assemble(mesh)
    g = oracle.dirichlet_values(case.grid, case.flow, case.circles)
    dof, nfree, ndof = oracle.dof_numbering(case.grid, mesh.body, case.flow, len(case.circles))
    A, b, _ = oracle.reduced_system(K, dof, ndof, np.where(
        oracle.dirichlet_mask(case.grid, case.flow).ravel(), g, 0.0))
    A = A.tocsr()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, k, _ = cg(A, b, rtol=1e-300, max_iters=iters)
        dt = time.perf_counter() - t0
    return {"value": ndof * k / dt, "unit": "DOF·iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} iterations of the oracle's plain FP64 CG on the assembled "
                      f"reduced CSR system of the same workload ({ndof} DOF, scipy.sparse "
                      f"SpMV, 1 thread); assembly not timed; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-iters", type=int, default=1500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="time every n-th apply launch with HIP events (0: off)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    import paper_2512_12232_amd as mfp

    mfp.load()
    if args.calibrate_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes": a.numel() * 8}), flush=True)
        return
    case = W.five_cyl_1024()
    dev = "cuda:0"
    torch.cuda.set_device(0)

    def step(profile):
        disp, kind, body = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=dev)
        res = mfp.psi_solve(case.grid, case.circles, disp, kind, body, case.flow, rtol=1e-12,
                            pair=case.pair, profile_every=profile)
        return disp, body, res

    for _ in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step(args.profile_every) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    disp, body, res = outs[-1]
    dof_iters = sum(r.stats["n_dof"] * r.stats["iters"] for _, _, r in outs)
    value = dof_iters / wall
    apply_ms = [r.stats["apply_ms"] for _, _, r in outs if r.stats["apply_samples"] > 0]
    nbytes, moved = apply_bytes(case, disp, body)
    roofline = None
    if apply_ms:
        ms = sum(apply_ms) / len(apply_ms)
        achieved = nbytes / (ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None, "kernel": "k_apply<double, fused>",
                    "launch_ms": round(ms, 5), "bytes_per_launch": nbytes,
                    "samples": int(sum(r.stats["apply_samples"] for _, _, r in outs))}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, args.cpu_iters)
    s = res.stats
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF·iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "five cylinders D=1 at (-3,0),(0,0),(3,0),(0,+-1.25); "
                               "1024x512 Q1 cells on [-20,20]x[-10,10]; 200 Jacobi sweeps; "
                               "U=1; FP64 CG to relative residual 1e-12",
                   "nx": 1024, "ny": 512, "delta": 0.25, "rtol": 1e-12, "precision": "fp64",
                   "n_dof": s["n_dof"], "nodes": case.grid.nodes, "moved_nodes": moved},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "iters": s["iters"],
        "solve_ms": s["solve_ms"],
        "relres_true": s["relres_true"],
        "plain_tile_frac": s["n_plain_tiles"] / max(1, s["n_tiles"]),
        "psi_b": res.psi_b,
        "copfi": res.copfi,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
