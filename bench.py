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
roofline entry is for the dominant kernel, the one-kernel CG iteration (element
apply fused with the vector updates and dot products), timed with HIP events
inside the timed steps on the solver's stream.
The CPU baseline is the oracle's plain CG on its assembled sparse matrix, timed
on a bounded number of iterations on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CG DOF·iter/s + matvec HBM GB/s (% peak); adjoint/forward time; err vs FP64"
HBM_PEAK_GBS = 8000.0


def step_bytes(case, disp, body, esz=8):
    """Algorithmic bytes of one launch of the one-kernel CG iteration, averaged over the
    two launch parities: every node reads the previous residual, direction and K p
    (3 x 8 B) and writes the new ones (3 x 8 B); odd launches also read the iterate and
    the direction before last and write the iterate (3 x 8 B), i.e. 12 B per launch on
    average; every node with a non-zero displacement also reads it (2 x 8 B); every
    node that is not a free fluid node is identified by its one-byte tag.  esz = 4:
    the FP32 iteration (4-byte vectors and displacements)."""
    n = case.grid.nodes
    d = disp.view(2, n)
    moved = int(((d[0] != 0) | (d[1] != 0)).sum().item())
    nx, ny = case.grid.nx, case.grid.ny
    boundary = 2 * (nx + 1) + 2 * (ny - 1)
    bodies = int((body >= 0).sum().item())
    return (15 * esz * n) // 2 + 2 * esz * moved + (boundary + bodies), moved


COUNTERS = os.path.join(ROOT, "profiles", "k_step_fp64_five_cyl_1024x512_counters.md")


def traffic_from_profile():
    """HBM bytes per launch of the CG iteration kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by the copy-kernel calibration), or None
    when the kernel or solver source has changed since those counters were taken."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line
                  and line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "source_sha256_16"))
    h = hashlib.sha256()
    for f in ("apply.h", "step.h", "solve.hip", "reduce.h"):
        with open(os.path.join(ROOT, "paper_2512_12232_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def host_info():
    """CPU model and the cores this process may use on the benchmark host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(case, seconds):
    """The oracle's plain CG on the assembled reduced system, one thread, run for a
    bounded number of iterations chosen from a short calibration run so that the
    timed part takes about `seconds`; and the oracle's time to solution by sparse LU
    (assembly, factorisation and solve: oracle.solve), whose solution is returned for
    the error figures."""
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
        cg(A, b, rtol=1e-300, max_iters=50)
        per_iter = (time.perf_counter() - t0) / 50
        iters = max(100, int(seconds / per_iter))
        t0 = time.perf_counter()
        _, k, _ = cg(A, b, rtol=1e-300, max_iters=iters)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        sol = oracle.solve(mesh, case.flow)
        t_lu = time.perf_counter() - t0
    return {"value": ndof * k / dt, "unit": "DOF·iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} iterations of the oracle's plain FP64 CG on the assembled "
                      f"reduced CSR system of the same workload ({ndof} DOF, scipy.sparse "
                      f"SpMV, 1 thread); assembly not timed; {dt:.1f} s",
            "splu_time_to_solution_s": round(t_lu, 2),
            "splu_note": "oracle.solve: assembly, SuperLU factorisation and solve, 1 thread",
            "host": host_info()}, mesh, sol


def errors_vs_oracle(case, res, mesh, sol, kappa):
    """The GPU result of the benchmark workload against the oracle's direct solve:
    psi (relative L2 over all nodes, and the largest nodal difference relative to
    max|psi|), psi_b, Q, CoPFI and u_t (relative to max|u_t|), each stated beside the
    condition number (the GPU's Lanczos estimate from this solve's CG scalars and the
    oracle's extreme eigenvalues of the reduced operator)."""
    import numpy as np

    import oracle
    from oracle.spectrum import condition_number
    psi = res.psi.cpu().numpy()
    lo, hi = case.pair
    Q, J = oracle.copfi(sol.psi_b, lo, hi, case.flow.U, case.circles[lo][1], case.circles[hi][1])
    th, ut, _ = oracle.surface_samples(mesh, sol.psi, sol.psi_b)
    t0 = time.perf_counter()
    lmin, lmax, kap = condition_number(sol.A)
    return {"psi_rel_l2": float(np.linalg.norm(psi - sol.psi) / np.linalg.norm(sol.psi)),
            "psi_node_max_rel": float(np.abs(psi - sol.psi).max() / np.abs(sol.psi).max()),
            "psi_b_max_abs": float(np.abs(np.array(res.psi_b) - sol.psi_b).max()),
            "Q_abs": abs(res.Q - Q), "copfi_abs": abs(res.copfi - J),
            "u_t_max_rel": float(np.abs(res.ut.cpu().numpy() - ut).max() / np.abs(ut).max()),
            "kappa_gpu_lanczos": kappa,
            "kappa_oracle": {"lambda_min": lmin, "lambda_max": lmax, "kappa": kap,
                             "seconds": round(time.perf_counter() - t0, 1),
                             "note": "ARPACK on the assembled reduced matrix (largest "
                                     "eigenvalue, and shift-invert about 0 for the "
                                     "smallest)"},
            "note": "the Lanczos estimate sees the eigenvectors the odd (mirror-symmetric) "
                    "right-hand side reaches; the oracle's kappa is the whole operator's"}


def potential_vs_oracle(case_phi, phi, mesh):
    """The GPU potential against the oracle's direct solve of the same problem."""
    import numpy as np

    import oracle
    ref = oracle.phi_solve(mesh, case_phi.flow)
    p = phi.cpu().numpy()
    dom = ~np.isnan(ref.phi)
    return {"phi_rel_l2": float(np.linalg.norm(p[dom] - ref.phi[dom]) / np.linalg.norm(ref.phi[dom])),
            "phi_node_max_rel": float(np.abs(p[dom] - ref.phi[dom]).max()
                                      / np.abs(ref.phi[dom]).max()),
            "nan_pattern_equal": bool(np.array_equal(np.isnan(p), ~dom))}


def _sync():
    import torch
    torch.cuda.synchronize()


def _timed(fn, reps=1):
    """Wall time of fn() (ms, best of reps) after one untimed call."""
    out = fn()
    _sync()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        _sync()
        best = min(best, time.perf_counter() - t0)
    return out, 1e3 * best


def _kernel_label(case, stats, prec="fp64"):
    """The iteration kernel of a solve: element type, task rows, element mode and launch
    shape."""
    label = "k_step<%s, %d>" % ("double" if prec == "fp64" else "float",
                                _task_height(case, stats["n_tiles"]))
    notes = []
    if stats.get("step_element_mode") == 2:
        notes.append("stored entries")
    if stats.get("step_block_waves") == 8:
        notes.append("8-wavefront blocks, task table")
    return label + (" (%s)" % ", ".join(notes) if notes else "")


def _launch_bytes(case, disp, body, stats, esz=8):
    """Algorithmic bytes per iteration launch for the solve's element mode."""
    if stats.get("step_element_mode") == 2:
        return stored_step_bytes(case, body, stats["n_tiles"], stats["n_plain_tiles"],
                                 _task_height(case, stats["n_tiles"]), esz)
    return step_bytes(case, disp, body, esz)[0]


def _task_height(case, n_tiles):
    """Node rows per task of a solve's layout, from its task count (strips of 62 node
    columns x chunks of hc node rows)."""
    strips = -(-(case.grid.nx + 1) // 62)
    for hc in (4, 5, 8):
        if strips * -(-(case.grid.ny + 1) // hc) == n_tiles:
            return hc
    return 0


def mixed_precision(mfp, W, kmax=10 ** 7):
    """4096 x 2048 cells (delta 0.5): FP32 apply with FP64 refinement against plain
    FP64 CG, both to relative residual 1e-10, and plain FP32 CG to 1e-6.  A small kmax
    cuts every solve short (profiling runs: per-launch figures only)."""
    case = W.five_cyl_4096()
    disp, kind, body = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device="cuda:0")
    out = {"workload": "five cylinders, 4096x2048 cells, delta 0.5, rtol 1e-10"}
    res = {}
    for prec, rtol in (("fp64", 1e-10), ("fp32_ir", 1e-10), ("fp32", 1e-6)):
        r, ms = _timed(lambda: mfp.psi_solve(case.grid, case.circles, disp, kind, body,
                                             case.flow, precision=prec, rtol=rtol, kmax=kmax,
                                             pair=case.pair, sample_cap=0, profile_every=1))
        res[prec] = r
        out[prec] = {"solve_ms": round(ms, 2), "iters": r.stats["iters"],
                     "relres_true": r.stats["relres_true"], "rtol": rtol,
                     "dof_iter_per_s": r.stats["n_dof"] * r.stats["iters"] / (ms * 1e-3)}
        if r.stats["apply_samples"] > 0:
            nbytes = _launch_bytes(case, disp, body, r.stats, 8 if prec == "fp64" else 4)
            kms = r.stats["apply_ms"]
            out[prec]["roofline"] = {
                "kernel": _kernel_label(case, r.stats, prec),
                "launch_ms": round(kms, 5), "bytes_per_launch": nbytes,
                "achieved_GBs": round(nbytes / (kms * 1e-3) / 1e9, 1),
                "frac": round(nbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # condition estimate of this operator from an FP64 solve's CG scalars (untimed)
    rk = mfp.psi_solve(case.grid, case.circles, disp, kind, body, case.flow, rtol=1e-10,
                       kmax=kmax, pair=case.pair, sample_cap=0, estimate_kappa=True)
    out["kappa_gpu_lanczos"] = {"kappa": rk.stats["kappa_est"], "ritz_min": rk.stats["ritz_min"],
                                "ritz_max": rk.stats["ritz_max"], "steps": rk.stats["kappa_steps"]}
    ref = res["fp64"].psi
    for prec in ("fp32_ir", "fp32"):
        d = res[prec].psi - ref
        out[prec]["psi_rel_l2_vs_fp64"] = float(d.norm() / ref.norm())
        out[prec]["max_abs_dpsi_b"] = max(abs(a - b) for a, b in
                                          zip(res[prec].psi_b, res["fp64"].psi_b))
        out[prec]["abs_dcopfi"] = abs(res[prec].copfi - res["fp64"].copfi)
    out["fp32_ir_speedup_vs_fp64"] = out["fp64"]["solve_ms"] / out["fp32_ir"]["solve_ms"]
    ref_o = _oracle_reference_4096()
    if ref_o is not None and kmax >= 10 ** 6:
        # the same two forms at the accuracy the refined-FP32 target states (psi within
        # 1e-10 of the oracle, relative L2): the tolerances that reach it
        acc = {}
        nodes, vals, _, _ = ref_o
        for prec, rtol in (("fp64", 1e-12), ("fp32_ir", 3e-13)):
            r, ms = _timed(lambda: mfp.psi_solve(case.grid, case.circles, disp, kind, body,
                                                 case.flow, precision=prec, rtol=rtol,
                                                 pair=case.pair, sample_cap=0))
            p = r.psi.cpu().numpy()[nodes]
            acc[prec] = {"rtol": rtol, "solve_ms": round(ms, 2), "iters": r.stats["iters"],
                         "psi_rel_l2_vs_oracle": float(((p - vals) ** 2).sum() ** 0.5
                                                       / (vals ** 2).sum() ** 0.5)}
        acc["fp32_ir_speedup_vs_fp64"] = acc["fp64"]["solve_ms"] / acc["fp32_ir"]["solve_ms"]
        out["at_1e-10_vs_oracle"] = acc
    if ref_o is not None:
        nodes, vals, psi_b, copfi = ref_o
        for prec in ("fp64", "fp32_ir", "fp32"):
            p = res[prec].psi.cpu().numpy()[nodes]
            out[prec]["vs_oracle"] = {
                "psi_rel_l2_at_2000_nodes": float(((p - vals) ** 2).sum() ** 0.5
                                                  / (vals ** 2).sum() ** 0.5),
                "max_abs_dpsi_b": max(abs(a - b) for a, b in zip(res[prec].psi_b, psi_b)),
                "abs_dcopfi": abs(res[prec].copfi - copfi)}
    return out


def _oracle_reference_4096():
    """The stored oracle solution of the 4096x2048 workload (tests/golden): the refined
    one (residuals in extended precision, FP64 CG corrections) when present, else the
    plain CG one (true relative residual <= 1e-13); None if neither exists."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "five_cyl_4096x2048_refined.txt")
    if not os.path.exists(path):
        path = os.path.join(ROOT, "tests", "golden", "five_cyl_4096x2048_reference.txt")
    if not os.path.exists(path):
        return None
    psi_b, copfi, rows = None, None, []
    with open(path) as f:
        for line in f:
            if line.startswith("# psi_b"):
                psi_b = [float(v) for v in line.split()[2:]]
            elif line.startswith("# copfi"):
                copfi = float(line.split()[2])
            elif not line.startswith("#"):
                n, v = line.split()
                rows.append((int(n), float(v)))
    nodes = np.array([r[0] for r in rows])
    vals = np.array([r[1] for r in rows])
    return nodes, vals, psi_b, copfi


def adjoint_ratio(mfp, W):
    """2048 x 1024 cells (delta 0.15): forward (mesh + FP64 solve to 1e-12 + outputs)
    against backward (adjoint solve, shape derivative, transposed smoother,
    projection) for dCoPFI/d(centres, delta)."""
    case = W.five_cyl_2048_adjoint()
    dev = "cuda:0"

    def fwd():
        d, k, b = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=dev)
        r = mfp.psi_solve(case.grid, case.circles, d, k, b, case.flow, rtol=1e-12,
                          pair=case.pair, sample_cap=0)
        return d, k, b, r

    (d, k, b, r), fwd_ms = _timed(fwd, reps=2)

    def bwd():
        g, expl, st, _, _ = mfp.psi_grad(case.grid, case.circles, d, k, b, case.flow, r.psi,
                                      r.psi_b, dL_dcopfi=1.0, pair=case.pair, rtol=1e-12)
        dc, _ = mfp.mesh_conform_grad(case.grid, case.circles, k, b, g, case.nsweeps,
                                      dL_dcentre=expl)
        return dc, st

    (dc, st), bwd_ms = _timed(bwd, reps=2)
    out = {"workload": "five cylinders, 2048x1024 cells, delta 0.15, rtol 1e-12",
           "forward_ms": round(fwd_ms, 2), "backward_ms": round(bwd_ms, 2),
           "ratio": bwd_ms / fwd_ms, "forward_iters": r.stats["iters"],
           "adjoint_iters": st["iters"], "copfi": r.copfi,
           "dcopfi_ddelta": dc[4][1] - dc[3][1]}
    gold = _gradient_golden()
    if gold is not None:
        hdr, gref = gold
        g = [[float(v) for v in row] for row in dc]
        scale = max(abs(v) for row in gref for v in row)
        err = max(abs(g[b][k] - gref[b][k]) for b in range(5) for k in range(2))
        out["vs_oracle_gradient"] = {
            "max_abs_err_centres": err, "abs_err_ddelta": abs(out["dcopfi_ddelta"] -
                                                               hdr["dcopfi_ddelta"]),
            "max_abs_grad": scale, "rel_to_max_grad": err / scale,
            "source": "tests/golden/five_cyl_2048x1024_gradient.txt (oracle discrete "
                      "adjoint, sparse LU)"}
    return out


def _gradient_golden():
    """The oracle's gradient of the 2048x1024 workload (tests/golden), or None."""
    path = os.path.join(ROOT, "tests", "golden", "five_cyl_2048x1024_gradient.txt")
    if not os.path.exists(path):
        return None
    hdr, rows = {}, []
    for line in open(path):
        if line.startswith("#"):
            parts = line[1:].split()
            if parts and parts[0] in ("copfi", "dcopfi_ddelta"):
                hdr[parts[0]] = float(parts[1])
            continue
        _, gx, gy = line.split()
        rows.append((float(gx), float(gy)))
    return hdr, rows


def autotune_effect(mfp, W):
    """Tuned schedule (the package's tuning cache) against the built-in rules
    (MFP_TUNE_CACHE=none) on the workloads the cache was tuned on (the tuner's: five
    cylinders, gap 0.25, on [-20, 20] x [-10, 10]): 1024x512 (the benchmark's) and
    2048x1024 to rtol 1e-12, 4096x2048 to 1e-10, each in FP64 and FP32 + refinement,
    and the 256-variant batched sweep in FP32 + refinement.  Iteration-phase times
    (ms, best of two)."""
    import numpy as np
    out = {}

    def both(fn):
        old = os.environ.get("MFP_TUNE_CACHE")
        res = {}
        for label, val in (("builtin", "none"), ("tuned", None)):
            if val is None:
                os.environ.pop("MFP_TUNE_CACHE", None)
            else:
                os.environ["MFP_TUNE_CACHE"] = val
            res[label] = min(fn() for _ in range(2))
        if old is None:
            os.environ.pop("MFP_TUNE_CACHE", None)
        else:
            os.environ["MFP_TUNE_CACHE"] = old
        res["speedup"] = res["builtin"] / res["tuned"]
        return res

    for case, prec, rtol, key in ((W.five_cyl_1024(), "fp64", 1e-12, "1024x512_fp64"),
                                  (W.five_cyl_1024(), "fp32_ir", 1e-12, "1024x512_fp32_ir"),
                                  (W.five_cylinders(2048, 1024, 0.25), "fp64", 1e-12,
                                   "2048x1024_fp64"),
                                  (W.five_cylinders(2048, 1024, 0.25), "fp32_ir", 1e-12,
                                   "2048x1024_fp32_ir"),
                                  (W.five_cylinders(4096, 2048, 0.25), "fp64", 1e-10,
                                   "4096x2048_fp64"),
                                  (W.five_cylinders(4096, 2048, 0.25), "fp32_ir", 1e-10,
                                   "4096x2048_fp32_ir")):
        d, k, b = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device="cuda:0")
        out[key] = both(lambda: mfp.psi_solve(case.grid, case.circles, d, k, b, case.flow,
                                              rtol=rtol, precision=prec, pair=case.pair,
                                              sample_cap=0).stats["solve_ms"])
    cases = W.batch_variants(256, seed=0)
    systems = []
    for c in cases:
        d, k, b = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device="cuda:0")
        systems.append((c.grid, c.circles, d, k, b))
    out["sweep256_fp32_ir"] = both(lambda: mfp.psi_solve_batched(
        systems, cases[0].flow, precision="fp32_ir", rtol=1e-10,
        pair=cases[0].pair).stats[0]["solve_ms"])
    for v in out.values():
        for kk in ("builtin", "tuned"):
            v[kk] = round(float(np.float64(v[kk])), 3)
    return out


def potential_solve(mfp, W):
    """The velocity potential of the benchmark workload (1024 x 512 cells, five
    cylinders): phi = U x on inlet and outlet, natural walls and bodies, FP64 CG to
    1e-12 on the same mesh, with the iteration kernel's roofline (the stream
    function's byte model for the element mode the solve used: the same vectors,
    tags, and displacements or stored entries)."""
    case = W.potential_flow(W.five_cyl_1024())
    dev = "cuda:0"
    d, k, b = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=dev)
    r, ms = _timed(lambda: mfp.phi_solve(case.grid, case.circles, d, k, b, case.flow,
                                         rtol=1e-12, profile_every=1), reps=2)
    potential_solve.last = (case, r.phi)
    s = r.stats
    nbytes = _launch_bytes(case, d, b, s)
    out = {"workload": "five cylinders, 1024x512 cells, delta 0.25; phi = U x on inlet and "
                       "outlet, natural walls and bodies; FP64 CG to 1e-12",
           "solve_ms": round(ms, 2), "iters": s["iters"], "n_dof": s["n_dof"],
           "relres_true": s["relres_true"],
           "dof_iter_per_s": s["n_dof"] * s["iters"] / (ms * 1e-3)}
    if s["apply_samples"] > 0:
        kms = s["apply_ms"]
        out["roofline"] = {"kernel": _kernel_label(case, s),
                           "launch_ms": round(kms, 5), "bytes_per_launch": nbytes,
                           "achieved_GBs": round(nbytes / (kms * 1e-3) / 1e9, 1),
                           "frac": round(nbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def delta_sweep(mfp, W, count=256):
    """256 seeded five-cylinder variants (delta ~ U[0.05, 2], 256x128 .. 1024x512
    cells): one batched graph-replayed solve (FP32 apply + FP64 refinement, and plain
    FP64) against the same systems solved one after another with the single-system
    FP64 solver, all to relative residual 1e-10."""
    cases = W.batch_variants(count, seed=0)
    systems = []
    for c in cases:
        d, k, b = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device="cuda:0")
        systems.append((c.grid, c.circles, d, k, b))
    _sync()
    flow, pair = cases[0].flow, cases[0].pair
    out = {"workload": f"{count} five-cylinder variants, delta ~ U[0.05,2], "
                       "256x128..1024x512 cells, rtol 1e-10",
           "nodes": sum(c.grid.nodes for c in cases)}
    res = {}
    # algorithmic bytes of one iteration launch of each system (geometry on the fly,
    # the batched layouts' element mode), FP64 and FP32 vectors
    per_launch = {esz: [step_bytes(c, d, b, esz)[0] for c, (_, _, d, _, b) in zip(cases, systems)]
                  for esz in (8, 4)}
    for prec in ("fp32_ir", "fp64"):
        ws = mfp.binding.workspace(mfp.binding.batched_workspace_size(systems, prec), "cuda:0")
        r, ms = _timed(lambda: mfp.psi_solve_batched(systems, flow, precision=prec,
                                                     rtol=1e-10, pair=pair, ws=ws))
        del ws
        res[prec] = r
        its = [s["iters"] for s in r.stats]
        # every system's iteration launches (FP32 ones for FP32 + refinement); their
        # bytes over the whole batched solve's wall time (set-up, refinement residuals
        # and the other kernels included) bound the iteration kernel's rate from below
        nbytes = sum(k * v for k, v in zip(its, per_launch[4 if prec == "fp32_ir" else 8]))
        out["batched_" + prec] = {
            "ms": round(ms, 1), "iters_mean": sum(its) / len(its), "iters_max": max(its),
            "max_relres_true": max(s["relres_true"] for s in r.stats),
            "dof_iter_per_s": sum(s["n_dof"] * s["iters"] for s in r.stats) / (ms * 1e-3),
            "iteration_bytes": nbytes,
            "achieved_GBs_wall": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_wall": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    def seq():
        return [mfp.psi_solve(g, c, d, k, b, flow, rtol=1e-10, pair=pair, sample_cap=0)
                for g, c, d, k, b in systems]

    rs, ms = _timed(seq)
    out["sequential_fp64"] = {"ms": round(ms, 1), "dof_iter_per_s": sum(
        r.stats["n_dof"] * r.stats["iters"] for r in rs) / (ms * 1e-3)}
    for prec in ("fp32_ir", "fp64"):
        b = out["batched_" + prec]
        b["speedup_vs_sequential_fp64"] = out["sequential_fp64"]["ms"] / b["ms"]
        b["max_abs_dcopfi_vs_sequential_fp64"] = max(
            abs(x - r.copfi) for x, r in zip(res[prec].copfi, rs))
    # the paper's post-processing of a gap-ratio study: cubic fit of CoPFI(delta)
    coef, r2, mse = mfp.cubic_fit([c.delta for c in cases], list(res["fp32_ir"].copfi))
    out["copfi_cubic_fit"] = {"coef_d3_d2_d1_d0": [round(v, 6) for v in coef], "r2": r2,
                              "mse": mse}
    return out


def mixed_apply_bytes(gm):
    """Algorithmic bytes of one mixed-node product (k_mx_apply): every mixed node reads
    its input value and writes its output (2 x 8 B); every plain quadrilateral cell's
    six coefficients (48 B) and every cell's kind (1 B) are read once; every element
    of a cut cell is read whole (16 x 8 B matrix, 4 x 4 B node ids, 1 B size) with its
    cell's first-element pair (8 B per cut cell); every cut point reads its edge
    (4 B)."""
    import torch
    nc = gm.grid.nx * gm.grid.ny
    first = gm.cell_first.to(torch.int64)
    cnt = first[1:] - first[:-1]
    nn = (gm.grid.nx + 1) * (gm.grid.ny + 1)
    quad_like = (cnt == 1) & (gm.nne[first[:-1].clamp(max=max(gm.n_elems - 1, 0))] == 4)
    ids = gm.elem[first[:-1].clamp(max=max(gm.n_elems - 1, 0))].to(torch.int64)
    plain = quad_like & (ids < nn).all(dim=1)
    n_plain = int(plain.sum().item())
    cut_cells = (cnt > 0) & ~plain
    n_cut_cells = int(cut_cells.sum().item())
    n_cut_elems = int(cnt[cut_cells].sum().item())
    return (16 * gm.n_nodes + 48 * n_plain + nc + 145 * n_cut_elems + 8 * n_cut_cells
            + 4 * gm.n_points), n_plain, n_cut_cells, n_cut_elems


def stored_step_bytes(case, body, n_tiles, n_plain, hc, esz=8):
    """Algorithmic bytes of one iteration launch that reads stored element entries:
    the vectors and tags of step_bytes, and instead of displacements the slab of every
    geometry task ((hc + 1) cell rows x 6 entries x 64 lanes)."""
    import torch
    n = case.grid.nodes
    nx, ny = case.grid.nx, case.grid.ny
    boundary = 2 * (nx + 1) + 2 * (ny - 1)
    bodies = int((body >= 0).sum().item())
    return (15 * esz * n) // 2 + (boundary + bodies) + (n_tiles - n_plain) * (hc + 1) * 6 * 64 * esz


def mixed_cell_mesh(mfp, W):
    """The paper's mixed-cell mesh of the benchmark geometry (1024 x 512, five
    cylinders): mesh time, the mixed-node product's roofline, and the constrained
    solve (FP64 and FP32 + FP64 refinement to 1e-12) on the one-kernel iteration with
    the cut cells condensed onto their corners, with its iteration kernel's roofline."""
    import numpy as np
    import torch
    case = W.five_cyl_1024()
    dev = "cuda:0"
    gm, mesh_ms = _timed(lambda: mfp.mixed_mesh(case.grid, case.circles, case.nsweeps,
                                                device=dev), reps=3)
    p = torch.from_numpy(W.random_vector(gm.n_nodes, 1)).to(dev)
    _, apply_ms = mfp.mixed_element_apply(gm, p, repeat=200)
    nbytes, n_plain, n_cut_cells, n_cut_elems = mixed_apply_bytes(gm)
    out = {"workload": "five cylinders, 1024x512 cells, delta 0.25; mixed-cell mesh (cut "
                       "points on grid lines, triangles and split pentagons); rtol 1e-12",
           "mesh_ms": round(mesh_ms, 3), "cut_points": gm.n_points, "elements": gm.n_elems,
           "triangles": gm.n_tri, "plain_quad_cells": n_plain, "cut_cells": n_cut_cells,
           "cut_cell_elements": n_cut_elems,
           "product": {"kernel": "k_mx_apply", "ms": round(apply_ms, 5),
                       "bytes": nbytes,
                       "achieved_GBs": round(nbytes / (apply_ms * 1e-3) / 1e9, 1),
                       "frac": round(nbytes / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    res = {}
    for prec in ("fp64", "fp32_ir"):
        r, ms = _timed(lambda: mfp.mixed_psi_solve(gm, case.flow, precision=prec, rtol=1e-12,
                                                   pair=case.pair, profile_every=1), reps=2)
        res[prec] = r
        s = r.stats
        e = {"solve_ms": round(ms, 2), "iters": s["iters"], "n_dof": s["n_dof"],
             "relres_true": s["relres_true"], "copfi": r.copfi,
             "dof_iter_per_s": s["n_dof"] * s["iters"] / (ms * 1e-3)}
        if s["apply_samples"] > 0 and prec == "fp64":
            hc = _task_height(case, s["n_tiles"])
            sb = stored_step_bytes(case, gm.body, s["n_tiles"], s["n_plain_tiles"], hc)
            kms = s["apply_ms"]
            e["roofline"] = {"kernel": _kernel_label(case, s),
                             "launch_ms": round(kms, 5), "bytes_per_launch": sb,
                             "achieved_GBs": round(sb / (kms * 1e-3) / 1e9, 1),
                             "frac": round(sb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[prec] = e
    rk = mfp.mixed_psi_solve(gm, case.flow, rtol=1e-12, pair=case.pair, estimate_kappa=True)
    out["kappa_gpu_lanczos"] = {"kappa": rk.stats["kappa_est"], "ritz_min": rk.stats["ritz_min"],
                                "ritz_max": rk.stats["ritz_max"]}
    mixed_cell_mesh.last = (case, gm, res)
    return out


def airfoils_kutta(mfp, W):
    """Two cambered Joukowski airfoils (chord 2, sharp trailing edges) in the 1024 x 512
    channel, mixed-cell mesh, each with a Kutta point 0.3 behind its trailing edge:
    mesh time and the Kutta solve (three constrained FP64 solves to 1e-12 combined on
    the host), with the circulation the flow gives each airfoil."""
    import torch
    bodies = [("joukowski", -1.0, 0.5, 0.5, -0.04, 0.05, 0.08),
              ("joukowski", 1.5, -0.8, 0.5, -0.04, 0.05, 0.08)]
    grid = W.Grid(1024, 512, -20.0, 20.0, -10.0, 10.0)
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UY, W.BC_NATURAL, W.BC_DIRICHLET_UY,
                        W.BC_DIRICHLET_UY))
    gm, mesh_ms = _timed(lambda: mfp.mixed_mesh_bodies(grid, bodies, 200, device="cuda:0"),
                         reps=3)
    pts = []
    for b in bodies:
        ca, sa = math.cos(b[6]), math.sin(b[6])
        te = (b[1] + ca * 2.0 * b[3], b[2] - sa * 2.0 * b[3])
        pts.append((te[0] + 0.3 * ca, te[1] - 0.3 * sa))
    r, ms = _timed(lambda: mfp.mixed_psi_solve_kutta(gm, flow, pts, rtol=1e-12), reps=2)
    airfoils_kutta.last = (grid, bodies, flow, pts, gm, r)
    return {"workload": "two Joukowski airfoils (c = 0.5, xi0 = -0.04, eta0 = 0.05, "
                        "alpha = 0.08) at (-1, 0.5) and (1.5, -0.8), 1024x512 cells on "
                        "[-20,20]x[-10,10]; Kutta points 0.3 behind the trailing edges; "
                        "FP64 to 1e-12",
            "mesh_ms": round(mesh_ms, 3), "cut_points": gm.n_points, "elements": gm.n_elems,
            "triangles": gm.n_tri, "kutta_nodes": r.kutta_nodes,
            "solve_ms": round(ms, 2), "iters_all_subsolves": r.stats["iters"],
            "relres_true_max": r.stats["relres_true"], "psi_b": r.psi_b}


def airfoils_vs_oracle(grid, bodies, flow, pts, gm, r):
    """CPU leg: the oracle's airfoil mesh and direct nonsymmetric Kutta solve against the
    GPU's (mesh bit for bit; psi, psi_b; the circulation of each airfoil)."""
    import numpy as np
    from oracle import airfoil as OA
    from oracle import kutta as OK
    from oracle import mixed as OM
    t0 = time.perf_counter()
    obodies = [OA.Joukowski(*b[1:]) for b in bodies]
    mm = OM.mixed_mesh_bodies(grid, obodies, 200)
    sol = OK.mixed_solve_kutta(mm, flow, pts)
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    psi = r.psi.cpu().numpy()
    scale = np.abs(sol.psi).max()
    return {"oracle_s": round(time.perf_counter() - t0, 1),
            "mesh_bitwise": bool(np.array_equal(gm.pxy.cpu().numpy(), mm.pxy)
                                 and np.array_equal(gm.disp.cpu().numpy(), mm.disp.reshape(-1))
                                 and np.array_equal(gm.elem.cpu().numpy(), mm.elem_nodes)),
            "psi_node_max_rel": float(np.abs(psi - sol.psi)[used].max() / scale),
            "psi_b_max_abs": float(np.abs(np.asarray(r.psi_b) - sol.psi_b).max()),
            "circulation": [float(v) for v in sol.body_rows],
            "kutta_circulation_isolated": [OA.Joukowski(*b[1:]).kutta_circulation(1.0)
                                           for b in bodies]}


def mixed_vs_oracle(case, gm, res):
    """CPU leg: the oracle's mixed-cell mesh and direct solve of the same workload
    against the GPU's (mesh bit for bit; psi, psi_b and CoPFI errors)."""
    import numpy as np
    from oracle import mixed as OM
    t0 = time.perf_counter()
    mm = OM.mixed_mesh(case.grid, case.circles, case.nsweeps)
    sol = OM.mixed_solve(mm, case.flow)
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    scale = np.abs(sol.psi).max()
    v = {"oracle_s": round(time.perf_counter() - t0, 1),
         "mesh_bitwise": bool(np.array_equal(gm.disp.cpu().numpy(), mm.disp.reshape(-1))
                              and np.array_equal(gm.pxy.cpu().numpy(), mm.pxy)
                              and np.array_equal(gm.elem.cpu().numpy(), mm.elem_nodes))}
    lo, hi = case.pair
    ref_cop = (sol.psi_b[hi] - sol.psi_b[lo]) / (
        case.flow.U * (case.circles[hi][1] - case.circles[lo][1]))
    for prec, r in res.items():
        psi = r.psi.cpu().numpy()
        v[prec] = {"psi_node_max_rel": float(np.abs(psi - sol.psi)[used].max() / scale),
                   "psi_b_max_abs": float(np.abs(np.asarray(r.psi_b) - sol.psi_b).max()),
                   "copfi_abs": float(abs(r.copfi - ref_cop))}
    return v


def streamlines(mfp, W):
    """Stagnation streamlines psi = psi_4 and psi = psi_5 of the benchmark workload
    (1024 x 512): mfp_contour on the FP64 solution, timed (both lines, ms)."""
    case = W.five_cyl_1024()
    dev = "cuda:0"
    d, k, b = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=dev)
    r = mfp.psi_solve(case.grid, case.circles, d, k, b, case.flow, rtol=1e-12,
                      pair=case.pair, sample_cap=0)

    def lines():
        return [mfp.contour(case.grid, d, b, r.psi, r.psi_b[q]) for q in (3, 4)]

    segs, ms = _timed(lines, reps=3)
    return {"workload": "five cylinders, 1024x512 cells; contours psi = psi_4, psi_5",
            "ms": round(ms, 3), "segments": [int(s.shape[0]) for s in segs],
            "lengths": [round(float((s[:, 2:] - s[:, :2]).norm(dim=1).sum()), 4)
                        for s in segs]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="length of the timed oracle CG run on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 4096x2048 mixed-precision, adjoint and delta-sweep "
                         "measurements")
    ap.add_argument("--profile-every", type=int, default=1,
                    help="time every n-th batch of iteration launches with HIP events "
                         "(0: off); a batch is timed between the events that end it and "
                         "the batch before it, which the host loop records anyway")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only run the 4096x2048 FP64 / FP32+refinement / FP32 comparison "
                         "and print its JSON (for profiling that workload)")
    ap.add_argument("--mixed-kmax", type=int, default=10 ** 7,
                    help="with --mixed-only: iteration cap of every solve (short "
                         "profiling runs)")
    ap.add_argument("--mixed-cell-only", action="store_true",
                    help="only run the mixed-cell mesh leg (1024x512) and print its JSON "
                         "(for profiling that workload)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only run the 256-system batched delta sweep and print its JSON "
                         "(for profiling that workload)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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
    if args.mixed_only:
        print(json.dumps({"mixed_precision_4096x2048": mixed_precision(mfp, W, args.mixed_kmax)}),
              flush=True)
        return
    if args.sweep_only:
        print(json.dumps({"delta_sweep_256": delta_sweep(mfp, W)}), flush=True)
        return
    if args.mixed_cell_only:
        out = {"mixed_cell_mesh_1024x512": mixed_cell_mesh(mfp, W),
               "airfoils_kutta_1024x512": airfoils_kutta(mfp, W)}
        print(json.dumps(out), flush=True)
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
    timed = [(r.stats["apply_ms"], r.stats["apply_samples"]) for _, _, r in outs
             if r.stats["apply_samples"] > 0]
    nbytes = _launch_bytes(case, disp, body, res.stats)
    _, moved = step_bytes(case, disp, body)
    roofline = None
    if timed:
        ms = sum(m * n for m, n in timed) / sum(n for _, n in timed)
        achieved = nbytes / (ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_from_profile(),
                    "kernel": _kernel_label(case, res.stats),
                    "launch_ms": round(ms, 5), "bytes_per_launch": nbytes,
                    "samples": int(sum(r.stats["apply_samples"] for _, _, r in outs))}
    # condition estimate of the benchmark solve from its CG scalars (an extra,
    # untimed solve of the same system)
    dk, kk, bk = mfp.mesh_conform(case.grid, case.circles, case.nsweeps, device=dev)
    rk = mfp.psi_solve(case.grid, case.circles, dk, kk, bk, case.flow, rtol=1e-12,
                       pair=case.pair, sample_cap=0, estimate_kappa=True)
    kappa = {"kappa": rk.stats["kappa_est"], "ritz_min": rk.stats["ritz_min"],
             "ritz_max": rk.stats["ritz_max"], "steps": rk.stats["kappa_steps"]}
    extras = {}
    if not args.no_extras:
        extras["mixed_precision_4096x2048"] = mixed_precision(mfp, W)
        extras["adjoint_2048x1024"] = adjoint_ratio(mfp, W)
        extras["potential_1024x512"] = potential_solve(mfp, W)
        extras["stagnation_streamlines_1024x512"] = streamlines(mfp, W)
        extras["delta_sweep_256"] = delta_sweep(mfp, W)
        extras["autotune"] = autotune_effect(mfp, W)
        extras["mixed_cell_mesh_1024x512"] = mixed_cell_mesh(mfp, W)
        extras["airfoils_kutta_1024x512"] = airfoils_kutta(mfp, W)
    cpu = None
    vs_oracle = {"kappa_gpu_lanczos": kappa}
    if not args.no_cpu_baseline:
        cpu, mesh_o, sol_o = cpu_baseline(case, args.cpu_seconds)
        vs_oracle = errors_vs_oracle(case, res, mesh_o, sol_o, kappa)
        if "potential_1024x512" in extras:
            pc, phi = potential_solve.last
            extras["potential_1024x512"]["vs_oracle"] = potential_vs_oracle(pc, phi, mesh_o)
        if "mixed_cell_mesh_1024x512" in extras:
            extras["mixed_cell_mesh_1024x512"]["vs_oracle"] = mixed_vs_oracle(
                *mixed_cell_mesh.last)
        if "airfoils_kutta_1024x512" in extras:
            extras["airfoils_kutta_1024x512"]["vs_oracle"] = airfoils_vs_oracle(
                *airfoils_kutta.last)
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
        "vs_oracle": vs_oracle,
        "iters": s["iters"],
        "solve_ms": s["solve_ms"],
        "relres_true": s["relres_true"],
        "plain_tile_frac": s["n_plain_tiles"] / max(1, s["n_tiles"]),
        "psi_b": res.psi_b,
        "copfi": res.copfi,
        **extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
