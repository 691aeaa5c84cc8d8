"""Oracle: plain conjugate gradients on the assembled reduced system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Appendix, Algorithm 1 writes CG with r = A x - b and the product sign folded
into the element loop (v_e = -A_e xp_e); that is the textbook method in
different signs.  This is the textbook form: r = b - A x, p = r, and per
iteration alpha = r.r / p.Ap, x += alpha p, r -= alpha Ap,
beta = r_new.r_new / r.r, p = r + beta p.  Readings: the epsilon in the
paper's alpha and beta denominators is taken as 0, the initial guess is 0 and
the stopping test is ||r_k|| <= rtol ||r_0|| (the paper's absolute 1e-12 on the
residual norm, made relative).  Used as the CPU timing baseline.
"""
from __future__ import annotations

import numpy as np


def cg(A, b, rtol=1e-12, kmax=10**6, x0=None, max_iters=None):
    """Returns (x, iterations, ||r||/||r0||)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    p = r.copy()
    rr = float(r @ r)
    rr0 = rr
    k = 0
    limit = kmax if max_iters is None else min(kmax, max_iters)
    while k < limit and rr > (rtol * rtol) * rr0:
        Ap = A @ p
        alpha = rr / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
    return x, k, (np.sqrt(rr / rr0) if rr0 > 0 else 0.0)
