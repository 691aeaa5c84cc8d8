"""Oracle: post-processing of a gap-ratio sweep.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Effect of Gap Ratio" fits CoPFI as a cubic polynomial of the gap ratio
delta and reports the fit's R^2 and mean square error.  Reading: an ordinary
least-squares fit (the paper names no weighting), R^2 = 1 - SS_res / SS_tot
about the mean, MSE = SS_res / n.
"""
from __future__ import annotations

import numpy as np


def cubic_fit(delta, copfi):
    """Least-squares cubic CoPFI(delta) = c3 delta^3 + c2 delta^2 + c1 delta + c0.
    Returns ((c3, c2, c1, c0), R^2, MSE)."""
    x = np.asarray(delta, dtype=np.float64)
    y = np.asarray(copfi, dtype=np.float64)
    c = np.polyfit(x, y, 3)
    res = y - np.polyval(c, x)
    ss_res = float(res @ res)
    ss_tot = float(((y - y.mean()) ** 2).sum())
    return tuple(float(v) for v in c), 1.0 - ss_res / ss_tot, ss_res / x.size
