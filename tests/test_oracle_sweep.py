"""Pins of the oracle's sweep post-processing (no GPU): the cubic fit of CoPFI over
the gap ratio (section "Effect of Gap Ratio").

Pins: exact recovery of a cubic from exact samples (R^2 = 1, MSE = 0); and the
paper's own numbers: fitted to the CoPFI column of Table 1 (tests/golden, values
as printed), the least-squares cubic rounds to the coefficients the paper prints
(0.80417, -1.38561, 2.21409, -0.22171), and the paper's mean square error
1.40428920e-07 is the MSE of that printed (rounded) cubic on the same data.
"""
import os

import numpy as np

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER_CUBIC = (0.80417, -1.38561, 2.21409, -0.22171)


def test_exact_cubic_is_recovered():
    rng = np.random.default_rng(5)
    x = np.sort(rng.uniform(0.05, 2.0, 40))
    c = (0.7, -1.1, 2.3, -0.4)
    y = np.polyval(c, x)
    got, r2, mse = O.cubic_fit(x, y)
    np.testing.assert_allclose(got, c, rtol=0, atol=1e-11)
    assert abs(r2 - 1.0) < 1e-14 and mse < 1e-26


def test_table1_fit_gives_the_papers_cubic():
    t = np.loadtxt(os.path.join(HERE, "golden", "table1_gap_ratio.txt"), comments="#")
    delta, copfi = t[:, 0], t[:, 5]
    got, r2, mse = O.cubic_fit(delta, copfi)
    assert tuple(round(v, 5) for v in got) == PAPER_CUBIC
    assert 0.99999 < r2 < 1.0
    # the paper's MSE is that of its printed cubic
    res = copfi - np.polyval(PAPER_CUBIC, delta)
    assert abs((res @ res) / res.size - 1.40428920e-07) < 5e-16
    assert mse <= (res @ res) / res.size
