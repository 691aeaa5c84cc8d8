"""Oracle: bodies with a sharp trailing edge -- Joukowski airfoils -- for the mixed-cell
mesh, and their exact potential flow.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Boundary Conditions" treats bodies with corners, trailing edges above all,
and section "Practical Applications" names airfoil and hydrofoil clusters.  The
Joukowski airfoil is the sharp-edged body whose potential flow is known in closed
form, so it pins both the mesh and the Kutta constraint.

Body.  The Joukowski map z' = zeta + c^2 / zeta takes the circle
|zeta - zeta0| = R through zeta = c (R^2 = (c - xi0)^2 + eta0^2, zeta0 = (xi0, eta0)) to an
airfoil with a cusped trailing edge at z' = 2c (chord about 4c; xi0 < 0 gives
thickness, eta0 > 0 camber).  It is placed by a rotation through -alpha (the angle
of attack against the horizontal free stream) and a translation:
z = zc + e^{-i alpha} z'.

Inside test, in plain FP64 real arithmetic: w = e^{i alpha} (z - zc); the roots of
zeta^2 - w zeta + c^2 = 0 are (w +- s) / 2 with s a square root of w^2 - 4 c^2
(taken as: m = sqrt(a_r^2 + a_i^2); a_r >= 0: s_r = sqrt((m + a_r)/2),
s_i = a_i / (2 s_r); else s_i = sqrt((m - a_r)/2) with the sign of a_i,
s_r = a_i / (2 s_i); s = 0 when a = 0).  The map takes the outside of the circle
one to one onto the outside of the airfoil, so a point is outside the body iff one
of its two preimages lies outside the circle: with zeta the root of larger
|zeta - zeta0|^2 (the first on a tie), z is in the body (boundary included) iff
|zeta - zeta0|^2 - R^2 <= 0 (cos alpha and sin alpha from the C library).  (Of a cambered airfoil's two preimages the one outside
|zeta| = c is not always the one outside the circle: near the trailing edge part
of the slit [-2c, 2c] lies outside the body.)  The level |zeta - zeta0|^2 - R^2 is
continuous, since the two roots only swap across the branch cut.

Cut point of a grid edge from an inside node I to a fluid node O (the projection
along the grid line): f(t) = |zeta(I + t (O - I)) - zeta0|^2 - R^2 is <= 0 at t = 0
and > 0 at t = 1; the bracket [t_k, t_(k+1)], t_k = k / 64, of its first sign change
(first k with f(t_(k+1)) > 0) is bisected 60 times (midpoint, keep the half whose
lower end is inside), and the cut point is I + t (O - I) with t the final lower
end.  A grid edge whose two nodes are fluid is not cut even if a thin part of the
body passes between them: a trailing edge thinner than the grid is not resolved.

Exact flow.  In the body's frame W(zeta) = U [(zeta - zeta0) e^{-i alpha}
+ R^2 e^{i alpha} / (zeta - zeta0)] - i Gamma/(2 pi) ln((zeta - zeta0)/R) (Gamma
counter-clockwise positive); psi = Im W at the exterior root, zero on the body.
Far away psi -> U (y - yc).  The Kutta condition (finite velocity at the trailing
edge zeta = c) gives Gamma = 4 pi U R sin(theta_c - alpha), theta_c = arg(c - zeta0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _csqrt(ar, ai):
    """Square root of a_r + i a_i in the stated real arithmetic (arrays)."""
    ar = np.asarray(ar, dtype=float)
    ai = np.asarray(ai, dtype=float)
    m = np.sqrt(ar * ar + ai * ai)
    pos = ar >= 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        sr_p = np.sqrt((m + ar) * 0.5)
        si_p = np.where(sr_p > 0.0, ai / (2.0 * sr_p), 0.0)
        si_n = np.copysign(np.sqrt((m - ar) * 0.5), ai)
        sr_n = np.where(si_n != 0.0, ai / (2.0 * si_n), 0.0)
    return np.where(pos, sr_p, sr_n), np.where(pos, si_p, si_n)


@dataclass(frozen=True)
class Joukowski:
    xc: float      # placement of the airfoil's origin (the image of zeta = 0)
    yc: float
    c: float       # map constant (chord about 4c)
    xi0: float     # centre of the generating circle
    eta0: float
    alpha: float   # angle of attack (radians): the body is rotated through -alpha

    @property
    def R2(self):
        """R^2 = (c - xi0)^2 + eta0^2 (the circle passes through zeta = c)."""
        return (self.c - self.xi0) * (self.c - self.xi0) + self.eta0 * self.eta0

    @property
    def R(self):
        return math.sqrt(self.R2)

    def cs(self):
        return math.cos(self.alpha), math.sin(self.alpha)

    def zeta(self, X, Y):
        """The preimage zeta (real, imaginary parts) of points (X, Y) farther from the
        circle's centre."""
        ca, sa = self.cs()
        dx = np.asarray(X, dtype=float) - self.xc
        dy = np.asarray(Y, dtype=float) - self.yc
        wr = ca * dx - sa * dy
        wi = sa * dx + ca * dy
        c2 = self.c * self.c
        ar = wr * wr - wi * wi - 4.0 * c2
        ai = 2.0 * wr * wi
        sr, si = _csqrt(ar, ai)
        z1r, z1i = (wr + sr) * 0.5, (wi + si) * 0.5
        z2r, z2i = (wr - sr) * 0.5, (wi - si) * 0.5
        e1r, e1i = z1r - self.xi0, z1i - self.eta0
        e2r, e2i = z2r - self.xi0, z2i - self.eta0
        first = (e1r * e1r + e1i * e1i) >= (e2r * e2r + e2i * e2i)
        return np.where(first, z1r, z2r), np.where(first, z1i, z2i)

    def level(self, X, Y):
        """|zeta - zeta0|^2 - R^2 (<= 0: in the body)."""
        zr, zi = self.zeta(X, Y)
        er = zr - self.xi0
        ei = zi - self.eta0
        return er * er + ei * ei - self.R2

    def contains(self, X, Y):
        return self.level(X, Y) <= 0.0

    def cut(self, xi, yi, xo, yo):
        """Cut point of the grid edge from inside node (xi, yi) to fluid node (xo, yo)."""
        vx, vy = xo - xi, yo - yi
        k = 0
        while k < 63 and not (self.level(xi + ((k + 1) / 64.0) * vx,
                                         yi + ((k + 1) / 64.0) * vy) > 0.0):
            k += 1
        lo, hi = k / 64.0, (k + 1) / 64.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if self.level(xi + mid * vx, yi + mid * vy) > 0.0:
                hi = mid
            else:
                lo = mid
        return xi + lo * vx, yi + lo * vy

    def trailing_edge(self):
        """Physical position of the trailing edge (z' = 2c) and the chord direction."""
        ca, sa = self.cs()
        te = (self.xc + ca * 2.0 * self.c, self.yc - sa * 2.0 * self.c)
        return te, (ca, -sa)

    def bounding_circle(self):
        """A circle holding the whole body (for the geometry checks): about its origin
        image, radius max |z'| over the boundary plus a margin."""
        th = np.linspace(0.0, 2.0 * np.pi, 4097)
        zr = self.xi0 + self.R * np.cos(th)
        zi = self.eta0 + self.R * np.sin(th)
        d = zr * zr + zi * zi
        xr = zr + self.c * self.c * zr / d
        xi = zi - self.c * self.c * zi / d
        return (self.xc, self.yc, float(np.sqrt(xr * xr + xi * xi).max()) * 1.01)

    def kutta_circulation(self, U):
        theta_c = math.atan2(-self.eta0, self.c - self.xi0)
        return 4.0 * math.pi * U * self.R * math.sin(theta_c - self.alpha)

    def psi_exact(self, X, Y, U, gamma):
        """Stream function of the flow past the airfoil with circulation gamma; zero on
        the body, U (y - yc) far away."""
        zr, zi = self.zeta(X, Y)
        er = zr - self.xi0
        ei = zi - self.eta0
        R = self.R
        ca, sa = self.cs()
        # Im[(e) e^{-i a}] = ei ca - er sa;  Im[R^2 e^{i a} / e] = R^2 (sa er - ca ei)/|e|^2
        r2 = er * er + ei * ei
        with np.errstate(divide="ignore", invalid="ignore"):
            return (U * ((ei * ca - er * sa) + R * R * (sa * er - ca * ei) / r2)
                    - gamma / (2.0 * np.pi) * 0.5 * np.log(r2 / (R * R)))

    def circulation_through(self, point, U):
        """Gamma for which psi_exact vanishes at point (a Kutta point on the zero
        streamline)."""
        p0 = self.psi_exact(np.array([point[0]]), np.array([point[1]]), U, 0.0)[0]
        zr, zi = self.zeta(np.array([point[0]]), np.array([point[1]]))
        r2 = (zr[0] - self.xi0) ** 2 + (zi[0] - self.eta0) ** 2
        return 2.0 * np.pi * p0 / (0.5 * math.log(r2 / self.R ** 2))


@dataclass(frozen=True)
class Circle:
    cx: float
    cy: float
    r: float

    def contains(self, X, Y):
        dx = np.asarray(X, dtype=float) - self.cx
        dy = np.asarray(Y, dtype=float) - self.cy
        return (dx * dx + dy * dy) <= self.r * self.r

    def cut(self, xi, yi, xo, yo):
        vx, vy = xo - xi, yo - yi
        ux, uy = xi - self.cx, yi - self.cy
        vv = vx * vx + vy * vy
        uv = ux * vx + uy * vy
        uu = ux * ux + uy * uy
        t = (-uv + np.sqrt(uv * uv - vv * (uu - self.r * self.r))) / vv
        return xi + t * vx, yi + t * vy

    def bounding_circle(self):
        return (self.cx, self.cy, self.r)
