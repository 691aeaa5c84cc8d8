"""Oracle: contour lines of a nodal field on the conformed mesh.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper draws the flow net (contours of psi and phi, section "Governing
Equation") and the stagnation streamlines of the transverse cylinders (section
"Effect of Gap Ratio": the streamlines psi = psi_4 and psi = psi_5 that bound the
stream tube between them).  It does not say how its lines were drawn.  Reading:
marching squares over the active cells of the conformed mesh, in the displaced
node coordinates:

* a node is above the level when its value is >= the level;
* on every cell edge whose two nodes differ, the crossing is the linear
  interpolation x_a + t (x_b - x_a), t = (level - f_a) / (f_b - f_a), between
  the edge's end nodes a -> b (edges 0-1, 1-2, 2-3, 3-0);
* two crossings give one segment (from the lower-numbered edge to the other);
  four crossings (a saddle) give two segments, paired by the cell-centre value
  (the mean of the four): if the centre is on node 0's side, the segments cut
  off nodes 1 and 3 (edges 0,1 and 2,3), otherwise nodes 0 and 2 (edges 3,0 and
  1,2), in that order;
* cells inside a body (inactive) and cells with a non-finite nodal value are
  skipped;
* segments are ordered by cell id (j nx + i), then as above.
"""
from __future__ import annotations

import numpy as np

from .mesh import active_cells, cell_nodes


def contour(mesh, field, level):
    """Segments (k, 4) array of (x0, y0, x1, y1) of the level set field = level."""
    grid = mesh.grid
    X, Y = mesh.coords()
    Xf, Yf = X.ravel(), Y.ravel()
    f = np.asarray(field, dtype=np.float64).ravel()
    cn = cell_nodes(grid)
    segs = []
    act = active_cells(grid, mesh.body)
    for cid in np.flatnonzero(act):
        nd = cn[cid]
        v = f[nd]
        if not np.all(np.isfinite(v)):
            continue
        up = v >= level
        cross = {}
        for e in range(4):
            a, b = e, (e + 1) % 4
            if up[a] != up[b]:
                t = (level - v[a]) / (v[b] - v[a])
                cross[e] = (Xf[nd[a]] + t * (Xf[nd[b]] - Xf[nd[a]]),
                            Yf[nd[a]] + t * (Yf[nd[b]] - Yf[nd[a]]))
        if len(cross) == 2:
            e0, e1 = sorted(cross)
            segs.append((*cross[e0], *cross[e1]))
        elif len(cross) == 4:
            centre_up = v.mean() >= level
            pairs = ((0, 1), (2, 3)) if centre_up == up[0] else ((3, 0), (1, 2))
            for e0, e1 in pairs:
                segs.append((*cross[e0], *cross[e1]))
    return np.array(segs, dtype=np.float64).reshape(-1, 4)
