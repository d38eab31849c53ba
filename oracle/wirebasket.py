"""Oracle: structured wirebaskets on a periodic L_t x L_x grid (test infrastructure).

Paper, SM-AMG for LQCD subsection and the wirebasket figure: the grid is covered by
compact aggregates (wirebaskets) whose borders overlap.  Each point is a vertex (V),
an edge point (E) or an interior point (I); vertices form the coarse grid, edges are
interpolated from vertices and couple to neighbouring wirebaskets, interior points
couple only inside their wirebasket.  The figure shows two 3 x 3 wirebaskets sharing
one column: 4 vertices, 4 edge points and 1 interior point each.

Reading for aggregate size a and overlap o (the paper only draws a = 2, o = 1):
* wirebasket W(I, J), 0 <= I < L_t / a, 0 <= J < L_x / a, is the (a + o) x (a + o) block
  of points {(a I + d_t, a J + d_x) mod L : 0 <= d_t, d_x < a + o}; neighbours share an
  o-wide strip;
* the multiplicity of a point is the number of wirebaskets containing it: 4 -> V,
  2 -> E, 1 -> I;
* the coarse node (I, J) is the o x o block of vertices {(a I + p_t, a J + p_x), p < o};
  its coarse degrees of freedom are numbered (I * L_x/a + J) * b_c + (p_t * o + p_x) * b + q
  with b the degrees of freedom per fine point and b_c = o^2 b;
* an edge point belongs to two wirebaskets; it is interpolated only from its primary
  wirebasket, the first one it was assigned to (paper, end of the SM-AMG subsection),
  read as the lowest wirebasket index w = I * (L_x / a) + J.
"""
from __future__ import annotations

import numpy as np

KIND_I, KIND_E, KIND_V = 0, 1, 2


def footprint(I: int, J: int, Lt: int, Lx: int, a: int, o: int):
    """Points of W(I, J) in row-major local order (d_t, d_x); returns list of (t, x, d_t, d_x)."""
    pts = []
    for dt in range(a + o):
        for dx in range(a + o):
            pts.append(((a * I + dt) % Lt, (a * J + dx) % Lx, dt, dx))
    return pts


def classify(Lt: int, Lx: int, a: int, o: int):
    """Multiplicity, kind, owner wirebasket and node id of every grid point.

    Returns dict with int arrays of shape [Lt * Lx] (point index t * Lx + x):
      mult  -- number of wirebaskets containing the point,
      kind  -- KIND_V / KIND_E / KIND_I,
      owner -- primary wirebasket (lowest index containing the point; -1 for vertices),
      node  -- coarse node of a vertex (-1 otherwise).
    """
    if Lt % a or Lx % a:
        raise ValueError("aggregate size must divide the grid")
    nI, nJ = Lt // a, Lx // a
    if nI < 2 or nJ < 2 or not (1 <= o < a):
        raise ValueError("need L / a >= 2 and 1 <= o < a")
    n = Lt * Lx
    mult = np.zeros(n, dtype=np.int64)
    owner = np.full(n, -1, dtype=np.int64)
    for I in range(nI):
        for J in range(nJ):
            w = I * nJ + J
            for t, x, _, _ in footprint(I, J, Lt, Lx, a, o):
                p = t * Lx + x
                mult[p] += 1
                if owner[p] < 0:          # wirebaskets are visited in increasing index
                    owner[p] = w
    kind = np.full(n, -1, dtype=np.int64)
    kind[mult == 1] = KIND_I
    kind[mult == 2] = KIND_E
    kind[mult == 4] = KIND_V
    if np.any(kind < 0):
        raise AssertionError("multiplicity outside {1, 2, 4}")
    node = np.full(n, -1, dtype=np.int64)
    for p in np.nonzero(kind == KIND_V)[0]:
        t, x = divmod(int(p), Lx)
        node[p] = (t // a) * nJ + (x // a)
    owner[kind == KIND_V] = -1
    return {"mult": mult, "kind": kind, "owner": owner, "node": node,
            "nI": nI, "nJ": nJ}


def coarse_dof_of_vertex(p: int, q: int, Lx: int, a: int, o: int, b: int, node_id: int) -> int:
    """Coarse degree of freedom that vertex point p, component q, is injected into."""
    t, x = divmod(p, Lx)
    pt, px = t % a, x % a
    return node_id * (o * o * b) + (pt * o + px) * b + q
