"""Knot diagram -> signed Tait graph (Sec. II of the paper).

Test infrastructure (see ``oracle/__init__``).

Definitions followed (Sec. II, "For any knot diagram, a planar graph G called
the Tait graph ..."):

* the regions of the diagram are bicoloured so that adjacent regions differ;
  the unbounded region is white;
* vertices of G are the black regions; every crossing c gives an edge joining
  the two black regions that meet at c;
* twist sign: +1 for a right-handed crossing; writhe w = sum of twist signs;
* Tait sign eps_c: +1 iff the region on the left of the over-strand, as it
  leaves the crossing, is black; Tait number tau = sum of eps_c.

PD convention: ``pd[i] = (a, b, c, d)`` lists the arcs at crossing i counter-
clockwise from the incoming under-arc; arcs are numbered 0..2n-1 along the
orientation; crossing i is positive iff b == d + 1 (mod 2n).  The unbounded
region is taken to be the one on the left of arc 0 unless another is named.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class TaitGraph:
    n_vertices: int
    edges: list          # list of (u, v) with u, v black-region ids (u == v: loop)
    eps: list            # Tait sign per edge, +1 / -1; edge k <-> crossing k
    writhe: int
    tait_number: int
    twist: list          # twist sign per crossing


def crossing_signs(pd) -> list:
    """Twist sign of every crossing read off the labels (b == d+1 -> +1)."""
    n = len(pd)
    m = 2 * n
    out = []
    for (a, b, c, d) in pd:
        out.append(1 if (b - d) % m == 1 else -1)
    return out


def faces(pd):
    """Regions of the diagram as cycles of crossing corners.

    Corner (i, k) is the wedge at crossing i between slot k and slot k+1
    (counter-clockwise).  Walking out of crossing i along slot k, corner (i, k)
    is on the left; arriving at the far end (j, p) of that arc, the same region
    continues in corner (j, p-1).  Returns ``face_of[(i, k)]`` and the count.
    """
    n = len(pd)
    where = {}
    for i in range(n):
        for k in range(4):
            where.setdefault(int(pd[i][k]), []).append((i, k))
    for lab, occ in where.items():
        if len(occ) != 2:
            raise ValueError(f"arc {lab} appears {len(occ)} times")

    def far_end(i, k):
        lab = int(pd[i][k])
        o0, o1 = where[lab]
        return o1 if o0 == (i, k) else o0

    face_of = {}
    nf = 0
    for i in range(n):
        for k in range(4):
            if (i, k) in face_of:
                continue
            cur = (i, k)
            while cur not in face_of:
                face_of[cur] = nf
                j, p = far_end(*cur)
                cur = (j, (p - 1) % 4)
            nf += 1
    return face_of, nf


def tait_graph(pd, signs=None, outer_arc: int = 0, outer_left: bool = True) -> TaitGraph:
    """Signed Tait graph of a PD code (Sec. II).

    ``signs`` gives the twist signs when they cannot be read from the labels
    (one crossing).  The unbounded (white) region is the one on the left
    (``outer_left``) or right of arc ``outer_arc`` where that arc starts.
    """
    pd = [tuple(int(v) for v in row) for row in pd]
    n = len(pd)
    if n == 0:
        # a circle: the disc it bounds is the single black region
        return TaitGraph(1, [], [], 0, 0, [])
    if signs is None:
        if n == 1:
            raise ValueError("a one-crossing PD code needs explicit signs")
        signs = crossing_signs(pd)
    signs = [int(s) for s in signs]
    face_of, nf = faces(pd)

    # 2-colour the regions: the two corners on either side of a slot are in
    # regions of opposite colour.
    adj = [[] for _ in range(nf)]
    for i in range(n):
        for k in range(4):
            f1 = face_of[(i, k)]
            f2 = face_of[(i, (k - 1) % 4)]
            adj[f1].append(f2)
            adj[f2].append(f1)
    # the region to the left of arc `outer_arc` where it leaves its crossing
    start = None
    for i in range(n):
        a, b, c, d = pd[i]
        out_slots = [2, 1 if signs[i] > 0 else 3]   # outgoing under, outgoing over
        for s in out_slots:
            if pd[i][s] == outer_arc:
                start = (i, s) if outer_left else (i, (s - 1) % 4)
    if start is None:
        raise ValueError("outer_arc not found")
    colour = [-1] * nf
    root = face_of[start]
    colour[root] = 0                      # 0 = white, 1 = black
    stack = [root]
    while stack:
        f = stack.pop()
        for g in adj[f]:
            if colour[g] < 0:
                colour[g] = 1 - colour[f]
                stack.append(g)
            elif colour[g] == colour[f]:
                raise ValueError("regions are not 2-colourable")

    black = [f for f in range(nf) if colour[f] == 1]
    vid = {f: k for k, f in enumerate(black)}
    edges, eps = [], []
    for i in range(n):
        # outgoing over-slot: b for a positive crossing, d for a negative one
        s_out_over = 1 if signs[i] > 0 else 3
        left = face_of[(i, s_out_over)]
        e = 1 if colour[left] == 1 else -1
        if e > 0:
            c1, c2 = face_of[(i, s_out_over)], face_of[(i, (s_out_over + 2) % 4)]
        else:
            c1, c2 = face_of[(i, (s_out_over + 1) % 4)], face_of[(i, (s_out_over + 3) % 4)]
        edges.append((vid[c1], vid[c2]))
        eps.append(e)
    return TaitGraph(len(black), edges, eps, int(sum(signs)), int(sum(eps)), signs)

