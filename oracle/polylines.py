"""Sub-pixel contour segments and their chaining into polylines: the step
after marching squares (Sec. 4 stops at rough boundary curves from the
binary image; toolpaths need ordered, closed curves).

Test infrastructure (see the package docstring).

Readings fixed here (the paper gives neither):

* Sub-pixel endpoints.  The cells, segments and output order are those of
  contours.segments on the binary image g >= C; only the endpoint positions
  move.  A segment end on the cell edge between grid points P and Q (P the
  point with the smaller (j, i)) sits at P + t (Q - P) with
  t = (C - g(P)) / (g(Q) - g(P)), the zero of g - C interpolated linearly
  along the edge.  Exactly one of P and Q is inside, so g(Q) != g(P).
* Chains.  Each segment ends on a cell edge; the segment that starts on that
  edge (it lies in the neighbouring cell) follows it.  With the inside on the
  left of every segment, an edge crossed by the contour is the end of exactly
  one segment and the start of exactly one, unless the contour leaves the
  grid.  A chain starts at a segment with no predecessor; a closed loop starts
  at its smallest segment index.  Per plane, chain[s] is the index of the
  start segment of s's chain and rank[s] the number of steps from it along the
  successors.
"""
from __future__ import annotations

import numpy as np

from . import contours as C

# cell-local edge of each table point, as (corner P, corner Q) offsets with P
# the smaller (j, i): B bottom, E right, T top, L left
EDGE = {
    C.B: ((0, 0), (1, 0)),
    C.E: ((1, 0), (1, 1)),
    C.T: ((0, 1), (1, 1)),
    C.L: ((0, 0), (0, 1)),
}


def edge_id(i: int, j: int, pt) -> tuple:
    """Global id of the cell edge of table point pt in cell (i, j):
    ('h', x, y) joins (x, y)-(x+1, y); ('v', x, y) joins (x, y)-(x, y+1)."""
    (pi, pj), (qi, qj) = EDGE[pt]
    kind = "h" if pj == qj else "v"
    return (kind, i + pi, j + pj)


def crossing(field: np.ndarray, Cval: float, i: int, j: int, pt):
    """Point where g - C, linear along the edge, vanishes (grid units)."""
    (pi, pj), (qi, qj) = EDGE[pt]
    P = (i + pi, j + pj)
    Q = (i + qi, j + qj)
    gP = float(field[P[1], P[0]])
    gQ = float(field[Q[1], Q[0]])
    t = (Cval - gP) / (gQ - gP)
    return (P[0] + t * (Q[0] - P[0]), P[1] + t * (Q[1] - P[1]))


def segments_subpixel(field: np.ndarray, Cval: float) -> np.ndarray:
    """[n, 4] float64 segments (x0, y0, x1, y1), same cells and order as
    contours.segments(field >= Cval), endpoints interpolated."""
    field = np.asarray(field, dtype=np.float64)
    codes = C.case_codes(field >= Cval)
    out = []
    js, is_ = np.nonzero((codes != 0) & (codes != 15))
    for j, i in zip(js, is_):
        for s, e in C.TABLE[int(codes[j, i])]:
            out.append(crossing(field, Cval, i, j, s) + crossing(field, Cval, i, j, e))
    return np.array(out, dtype=np.float64).reshape(-1, 4)


def segment_edges(inside: np.ndarray):
    """Start and end edge ids of every segment of contours.segments(inside),
    in output order."""
    codes = C.case_codes(inside)
    start, end = [], []
    js, is_ = np.nonzero((codes != 0) & (codes != 15))
    for j, i in zip(js, is_):
        for s, e in C.TABLE[int(codes[j, i])]:
            start.append(edge_id(i, j, s))
            end.append(edge_id(i, j, e))
    return start, end


def chains(inside: np.ndarray):
    """(succ, chain, rank) int64 arrays over the segments of one plane:
    succ[s] the following segment or -1; chain and rank as in the module
    docstring."""
    start, end = segment_edges(inside)
    n = len(start)
    starts_on = {}
    for s, e in enumerate(start):
        assert e not in starts_on, "two segments start on one edge"
        starts_on[e] = s
    succ = np.array([starts_on.get(e, -1) for e in end], dtype=np.int64)
    pred = np.full(n, -1, dtype=np.int64)
    for s in range(n):
        if succ[s] >= 0:
            assert pred[succ[s]] < 0, "two segments end on one edge"
            pred[succ[s]] = s
    chain = np.full(n, -1, dtype=np.int64)
    rank = np.full(n, -1, dtype=np.int64)

    def walk(head):
        s, r = head, 0
        while s >= 0 and chain[s] < 0:
            chain[s] = head
            rank[s] = r
            s = succ[s]
            r += 1

    for s in range(n):                 # open chains: from their first segment
        if pred[s] < 0:
            walk(s)
    for s in range(n):                 # closed loops: from their smallest index
        if chain[s] < 0:
            walk(s)
    return succ, chain, rank
