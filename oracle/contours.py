"""Marching squares on the binary slice image (Sec. 4: rough boundary curves
from the binary image).

Test infrastructure (see the package docstring).

The paper names the algorithm and its input (the binary image) but no
convention, so this module fixes one:

* Grid units: pixel (i, j) is the point (i, j); x grows with i, y with j.
* Cell (i, j), 0 <= i < W-1, 0 <= j < H-1, has corners c0 = (i, j),
  c1 = (i+1, j), c2 = (i+1, j+1), c3 = (i, j+1) and case code
  b0 | b1 << 1 | b2 << 2 | b3 << 3 with b = inside.
* Segment ends sit at edge midpoints (the image is binary, so there is no
  field to interpolate): bottom B = (1/2, 0), right E = (1, 1/2),
  top T = (1/2, 1), left L = (0, 1/2) in cell-local coordinates.
* Each segment runs with the inside on its left, so boundaries of inside
  regions turn counter-clockwise.
* The two saddle cases (5, 10) keep the two inside corners apart (inside is
  4-connected, outside 8-connected).
* Output order: cells row by row (j outer, i inner), segments of a cell in
  table order.  All coordinates are multiples of 1/2.
"""
from __future__ import annotations

import numpy as np

B = (0.5, 0.0)
E = (1.0, 0.5)
T = (0.5, 1.0)
L = (0.0, 0.5)

# case -> list of (start, end); inside on the left of start -> end
TABLE = {
    0: [],
    1: [(B, L)],            # c0
    2: [(E, B)],            # c1
    3: [(E, L)],            # c0 c1
    4: [(T, E)],            # c2
    5: [(B, L), (T, E)],    # c0 c2, kept apart
    6: [(T, B)],            # c1 c2
    7: [(T, L)],            # c0 c1 c2
    8: [(L, T)],            # c3
    9: [(B, T)],            # c0 c3
    10: [(E, B), (L, T)],   # c1 c3, kept apart
    11: [(E, T)],           # c0 c1 c3
    12: [(L, E)],           # c2 c3
    13: [(B, E)],           # c0 c2 c3
    14: [(L, B)],           # c1 c2 c3
    15: [],
}

# area of the inside part of a cell, by case (for the shoelace check)
CASE_AREA = {0: 0.0, 1: 1 / 8, 2: 1 / 8, 4: 1 / 8, 8: 1 / 8,
             3: 0.5, 6: 0.5, 12: 0.5, 9: 0.5,
             5: 0.25, 10: 0.25,
             7: 7 / 8, 11: 7 / 8, 13: 7 / 8, 14: 7 / 8, 15: 1.0}


def case_codes(inside: np.ndarray) -> np.ndarray:
    """[H-1, W-1] uint8 case codes of a boolean image inside[j, i]."""
    b = np.asarray(inside, dtype=np.uint8)
    c0 = b[:-1, :-1]
    c1 = b[:-1, 1:]
    c2 = b[1:, 1:]
    c3 = b[1:, :-1]
    return (c0 | (c1 << 1) | (c2 << 2) | (c3 << 3)).astype(np.uint8)


def segments(inside: np.ndarray) -> np.ndarray:
    """[n, 4] float64 segments (x0, y0, x1, y1) in grid units, in output
    order."""
    codes = case_codes(inside)
    out = []
    js, is_ = np.nonzero((codes != 0) & (codes != 15))
    for j, i in zip(js, is_):          # nonzero walks row-major
        for (sx, sy), (ex, ey) in TABLE[int(codes[j, i])]:
            out.append((i + sx, j + sy, i + ex, j + ey))
    return np.array(out, dtype=np.float64).reshape(-1, 4)


def segment_counts(inside: np.ndarray) -> np.ndarray:
    codes = case_codes(inside)
    n = np.zeros(16, dtype=np.int64)
    for c, segs in TABLE.items():
        n[c] = len(segs)
    return n[codes]
