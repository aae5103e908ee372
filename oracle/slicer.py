"""The streaming slicer of Sec. 4, in float64.

Test infrastructure (see the package docstring).

* slice_heights: the sweep of Sec. 4 puts the first plane half a layer above
  the start height and moves up one layer per plane, so plane k is
  z0 + (k + 1/2) t.
* active_set: Eq. (8), the struts whose swept sphere of radius R meets the
  plane, with the lower end written v_s (the paper orders the ends by z).
* sweep_active_sets: the same sets from sorted events along z (where each
  swept sphere starts and ends), as a second route to them.
* slice_field: the field at every pixel centre of one plane using the
  active struts only (Sec. 4); inside where the sum reaches the iso-value.

R is one support for every strut, or an array with one per strut (the
per-strut variant); the sweep's start events are then ordered by z_lo - R_i,
the lower end of each swept sphere, which is z_lo ordering when R is shared.
"""
from __future__ import annotations

import numpy as np

from .field import strut_term, support_of


def slice_heights(z0: float, t: float, n: int) -> np.ndarray:
    return z0 + (np.arange(n, dtype=np.float64) + 0.5) * t


def strut_z_range(nodes, edges):
    """(lower z, upper z) of each strut's two ends."""
    z = np.asarray(nodes, dtype=np.float64)[:, 2]
    za = z[edges[:, 0]]
    zb = z[edges[:, 1]]
    return np.minimum(za, zb), np.maximum(za, zb)


def active_set(zlo, zhi, R, z: float) -> np.ndarray:
    """Eq. (8): ids j with v_s^z - R <= z and v_e^z + R >= z, ascending
    (R per strut when given as an array)."""
    return np.nonzero((zlo - R <= z) & (zhi + R >= z))[0]


def sweep_active_sets(zlo, zhi, R, heights):
    """Eq. (8)'s active sets by events along z, a second route to active_set:
    each strut's swept sphere spans [b, t] = [z_lo - R, z_hi + R]; sorting
    the b's and the t's once, the struts started by plane z are a prefix of
    the b order (b <= z) and those finished are a prefix of the t order
    (t < z); the active set is the first less the second.  The b order is the
    paper's edge list sorted by lower end (Sec. 4).  Returns the active set
    (ascending ids) of every plane."""
    Rv = np.broadcast_to(np.asarray(R, dtype=np.float64), np.shape(zlo))
    b = np.asarray(zlo, dtype=np.float64) - Rv
    t = np.asarray(zhi, dtype=np.float64) + Rv
    by_b = np.argsort(b, kind="stable")
    by_t = np.argsort(t, kind="stable")
    b_sorted, t_sorted = b[by_b], t[by_t]
    out = []
    for z in heights:
        started = by_b[:np.searchsorted(b_sorted, z, side="right")]
        finished = by_t[:np.searchsorted(t_sorted, z, side="left")]
        out.append(np.setdiff1d(started, finished).astype(np.int64))
    return out


def _pixel_window(lo, hi, origin, step, n):
    """Index range of pixel centres origin + (i + 1/2) step inside [lo, hi],
    widened by one pixel on each side (a superset; pixels outside the
    kernel's support add exact zeros)."""
    i0 = int(np.floor((lo - origin) / step - 0.5)) - 1
    i1 = int(np.ceil((hi - origin) / step - 0.5)) + 1
    return max(i0, 0), min(i1, n - 1)


def slice_field(nodes, edges, weight, R, grid, k: int, struts=None,
                kind: str = "quartic", sigma: float | None = None) -> np.ndarray:
    """g at every pixel centre of plane k: array [H, W] float64, g[j, i] at
    (x0 + (i+1/2) dx, y0 + (j+1/2) dy).  Struts of the active set (Eq. 8)
    are added in ascending id, each over the window of pixels its support
    can reach; outside that window its term is exactly zero.  R: one support
    or one per strut; kind, sigma: the kernel (see field.strut_term)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    weight = np.asarray(weight, dtype=np.float64)
    z = float(grid.slice_z(k))
    zlo, zhi = strut_z_range(nodes, edges)
    ids = active_set(zlo, zhi, R, z) if struts is None else struts
    g = np.zeros((grid.H, grid.W))
    xs = grid.pixel_x()
    ys = grid.pixel_y()
    for i in ids:
        if weight[i] == 0.0:
            continue
        a = nodes[edges[i, 0]]
        b = nodes[edges[i, 1]]
        Ri = support_of(R, i)
        ix0, ix1 = _pixel_window(min(a[0], b[0]) - Ri, max(a[0], b[0]) + Ri,
                                 grid.x0, grid.dx, grid.W)
        iy0, iy1 = _pixel_window(min(a[1], b[1]) - Ri, max(a[1], b[1]) + Ri,
                                 grid.y0, grid.dy, grid.H)
        if ix0 > ix1 or iy0 > iy1:
            continue
        X, Y = np.meshgrid(xs[ix0:ix1 + 1], ys[iy0:iy1 + 1], indexing="xy")
        P = np.stack([X, Y, np.full_like(X, z)], axis=-1)
        g[iy0:iy1 + 1, ix0:ix1 + 1] += weight[i] * strut_term(P, a, b, Ri, kind, sigma)
    return g


def slice_points(grid, k: int, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Pixel-centre points [n,3] of plane k for pixel indices (px, py)."""
    x = grid.x0 + (np.asarray(px, dtype=np.float64) + 0.5) * grid.dx
    y = grid.y0 + (np.asarray(py, dtype=np.float64) + 0.5) * grid.dy
    z = np.full(x.shape, float(grid.slice_z(k)))
    return np.stack([x, y, z], axis=-1)


def inside(g, C: float):
    """Binary slice image: inside where the field sum reaches C."""
    return np.asarray(g) >= C
