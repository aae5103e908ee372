"""The (slab, tile, strut) bin set: which struts a tile of a slab must visit.

Test infrastructure (see the package docstring).

Sec. 3.2: only struts within distance R of p contribute to the field at p.
Sec. 4: a strut's swept sphere of radius R bounds the region it reaches, and
the edge list is kept sorted by the z of each edge's lower end.  The binning
turns both facts into integer sets, evaluated in float64 with exactly the
operation order written here (no fused multiply-add), so that any
implementation evaluating the same formulas gets the same integers:

  per strut (ends a, b as given, promoted to float64), skipped when its weight
  is 0 or a == b:
    lo = min(a, b) - R,  hi = max(a, b) + R          (per axis x, y, z)
    slice/pixel index range along an axis with origin o, step s, count n:
      i0 = floor(((lo - o) * inv_s) - 0.5)
      i1 = ceil(((hi - o) * inv_s) - 0.5)            inv_s = 1 / s
      clamped to [0, n - 1]; the strut is dropped if any range is empty.
    (Pixel i's centre is o + (i + 1/2) s; the rounding is outward, so every
    pixel centre and plane within the swept box is covered.)
  slab range   [k0 // Sz, k1 // Sz]
  tile range   [i0 // T, i1 // T] x [j0 // T, j1 // T]

  The edge list order is ascending (z of the lower end in the input's own
  precision, id).  With per-strut supports R_i (R given as an array), lo and
  hi use R_i and the order is ascending (first slab, z of the lower end, id):
  the first slab then no longer follows from z alone, and a slab's window
  must stay a prefix of the list.  With one R the first slab is a monotone
  function of z, so both orders coincide.  A bucket (slab, tile_y, tile_x) holds every binned strut
  whose ranges cover it, in edge-list order.  Buckets are numbered row-major
  within a slab, slabs in order.
"""
from __future__ import annotations

import math

import numpy as np


def axis_range(lo, hi, origin: float, step: float, n: int):
    """Outward-rounded index range of the points origin + (i + 1/2) step that
    lie in [lo, hi]; returns (i0, i1, nonempty) with i0, i1 clamped."""
    inv = 1.0 / step
    f0 = np.floor((lo - origin) * inv - 0.5)
    f1 = np.ceil((hi - origin) * inv - 0.5)
    ok = (f1 >= 0.0) & (f0 <= float(n - 1)) & (f0 <= f1)
    i0 = np.clip(f0, 0.0, float(n - 1))
    i1 = np.clip(f1, 0.0, float(n - 1))
    i0 = np.where(ok, i0, 0.0).astype(np.int64)
    i1 = np.where(ok, i1, -1.0).astype(np.int64)
    return i0, i1, ok


def strut_ranges(nodes, edges, weight, R, grid, tile: int, slab: int):
    """Per-strut ranges.  Returns a dict of int64 arrays (slab0, slab1, tx0,
    tx1, ty0, ty1), the boolean mask `binned`, and `order`: the ids of the
    binned struts in edge-list order."""
    nd = np.asarray(nodes)
    a = nd[edges[:, 0]].astype(np.float64)
    b = nd[edges[:, 1]].astype(np.float64)
    w = np.asarray(weight)
    per_strut = np.ndim(R) > 0
    Rc = np.asarray(R, dtype=np.float64)[:, None] if per_strut else R
    lo = np.minimum(a, b) - Rc
    hi = np.maximum(a, b) + Rc
    k0, k1, okz = axis_range(lo[:, 2], hi[:, 2], grid.z0, grid.dz, grid.n_slices)
    i0, i1, okx = axis_range(lo[:, 0], hi[:, 0], grid.x0, grid.dx, grid.W)
    j0, j1, oky = axis_range(lo[:, 1], hi[:, 1], grid.y0, grid.dy, grid.H)
    degenerate = np.all(a == b, axis=1)
    binned = okz & okx & oky & (w != 0) & ~degenerate
    # the edge list: ascending lower-end z in the input precision, then id
    zin = nd[:, 2]
    zlo_in = np.minimum(zin[edges[:, 0]], zin[edges[:, 1]])
    ids = np.nonzero(binned)[0]
    if per_strut:
        order = ids[np.lexsort((ids, zlo_in[ids], (k0 // slab)[ids]))]
    else:
        order = ids[np.lexsort((ids, zlo_in[ids]))]
    return dict(slab0=k0 // slab, slab1=k1 // slab, tx0=i0 // tile, tx1=i1 // tile,
                ty0=j0 // tile, ty1=j1 // tile, binned=binned, order=order,
                k0=k0, k1=k1)


def tiles_xy(grid, tile: int):
    return (grid.W + tile - 1) // tile, (grid.H + tile - 1) // tile


def bucket_lists(nodes, edges, weight, R, grid, tile: int, slab: int,
                 slabs=None):
    """CSR of the buckets of the slabs in `slabs` (a range, default all):
    (offsets int64 [n_slabs * nty * ntx + 1], ids int64 [pairs]).  Built by
    walking the edge list in order and appending each strut to every bucket
    it covers, then grouping stably by bucket."""
    r = strut_ranges(nodes, edges, weight, R, grid, tile, slab)
    ntx, nty = tiles_xy(grid, tile)
    n_slabs_all = (grid.n_slices + slab - 1) // slab
    if slabs is None:
        slabs = range(n_slabs_all)
    s_a, s_b = slabs.start, slabs.stop - 1
    per_slab = ntx * nty
    keys = []
    vals = []
    for p, i in enumerate(r["order"]):
        sa = max(int(r["slab0"][i]), s_a)
        sb = min(int(r["slab1"][i]), s_b)
        if sa > sb:
            continue
        ty = np.arange(r["ty0"][i], r["ty1"][i] + 1)
        tx = np.arange(r["tx0"][i], r["tx1"][i] + 1)
        T = (ty[:, None] * ntx + tx[None, :]).ravel()
        S = np.arange(sa, sb + 1) - s_a
        k = (S[:, None] * per_slab + T[None, :]).ravel()
        keys.append(k)
        vals.append(np.full(k.shape, i))
    n_buckets = (s_b - s_a + 1) * per_slab
    if keys:
        keys = np.concatenate(keys)
        vals = np.concatenate(vals)
        srt = np.argsort(keys, kind="stable")
        keys = keys[srt]
        vals = vals[srt]
    else:
        keys = np.zeros(0, np.int64)
        vals = np.zeros(0, np.int64)
    counts = np.bincount(keys, minlength=n_buckets)
    offsets = np.zeros(n_buckets + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return offsets, vals.astype(np.int64)


def bucket_of(r, i, s, ty, tx) -> bool:
    """Whether strut i belongs to bucket (slab s, tile ty, tx)."""
    return bool(r["binned"][i] and r["slab0"][i] <= s <= r["slab1"][i]
                and r["ty0"][i] <= ty <= r["ty1"][i]
                and r["tx0"][i] <= tx <= r["tx1"][i])
