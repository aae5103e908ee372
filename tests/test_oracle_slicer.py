"""Pins of the oracle's slicer, binning and marching squares."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import binning as B
from oracle import contours as C
from oracle import field as F
from oracle import slicer as S
from paper_2101_05031_amd import synth


def test_slice_heights_half_layer_then_one_layer_apart():
    z = S.slice_heights(2.0, 0.1, 5)
    # the first plane half a layer up, then one layer per plane (Sec. 4)
    ref = [2.0 + 0.05]
    for _ in range(4):
        ref.append(ref[-1] + 0.1)
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sweep_equals_eq8(seed):
    """The event sweep (sorted starts and ends of the swept spheres) gives
    exactly Eq. (8)'s sets."""
    lat = synth.random_lattice(60, 300, 20.0, seed=seed)
    zlo, zhi = S.strut_z_range(lat.nodes, lat.edges)
    heights = S.slice_heights(-3.0, 0.37, 80)
    sets = S.sweep_active_sets(zlo, zhi, lat.R, heights)
    for z, got in zip(heights, sets):
        ref = S.active_set(zlo, zhi, lat.R, z)
        assert np.array_equal(got, ref)


def test_active_set_is_complete():
    """Every strut with a non-zero term at some pixel of a plane is in that
    plane's active set."""
    lat = synth.kuhn_lattice(2, 10.0, seed=7)
    grid = synth.grid_for(lat, 48, 48, 20, dz=0.5)
    zlo, zhi = S.strut_z_range(lat.nodes, lat.edges)
    for k in range(0, grid.n_slices, 3):
        act = set(S.active_set(zlo, zhi, lat.R, grid.slice_z(k)).tolist())
        X, Y = np.meshgrid(grid.pixel_x(), grid.pixel_y(), indexing="xy")
        P = np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1)
        for i in range(lat.n_edges):
            I = F.strut_integral(P, lat.nodes[lat.edges[i, 0]], lat.nodes[lat.edges[i, 1]], lat.R)
            if np.any(I > 0):
                assert i in act


# ---------------------------------------------------------------- binning
def _bins_by_loops(lat, grid, T, Sz):
    """Independent re-derivation with Python scalars and math.floor/ceil."""
    nd = lat.nodes
    ntx, nty = B.tiles_xy(grid, T)
    nslab = (grid.n_slices + Sz - 1) // Sz
    lists = {}
    recs = []
    for i, (ia, ib) in enumerate(lat.edges):
        if lat.weight[i] == 0:
            continue
        a = [float(v) for v in nd[ia]]
        b = [float(v) for v in nd[ib]]
        if a == b:
            continue
        rng = []
        for ax, o, s, n in ((0, grid.x0, grid.dx, grid.W), (1, grid.y0, grid.dy, grid.H),
                            (2, grid.z0, grid.dz, grid.n_slices)):
            inv = 1.0 / s
            lo = min(a[ax], b[ax]) - lat.R
            hi = max(a[ax], b[ax]) + lat.R
            i0 = math.floor((lo - o) * inv - 0.5)
            i1 = math.ceil((hi - o) * inv - 0.5)
            i0 = max(i0, 0)
            i1 = min(i1, n - 1)
            rng.append((i0, i1))
        if any(r[0] > r[1] for r in rng):
            continue
        zlo_in = min(nd[ia][2], nd[ib][2])
        recs.append((zlo_in, i, rng))
    recs.sort(key=lambda r: (r[0], r[1]))
    for _, i, ((i0, i1), (j0, j1), (k0, k1)) in recs:
        for s in range(k0 // Sz, k1 // Sz + 1):
            for ty in range(j0 // T, j1 // T + 1):
                for tx in range(i0 // T, i1 // T + 1):
                    lists.setdefault((s * nty + ty) * ntx + tx, []).append(i)
    nb = nslab * ntx * nty
    off = [0]
    ids = []
    for key in range(nb):
        ids += lists.get(key, [])
        off.append(len(ids))
    return np.array(off), np.array(ids, dtype=np.int64)


@pytest.mark.parametrize("T,Sz", [(8, 1), (16, 4), (32, 8)])
def test_bucket_lists_match_loops(T, Sz):
    lat = synth.random_lattice(50, 400, 12.0, seed=3, zero_frac=0.1)
    lat.edges[5] = [7, 7]          # a zero-length strut
    grid = synth.Grid(-1.0, -2.0, 0.11, 0.13, 123, 101, -0.5, 0.21, 57)
    off, ids = B.bucket_lists(lat.nodes, lat.edges, lat.weight, lat.R, grid, T, Sz)
    off2, ids2 = _bins_by_loops(lat, grid, T, Sz)
    assert np.array_equal(off, off2)
    assert np.array_equal(ids, ids2)


def test_bucket_lists_group_equals_slice_of_full():
    lat = synth.random_lattice(40, 200, 10.0, seed=4)
    grid = synth.Grid(-1.0, -1.0, 0.1, 0.1, 130, 130, -1.0, 0.25, 60)
    T, Sz = 16, 4
    off, ids = B.bucket_lists(lat.nodes, lat.edges, lat.weight, lat.R, grid, T, Sz)
    ntx, nty = B.tiles_xy(grid, T)
    per = ntx * nty
    off2, ids2 = B.bucket_lists(lat.nodes, lat.edges, lat.weight, lat.R, grid, T, Sz,
                                slabs=range(3, 9))
    ref_ids = ids[off[3 * per]:off[9 * per]]
    assert np.array_equal(ids2, ref_ids)
    assert np.array_equal(off2, off[3 * per:9 * per + 1] - off[3 * per])


def test_binning_complete():
    """Every (pixel, strut) pair with a non-zero term has the strut in the
    bucket of the pixel's tile and slab."""
    lat = synth.kuhn_lattice(2, 8.0, seed=9)
    grid = synth.grid_for(lat, 64, 64, 24, dz=0.4)
    T, Sz = 8, 4
    r = B.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.R, grid, T, Sz)
    X, Y = np.meshgrid(grid.pixel_x(), grid.pixel_y(), indexing="xy")
    for k in range(0, grid.n_slices, 2):
        P = np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1)
        for i in range(lat.n_edges):
            I = F.strut_integral(P, lat.nodes[lat.edges[i, 0]], lat.nodes[lat.edges[i, 1]], lat.R)
            jj, ii = np.nonzero(I > 0)
            for j, i_ in zip(jj[::7], ii[::7]):
                assert B.bucket_of(r, i, k // Sz, j // T, i_ // T)


def test_edge_list_sorted_by_lower_z():
    lat = synth.random_lattice(80, 500, 15.0, seed=5)
    grid = synth.Grid(-2.0, -2.0, 0.2, 0.2, 100, 100, -2.0, 0.2, 100)
    r = B.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.R, grid, 16, 4)
    z = lat.nodes[:, 2]
    zlo = np.minimum(z[lat.edges[:, 0]], z[lat.edges[:, 1]])[r["order"]]
    assert np.all(np.diff(zlo) >= 0)
    ties = np.diff(zlo) == 0
    assert np.all(np.diff(r["order"])[ties] > 0)


# ---------------------------------------------------------------- contours
def _padded_random_image(rng, H, W, p):
    img = rng.uniform(size=(H, W)) < p
    img[0, :] = img[-1, :] = False
    img[:, 0] = img[:, -1] = False
    return img


def _loops(segs):
    nxt = {}
    indeg = {}
    for x0, y0, x1, y1 in segs:
        s, e = (x0, y0), (x1, y1)
        assert s not in nxt          # out-degree 1
        nxt[s] = e
        indeg[e] = indeg.get(e, 0) + 1
    assert all(v == 1 for v in indeg.values())   # in-degree 1
    assert set(indeg) == set(nxt)
    seen = set()
    n = 0
    for s in nxt:
        if s in seen:
            continue
        n += 1
        v = s
        while v not in seen:
            seen.add(v)
            v = nxt[v]
    return n


@pytest.mark.parametrize("p", [0.3, 0.5, 0.7])
def test_marching_squares_topology_and_area(rng, p):
    for _ in range(15):
        img = _padded_random_image(rng, 30, 37, p)
        segs = C.segments(img)
        # closed loops; #loops = 4-connected inside parts + holes
        n_loops = _loops(segs)
        n_in = ndimage.label(img, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])[1]
        lab_out, n_out = ndimage.label(~img, structure=np.ones((3, 3)))
        n_holes = n_out - 1            # the border-touching outside part
        assert n_loops == n_in + n_holes
        # shoelace area of all loops = sum of per-cell inside areas
        area = 0.5 * np.sum(segs[:, 0] * segs[:, 3] - segs[:, 2] * segs[:, 1])
        codes = C.case_codes(img)
        ref = sum(C.CASE_AREA[int(c)] for c in codes.ravel())
        assert area == pytest.approx(ref, abs=1e-9)


def test_marching_squares_inside_on_left():
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]
    edges = {C.B: (0, 1), C.E: (1, 2), C.T: (2, 3), C.L: (3, 0)}
    for case, segs in C.TABLE.items():
        bits = [(case >> k) & 1 for k in range(4)]
        crossing = {e for e, (i, j) in edges.items() if bits[i] != bits[j]}
        used = {pt for seg in segs for pt in seg}
        assert used == crossing
        for s, e in segs:
            for pt in (s, e):
                i, j = edges[pt]
                cin = corners[i] if bits[i] else corners[j]
                cross = (e[0] - s[0]) * (cin[1] - s[1]) - (e[1] - s[1]) * (cin[0] - s[0])
                assert cross > 0


def test_marching_squares_order_and_counts(rng):
    img = _padded_random_image(rng, 20, 25, 0.5)
    segs = C.segments(img)
    cnt = C.segment_counts(img)
    assert cnt.sum() == len(segs)
    # row-major cell order
    cell = np.floor(np.minimum(segs[:, 1], segs[:, 3])).astype(int) * 1000 + \
        np.floor(np.minimum(segs[:, 0], segs[:, 2])).astype(int)
    assert np.all(np.diff(cell) >= 0)
    # all coordinates are multiples of 1/2
    assert np.all((segs * 2) == np.round(segs * 2))
