"""Pins of the oracle's kernel variants: per-strut supports and the compact
Gaussian kernel (oracle/field.py, slicer.py, binning.py, gradient.py)."""
import math

import numpy as np
import pytest

from oracle import binning as OB
from oracle import field as OF
from oracle import gradient as OG
from oracle import slicer as OS
from paper_2101_05031_amd import synth


def _long_strut():
    return np.array([[0.0, 0.0, -40.0], [0.0, 0.0, 40.0]]), np.array([[0, 1]], dtype=np.int32)


def test_per_strut_supports_reduce_to_one_support():
    lat = synth.random_lattice(30, 80, 6.0, seed=3, dtype=np.float64)
    rng = np.random.default_rng(1)
    P = rng.uniform(0, 6, size=(200, 3))
    one = OF.field_at(P, lat.nodes, lat.edges, lat.weight, lat.R)
    many = OF.field_at(P, lat.nodes, lat.edges, lat.weight, np.full(lat.n_edges, lat.R))
    assert np.array_equal(one, many)
    grid = synth.grid_for(lat, 61, 57, 9, dz=0.7)
    for k in (0, 4, 8):
        a = OS.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k)
        b = OS.slice_field(lat.nodes, lat.edges, lat.weight, np.full(lat.n_edges, lat.R), grid, k)
        assert np.array_equal(a, b)
    ra = OB.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.R, grid, 16, 4)
    rb = OB.strut_ranges(lat.nodes, lat.edges, lat.weight, np.full(lat.n_edges, lat.R), grid,
                         16, 4)
    assert np.array_equal(ra["order"], rb["order"])     # (slab, z, id) = (z, id) order here


def test_per_strut_support_closed_forms_and_quadrature():
    """Each strut uses its own R_j: the infinite-line value 16 h^5/(15 R_j^4),
    quadrature of Eq. (6) with R_j, and the weight convention putting each
    strut's surface at its own radius."""
    nodes, edges = _long_strut()
    for Rj, d in ((0.7, 0.3), (2.2, 1.9), (1.0, 0.0)):
        g = OF.field_at(np.array([[d, 0.0, 0.0]]), nodes, edges, [1.0], np.array([Rj]))[0]
        assert g == pytest.approx(16 * (Rj * Rj - d * d) ** 2.5 / (15 * Rj ** 4), rel=1e-13)
    rng = np.random.default_rng(4)
    lat = synth.random_lattice(12, 20, 4.0, seed=9, dtype=np.float64)
    Rs = rng.uniform(0.4, 1.6, size=lat.n_edges)
    for _ in range(20):
        p = rng.uniform(0, 4, size=3)
        g = OF.field_at(p[None], lat.nodes, lat.edges, lat.weight, Rs)[0]
        q = sum(lat.weight[j] * OF.line_integral_quadrature(p, lat.nodes[lat.edges[j, 0]],
                                                            lat.nodes[lat.edges[j, 1]], Rs[j])
                for j in range(lat.n_edges))
        assert g == pytest.approx(q, rel=1e-9, abs=1e-12)
    # two parallel long struts far apart, each with its own support and radius
    nodes = np.array([[0.0, 0, -40], [0.0, 0, 40], [10.0, 0, -40], [10.0, 0, 40]])
    edges = np.array([[0, 1], [2, 3]], dtype=np.int32)
    rho = np.array([0.3, 0.8])
    Rs = 1.5 * rho
    w = synth.weight_for_radius(rho, Rs)
    for j, x in ((0, 0.0), (1, 10.0)):
        g = OF.field_at(np.array([[x + rho[j], 0.0, 0.0]]), nodes, edges, w, Rs)[0]
        assert g == pytest.approx(1.0, rel=1e-12)


def test_per_strut_binning_order_and_sweep():
    lat = synth.with_supports(synth.kuhn_lattice(3, 12.0, seed=5, dtype=np.float64))
    grid = synth.grid_for(lat, 97, 91, 23, dz=0.6)
    for tile, slab in ((16, 4), (8, 1), (32, 16)):
        r = OB.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.support, grid, tile, slab)
        order = r["order"]
        s0 = r["slab0"][order]
        assert np.all(np.diff(s0) >= 0)                 # every slab's window is a prefix
        zlo = np.minimum(lat.nodes[lat.edges[:, 0], 2], lat.nodes[lat.edges[:, 1], 2])
        for a, b in zip(order[:-1], order[1:]):
            assert (s0_a := r["slab0"][a]) < r["slab0"][b] or (
                s0_a == r["slab0"][b] and (zlo[a], a) < (zlo[b], b))
        # bucket lists against a direct loop over (slab, tile, strut)
        off, ids = OB.bucket_lists(lat.nodes, lat.edges, lat.weight, lat.support, grid, tile,
                                   slab)
        ntx, nty = OB.tiles_xy(grid, tile)
        ns = (grid.n_slices + slab - 1) // slab
        for s in range(0, ns, max(1, ns // 3)):
            for ty in range(nty):
                for tx in range(ntx):
                    bk = (s * nty + ty) * ntx + tx
                    want = [i for i in order if OB.bucket_of(r, i, s, ty, tx)]
                    assert list(ids[off[bk]:off[bk + 1]]) == want
    # the event sweep, its starts ordered by z_lo - R_j, gives Eq. (8)'s sets
    zlo, zhi = OS.strut_z_range(lat.nodes, lat.edges)
    hs = OS.slice_heights(grid.z0, grid.dz, grid.n_slices)
    for z, got in zip(hs, OS.sweep_active_sets(zlo, zhi, lat.support, hs)):
        assert np.array_equal(got, OS.active_set(zlo, zhi, lat.support, z))


def test_per_strut_gradient_matches_finite_differences():
    lat = synth.random_lattice(10, 16, 3.0, seed=12, dtype=np.float64)
    rng = np.random.default_rng(6)
    Rs = rng.uniform(0.8, 1.6, size=lat.n_edges)
    P = rng.uniform(0, 3, size=(60, 3))
    G = rng.normal(size=60)
    gw, gn = OG.field_vjp(P, G, lat.nodes, lat.edges, lat.weight, Rs)
    h = 1e-6

    def L(nodes, w):
        return float(G @ OF.field_at(P, nodes, lat.edges, w, Rs))

    for j in range(0, lat.n_edges, 3):
        wp, wm = lat.weight.copy(), lat.weight.copy()
        wp[j] += h
        wm[j] -= h
        assert gw[j] == pytest.approx((L(lat.nodes, wp) - L(lat.nodes, wm)) / (2 * h),
                                      rel=1e-6, abs=1e-9)
    for n in range(0, lat.n_nodes, 2):
        for c in range(3):
            npp, nm = lat.nodes.copy(), lat.nodes.copy()
            npp[n, c] += h
            nm[n, c] -= h
            fd = (L(npp, lat.weight) - L(nm, lat.weight)) / (2 * h)
            assert gn[n, c] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_gauss_kernel_closed_form():
    """The compact Gaussian: zero at and beyond R (continuous), quadrature of
    the kernel along the edge, and the textbook line integral
    int exp(-t^2/2s^2) dt = s sqrt(2 pi) for an infinite line."""
    R, s = 1.5, 0.5
    assert OF.kernel_gauss(R, R, s) == 0.0 and OF.kernel_gauss(2.0, R, s) == 0.0
    assert OF.kernel_gauss(R - 1e-9, R, s) == pytest.approx(0.0, abs=1e-8)
    assert OF.kernel_gauss(0.0, R, s) == pytest.approx(1 - math.exp(-4.5), rel=1e-15)
    rng = np.random.default_rng(2)
    for _ in range(30):
        p = rng.uniform(-1, 1, size=3)
        a = rng.uniform(-2, 2, size=3)
        b = a + rng.uniform(-2, 2, size=3)
        got = float(OF.strut_integral_gauss(p, a, b, R, s))
        q = OF.line_integral_quadrature(p, a, b, R, kind="gauss", sigma=s)
        assert got == pytest.approx(q, rel=1e-9, abs=1e-12)
    nodes, edges = _long_strut()
    for d in (0.0, 0.4, 1.2):
        g = OF.field_at(np.array([[d, 0, 0]]), nodes, edges, [1.0], R, kind="gauss", sigma=s)[0]
        h = math.sqrt(R * R - d * d)
        want = (math.exp(-d * d / (2 * s * s)) * s * math.sqrt(2 * math.pi) *
                math.erf(h / (s * math.sqrt(2))) - math.exp(-R * R / (2 * s * s)) * 2 * h)
        assert g == pytest.approx(want, rel=1e-12)
    # wide support: the truncated integral tends to the full Gaussian's
    g = OF.field_at(np.array([[0.0, 0, 0]]), nodes, edges, [1.0], 12 * s, kind="gauss",
                    sigma=s)[0]
    assert g == pytest.approx(s * math.sqrt(2 * math.pi), rel=1e-12)
    # the weight convention puts an isolated strut's surface at its radius
    w = synth.weight_for_radius_gauss(0.4, R, s)
    g = OF.field_at(np.array([[0.4, 0, 0]]), nodes, edges, [w], R, kind="gauss", sigma=s)[0]
    assert g == pytest.approx(1.0, rel=1e-12)
