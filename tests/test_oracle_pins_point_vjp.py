"""Pins of the two oracle routes the full-size GPU checks lean on:
field_at_point (one point, every strut at once; Eq. 6) and slice_vjp (the
gradient over a slice grid, windowed per strut; the radius-tuning step of
Sec. 5.3).  Each is held to a route of different construction: the per-strut
loop of field_at, the windowed plane sum of slice_field, adaptive quadrature
of Eq. (6), the all-pixel field_vjp, and float64 central differences of the
loss."""
import numpy as np
import pytest

from oracle import field as F
from oracle import gradient as G
from oracle import slicer as S
from paper_2101_05031_amd import synth


def _lattice_crossing_border():
    """A small jittered Kuhn lattice whose grid window cuts struts (some
    struts leave the grid), float64."""
    lat = synth.kuhn_lattice(2, 8.0, seed=41, dtype=np.float64)
    grid = synth.grid_for(lat, 40, 36, 6)
    # shrink the window so that struts cross its border
    grid = synth.Grid(grid.x0 + 6 * grid.dx, grid.y0 + 5 * grid.dy, grid.dx, grid.dy,
                      28, 26, grid.z0, grid.dz, grid.n_slices)
    return lat, grid


def _variants():
    lat, grid = _lattice_crossing_border()
    yield "one support", lat, lat.R, "quartic", None
    sup = synth.with_supports(lat)
    yield "per-strut supports", sup, sup.support.astype(np.float64), "quartic", None
    gs = synth.with_gauss(lat)
    yield "gaussian", gs, gs.R, "gauss", gs.sigma


@pytest.mark.parametrize("case", ["one support", "per-strut supports", "gaussian"])
def test_field_at_point_equals_field_at_and_slice_field(case):
    lat, grid = _lattice_crossing_border()
    _, lat, R, kind, sigma = next(v for v in _variants() if v[0] == case)
    rng = np.random.default_rng(3)
    for k in (0, 2, 5):
        plane = S.slice_field(lat.nodes, lat.edges, lat.weight, R, grid, k, kind=kind,
                              sigma=sigma)
        js = rng.integers(0, grid.H, 25)
        is_ = rng.integers(0, grid.W, 25)
        P = S.slice_points(grid, k, is_, js)
        via_loop = F.field_at(P, lat.nodes, lat.edges, lat.weight, R, kind=kind, sigma=sigma)
        for n in range(len(P)):
            g = F.field_at_point(P[n], lat.nodes, lat.edges, lat.weight, R, kind=kind,
                                 sigma=sigma)
            for ref in (via_loop[n], plane[js[n], is_[n]]):
                assert abs(g - ref) <= 1e-15 * max(abs(ref), 1.0)
        assert np.count_nonzero(plane) > 50        # the sample sees the lattice


def test_field_at_point_matches_quadrature():
    """field_at_point against the weighted sum of adaptive quadratures of the
    kernel along each strut (Eq. 6 integrated numerically)."""
    lat = synth.tiny_lattice("tjoint")
    rng = np.random.default_rng(9)
    for _ in range(12):
        p = rng.uniform(-1.0, 1.0, 3)
        got = F.field_at_point(p, lat.nodes, lat.edges, lat.weight, lat.R)
        ref = sum(lat.weight[i] * F.line_integral_quadrature(
            p, lat.nodes[lat.edges[i, 0]], lat.nodes[lat.edges[i, 1]], lat.R)
            for i in range(lat.n_edges))
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-12)


def _grid_points(grid, ks):
    pts = []
    for k in ks:
        X, Y = np.meshgrid(grid.pixel_x(), grid.pixel_y(), indexing="xy")
        pts.append(np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1).reshape(-1, 3))
    return np.concatenate(pts)


@pytest.mark.parametrize("case", ["one support", "per-strut supports"])
def test_slice_vjp_equals_field_vjp(case):
    """The windowed per-plane route equals the all-pixel route."""
    _, lat, R, _, _ = next(v for v in _variants() if v[0] == case)
    _, grid = _lattice_crossing_border()
    ks = range(grid.n_slices)
    rng = np.random.default_rng(6)
    Gs = rng.normal(size=(len(ks), grid.H, grid.W))
    gw, gn = G.slice_vjp(lat.nodes, lat.edges, lat.weight, R, grid, ks, Gs)
    rw, rn = G.field_vjp(_grid_points(grid, ks), Gs.reshape(-1), lat.nodes, lat.edges,
                         lat.weight, R)
    assert np.abs(gw).max() > 0 and np.abs(gn).max() > 0
    np.testing.assert_allclose(gw, rw, rtol=1e-12, atol=1e-12 * np.abs(rw).max())
    np.testing.assert_allclose(gn, rn, rtol=1e-12, atol=1e-12 * np.abs(rn).max())


def test_slice_vjp_matches_finite_differences():
    """slice_vjp against central differences of L = sum G g over the planes
    (slice_field), per weight (h = 1e-4 w) and per node coordinate
    (h = 1e-4 mm)."""
    lat = synth.kuhn_lattice(1, 4.0, seed=12, dtype=np.float64)
    grid = synth.grid_for(lat, 22, 20, 3)
    ks = range(grid.n_slices)
    Gs = np.random.default_rng(2).normal(size=(len(ks), grid.H, grid.W))

    def loss(nodes, w):
        return sum(float(np.sum(Gs[kk] * S.slice_field(nodes, lat.edges, w, lat.R, grid, k)))
                   for kk, k in enumerate(ks))

    gw, gn = G.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, Gs)
    for i in range(lat.n_edges):
        h = 1e-4 * lat.weight[i]
        wp, wm = lat.weight.copy(), lat.weight.copy()
        wp[i] += h
        wm[i] -= h
        fd = (loss(lat.nodes, wp) - loss(lat.nodes, wm)) / (2 * h)
        assert gw[i] == pytest.approx(fd, rel=1e-7, abs=1e-9)
    for n in range(lat.n_nodes):
        for c in range(3):
            npl, nmi = lat.nodes.copy(), lat.nodes.copy()
            npl[n, c] += 1e-4
            nmi[n, c] -= 1e-4
            fd = (loss(npl, lat.weight) - loss(nmi, lat.weight)) / 2e-4
            assert gn[n, c] == pytest.approx(fd, rel=1e-5, abs=1e-6)


def test_slice_vjp_restricted_to_struts():
    """With `struts`, the listed struts' weight gradients are exact, and so is
    the gradient of every node whose struts are all listed."""
    lat, grid = _lattice_crossing_border()
    ks = range(1, 4)
    Gs = np.random.default_rng(7).normal(size=(len(ks), grid.H, grid.W))
    gw, gn = G.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, Gs)
    node = 4
    sub = np.nonzero((lat.edges[:, 0] == node) | (lat.edges[:, 1] == node))[0]
    sw, sn = G.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, Gs, struts=sub)
    np.testing.assert_array_equal(sw[sub], gw[sub])
    other = np.setdiff1d(np.arange(lat.n_edges), sub)
    assert not sw[other].any()
    np.testing.assert_allclose(sn[node], gn[node], rtol=1e-13, atol=1e-15)


def test_zero_weight_strut_has_the_linear_gradient():
    """A strut of weight 0 contributes nothing, but Eq. (6) is linear in its
    weight, so dL/dr = sum_p G I (central differences through r = 0, which
    the field evaluates for negative r as well)."""
    lat = synth.kuhn_lattice(1, 4.0, seed=13, dtype=np.float64)
    grid = synth.grid_for(lat, 22, 20, 3)
    w0 = lat.weight.copy()
    w0[[2, 5]] = 0.0
    ks = range(grid.n_slices)
    Gs = np.random.default_rng(4).normal(size=(len(ks), grid.H, grid.W))

    def loss(w):
        return sum(float(np.sum(Gs[kk] * np.stack([
            F.field_at(S.slice_points(grid, k, *np.meshgrid(np.arange(grid.W), np.arange(grid.H),
                                                               indexing="xy")).reshape(-1, 3),
                       lat.nodes, lat.edges, w, lat.R).reshape(grid.H, grid.W)])[0]))
                   for kk, k in enumerate(ks))

    gw, _ = G.slice_vjp(lat.nodes, lat.edges, w0, lat.R, grid, ks, Gs)
    for i in (2, 5):
        h = 1e-3
        wp, wm = w0.copy(), w0.copy()
        wp[i] += h
        wm[i] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert abs(fd) > 1e-6                    # the strut matters to the loss
        assert gw[i] == pytest.approx(fd, rel=1e-7, abs=1e-10)
