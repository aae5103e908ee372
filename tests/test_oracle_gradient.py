"""Pins of the oracle's gradient against float64 central finite differences
of the oracle's field, and against the translation identity."""
import numpy as np
import pytest

from oracle import field as F
from oracle import gradient as G
from paper_2101_05031_amd import synth


def test_partials_match_finite_differences(rng):
    R = 1.4
    h = 1e-6
    n = 0
    for _ in range(80):
        a = rng.uniform(-1, 1, 3)
        b = a + rng.normal(0, 1.2, 3)
        P = 0.5 * (a + b) + rng.normal(0, 0.8, (4, 3))
        I, dA, dB = G.strut_partials(P, a, b, R)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fdA = (F.strut_integral(P, a + e, b, R) - F.strut_integral(P, a - e, b, R)) / (2 * h)
            fdB = (F.strut_integral(P, a, b + e, R) - F.strut_integral(P, a, b - e, R)) / (2 * h)
            np.testing.assert_allclose(dA[:, c], fdA, rtol=1e-6, atol=1e-8)
            np.testing.assert_allclose(dB[:, c], fdB, rtol=1e-6, atol=1e-8)
        n += np.count_nonzero(I)
    assert n > 100


def test_translation_identity(rng):
    """dI/da + dI/db = -dI/dp."""
    R = 1.1
    h = 1e-6
    for _ in range(40):
        a = rng.uniform(-1, 1, 3)
        b = a + rng.normal(0, 1.0, 3)
        P = 0.5 * (a + b) + rng.normal(0, 0.6, (3, 3))
        _, dA, dB = G.strut_partials(P, a, b, R)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            dp = (F.strut_integral(P + e, a, b, R) - F.strut_integral(P - e, a, b, R)) / (2 * h)
            np.testing.assert_allclose(dA[:, c] + dB[:, c], -dp, rtol=1e-6, atol=1e-8)


def test_vjp_matches_fd_of_loss():
    """Gradient of L = sum_p G(p) g(p) over a slice grid, per weight and per
    node coordinate, vs FP64 central differences (h = 1e-4 mm on positions,
    1e-4 * w on weights)."""
    lat = synth.kuhn_lattice(1, 4.0, seed=11, dtype=np.float64)
    grid = synth.grid_for(lat, 24, 24, 3)
    rng = np.random.default_rng(0)
    pts = []
    for k in range(grid.n_slices):
        X, Y = np.meshgrid(grid.pixel_x(), grid.pixel_y(), indexing="xy")
        pts.append(np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1).reshape(-1, 3))
    P = np.concatenate(pts)
    Gp = rng.normal(size=P.shape[0])

    def loss(nodes, w):
        return float(np.dot(Gp, F.field_at(P, nodes, lat.edges, w, lat.R)))

    gw, gn = G.field_vjp(P, Gp, lat.nodes, lat.edges, lat.weight, lat.R)
    for i in range(lat.n_edges):
        hw = 1e-4 * lat.weight[i]
        wp = lat.weight.copy(); wp[i] += hw
        wm = lat.weight.copy(); wm[i] -= hw
        fd = (loss(lat.nodes, wp) - loss(lat.nodes, wm)) / (2 * hw)
        assert gw[i] == pytest.approx(fd, rel=1e-7, abs=1e-9)
    for n in range(lat.n_nodes):
        for c in range(3):
            npl = lat.nodes.copy(); npl[n, c] += 1e-4
            nmi = lat.nodes.copy(); nmi[n, c] -= 1e-4
            fd = (loss(npl, lat.weight) - loss(nmi, lat.weight)) / 2e-4
            assert gn[n, c] == pytest.approx(fd, rel=1e-5, abs=1e-6)


def test_weight_gradient_is_integral():
    """dg/dr_i = I_i exactly (g is linear in the weights)."""
    lat = synth.tiny_lattice("tjoint")
    P = np.array([[0.1, 0.2, 0.3], [1.0, -0.4, 0.2], [-1.2, 0.3, 1.0]])
    for j in range(3):
        Gp = np.zeros(3); Gp[j] = 1.0
        gw, _ = G.field_vjp(P, Gp, lat.nodes, lat.edges, lat.weight, lat.R)
        for i in range(lat.n_edges):
            ref = F.strut_integral(P[j:j + 1], lat.nodes[lat.edges[i, 0]],
                                   lat.nodes[lat.edges[i, 1]], lat.R)[0]
            assert gw[i] == ref


def test_mirror_symmetry_of_gradients():
    lat = synth.tiny_lattice("mirror")
    P = np.array([[0.0, 0.3, 0.1], [0.0, 0.8, 0.4]])
    Gp = np.array([1.0, -0.5])
    gw, gn = G.field_vjp(P, Gp, lat.nodes, lat.edges, lat.weight, lat.R)
    assert gw[0] == pytest.approx(gw[1], rel=1e-12)
    np.testing.assert_allclose(gn[0] * [-1, 1, 1], gn[2], rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(gn[1] * [-1, 1, 1], gn[3], rtol=1e-10, atol=1e-14)


def test_soft_occupancy_loss_pins():
    """The per-pixel soft-occupancy loss: its gradient against central
    differences, equality with the voxel-density loss of one-sample voxels
    (a separate route), and the exp(-|z|) tails of the gradient."""
    from oracle import density as D
    rng = np.random.default_rng(8)
    g = rng.uniform(0.7, 1.3, size=(3, 5, 7))
    t = rng.uniform(0.0, 1.0, size=g.shape)
    tau, h = 0.05, 1e-6
    Gr = G.soft_occupancy_grad(g, t, 1.0, tau)
    for _ in range(20):
        k, y, x = (int(rng.integers(n)) for n in g.shape)
        p, q = g.copy(), g.copy()
        p[k, y, x] += h
        q[k, y, x] -= h
        fd = (G.soft_occupancy_loss(p, t, 1.0, tau) - G.soft_occupancy_loss(q, t, 1.0, tau)) / (2 * h)
        assert Gr[k, y, x] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    loss, _, grad = D.density_loss(g, t, 1.0, tau, 1, 1, 1)
    assert G.soft_occupancy_loss(g, t, 1.0, tau) == pytest.approx(loss, rel=1e-14)
    assert np.allclose(Gr, grad, rtol=1e-13, atol=0)
    deep = G.soft_occupancy_grad(np.array([1.0 + 70 * tau]), np.array([0.0]), 1.0, tau)[0]
    assert deep == pytest.approx(2.0 * np.exp(-70.0) / tau, rel=1e-12)
