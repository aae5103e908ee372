"""Pins of the per-voxel density oracle (oracle/density.py, Eq. 9)."""
import numpy as np
import pytest

from oracle import density as OD
from oracle import field as OF
from paper_2101_05031_amd import synth


def test_constant_and_half_space():
    f = np.full((5, 9, 13), 2.0)
    assert np.all(OD.voxel_density(f, 1.0, 4, 3, 2) == 1.0)
    assert np.all(OD.voxel_density(f, 3.0, 4, 3, 2) == 0.0)
    # inside where column >= 6: voxels of 4 columns hold 0, 2/4, 4/4, 1/1 inside
    g = np.zeros((3, 5, 13))
    g[:, :, 6:] = 1.0
    d = OD.voxel_density(g, 0.5, 4, 5, 3)
    assert d.shape == (1, 1, 4)
    assert np.array_equal(d[0, 0], [0.0, 0.5, 1.0, 1.0])


def test_brute_force_counts():
    rng = np.random.default_rng(1)
    f = rng.random((7, 11, 10))
    d = OD.voxel_density(f, 0.4, 3, 4, 2)
    for l in range(d.shape[0]):
        for j in range(d.shape[1]):
            for i in range(d.shape[2]):
                n = inn = 0
                for k in range(2 * l, min(2 * l + 2, 7)):
                    for y in range(4 * j, min(4 * j + 4, 11)):
                        for x in range(3 * i, min(3 * i + 3, 10)):
                            n += 1
                            inn += f[k, y, x] >= 0.4
                assert d[l, j, i] == pytest.approx(inn / n, abs=0)


def test_isolated_strut_density_is_its_cross_section():
    """A long vertical strut whose weight puts its iso-surface at radius rho
    fills pi rho^2 of the voxel's area, up to the sampling error of the pixel
    grid."""
    R, rho, C = 1.5, 0.8, 1.0
    w = synth.weight_for_radius(rho, R, C)
    nodes = np.array([[0.0, 0.0, -50.0], [0.0, 0.0, 50.0]])
    edges = np.array([[0, 1]], dtype=np.int32)
    side, n = 4.0, 200                       # a 4 mm voxel sampled by 200 x 200 pixels
    xs = -side / 2 + (np.arange(n) + 0.5) * side / n
    X, Y = np.meshgrid(xs, xs)
    P = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    g = OF.field_at(P, nodes, edges, np.array([w]), R).reshape(1, n, n)
    d = OD.voxel_density(g, C, n, n, 1)
    assert d[0, 0, 0] == pytest.approx(np.pi * rho * rho / side ** 2, abs=2 * 2 * np.pi * rho * (side / n) / side ** 2)


def test_soft_density_limits():
    rng = np.random.default_rng(3)
    f = rng.uniform(0.0, 2.0, size=(5, 9, 11))
    f[np.abs(f - 1.0) < 1e-3] = 1.5                      # keep samples off the iso-surface
    assert np.allclose(OD.soft_density(f, 1.0, 1e-6, 3, 4, 2), OD.voxel_density(f, 1.0, 3, 4, 2),
                       atol=1e-12, rtol=0)
    g = np.full((3, 4, 5), 1.0)
    t = rng.uniform(0, 1, size=(1, 2, 2))
    loss, rho, _ = OD.density_loss(g, t, 1.0, 0.05, 3, 3, 3)
    assert np.all(rho == 0.5)
    assert loss == pytest.approx(np.sum((0.5 - t) ** 2), rel=1e-15)


def test_density_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    f = rng.uniform(0.8, 1.2, size=(3, 7, 6))
    t = rng.uniform(0, 1, size=(2, 3, 2))
    tau, h = 0.05, 1e-6
    loss, _, grad = OD.density_loss(f, t, 1.0, tau, 4, 3, 2)
    for _ in range(25):
        k, y, x = (int(rng.integers(n)) for n in f.shape)
        p, q = f.copy(), f.copy()
        p[k, y, x] += h
        q[k, y, x] -= h
        fd = (OD.density_loss(p, t, 1.0, tau, 4, 3, 2)[0] -
              OD.density_loss(q, t, 1.0, tau, 4, 3, 2)[0]) / (2 * h)
        assert abs(fd - grad[k, y, x]) <= 1e-7 * max(1.0, abs(fd))


def test_density_gradient_deep_inside_and_outside():
    """Far from the iso-surface s (1 - s) is tiny but not zero: the gradient
    keeps its sign and size there, matching exp(-|z|) to leading order."""
    tau = 0.05
    g = np.array([[[1.0 + 70 * tau, 1.0 - 19 * tau]]])
    _, rho, grad = OD.density_loss(g, np.array([[[0.0]]]), 1.0, tau, 2, 1, 1)
    r = rho[0, 0, 0]
    assert grad[0, 0, 0] == pytest.approx(2 * r / 2 * np.exp(-70.0) / tau, rel=1e-12)
    assert grad[0, 0, 1] == pytest.approx(2 * r / 2 * np.exp(-19.0) / (1 + np.exp(-19.0)) ** 2 / tau,
                                          rel=1e-12)
