"""Pins of the self-support oracle (oracle/support.py: Sec. 5.2, Eqs. 11-14,
Appendix II)."""
import numpy as np
import pytest

from oracle import support as SP


def test_polynomial_fits_the_exact_ratio():
    """Eq. (12) approximates Appendix II's arc-length ratio (quadrature): a
    wrong or mistyped coefficient moves it far off this band."""
    th = np.linspace(0.9, np.pi / 2, 40)
    ex = np.array([SP.g_exact(t) for t in th])
    assert np.max(np.abs(SP.g_poly(th) - ex)) < 0.04
    # the exact ratio: 0 up to alpha, 1/sqrt(2) for a horizontal strut
    assert SP.g_exact(SP.ALPHA - 1e-9) == 0.0
    assert SP.g_exact(np.pi / 2) == pytest.approx(np.sqrt(0.5), abs=1e-9)
    assert SP.g_poly(0.5) == 0.0 and SP.g_poly(np.pi / 4) == 0.0


def test_theta_of_a_tilted_strut():
    nodes = np.array([[0.0, 0, 0], [np.sin(np.pi / 3), 0, np.cos(np.pi / 3)]])
    L, u, c, theta, ok = SP.edge_geometry(nodes, np.array([[0, 1]]), [0, 0, 1])
    assert theta[0] == pytest.approx(np.pi / 3, abs=1e-12)
    L, u, c, theta, ok = SP.edge_geometry(nodes, np.array([[1, 0]]), [0, 0, 1])
    assert theta[0] == pytest.approx(np.pi / 3, abs=1e-12)      # |u . t|: orientation free


def _lattice(rng, n=40, m=90):
    nodes = rng.uniform(0, 10, size=(n, 3))
    e = rng.integers(0, n, size=(m, 2))
    e = e[e[:, 0] != e[:, 1]].astype(np.int32)
    w = rng.uniform(0.1, 1.0, size=len(e))
    return nodes, e, w


def test_vertical_horizontal_and_mixed():
    t = np.array([0.0, 0.0, 1.0])
    nodes = np.array([[0, 0, 0], [0, 0, 2.0], [3.0, 0, 0], [3.0, 0.0, 5.0], [7.0, 0, 0]])
    vert = np.array([[0, 1], [2, 3]], dtype=np.int32)
    horiz = np.array([[0, 2], [2, 4]], dtype=np.int32)
    m = SP.metrics(nodes, vert, [0.5, 0.7], t)
    assert m["gamma"] == 0.0 and m["psi"] == 100.0
    m = SP.metrics(nodes, horiz, [0.5, 0.7], t)
    g90 = sum(a * (np.pi / 2) ** i for i, a in enumerate(SP.A))
    assert m["psi"] == 0.0 and m["gamma"] == pytest.approx(g90, abs=1e-12)
    both = np.concatenate([vert, horiz])
    r = np.array([0.5, 0.7, 0.2, 0.9])
    m = SP.metrics(nodes, both, r, t)
    Lv, Lh = np.array([2.0, 5.0]), np.array([3.0, 4.0])
    assert m["gamma"] == pytest.approx(g90 * (0.2 * 3 + 0.9 * 4) /
                                       (0.5 * 2 + 0.7 * 5 + 0.2 * 3 + 0.9 * 4), abs=1e-12)
    assert m["psi"] == pytest.approx(100 * Lv.sum() / (Lv.sum() + Lh.sum()), abs=1e-12)


def test_invariances():
    rng = np.random.default_rng(2)
    nodes, e, w = _lattice(rng)
    t = np.array([0.0, 0.0, 1.0])
    m0 = SP.metrics(nodes, e, w, t)
    a = 0.73
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1.0]])
    for moved in (nodes @ Rz.T, nodes * 3.7, nodes + [4.0, -2.0, 9.0]):
        m1 = SP.metrics(moved, e, w, t)
        assert m1["gamma"] == pytest.approx(m0["gamma"], abs=1e-12)
        assert m1["psi"] == pytest.approx(m0["psi"], abs=1e-12)
    m2 = SP.metrics(nodes, e[:, ::-1].copy(), w, t)
    assert m2["gamma"] == pytest.approx(m0["gamma"], abs=1e-12)
    # a general printing direction: rotate the lattice and the direction together
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    m3 = SP.metrics(nodes @ R.T, e, w, R @ t)
    assert m3["gamma"] == pytest.approx(m0["gamma"], abs=1e-12)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    nodes, e, w = _lattice(rng, 25, 60)
    t = np.array([0.3, -0.2, 0.9])
    t = t / np.linalg.norm(t)
    L, u, c, theta, ok = SP.edge_geometry(nodes, e, t)
    assert np.min(np.abs(theta - SP.ALPHA)) > 1e-3          # away from the step of g
    gr = SP.gamma_grad(nodes, e, w, t)
    h = 1e-6
    for _ in range(30):
        i, k = int(rng.integers(len(nodes))), int(rng.integers(3))
        p, q = nodes.copy(), nodes.copy()
        p[i, k] += h
        q[i, k] -= h
        fd = (SP.metrics(p, e, w, t)["gamma"] - SP.metrics(q, e, w, t)["gamma"]) / (2 * h)
        assert abs(fd - gr[i, k]) <= 1e-6 * max(1.0, abs(fd))
    # Gamma is invariant under translation and rotation about t
    assert np.allclose(gr.sum(axis=0), 0.0, atol=1e-12)
    torque = np.cross(nodes, gr).sum(axis=0) @ t
    assert abs(torque) < 1e-10
