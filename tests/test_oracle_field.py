"""Pins of the oracle's field (Eqs. 5-7) against things other than itself:
numerical quadrature of the definition, closed-form special cases, geometric
invariants, brute force, and the radius -> weight input convention."""
import numpy as np
import pytest

from oracle import field as F
from oracle import slicer as S
from paper_2101_05031_amd import synth


def _rand_case(rng, R):
    a = rng.uniform(-2, 2, 3)
    b = a + rng.normal(0, 1.5, 3)
    p = 0.5 * (a + b) + rng.normal(0, 0.6 * R, 3)
    return p, a, b


def test_closed_form_matches_quadrature(rng):
    """Eq. (6) by adaptive quadrature along the edge vs the closed form."""
    worst = 0.0
    n_nonzero = 0
    for _ in range(200):
        R = rng.uniform(0.5, 2.0)
        p, a, b = _rand_case(rng, R)
        ref = F.line_integral_quadrature(p, a, b, R)
        got = float(F.strut_integral(p[None], a, b, R)[0])
        if ref == 0.0:
            assert got == 0.0
            continue
        n_nonzero += 1
        worst = max(worst, abs(got - ref) / abs(ref))
    assert n_nonzero > 100
    assert worst < 1e-9


def test_printed_form_lacks_arclength_jacobian(rng):
    """The s-integral printed in Eq. (7) equals the arclength integral of
    Eq. (6) divided by the chord length l = 2h (so the oracle's factor l is
    the Jacobian of x(s), not a scale error)."""
    for _ in range(50):
        R = 1.3
        p, a, b = _rand_case(rng, R)
        u = (b - a) / np.linalg.norm(b - a)
        t0 = np.dot(p - a, u)
        dp2 = np.dot(p - a - t0 * u, p - a - t0 * u)
        if dp2 >= R * R:
            continue
        h = np.sqrt(R * R - dp2)
        # direct quadrature of the printed s-integrand over [s1, s2]
        from scipy.integrate import quad
        p1 = a + (t0 - h) * u
        p2 = a + (t0 + h) * u
        l2 = np.dot(p2 - p1, p2 - p1)
        s1 = max(0.0, np.dot(a - p1, p2 - p1) / l2)
        s2 = min(1.0, np.dot(b - p1, p2 - p1) / l2)
        if s2 <= s1:
            continue
        val, _ = quad(lambda s: (1 - np.dot(p - ((1 - s) * p1 + s * p2),
                                            p - ((1 - s) * p1 + s * p2)) / R**2) ** 2,
                      s1, s2, epsabs=1e-14, epsrel=1e-12)
        got = float(F.strut_integral(p[None], a, b, R)[0])
        assert got == pytest.approx(2 * h * val, rel=1e-9, abs=1e-14)


@pytest.mark.parametrize("R,d", [(1.3, 0.4), (1.5, 0.0), (0.75, 0.5), (2.0, 1.99)])
def test_infinite_line(R, d):
    """Both ends far outside the support: 16 (R^2-d^2)^(5/2) / (15 R^4)."""
    a = np.array([-50.0, 0.0, 0.0])
    b = np.array([50.0, 0.0, 0.0])
    p = np.array([[0.3, d, 0.0]])
    got = float(F.strut_integral(p, a, b, R)[0])
    ref = 16.0 * (R * R - d * d) ** 2.5 / (15.0 * R ** 4)
    assert got == pytest.approx(ref, rel=1e-12)


def test_axis_point_and_half_strut():
    R = 1.5
    a = np.array([0.0, 0.0, -10.0])
    b = np.array([0.0, 0.0, 10.0])
    # on the axis, mid strut: integral of (1 - t^2/R^2)^2 over [-R, R] = 16R/15
    assert float(F.strut_integral(np.array([[0.0, 0.0, 0.0]]), a, b, R)[0]) == \
        pytest.approx(16 * R / 15, rel=1e-13)
    # foot exactly at an end: half of the infinite-line value
    p = np.array([[0.7, 0.0, 10.0]])
    ref = 0.5 * 16.0 * (R * R - 0.49) ** 2.5 / (15.0 * R ** 4)
    assert float(F.strut_integral(p, a, b, R)[0]) == pytest.approx(ref, rel=1e-12)


def test_zero_outside_support(rng):
    R = 1.1
    for _ in range(100):
        a = rng.uniform(-3, 3, 3)
        b = rng.uniform(-3, 3, 3)
        # points at distance >= R from the segment
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        t = rng.uniform(0, 1)
        base = a + t * (b - a)
        p = base + u * rng.uniform(R, R + 3)
        seg = b - a
        tt = np.clip(np.dot(p - a, seg) / np.dot(seg, seg), 0, 1)
        if np.linalg.norm(p - (a + tt * seg)) < R:
            continue
        assert float(F.strut_integral(p[None], a, b, R)[0]) == 0.0
    # zero-length strut
    assert float(F.strut_integral(np.zeros((1, 3)), np.ones(3), np.ones(3), R)[0]) == 0.0


def test_invariants(rng):
    """Reversal, mirror, translation, collinear split, and scaling by lambda
    (arclength integral => the value scales by lambda)."""
    R = 1.2
    for _ in range(60):
        p, a, b = _rand_case(rng, R)
        P = p[None]
        I = float(F.strut_integral(P, a, b, R)[0])
        assert float(F.strut_integral(P, b, a, R)[0]) == pytest.approx(I, rel=1e-12, abs=1e-15)
        M = np.array([-1.0, 1.0, 1.0])
        assert float(F.strut_integral(P * M, a * M, b * M, R)[0]) == \
            pytest.approx(I, rel=1e-12, abs=1e-15)
        t = rng.uniform(-100, 100, 3)
        assert float(F.strut_integral(P + t, a + t, b + t, R)[0]) == \
            pytest.approx(I, rel=1e-9, abs=1e-12)
        c = a + rng.uniform(0.1, 0.9) * (b - a)
        split = float(F.strut_integral(P, a, c, R)[0]) + float(F.strut_integral(P, c, b, R)[0])
        assert split == pytest.approx(I, rel=1e-11, abs=1e-14)
        lam = rng.uniform(0.3, 3.0)
        assert float(F.strut_integral(P * lam, a * lam, b * lam, R * lam)[0]) == \
            pytest.approx(lam * I, rel=1e-11, abs=1e-14)


def test_kernel_eq5():
    R = 2.0
    d = np.array([0.0, 1.0, 1.999, 2.0, 3.0])
    np.testing.assert_allclose(F.kernel(d, R), [1.0, (1 - 0.25) ** 2,
                                                (1 - 1.999 ** 2 / 4) ** 2, 0.0, 0.0])


@pytest.mark.parametrize("kind", ["one", "collinear", "tjoint", "mirror"])
def test_brute_equals_culled_bitwise(kind):
    """All-pairs sum over every strut equals the active-set, windowed sum of
    the slicer bit for bit (omitted terms are exact zeros)."""
    lat = synth.tiny_lattice(kind)
    grid = synth.grid_for(lat, 40, 36, 12, dz=0.31)
    xs, ys = grid.pixel_x(), grid.pixel_y()
    for k in range(grid.n_slices):
        X, Y = np.meshgrid(xs, ys, indexing="xy")
        P = np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1)
        brute = F.field_at(P, lat.nodes, lat.edges, lat.weight, lat.R)
        culled = S.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k)
        assert np.array_equal(brute, culled)


def test_brute_equals_culled_bcc_cell():
    lat = synth.bcc_lattice(1, 5.0, 0.5)
    grid = synth.grid_for(lat, 48, 48, 6, dz=0.9)
    xs, ys = grid.pixel_x(), grid.pixel_y()
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    for k in range(grid.n_slices):
        P = np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1)
        brute = F.field_at(P, lat.nodes, lat.edges, lat.weight, lat.R)
        culled = S.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k)
        assert np.array_equal(brute, culled)
        assert brute.max() > 0


def test_radius_to_weight_places_iso_surface():
    """An isolated long strut with weight w(rho) has g = C at distance rho."""
    R = 1.5
    for rho in (0.2, 0.5, 0.99):
        w = float(synth.weight_for_radius(rho, R))
        a = np.array([0.0, 0.0, -40.0])
        b = np.array([0.0, 0.0, 40.0])
        g = w * float(F.strut_integral(np.array([[rho, 0.0, 0.3]]), a, b, R)[0])
        assert g == pytest.approx(1.0, rel=1e-12)
        # inside at smaller distance, outside at larger
        gi = w * float(F.strut_integral(np.array([[rho * 0.99, 0, 0]]), a, b, R)[0])
        go = w * float(F.strut_integral(np.array([[rho * 1.01, 0, 0]]), a, b, R)[0])
        assert gi > 1.0 > go


def test_smaller_weight_thinner_strut():
    """Sec. 3.2: decreasing r_i moves the iso-surface towards the edge."""
    R = 1.5
    a = np.array([0.0, 0.0, -40.0])
    b = np.array([0.0, 0.0, 40.0])
    d = np.linspace(0, R, 3001)[:-1]
    P = np.stack([d, 0 * d, 0 * d], 1)
    I = F.strut_integral(P, a, b, R)
    radii = []
    for w in (1.0, 1.5, 2.0, 3.0):
        radii.append(d[np.nonzero(w * I >= 1.0)[0].max()])
    assert all(r1 < r2 for r1, r2 in zip(radii, radii[1:]))
