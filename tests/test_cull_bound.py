"""The reach test the field and adjoint kernels stage with, checked on the
CPU: for a flat 8x8 block of pixel centres around c and a segment whose
point nearest to c is F* (e = F* - c, D = |e|), every pixel c + d of the
block is at least D - (hx |e_x| + hy |e_y|) / D from the segment, with hx,
hy the block's half extents.  A strut the test drops therefore reaches no
pixel within R (the field is unchanged by the cull), and the test drops at
least every strut that the bounding circle of radius R + r_block drops."""
import numpy as np


def _seg_dist(P, a, b):
    u = b - a
    L2 = float(u @ u)
    t = np.clip((P - a) @ u / L2, 0.0, 1.0) if L2 > 0 else np.zeros(len(P))
    return np.linalg.norm(a + t[:, None] * u - P, axis=1)


def _reach(c, a, b, hx, hy, R):
    """(keep, D, bound): the kernels' test in float64, R widened by 1e-7."""
    u = b - a
    L = np.linalg.norm(u)
    u = u / L
    tc = (c - a) @ u
    F = a + np.clip(tc, 0.0, L) * u
    e = F - c
    D2 = float(e @ e)
    q = D2 - (hx * abs(e[0]) + hy * abs(e[1]))
    Rc = R * (1.0 + 1e-7)
    keep = q <= 0.0 or q * q < Rc * Rc * D2
    return keep, np.sqrt(D2), q


def test_bound_holds_and_drops_only_unreachable_struts():
    rng = np.random.default_rng(17)
    dx, dy, R = 0.049, 0.061, 1.5
    hx, hy = 3.5 * dx, 3.5 * dy
    rb = np.hypot(hx, hy)
    offs = np.array([[(i - 3.5) * dx, (j - 3.5) * dy, 0.0] for j in range(8) for i in range(8)])
    n_drop = n_circle = 0
    for trial in range(4000):
        c = rng.uniform(-1, 1, size=3)
        a = c + rng.normal(size=3) * 1.3
        b = a + rng.normal(size=3) * rng.choice([0.05, 1.0, 4.0])
        if np.allclose(a, b):
            continue
        keep, D, q = _reach(c, a, b, hx, hy, R)
        dist = _seg_dist(c + offs, a, b)
        # the bound itself: every pixel is at least D - h(n) away
        e_unit = None
        if D > 0:
            u = (b - a) / np.linalg.norm(b - a)
            F = a + np.clip((c - a) @ u, 0.0, np.linalg.norm(b - a)) * u
            e_unit = (F - c) / D
            lower = D - (hx * abs(e_unit[0]) + hy * abs(e_unit[1]))
            assert dist.min() >= lower - 1e-12
        if not keep:
            n_drop += 1
            assert dist.min() >= R              # nothing of the block within R
        if D >= R + rb:                         # the bounding circle drops it
            n_circle += 1
            assert not keep                     # so does the reach test
    assert n_drop > n_circle > 100               # strictly tighter on this sample


def test_struts_above_the_block_go_sooner_than_under_a_circle():
    """A strut parallel to the block, just over R above it: the circle keeps
    it (D < R + r_block), the flat block's support function drops it."""
    dx = dy = 0.05
    hx, hy = 3.5 * dx, 3.5 * dy
    R = 1.0
    c = np.zeros(3)
    a, b = np.array([-2.0, 0.3, R + 0.01]), np.array([2.0, 0.3, R + 0.01])
    keep, D, _ = _reach(c, a, b, hx, hy, R)
    assert D < R + np.hypot(hx, hy)
    assert not keep
    # a little lower it reaches the block and is kept
    keep2, _, _ = _reach(c, a - [0, 0, 0.02], b - [0, 0, 0.02], hx, hy, R)
    assert keep2
