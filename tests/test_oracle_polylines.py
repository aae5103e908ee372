"""Pins of the sub-pixel contour and chaining oracle (oracle/polylines.py)
against exact geometry and topology."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import contours as C
from oracle import polylines as PL


def _grid(W, H):
    return np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))


def _shoelace(pts):
    x, y = pts[:, 0], pts[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


def _loops(segs, chain, rank):
    """Closed polygons (start points in rank order) of each chain."""
    out = {}
    for c in np.unique(chain):
        idx = np.nonzero(chain == c)[0]
        idx = idx[np.argsort(rank[idx])]
        out[int(c)] = segs[idx, :2]
    return out


@pytest.mark.parametrize("a,b,c", [(0.37, -0.81, 3.0), (1.0, 0.0, -7.25), (-0.2, 0.9, 1.5)])
def test_linear_field_crossings_lie_on_the_line(a, b, c):
    """Linear interpolation is exact for a linear field: every endpoint lies
    on a x + b y + c = C."""
    X, Y = _grid(23, 19)
    g = a * X + b * Y + c
    Cval = 0.5
    segs = PL.segments_subpixel(g, Cval)
    assert len(segs) > 5
    for x, y in np.concatenate([segs[:, :2], segs[:, 2:]]):
        assert abs(a * x + b * y + c - Cval) < 1e-12


def test_two_level_field_gives_midpoints():
    rng = np.random.default_rng(3)
    img = rng.random((21, 26)) < 0.5
    g = np.where(img, 2.0, 0.0)          # C +- 1: t = 1/2 on every edge
    assert np.array_equal(PL.segments_subpixel(g, 1.0), C.segments(img))


def test_circle_is_traced_closely():
    """g = r0^2 - |p - c|^2: the chained loop is a polygon inscribed close to
    the circle, enclosing about pi r0^2, oriented with the inside on the
    left (positive area)."""
    X, Y = _grid(40, 36)
    r0, cx, cy = 11.3, 19.4, 17.2
    g = r0 * r0 - (X - cx) ** 2 - (Y - cy) ** 2
    segs = PL.segments_subpixel(g, 0.0)
    d = np.hypot(segs[:, 0] - cx, segs[:, 1] - cy)
    assert np.max(np.abs(d - r0)) < 0.02                # quadratic error, well under a pixel
    mid = C.segments(g >= 0.0)
    dm = np.hypot(mid[:, 0] - cx, mid[:, 1] - cy)
    assert np.max(np.abs(dm - r0)) > 10 * np.max(np.abs(d - r0))
    succ, chain, rank = PL.chains(g >= 0.0)
    loops = _loops(segs, chain, rank)
    assert len(loops) == 1 and np.all(succ >= 0)
    area = _shoelace(next(iter(loops.values())))
    assert area == pytest.approx(np.pi * r0 * r0, rel=5e-3)   # inscribed: chords cut ~0.3%


def _padded_random_image(rng, H, W, p):
    img = np.zeros((H, W), dtype=bool)
    img[2:-2, 2:-2] = rng.random((H - 4, W - 4)) < p
    return img


@pytest.mark.parametrize("p", [0.3, 0.5, 0.7])
def test_closed_loops_match_topology(p):
    """Away from the border every contour closes: #chains = 4-connected
    inside parts + holes; consecutive segments share their joint exactly;
    ranks run 0..len-1 from the smallest index of each loop."""
    rng = np.random.default_rng(int(p * 10))
    for _ in range(10):
        img = _padded_random_image(rng, 27, 33, p)
        g = np.where(img, 1.0 + rng.random(img.shape), -rng.random(img.shape))
        segs = PL.segments_subpixel(g, 0.5)
        succ, chain, rank = PL.chains(img)
        assert np.all(succ >= 0)
        n_in = ndimage.label(img, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])[1]
        n_out = ndimage.label(~img, structure=np.ones((3, 3)))[1]
        assert len(np.unique(chain)) == n_in + n_out - 1
        assert np.array_equal(segs[:, 2:], segs[succ, :2])         # joints coincide
        for c in np.unique(chain):
            idx = np.nonzero(chain == c)[0]
            assert c == idx.min()
            assert np.array_equal(np.sort(rank[idx]), np.arange(len(idx)))
            first = idx[rank[idx] == 0][0]
            assert first == c


def test_open_chains_start_at_the_border():
    """A shape cut by the grid border gives open chains: each starts at a
    segment with no predecessor, on the border, and ends on the border."""
    rng = np.random.default_rng(9)
    img = rng.random((15, 18)) < 0.6
    img[:, 0] = True                                   # touches the left border
    succ, chain, rank = PL.chains(img)
    pred = np.full(len(succ), -1)
    pred[succ[succ >= 0]] = np.nonzero(succ >= 0)[0]
    heads = np.nonzero(pred < 0)[0]
    assert len(heads) > 0
    segs = C.segments(img)
    H, W = img.shape
    for h in heads:
        assert chain[h] == h and rank[h] == 0
        x, y = segs[h, :2]
        assert x in (0.0, W - 1.0) or y in (0.0, H - 1.0)
    tails = np.nonzero(succ < 0)[0]
    assert len(tails) == len(heads)
    for t in tails:
        x, y = segs[t, 2:]
        assert x in (0.0, W - 1.0) or y in (0.0, H - 1.0)
    # every segment is reached from its chain's start
    for s in range(len(succ)):
        h, r = chain[s], rank[s]
        q = h
        for _ in range(r):
            q = succ[q]
        assert q == s
