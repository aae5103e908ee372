"""GPU parity on the degenerate geometry the closed form's "without loss of
generality" reading leaves open (Sec. 3.2, Eq. 7): planes exactly through
nodes and through a horizontal strut lying in the plane, a strut whose axis
passes through pixel centres (distance 0, H = R^2), pixel centres at exactly
distance R from a strut, and duplicated struts (the same edge twice, once
reversed).  The field, its classification and the adjoint are compared with
the oracle, and the field bits are compared across tilings."""
import numpy as np
import pytest
import torch

from oracle import contours as OC
from oracle import gradient as OG
from oracle import slicer as OS
from paper_2101_05031_amd import api, synth

from gpu_util import assert_field_close, bin_lattice, field_tol, unpack_bits

pytestmark = pytest.mark.gpu


def degenerate_case(dtype=np.float32):
    """Every coordinate below is a multiple of 1/8, exact in float32.
    Pixel centres: x = -3 + (i + 1/2)/4, y = -3 + (j + 1/2)/4; planes:
    z = (k + 1/2)/2, so the nodes at z = 0.25, 1.25, 2.25 lie on planes 0, 2
    and 4."""
    R = 1.0
    grid = synth.Grid(-3.0, -3.0, 0.25, 0.25, 26, 25, 0.0, 0.5, 7)
    px = lambda i: -3.0 + (i + 0.5) * 0.25            # noqa: E731
    nodes = np.array([
        [px(8), px(9), 0.25],       # 0: vertical strut 0-1 through pixel centres
        [px(8), px(9), 2.25],       # 1
        [-2.0, px(4), 1.25],        # 2: horizontal strut 2-3 in plane 2, along x,
        [1.5, px(4), 1.25],         # 3:   pixel rows j = 0 and 8 at exactly R
        [px(16), px(16), 0.25],     # 4: a node on plane 0 and on a pixel centre
        [px(20), px(12), 2.25],     # 5
        [px(12), px(20), 1.25],     # 6: node on plane 2
        [px(12), px(20), 1.25],     # 7: a second node at the same place
    ], dtype=dtype)
    edges = np.array([[0, 1], [2, 3], [4, 5], [4, 6], [6, 5],
                      [4, 6],        # duplicate of edge 3
                      [6, 4],        # and reversed
                      [2, 3],        # duplicate of the in-plane strut
                      [6, 7]],       # zero length (coincident nodes)
                     dtype=np.int32)
    rho = np.array([0.3, 0.35, 0.25, 0.3, 0.2, 0.3, 0.3, 0.35, 0.3])
    w = synth.weight_for_radius(rho, R).astype(dtype)
    lat = synth.Lattice(nodes, edges, w, R, 1.0, radius=rho)
    return lat, grid


def oracle_field(lat, grid, ks):
    return np.stack([OS.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k)
                     for k in ks])


def test_degenerate_case_is_what_it_says():
    """The construction: pixels on the axis, at exactly R, planes through
    nodes and through the horizontal strut (checked in float64)."""
    lat, grid = degenerate_case()
    n = lat.nodes.astype(np.float64)
    zs = grid.z0 + (np.arange(grid.n_slices) + 0.5) * grid.dz
    assert {0.25, 1.25, 2.25} <= set(zs.tolist())
    assert n[2, 2] == n[3, 2] == zs[2]
    assert n[0, 0] in grid.pixel_x() and n[0, 1] in grid.pixel_y()
    ys = grid.pixel_y()
    assert (n[2, 1] + lat.R) in ys and (n[2, 1] - lat.R) in ys


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_degenerate_field_and_contours(dtype):
    lat, grid = degenerate_case(dtype)
    ks = range(grid.n_slices)
    ref = oracle_field(lat, grid, ks)
    assert ref.max() > 2 * lat.C                     # overlapping struts
    base = None
    for tile, slab in ((8, 1), (16, 4), (32, 8), (16, 3)):
        print(f"degenerate {np.dtype(dtype).name} tile={tile} slab={slab}", flush=True)
        b = bin_lattice(lat, grid, tile=tile, slab=slab)
        f, bits = api.slice_field(b, 0, grid.n_slices, bits=True)
        fh = f.cpu().numpy()
        assert_field_close(fh, ref, lat.C, field_tol(dtype), "degenerate field")
        img = unpack_bits(bits, grid.W)
        assert np.array_equal(img, fh >= lat.C)
        sure = np.abs(ref - lat.C) > 1e-5
        assert np.array_equal(img[sure], (ref >= lat.C)[sure])
        if base is None:
            base = fh
        else:
            assert np.array_equal(fh.view(np.uint8), base.view(np.uint8))
        segs, off, _ = api.slice_contours(b, f)
        segs = segs.cpu().numpy().astype(np.float64)
        off = off.cpu().numpy()
        for k in ks:
            assert np.array_equal(segs[off[k]:off[k + 1]], OC.segments(fh[k] >= lat.C))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_degenerate_adjoint(dtype):
    lat, grid = degenerate_case(dtype)
    ks = range(grid.n_slices)
    G = np.random.default_rng(17).normal(size=(grid.n_slices, grid.H, grid.W)).astype(dtype)
    b = bin_lattice(lat, grid, tile=16, slab=4)
    gw, gn = api.slice_field_backward(b, 0, grid.n_slices, torch.from_numpy(G).cuda())
    rw, rn = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G)
    rtol = 1e-4 if dtype == np.float32 else 1e-10
    for got, ref, what in ((gw.cpu().numpy(), rw, "dL/dr"), (gn.cpu().numpy(), rn, "dL/dv")):
        got = np.asarray(got, dtype=np.float64).ravel()
        ref = np.asarray(ref, dtype=np.float64).ravel()
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        per = np.abs(got - ref) / scale
        norm = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"degenerate adjoint {what}: per-parameter {per.max():.2e}, normwise {norm:.2e}",
              flush=True)
        assert per.max() <= rtol and norm <= rtol
    # duplicated struts carry equal weight gradients (the reversed copy too)
    gwh = gw.cpu().numpy()
    assert gwh[3] == pytest.approx(gwh[5], rel=1e-6) and gwh[3] == pytest.approx(gwh[6], rel=1e-6)
    assert gwh[8] == 0.0                               # the zero-length strut is absent
