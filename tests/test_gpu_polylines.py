"""GPU parity of slice_polylines (sub-pixel contours and chaining) with the
oracle (oracle/polylines.py), on the GPU's own field."""
import copy

import numpy as np
import pytest
import torch

from oracle import contours as OC
from oracle import polylines as PL
from paper_2101_05031_amd import _native as N
from paper_2101_05031_amd import api, synth

from gpu_util import bin_lattice

pytestmark = pytest.mark.gpu


def small_kuhn():
    lat = synth.kuhn_lattice(6, 24.0, seed=21)
    grid = synth.grid_for(lat, 301, 283, 27, dz=0.83)     # ragged W, H
    return lat, grid


def p1():
    lat, grid = synth.config("P1")
    return lat, grid


def _close(got, ref):
    """float32 output of a float64-exact value: a few units in the last place."""
    return np.all(np.abs(got - ref) <= 4e-7 * np.maximum(1.0, np.abs(ref)) + 1e-6)


def check_planes(lat, field, segs, off, chain, rank, what):
    fh = field.cpu().numpy().astype(np.float64)
    segs = segs.cpu().numpy().astype(np.float64)
    off = off.cpu().numpy()
    chain = chain.cpu().numpy()
    rank = rank.cpu().numpy()
    n_open = 0
    for k in range(fh.shape[0]):
        a, b = off[k], off[k + 1]
        ref = PL.segments_subpixel(fh[k], lat.C)
        assert b - a == len(ref), what
        assert _close(segs[a:b], ref), f"{what}: plane {k} endpoints"
        succ, rc, rr = PL.chains(fh[k] >= lat.C)
        assert np.array_equal(chain[a:b], rc), f"{what}: plane {k} chains"
        assert np.array_equal(rank[a:b], rr), f"{what}: plane {k} ranks"
        # joints coincide bitwise: s ends where its successor starts
        has = succ >= 0
        assert np.array_equal(segs[a:b][has, 2:], segs[a:b][succ[has], :2])
        n_open += int(np.sum(~has))
    return n_open


@pytest.mark.parametrize("case", ["kuhn", "P1"])
def test_polylines_match_oracle(case):
    lat, grid = {"kuhn": small_kuhn, "P1": p1}[case]()
    b = bin_lattice(lat, grid)
    nk = min(grid.n_slices, 10)
    f = api.slice_field(b, 0, nk)
    segs, off, chain, rank = api.slice_polylines(b, f)
    # same segments and order as slice_contours, endpoints moved
    msegs, moff, _ = api.slice_contours(b, f)
    assert torch.equal(off, moff) and len(segs) == len(msegs) > 0
    n_open = check_planes(lat, f, segs, off, chain, rank, case)
    assert n_open == 0                  # the grid's margin closes every contour


def test_polylines_open_chains_on_a_window():
    """A grid window that cuts through the lattice: contours leave the window,
    so chains start and end on its border."""
    lat, grid = small_kuhn()
    win = copy.copy(grid)
    win.x0 = grid.x0 + 90 * grid.dx
    win.y0 = grid.y0 + 70 * grid.dy
    win.W, win.H = 131, 117
    win.n_slices = 6
    b = bin_lattice(lat, win)
    f = api.slice_field(b, 0, win.n_slices)
    segs, off, chain, rank = api.slice_polylines(b, f)
    n_open = check_planes(lat, f, segs, off, chain, rank, "window")
    assert n_open > 0


def test_polylines_capacity_and_repeatability():
    lat, grid = small_kuhn()
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, 3, 4)
    segs, off, chain, rank = api.slice_polylines(b, f)
    segs2, off2, chain2, rank2 = api.slice_polylines(b, f)
    assert torch.equal(segs.view(torch.int32), segs2.view(torch.int32))
    assert torch.equal(chain, chain2) and torch.equal(rank, rank2)
    import ctypes
    t = ctypes.c_int64()
    small = torch.empty((len(segs) - 1, 4), dtype=torch.float32, device="cuda")
    o3 = torch.empty(5, dtype=torch.int64, device="cuda")
    st = N.lib().slice_polylines(b.handle, 4, api._ptr(f), api._ptr(small), len(segs) - 1,
                                 api._ptr(o3), None, None, ctypes.byref(t), api._stream())
    assert st == N.LSL_ECAPACITY and t.value == len(segs)
    assert torch.equal(o3, off)
    # without chains: the same segments
    s3, _, c3, r3 = api.slice_polylines(b, f, chains=False)
    assert c3 is None and torch.equal(s3.view(torch.int32), segs.view(torch.int32))
