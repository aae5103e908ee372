"""GPU parity of the binning, field, binary image and contour passes against
the FP64 oracle (bit-exact for integer work, tolerance-bound for the field)."""
import numpy as np
import pytest
import torch

from oracle import binning as OB
from oracle import contours as OC
from oracle import field as OF
from oracle import slicer as OS
from paper_2101_05031_amd import _native as N
from paper_2101_05031_amd import api, synth

from gpu_util import assert_field_close, bin_lattice, field_tol, to_dev, unpack_bits

pytestmark = pytest.mark.gpu


def small_kuhn():
    lat = synth.kuhn_lattice(6, 24.0, seed=21)
    grid = synth.grid_for(lat, 301, 283, 27, dz=0.83)     # ragged W, H and slabs
    return lat, grid


def random_edge_cases():
    lat = synth.random_lattice(70, 500, 14.0, seed=8, zero_frac=0.1)
    lat.edges[3] = [5, 5]            # zero length
    lat.edges[4] = [6, 6]
    lat.nodes[69] = [500.0, 500.0, 500.0]     # struts to this node leave the grid
    grid = synth.Grid(-1.5, -2.0, 0.07, 0.09, 211, 179, -1.0, 0.31, 53)
    return lat, grid


CASES = {
    "P1": lambda: synth.config("P1"),
    "kuhn": small_kuhn,
    "random": random_edge_cases,
}


def oracle_field(lat, grid, ks):
    return np.stack([OS.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k)
                     for k in ks])


# ------------------------------------------------------------------ binning
@pytest.mark.parametrize("case,tile,slab,max_pairs", [
    ("P1", 16, 8, 0), ("kuhn", 16, 4, 0), ("kuhn", 8, 1, 0), ("kuhn", 32, 16, 0),
    ("kuhn", 16, 2, 3000), ("random", 64, 3, 0), ("random", 8, 5, 1500),
])
def test_bins_match_oracle(case, tile, slab, max_pairs):
    lat, grid = CASES[case]()
    print(f"bins {case} tile={tile} slab={slab} max_pairs={max_pairs}", flush=True)
    b = bin_lattice(lat, grid, tile=tile, slab=slab, max_pairs=max_pairs)
    info = b.info()
    r = OB.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.R, grid, tile, slab)
    assert info["n_binned"] == len(r["order"])
    assert np.array_equal(b.order().cpu().numpy(), r["order"])
    if max_pairs:
        assert info["n_groups"] > 1
    n_slabs = (grid.n_slices + slab - 1) // slab
    covered = []
    for g in range(info["n_groups"]):
        s0, s1, pairs = b.group(g)
        covered += list(range(s0, s1 + 1))
        off, ids = b.export(g)
        roff, rids = OB.bucket_lists(lat.nodes, lat.edges, lat.weight, lat.R, grid, tile, slab,
                                     slabs=range(s0, s1 + 1))
        assert pairs == len(rids)
        assert np.array_equal(off.cpu().numpy(), roff)
        assert np.array_equal(ids.cpu().numpy().astype(np.int64), rids)
    assert covered == list(range(n_slabs))


# ------------------------------------------------------------------ field
@pytest.mark.parametrize("case", ["P1", "kuhn", "random"])
def test_field_matches_oracle(case):
    lat, grid = CASES[case]()
    print(f"field {case}", flush=True)
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, 0, grid.n_slices)
    torch.cuda.synchronize()
    ref = oracle_field(lat, grid, range(grid.n_slices))
    assert_field_close(f.cpu().numpy(), ref, lat.C, field_tol(lat.nodes.dtype), case)
    assert ref.max() > lat.C       # the case has inside pixels


def test_field_independent_of_tiling_and_groups():
    """Each 8x8 block and plane gets the same candidate struts in the same
    order whatever the tile, slab or group split (the candidate counts agree
    exactly), so the float32 field, summed in runs of four candidates, is
    bitwise the same."""
    lat, grid = small_kuhn()
    base = base_stats = None
    for tile, slab, mp in [(16, 8, 0), (8, 1, 0), (32, 4, 0), (64, 16, 0), (16, 2, 2500)]:
        print(f"tiling tile={tile} slab={slab} max_pairs={mp}", flush=True)
        b = bin_lattice(lat, grid, tile=tile, slab=slab, max_pairs=mp)
        f = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
        st = api.slice_field_stats(b, 0, grid.n_slices)
        if base is None:
            base, base_stats = f, st
        else:
            assert np.array_equal(f.view(np.uint32), base.view(np.uint32))
            assert st == base_stats


def test_field_partial_ranges_and_repeatability():
    lat, grid = small_kuhn()
    b = bin_lattice(lat, grid, slab=4, max_pairs=4000)
    full = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
    again = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
    assert np.array_equal(full.view(np.uint32), again.view(np.uint32))
    for k0, nk in [(0, 1), (3, 5), (13, 14), (26, 1), (5, 17)]:
        part = api.slice_field(b, k0, nk).cpu().numpy()
        assert np.array_equal(part.view(np.uint32), full[k0:k0 + nk].view(np.uint32))


def test_bits_match_field():
    lat, grid = small_kuhn()
    b = bin_lattice(lat, grid)
    f, bits = api.slice_field(b, 2, 9, bits=True)
    img = unpack_bits(bits, grid.W)
    assert np.array_equal(img, f.cpu().numpy() >= lat.C)
    ref = oracle_field(lat, grid, range(2, 11))
    sure = np.abs(ref - lat.C) > 1e-5
    assert np.array_equal(img[sure], (ref >= lat.C)[sure])


# ------------------------------------------------------------------ contours
@pytest.mark.parametrize("case", ["kuhn", "P1"])
def test_contours_match_oracle(case):
    lat, grid = CASES[case]()
    b = bin_lattice(lat, grid)
    nk = min(grid.n_slices, 12)
    f = api.slice_field(b, 0, nk)
    segs, off, codes = api.slice_contours(b, f, case_codes=True)
    segs = segs.cpu().numpy().astype(np.float64)
    off = off.cpu().numpy()
    codes = codes.cpu().numpy()
    fh = f.cpu().numpy()
    ref = oracle_field(lat, grid, range(nk))
    assert off[0] == 0 and off[-1] == len(segs)
    for k in range(nk):
        # exact: marching squares of the GPU's own binary image
        mine = fh[k] >= lat.C
        assert np.array_equal(codes[k], OC.case_codes(mine))
        assert np.array_equal(segs[off[k]:off[k + 1]], OC.segments(mine))
        # against the oracle field: identical wherever the four corners are
        # more than 1e-5 from the iso-value
        rin = ref[k] >= lat.C
        rc = OC.case_codes(rin)
        far = np.abs(ref[k] - lat.C) > 1e-5
        sure = far[:-1, :-1] & far[:-1, 1:] & far[1:, 1:] & far[1:, :-1]
        assert np.array_equal(codes[k][sure], rc[sure])
        assert sure.mean() > 0.95
    assert len(segs) > 0


def test_contours_capacity():
    lat, grid = small_kuhn()
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, 0, 4)
    segs, off, _ = api.slice_contours(b, f)
    total = len(segs)
    assert total > 10
    small = torch.empty((total - 1, 4), dtype=torch.float32, device="cuda")
    off2 = torch.empty(5, dtype=torch.int64, device="cuda")
    import ctypes
    t = ctypes.c_int64()
    st = N.lib().slice_contours(b.handle, 4, api._ptr(f), api._ptr(small), total - 1,
                                api._ptr(off2), None, ctypes.byref(t), api._stream())
    assert st == N.LSL_ECAPACITY and t.value == total
    assert np.array_equal(off2.cpu().numpy(), off.cpu().numpy())


# ------------------------------------------------------------------ edge cases
def test_empty_and_absent_lattices():
    lat, grid = small_kuhn()
    for kind in ("no_edges", "all_zero", "outside"):
        l2 = synth.Lattice(lat.nodes.copy(), lat.edges.copy(), lat.weight.copy(), lat.R, lat.C)
        if kind == "no_edges":
            l2.edges = np.zeros((0, 2), np.int32)
            l2.weight = np.zeros(0, np.float32)
        elif kind == "all_zero":
            l2.weight[:] = 0
        else:
            l2.nodes = l2.nodes + np.float32(1000.0)
        b = bin_lattice(l2, grid)
        assert b.info()["n_binned"] == 0
        f, bits = api.slice_field(b, 0, 3, bits=True)
        assert float(f.abs().max()) == 0.0 and int(bits.abs().max()) == 0
        # the batched path writes its outputs too: empty images, no segments
        field = torch.full((3, grid.H, grid.W), 7.0, dtype=f.dtype, device="cuda")
        bits = torch.full((3, grid.H, (grid.W + 31) // 32), -1, dtype=torch.int32, device="cuda")
        offs = torch.full((4,), -1, dtype=torch.int64, device="cuda")
        st, total, _, offs = api.slice_batch(b, 0, 3, field=field, bits=bits, capacity=4,
                                             segs=torch.empty((4, 4), device="cuda"),
                                             offsets=offs)
        assert st == N.LSL_OK and total == 0
        assert float(field.abs().max()) == 0.0 and int(bits.abs().max()) == 0
        assert offs.tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("bad", ["index", "negative", "nan_weight", "nan_node"])
def test_invalid_lattice_rejected(bad):
    lat, grid = small_kuhn()
    lat.weight = lat.weight.copy()
    if bad == "index":
        lat.edges = lat.edges.copy()
        lat.edges[10, 1] = lat.n_nodes
    elif bad == "negative":
        lat.weight[5] = -1.0
    elif bad == "nan_weight":
        lat.weight[5] = np.nan
    else:
        lat.nodes = lat.nodes.copy()
        lat.nodes[lat.edges[7, 0], 2] = np.nan
    n, e, w = to_dev(lat)
    with pytest.raises(N.LslError) as ei:
        api.lattice_bin(n, e, w, lat.R, lat.C, grid)
    assert ei.value.status == N.LSL_EINVAL


def test_stats_count_useful_pairs():
    lat, grid = synth.config("P1")
    b = bin_lattice(lat, grid)
    st = api.slice_field_stats(b, 0, 10)
    assert st["pixels"] == 10 * grid.W * grid.H
    # oracle: number of (pixel, strut) pairs with a non-zero term
    xs, ys = grid.pixel_x(), grid.pixel_y()
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    n = 0
    zlo, zhi = OS.strut_z_range(lat.nodes, lat.edges)
    for k in range(10):
        P = np.stack([X, Y, np.full_like(X, grid.slice_z(k))], -1)
        for i in OS.active_set(zlo, zhi, lat.R, grid.slice_z(k)):
            n += int(np.count_nonzero(OF.strut_integral(P, lat.nodes[lat.edges[i, 0]],
                                                        lat.nodes[lat.edges[i, 1]], lat.R)))
    assert abs(st["useful"] - n) <= 1e-5 * n
    assert st["candidates"] >= st["useful"]


# ------------------------------------------------------------------ full size
@pytest.mark.parametrize("name,k0,nk", [("A2", 480, 16), ("M1", 200, 8)])
def test_full_size_sampled(name, k0, nk):
    """The configuration at full size, in the launch configuration the
    benchmark uses; sampled pixels against the oracle one by one."""
    lat, grid = synth.config(name)
    print(f"full size {name}: E={lat.n_edges}", flush=True)
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, k0, nk).cpu().numpy()
    rng = np.random.default_rng(7)
    zlo, zhi = OS.strut_z_range(lat.nodes, lat.edges)
    worst = 0.0
    n_in = 0
    for _ in range(120):
        k = int(rng.integers(k0, k0 + nk))
        i = int(rng.integers(0, grid.W))
        j = int(rng.integers(0, grid.H))
        p = OS.slice_points(grid, k, np.array([i]), np.array([j]))[0]
        act = OS.active_set(zlo, zhi, lat.R, float(grid.slice_z(k)))
        ref = OF.field_at_point(p, lat.nodes, lat.edges, lat.weight, lat.R, act)
        got = float(f[k - k0, j, i])
        worst = max(worst, abs(got - ref) / max(abs(ref), lat.C))
        n_in += ref > 0
    assert worst <= 1e-5, worst
    assert n_in > 20
    # sampled buckets of the resident group against the oracle's definition
    r = OB.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.R, grid, 16, 8)
    off, ids = b.export(0)
    off = off.cpu().numpy()
    ids = ids.cpu().numpy()
    s0, s1, _ = b.group(0)
    ntx, nty = OB.tiles_xy(grid, 16)
    order = r["order"]
    for _ in range(25):
        s = int(rng.integers(s0, s1 + 1))
        ty = int(rng.integers(0, nty))
        tx = int(rng.integers(0, ntx))
        m = ((r["slab0"][order] <= s) & (r["slab1"][order] >= s) & (r["ty0"][order] <= ty) &
             (r["ty1"][order] >= ty) & (r["tx0"][order] <= tx) & (r["tx1"][order] >= tx))
        key = ((s - s0) * nty + ty) * ntx + tx
        assert np.array_equal(ids[off[key]:off[key + 1]], order[m])


def test_device_cache_reuse_and_trim():
    """Freed handles leave their buffers in the library's cache; new handles
    reuse them (dirty) with identical results; trimming empties the cache."""
    import gc
    lat, grid = small_kuhn()
    b = bin_lattice(lat, grid)
    f0 = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
    del b
    gc.collect()
    b = bin_lattice(lat, grid)
    f1 = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
    assert np.array_equal(f0.view(np.uint32), f1.view(np.uint32))
    del b
    gc.collect()
    assert api.cache_trim() > 0
    assert api.cache_trim() == 0
    b = bin_lattice(lat, grid)
    f2 = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
    assert np.array_equal(f0.view(np.uint32), f2.view(np.uint32))


def dense_bundle():
    """300 struts through a small ball: blocks near it hold several 64-entry
    chunks of candidates per plane, so runs of four straddle chunks."""
    rng = np.random.default_rng(29)
    c = np.array([5.0, 5.0, 2.0])
    dirs = rng.normal(size=(300, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    off = rng.normal(size=(300, 3)) * 0.3
    a = c + off - dirs * rng.uniform(0.5, 3.0, size=(300, 1))
    b = c + off + dirs * rng.uniform(0.5, 3.0, size=(300, 1))
    nodes = np.concatenate([a, b]).astype(np.float32)
    edges = np.stack([np.arange(300), np.arange(300) + 300], axis=1).astype(np.int32)
    w = rng.uniform(0.02, 0.2, size=300).astype(np.float32)
    lat = synth.Lattice(nodes, edges, w, 1.5, 1.0)
    grid = synth.grid_for(lat, 93, 87, 11, dz=0.37)
    return lat, grid


def test_dense_bundle_runs_straddle_chunks():
    """Candidate lists longer than one chunk: the open run carried from one
    chunk to the next gives the oracle's field and the same bits under every
    tiling."""
    lat, grid = dense_bundle()
    ref = oracle_field(lat, grid, range(grid.n_slices))
    assert ref.max() > 2.0                      # many struts overlap
    base = base_stats = None
    for tile, slab, mp in [(16, 8, 0), (64, 16, 0), (8, 3, 0), (32, 4, 3000)]:
        print(f"dense bundle tile={tile} slab={slab} max_pairs={mp}", flush=True)
        b = bin_lattice(lat, grid, tile=tile, slab=slab, max_pairs=mp)
        f = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
        assert_field_close(f, ref, lat.C, field_tol(np.float32), "dense bundle")
        st = api.slice_field_stats(b, 0, grid.n_slices)
        if base is None:
            base, base_stats = f, st
            # some block and plane sees more than 64 candidates
            assert st["candidates"] > 64 * 64
        else:
            assert np.array_equal(f.view(np.uint32), base.view(np.uint32))
            assert st == base_stats
