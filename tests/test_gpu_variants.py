"""GPU parity of the kernel variants (per-strut supports, compact Gaussian
kernel) with the oracle (oracle/field.py, slicer.py, binning.py,
gradient.py)."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import binning as OB
from oracle import contours as OC
from oracle import field as OF
from oracle import gradient as OG
from oracle import slicer as OS
from paper_2101_05031_amd import _native as N
from paper_2101_05031_amd import api, synth, tuning
from paper_2101_05031_amd.autograd import slice_field as sf_fn

from gpu_util import assert_field_close, bin_lattice, field_tol, to_dev, variant_kw

pytestmark = pytest.mark.gpu


def small_kuhn(dtype=np.float32):
    lat = synth.kuhn_lattice(6, 24.0, seed=21, dtype=dtype)
    grid = synth.grid_for(lat, 301, 283, 27, dz=0.83)
    return lat, grid


def oracle_field(lat, grid, ks):
    R = lat.support if lat.support is not None else lat.R
    return np.stack([OS.slice_field(lat.nodes, lat.edges, lat.weight, R, grid, k,
                                    kind=lat.kernel, sigma=lat.sigma) for k in ks])


def test_one_support_per_strut_is_bitwise_the_plain_path():
    lat, grid = small_kuhn()
    same = dataclasses.replace(lat, support=np.full(lat.n_edges, lat.R, dtype=np.float32))
    for tile, slab in ((16, 8), (32, 4)):
        print(f"uniform supports tile={tile} slab={slab}", flush=True)
        a = bin_lattice(lat, grid, tile=tile, slab=slab)
        b = bin_lattice(same, grid, tile=tile, slab=slab)
        assert torch.equal(a.order(), b.order())
        fa = api.slice_field(a, 0, grid.n_slices)
        fb = api.slice_field(b, 0, grid.n_slices)
        assert torch.equal(fa.view(torch.int32), fb.view(torch.int32))


def test_per_strut_supports_independent_of_tile_and_groups():
    """With per-strut supports the edge-list order has the first slab as its
    major key, so it is fixed once the slab depth is; then the tile size and
    the group split leave every block's candidates and the field bitwise the
    same."""
    lat, grid = small_kuhn()
    lat = synth.with_supports(lat)
    base = base_stats = None
    for tile, mp in ((16, 0), (8, 0), (32, 0), (64, 0), (16, 2500)):
        print(f"per-strut supports tile={tile} slab=4 max_pairs={mp}", flush=True)
        b = bin_lattice(lat, grid, tile=tile, slab=4, max_pairs=mp)
        f = api.slice_field(b, 0, grid.n_slices).cpu().numpy()
        st = api.slice_field_stats(b, 0, grid.n_slices)
        if base is None:
            base, base_stats = f, st
        else:
            assert np.array_equal(f.view(np.uint32), base.view(np.uint32))
            assert st == base_stats


@pytest.mark.parametrize("dtype,tile,slab,max_pairs", [
    (np.float32, 16, 8, 0), (np.float32, 8, 3, 2500), (np.float64, 32, 4, 0)])
def test_per_strut_supports_match_oracle(dtype, tile, slab, max_pairs):
    lat, grid = small_kuhn(dtype)
    lat = synth.with_supports(lat)
    print(f"per-strut supports {np.dtype(dtype).name} tile={tile} slab={slab} "
          f"max_pairs={max_pairs}", flush=True)
    b = bin_lattice(lat, grid, tile=tile, slab=slab, max_pairs=max_pairs)
    info = b.info()
    r = OB.strut_ranges(lat.nodes, lat.edges, lat.weight, lat.support, grid, tile, slab)
    assert np.array_equal(b.order().cpu().numpy(), r["order"])
    if max_pairs:
        assert info["n_groups"] > 1
    for g in range(info["n_groups"]):
        s0, s1, pairs = b.group(g)
        off, ids = b.export(g)
        roff, rids = OB.bucket_lists(lat.nodes, lat.edges, lat.weight, lat.support, grid, tile,
                                     slab, slabs=range(s0, s1 + 1))
        assert np.array_equal(off.cpu().numpy(), roff)
        assert np.array_equal(ids.cpu().numpy().astype(np.int64), rids)
    f = api.slice_field(b, 0, grid.n_slices)
    ref = oracle_field(lat, grid, range(grid.n_slices))
    assert_field_close(f.cpu().numpy(), ref, lat.C, field_tol(dtype), "per-strut field")
    assert ref.max() > lat.C
    # contours on the GPU's own image equal the oracle's marching squares
    segs, off, _ = api.slice_contours(b, f)
    fh = f.cpu().numpy()
    o = off.cpu().numpy()
    for k in (0, grid.n_slices // 2, grid.n_slices - 1):
        want = OC.segments(fh[k] >= np.asarray(lat.C, dtype=dtype))
        assert np.array_equal(segs[o[k]:o[k + 1]].cpu().numpy(), want)


def test_per_strut_supports_backward_matches_oracle():
    lat = synth.with_supports(synth.kuhn_lattice(4, 16.0, seed=31))
    grid = synth.grid_for(lat, 165, 151, 14, dz=1.1)
    ks = range(0, grid.n_slices)
    rng = np.random.default_rng(5)
    G = rng.normal(size=(len(ks), grid.H, grid.W)).astype(np.float32)
    b = bin_lattice(lat, grid)
    gw, gn = api.slice_field_backward(b, 0, len(ks), torch.from_numpy(G).cuda())
    rw, rn = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.support, grid, ks, G)
    for got, ref, what in ((gw, rw, "dL/dr"), (gn, rn, "dL/dv")):
        got = got.cpu().numpy().astype(np.float64).ravel()
        ref = ref.ravel()
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        per = np.max(np.abs(got - ref) / scale)
        norm = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"per-strut supports {what}: per-parameter {per:.2e}, normwise {norm:.2e}",
              flush=True)
        assert per <= 1e-4 and norm <= 1e-4, what


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_gauss_kernel_matches_oracle(dtype):
    lat, grid = small_kuhn(dtype)
    lat = synth.with_gauss(lat)
    print(f"gauss {np.dtype(dtype).name}", flush=True)
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, 0, grid.n_slices)
    ref = oracle_field(lat, grid, range(grid.n_slices))
    assert_field_close(f.cpu().numpy(), ref, lat.C, field_tol(dtype), "gauss field")
    assert ref.max() > lat.C
    # the batched path evaluates the same kernel, bitwise
    bits = torch.empty((grid.n_slices, grid.H, (grid.W + 31) // 32), dtype=torch.int32,
                       device="cuda")
    f2 = torch.empty_like(f)
    offsets = torch.empty(grid.n_slices + 1, dtype=torch.int64, device="cuda")
    api.slice_batch(b, 0, grid.n_slices, field=f2, bits=bits, capacity=0, offsets=offsets)
    assert torch.equal(f.view(torch.int64 if dtype == np.float64 else torch.int32),
                       f2.view(torch.int64 if dtype == np.float64 else torch.int32))
    # the adjoint covers the quartic kernel only
    with pytest.raises(N.LslError) as ei:
        api.slice_field_backward(b, 0, 2, torch.zeros_like(f[:2]))
    assert ei.value.status == N.LSL_EINVAL


def test_gauss_with_per_strut_supports():
    lat, grid = small_kuhn()
    lat = synth.with_supports(lat)
    sigma = float(lat.support.max()) / 4
    rho = np.asarray(lat.radius, dtype=np.float64)
    w = synth.weight_for_radius_gauss(rho, lat.support.astype(np.float64), sigma, lat.C)
    lat = dataclasses.replace(lat, weight=w.astype(np.float32), kernel="gauss", sigma=sigma)
    b = bin_lattice(lat, grid)
    ks = range(5, 14)
    f = api.slice_field(b, ks.start, len(ks))
    ref = oracle_field(lat, grid, ks)
    assert_field_close(f.cpu().numpy(), ref, lat.C, 1e-5, "gauss per-strut")


def test_variant_arguments_rejected():
    lat, grid = small_kuhn()
    n, e, w = to_dev(lat)
    bad_support = torch.full((lat.n_edges,), 1.0, device="cuda")
    bad_support[7] = 0.0
    with pytest.raises(N.LslError) as ei:
        api.lattice_bin(n, e, w, lat.R, lat.C, grid, support=bad_support)
    assert ei.value.status == N.LSL_EINVAL
    with pytest.raises(N.LslError) as ei:                  # support above 12 sigma
        api.lattice_bin(n, e, w, lat.R, lat.C, grid, kernel="gauss", sigma=lat.R / 13)
    assert ei.value.status == N.LSL_EINVAL
    with pytest.raises(N.LslError) as ei:                  # per strut, checked on the device
        api.lattice_bin(n, e, w, lat.R, lat.C, grid, support=torch.full_like(w, 2.0),
                        kernel="gauss", sigma=0.1)
    assert ei.value.status == N.LSL_EINVAL
    with pytest.raises(N.LslError):
        api.lattice_bin(n, e, w, lat.R, lat.C, grid, kernel="gauss", sigma=0.0)


@pytest.mark.parametrize("name", ["M1R", "M1G"])
def test_variants_full_size_sampled(name):
    """The 1M-strut workload's variants at full size (1000 planes of 2048^2)
    through the batched path: sampled pixels against the oracle."""
    lat, grid = synth.config(name)
    b = bin_lattice(lat, grid, tile=16, slab=8)
    S = grid.n_slices
    field = torch.empty((S, grid.H, grid.W), dtype=torch.float32, device="cuda")
    bits = torch.empty((S, grid.H, (grid.W + 31) // 32), dtype=torch.int32, device="cuda")
    offsets = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    api.slice_batch(b, 0, S, field=field, bits=bits, capacity=0, offsets=offsets)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    R = lat.support if lat.support is not None else lat.R
    zlo, zhi = OS.strut_z_range(lat.nodes, lat.edges)
    worst = 0.0
    for k in rng.integers(0, S, size=4):
        ix = rng.integers(0, grid.W, size=12)
        iy = rng.integers(0, grid.H, size=12)
        P = OS.slice_points(grid, int(k), ix, iy)
        act = OS.active_set(zlo, zhi, R, float(grid.slice_z(int(k))))
        ref = np.array([OF.field_at_point(p, lat.nodes, lat.edges, lat.weight, R, act,
                                          kind=lat.kernel, sigma=lat.sigma) for p in P])
        got = field[int(k)].cpu().numpy()[iy, ix].astype(np.float64)
        err = np.abs(got - ref) / np.maximum(np.abs(ref), lat.C)
        worst = max(worst, float(err.max()))
    print(f"{name}: worst scaled error {worst:.2e}", flush=True)
    assert worst <= 1e-5


def test_per_strut_supports_through_autograd_and_matching():
    """The autograd Function and the density-matching driver carry per-strut
    supports: gradients equal the adjoint's, and matching lowers the loss."""
    lat, grid = small_kuhn()
    lat = synth.with_supports(lat)
    n, e, w = to_dev(lat)
    sup = torch.from_numpy(lat.support).cuda()
    wt = w.clone().requires_grad_(True)
    nt = n.clone().requires_grad_(True)
    f = sf_fn(nt, wt, e, lat.R, lat.C, grid, 3, 6, support=sup)
    G = torch.randn_like(f)
    (f * G).sum().backward()
    b = bin_lattice(lat, grid)
    gw, gn = api.slice_field_backward(b, 3, 6, G.contiguous())
    assert torch.equal(wt.grad, gw) and torch.equal(nt.grad, gn)
    vx, vy, vz = 24, 24, 4
    bt = api.lattice_bin(n, e, w * 1.3, lat.R, lat.C, grid, support=sup)
    target = api.slice_density(bt, api.slice_field(bt, 0, grid.n_slices), vx, vy, vz)
    w1, hist = tuning.match_density(n, e, w, lat.R, lat.C, grid, target, vx, vy, vz, iters=8,
                                    lr=0.05 * float(w.mean()), support=sup)
    assert min(h["loss"] for h in hist) < 0.3 * hist[0]["loss"]
