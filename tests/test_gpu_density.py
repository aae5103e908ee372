"""GPU parity of slice_density (Sec. 5, Eq. 9) and slice_density_loss with the
oracle (oracle/density.py), on the GPU's own field, and the density-matching
driver built on them (Sec. 5.3)."""
import numpy as np
import pytest
import torch

from oracle import density as OD
from paper_2101_05031_amd import _native as N
from paper_2101_05031_amd import api, synth, tuning

from gpu_util import bin_lattice, to_dev

pytestmark = pytest.mark.gpu

# voxel extents (vx, vy, vz): several per block, ragged, one sample, wider
# than a block (two column passes per thread), clipped to the whole field
VOXELS = [(8, 8, 4), (5, 7, 3), (1, 1, 1), (64, 40, 27), (257, 3, 2), (1000, 1000, 100)]


def small_kuhn(dtype=np.float32):
    lat = synth.kuhn_lattice(6, 24.0, seed=21, dtype=dtype)
    grid = synth.grid_for(lat, 301, 283, 27, dz=0.83)     # ragged W, H
    return lat, grid


def c_in(lat, dtype):
    """C rounded to the field's dtype, as the inside test uses it."""
    return float(np.asarray(lat.C, dtype=dtype))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_density_matches_oracle(dtype):
    lat, grid = small_kuhn(dtype)
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, 0, grid.n_slices)
    fh = f.cpu().numpy().astype(np.float64)
    C = c_in(lat, dtype)
    for vx, vy, vz in VOXELS:
        print(f"density dtype={np.dtype(dtype).name} voxel={vx}x{vy}x{vz}", flush=True)
        d = api.slice_density(b, f, vx, vy, vz).cpu().numpy()
        ref = OD.voxel_density(fh, C, vx, vy, vz).astype(np.float32)
        assert d.shape == ref.shape
        assert np.array_equal(d, ref), (vx, vy, vz)
    assert 0.0 < ref[0, 0, 0] < 1.0                       # the whole-field voxel


def test_density_constant_fields_and_errors():
    lat, grid = small_kuhn()
    b = bin_lattice(lat, grid)
    for val, want in ((0.0, 0.0), (1.0, 1.0), (2.5, 1.0), (0.999, 0.0)):
        f = torch.full((5, grid.H, grid.W), val, dtype=torch.float32, device="cuda")
        d = api.slice_density(b, f, 7, 9, 2)
        assert torch.all(d == want), val
    f = torch.zeros((5, grid.H, grid.W), dtype=torch.float32, device="cuda")
    out = torch.empty(1, device="cuda")
    st = N.lib().slice_density(b.handle, 5, api._ptr(f), 0, 4, 4, api._ptr(out), api._stream())
    assert st == N.LSL_EINVAL
    t = torch.zeros(api.voxel_shape(5, grid.H, grid.W, 4, 4, 4), device="cuda")
    st = N.lib().slice_density_loss(b.handle, 5, api._ptr(f), 4, 4, 4, api._ptr(t), 0.0,
                                    None, None, None, api._stream())
    assert st == N.LSL_EINVAL
    with pytest.raises(ValueError):
        api.slice_density_loss(b, f, t[:1], 0.05, 4, 4, 4)
    st = N.lib().slice_occupancy_loss(b.handle, 5, api._ptr(f), api._ptr(f), -1.0, None, None,
                                      api._stream())
    assert st == N.LSL_EINVAL
    st = N.lib().slice_occupancy_loss(b.handle, 0, api._ptr(f), api._ptr(f), 0.05, None, None,
                                      api._stream())
    assert st == N.LSL_EINVAL


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_density_loss_matches_oracle(dtype):
    lat, grid = small_kuhn(dtype)
    b = bin_lattice(lat, grid)
    nk = grid.n_slices
    f = api.slice_field(b, 0, nk)
    fh = f.cpu().numpy().astype(np.float64)
    C = c_in(lat, dtype)
    rng = np.random.default_rng(9)
    f32 = dtype == np.float32
    for vx, vy, vz in [(8, 8, 4), (5, 7, 3), (257, 3, 2), (1, 1, 1)]:
        print(f"loss dtype={np.dtype(dtype).name} voxel={vx}x{vy}x{vz}", flush=True)
        shape = api.voxel_shape(nk, grid.H, grid.W, vx, vy, vz)
        target = rng.uniform(0.0, 0.6, size=shape).astype(np.float32)
        loss, soft, g = api.slice_density_loss(b, f, torch.from_numpy(target).cuda(), 0.05,
                                               vx, vy, vz)
        rl, rs, rg = OD.density_loss(fh, target.astype(np.float64), C, 0.05, vx, vy, vz)
        # float32 fields: sigmoid of a float32 argument (|dz| ~ 1e-6), then
        # float64 sums; float64 fields: only the float32 rounding of the output
        assert np.max(np.abs(soft.cpu().numpy() - rs)) <= (2e-6 if f32 else 1e-7)
        assert loss.item() == pytest.approx(rl, rel=1e-4 if f32 else 1e-10)
        gh = g.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(gh - rg)) <= (1e-4 if f32 else 1e-10) * np.abs(rg).max()
    # bitwise repeatable
    t = torch.from_numpy(target).cuda()
    l1, s1, g1 = api.slice_density_loss(b, f, t, 0.05, 1, 1, 1)
    l2, s2, g2 = api.slice_density_loss(b, f, t, 0.05, 1, 1, 1)
    assert torch.equal(l1, l2) and torch.equal(s1, s2) and torch.equal(g1, g2)


def test_density_full_size_sampled():
    """The 1M-strut workload at its full 1000 planes of 2048 x 2048, voxels of
    16 x 16 x 8 samples: sampled voxels against the oracle, and every inside
    sample counted once."""
    lat, grid = synth.config("M1")
    b = bin_lattice(lat, grid, tile=32, slab=8)
    nk = grid.n_slices
    f = api.slice_field(b, 0, nk)
    vx, vy, vz = 16, 16, 8
    d = api.slice_density(b, f, vx, vy, vz)
    nz, ny, nx = d.shape
    n = torch.from_numpy(OD.voxel_samples((nk, grid.H, grid.W), vx, vy, vz)).cuda()
    inside = int((f >= lat.C).sum())
    assert inside > 0
    assert int(torch.round(d.double() * n).sum()) == inside
    rng = np.random.default_rng(17)
    dh = d.cpu().numpy()
    shape = (nz, ny, nx)
    target = torch.from_numpy(rng.uniform(0.0, 0.5, size=shape).astype(np.float32)).cuda()
    loss, soft, g = api.slice_density_loss(b, f, target, 0.05, vx, vy, vz)
    sh = soft.cpu().numpy()
    busy = np.argwhere(dh > 0)
    picks = np.concatenate([busy[rng.integers(len(busy), size=40)],
                            np.array([[nz - 1, ny - 1, nx - 1], [0, 0, 0]])])
    for l, j, i in picks:
        blk = f[l * vz:(l + 1) * vz, j * vy:(j + 1) * vy, i * vx:(i + 1) * vx].cpu().numpy()
        blk = blk.astype(np.float64)
        ref = OD.voxel_density(blk, lat.C, vx, vy, vz)[0, 0, 0]
        assert dh[l, j, i] == np.float32(ref), (l, j, i)
        t = target[l, j, i].item()
        rl, rs, rg = OD.density_loss(blk, np.array([[[t]]]), lat.C, 0.05, *blk.shape[::-1])
        assert abs(sh[l, j, i] - rs[0, 0, 0]) <= 2e-6
        gb = g[l * vz:(l + 1) * vz, j * vy:(j + 1) * vy, i * vx:(i + 1) * vx].cpu().numpy()
        scale = max(np.abs(rg).max(), 1e-30)
        assert np.max(np.abs(gb - rg)) <= 1e-4 * scale, (l, j, i)


def test_match_density_reduces_the_loss():
    """Density matching (Sec. 5.3) on a small Kuhn lattice: the targets are
    the voxel densities of the same lattice with 1.3x the weights; gradient
    steps from the thinner lattice move its voxel densities toward them."""
    lat, grid = small_kuhn()
    n, e, w = to_dev(lat)
    vx, vy, vz = 24, 24, 4
    nk = grid.n_slices
    bt = api.lattice_bin(n, e, w * 1.3, lat.R, lat.C, grid)
    target = api.slice_density(bt, api.slice_field(bt, 0, nk), vx, vy, vz)
    w_min = float(synth.weight_for_radius(0.05, lat.R, lat.C))
    lr = 0.05 * float(w.mean())
    w1, hist = tuning.match_density(n, e, w, lat.R, lat.C, grid, target, vx, vy, vz,
                                    iters=12, lr=lr, w_min=w_min)
    for h in hist:
        print(f"loss {h['loss']:.6e} density error {h['density_error']:.6e}", flush=True)
    assert len(hist) == 13
    best = min(range(len(hist)), key=lambda i: hist[i]["loss"])
    assert hist[best]["loss"] < 0.1 * hist[0]["loss"]
    assert hist[best]["density_error"] < 0.4 * hist[0]["density_error"]
    assert hist[-1]["loss"] < 0.5 * hist[0]["loss"]
    assert float(w1.min()) >= w_min and float(w1.mean()) > float(w.mean())
    # the returned weights are the best iterate
    bb = api.lattice_bin(n, e, w1, lat.R, lat.C, grid)
    loss, _, _ = api.slice_density_loss(bb, api.slice_field(bb, 0, nk), target, 0.05, vx, vy, vz,
                                        want_grad=False)
    assert loss.item() == hist[best]["loss"]
    # deterministic: the same run gives the same weights bitwise
    w2, _ = tuning.match_density(n, e, w, lat.R, lat.C, grid, target, vx, vy, vz,
                                 iters=12, lr=lr, w_min=w_min)
    assert torch.equal(w1, w2)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_occupancy_loss_matches_oracle(dtype):
    """The per-pixel soft-occupancy loss (slice_occupancy_loss) against the
    oracle's (oracle/gradient.py), on the GPU's own field."""
    from oracle import gradient as OG
    lat, grid = small_kuhn(dtype)
    b = bin_lattice(lat, grid)
    f = api.slice_field(b, 2, 20)
    rng = np.random.default_rng(12)
    t = rng.uniform(0.0, 1.0, size=tuple(f.shape)).astype(dtype)
    loss, g = api.slice_occupancy_loss(b, f, torch.from_numpy(t).cuda(), 0.05)
    fh = f.cpu().numpy().astype(np.float64)
    C = c_in(lat, dtype)
    rl = OG.soft_occupancy_loss(fh, t.astype(np.float64), C, 0.05)
    rg = OG.soft_occupancy_grad(fh, t.astype(np.float64), C, 0.05)
    f32 = dtype == np.float32
    assert loss.item() == pytest.approx(rl, rel=1e-5 if f32 else 1e-12)
    gh = g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gh - rg)) <= (1e-4 if f32 else 1e-10) * np.abs(rg).max()
    l2, g2 = api.slice_occupancy_loss(b, f, torch.from_numpy(t).cuda(), 0.05)
    assert torch.equal(loss, l2) and torch.equal(g, g2)
    # the same loss as the voxel-density loss with one-sample voxels
    lv, _, gv = api.slice_density_loss(b, f, torch.from_numpy(t.astype(np.float32)).cuda(), 0.05,
                                       1, 1, 1)
    assert lv.item() == pytest.approx(rl, rel=1e-5)         # (float32 targets there)
