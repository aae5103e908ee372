"""Helpers shared by the GPU tests: device copies of synthetic lattices and
tolerance checks.  Inputs come from the seeded generators; expected values
come from the oracle only."""
import numpy as np
import torch

from paper_2101_05031_amd import api


def to_dev(lat):
    return (torch.from_numpy(np.ascontiguousarray(lat.nodes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(lat.edges)).cuda(),
            torch.from_numpy(np.ascontiguousarray(lat.weight)).cuda())


def variant_kw(lat):
    """lattice_bin arguments for a lattice's kernel variant (per-strut
    supports, Gaussian kernel), empty for the paper's kernel."""
    kw = {}
    if lat.support is not None:
        kw["support"] = torch.from_numpy(np.ascontiguousarray(lat.support)).cuda()
    if lat.kernel != "quartic":
        kw["kernel"], kw["sigma"] = lat.kernel, lat.sigma
    return kw


def bin_lattice(lat, grid, **kw):
    n, e, w = to_dev(lat)
    b = api.lattice_bin(n, e, w, lat.R, lat.C, grid, **variant_kw(lat), **kw)
    torch.cuda.synchronize()
    return b


def field_tol(dtype):
    """|gpu - oracle| <= tol * max(|oracle|, C): 1e-5 for float32 (the
    stated bound), 1e-12 for float64."""
    return 1e-5 if dtype == np.float32 else 1e-12


def assert_field_close(got, ref, C, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), C)
    worst = float(err.max()) if err.size else 0.0
    assert worst <= tol, f"{what}: max scaled error {worst:.3e} > {tol:.1e}"
    return worst


def unpack_bits(bits, W):
    b = bits.cpu().numpy().view(np.uint32)
    out = np.zeros(b.shape[:-1] + (W,), dtype=bool)
    for i in range(W):
        out[..., i] = (b[..., i // 32] >> np.uint32(i % 32)) & np.uint32(1)
    return out
