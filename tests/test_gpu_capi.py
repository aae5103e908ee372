"""The C ABI used without Python: the lsl_slice tool (tools/lsl_slice.cpp)
reads a lattice file, bins it, slices a plane range, extracts contours and
runs the adjoint through include/lsl.h alone; its output is checked against
the oracle."""
import os
import struct
import subprocess

import numpy as np
import pytest

from oracle import contours as OC
from oracle import gradient as OG
from oracle import slicer as OS
from paper_2101_05031_amd import build as B
from paper_2101_05031_amd import synth

from gpu_util import assert_field_close, field_tol


def write_lattice(path, lat, grid):
    with open(path, "wb") as f:
        f.write(b"LSL1")
        f.write(struct.pack("<qqi", lat.n_nodes, lat.n_edges,
                            0 if lat.nodes.dtype == np.float32 else 1))
        f.write(struct.pack("<8d", lat.R, lat.C, grid.x0, grid.y0, grid.dx, grid.dy, grid.z0,
                            grid.dz))
        f.write(struct.pack("<3i", grid.W, grid.H, grid.n_slices))
        f.write(np.ascontiguousarray(lat.nodes).tobytes())
        f.write(np.ascontiguousarray(lat.edges, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(lat.weight).tobytes())


def read_output(path, dtype, n_edges):
    b = open(path, "rb").read()
    nk, W, H, total = struct.unpack_from("<4q", b, 0)
    o = 32
    es = np.dtype(dtype).itemsize
    field = np.frombuffer(b, dtype, nk * H * W, o).reshape(nk, H, W)
    o += nk * H * W * es
    off = np.frombuffer(b, np.int64, nk + 1, o)
    o += (nk + 1) * 8
    segs = np.frombuffer(b, np.float32, total * 4, o).reshape(total, 4)
    o += total * 16
    gw = np.frombuffer(b, dtype, n_edges, o)
    assert o + n_edges * es == len(b)
    return field, off, segs, gw


def test_tool_rejects_bad_input(tmp_path):
    """Usage and header errors end the tool before it touches a GPU."""
    if not os.path.exists(B.TOOL):
        B.build(verbose=False)
    r = subprocess.run([B.TOOL], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"XXXX" + bytes(64))
    r = subprocess.run([B.TOOL, str(bad), str(tmp_path / "o.bin"), "0", "1"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "header" in r.stderr
    # a plane range outside the grid
    lat = synth.kuhn_lattice(2, 10.0, seed=1, dtype=np.float32)
    grid = synth.grid_for(lat, 40, 40, 3, dz=1.0)
    good = tmp_path / "lat.bin"
    write_lattice(good, lat, grid)
    for k0, nk in (("2", "5"), ("-1", "1"), ("0", "0")):
        r = subprocess.run([B.TOOL, str(good), str(tmp_path / "o.bin"), k0, nk],
                           capture_output=True, text=True, timeout=60)
        assert r.returncode == 1 and "planes" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_lsl_slice_tool_matches_oracle(tmp_path, dtype):
    lat = synth.kuhn_lattice(4, 16.0, seed=31, dtype=dtype)
    grid = synth.grid_for(lat, 165, 151, 14, dz=1.1)
    inp, out = tmp_path / "lattice.bin", tmp_path / "out.bin"
    write_lattice(inp, lat, grid)
    k0, nk = 3, 6
    print(f"lsl_slice {np.dtype(dtype).name} planes {k0}..{k0 + nk - 1}", flush=True)
    r = subprocess.run([B.TOOL, str(inp), str(out), str(k0), str(nk)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    field, off, segs, gw = read_output(out, dtype, lat.n_edges)
    ks = range(k0, k0 + nk)
    ref = np.stack([OS.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k) for k in ks])
    assert_field_close(field, ref, lat.C, field_tol(dtype), "lsl_slice field")
    C = float(np.asarray(lat.C, dtype=dtype))
    assert off[0] == 0 and off[-1] == len(segs) > 0
    for k in range(nk):
        assert np.array_equal(segs[off[k]:off[k + 1]], OC.segments(field[k] >= C).astype(np.float32))
    rw, _ = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks,
                         np.ones((nk, grid.H, grid.W)))
    g = gw.astype(np.float64)
    tol = 1e-4 if dtype == np.float32 else 1e-10
    scale = np.maximum(np.abs(rw), 1e-3 * np.abs(rw).max())
    assert np.max(np.abs(g - rw) / scale) <= tol
