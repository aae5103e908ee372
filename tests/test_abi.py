"""Host-side checks of the C ABI: the library loads, exports every function
include/lsl.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2101_05031_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        from paper_2101_05031_amd import build
        build.build(verbose=False)
    return N.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lsl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lsl_status|const char\*)\s+(\w+)\s*\(", src, re.M)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ("lattice_bin", "slice_field", "slice_contours", "slice_field_backward",
              "slice_batch", "slice_autotune", "lattice_bins_free"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in N.SIGNATURES, name


def test_status_strings(lib):
    for code in (N.LSL_OK, N.LSL_EINVAL, N.LSL_ENOMEM, N.LSL_ECAPACITY, N.LSL_EDEVICE,
                 N.LSL_EINTERNAL):
        assert lib.lsl_status_string(code)
    assert b"gfx950" in lib.lsl_version()


def _good():
    L = N.LslLattice(n_nodes=2, n_edges=1, dtype=N.LSL_F32, nodes=8, edges=8, weight=8,
                     R=1.5, C=1.0)
    G = N.LslGrid(x0=0.0, y0=0.0, dx=0.1, dy=0.1, W=16, H=16, z0=0.0, dz=0.1, n_slices=4)
    return L, G


@pytest.mark.parametrize("mutate,msg", [
    (lambda L, G, P: setattr(L, "dtype", 7), b"dtype"),
    (lambda L, G, P: setattr(L, "R", 0.0), b"R must"),
    (lambda L, G, P: setattr(L, "R", float("nan")), b"R must"),
    (lambda L, G, P: setattr(L, "C", -1.0), b"C must"),
    (lambda L, G, P: setattr(L, "n_nodes", 0), b"n_nodes"),
    (lambda L, G, P: setattr(L, "nodes", None), b"nodes"),
    (lambda L, G, P: setattr(L, "edges", None), b"edges"),
    (lambda L, G, P: setattr(G, "W", 1), b"W and H"),
    (lambda L, G, P: setattr(G, "dz", 0.0), b"steps"),
    (lambda L, G, P: setattr(G, "n_slices", 0), b"n_slices"),
    (lambda L, G, P: setattr(P, "tile", 12), b"tile"),
    (lambda L, G, P: setattr(P, "slab", 17), b"slab"),
    (lambda L, G, P: setattr(P, "max_pairs", -5), b"max_pairs"),
])
def test_lattice_bin_validation(lib, mutate, msg):
    L, G = _good()
    P = N.LslBinParams(0, 0, 0)
    mutate(L, G, P)
    h = ctypes.c_void_p()
    st = lib.lattice_bin(ctypes.byref(L), ctypes.byref(G), ctypes.byref(P), ctypes.byref(h), None)
    assert st == N.LSL_EINVAL
    assert msg in lib.lsl_last_error()
    assert not h.value


def test_null_handles_rejected(lib):
    assert lib.slice_field(None, 0, 1, None, None, None) == N.LSL_EINVAL
    assert lib.slice_field_backward(None, 0, 1, None, None, None, 0, None) == N.LSL_EINVAL
    assert lib.slice_contours(None, 1, None, None, 0, None, None, None, None) == N.LSL_EINVAL
    assert lib.slice_batch(None, 0, 1, None, None, None, 0, None, None, None) == N.LSL_EINVAL
    assert lib.lattice_bins_info(None, None) == N.LSL_EINVAL
    assert lib.lattice_bins_free(None) == N.LSL_OK
    h = ctypes.c_void_p()
    assert lib.lattice_bin(None, None, None, ctypes.byref(h), None) == N.LSL_EINVAL
    assert lib.slice_autotune(None, None, None, None, None) == N.LSL_EINVAL


def test_python_binding_needs_the_library(monkeypatch, tmp_path):
    """No fallback: a missing library is an error, not a slow path."""
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        N.lib()
