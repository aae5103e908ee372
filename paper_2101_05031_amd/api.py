"""Python binding of liblsl with the ABI's names.  Torch supplies device
memory and the current stream; every step of the slicing path runs in the
native library's kernels."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_float, c_int32, c_int64, c_void_p

import torch

from . import _native as N

_DTYPES = {torch.float32: N.LSL_F32, torch.float64: N.LSL_F64}


def _stream(stream=None) -> c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


def _ptr(t) -> c_void_p:
    return c_void_p(0 if t is None else t.data_ptr())


def _grid_struct(grid) -> N.LslGrid:
    g = N.LslGrid()
    for f in ("x0", "y0", "dx", "dy", "z0", "dz"):
        setattr(g, f, float(getattr(grid, f)))
    g.W, g.H, g.n_slices = int(grid.W), int(grid.H), int(grid.n_slices)
    return g


_KERNELS = {"quartic": N.LSL_KERNEL_QUARTIC, "gauss": N.LSL_KERNEL_GAUSS}


def _lattice_struct(nodes, edges, weight, R, C, support=None, kernel: str = "quartic",
                    sigma: float | None = None) -> N.LslLattice:
    if nodes.dtype not in _DTYPES:
        raise TypeError("nodes must be float32 or float64")
    for t, name in ((nodes, "nodes"), (edges, "edges"), (weight, "weight")):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor")
    if weight.dtype != nodes.dtype:
        raise TypeError("weight must have the dtype of nodes")
    if edges.dtype != torch.int32:
        raise TypeError("edges must be int32")
    if nodes.dim() != 2 or nodes.shape[1] != 3 or edges.dim() != 2 or edges.shape[1] != 2:
        raise ValueError("nodes must be [N,3] and edges [E,2]")
    if weight.shape != (edges.shape[0],):
        raise ValueError("weight must be [E]")
    L = N.LslLattice()
    L.n_nodes, L.n_edges = nodes.shape[0], edges.shape[0]
    L.dtype = _DTYPES[nodes.dtype]
    L.nodes, L.edges, L.weight = nodes.data_ptr(), edges.data_ptr(), weight.data_ptr()
    L.R, L.C = float(R), float(C)
    if support is not None:
        if (not support.is_cuda or not support.is_contiguous() or support.dtype != nodes.dtype
                or support.shape != (edges.shape[0],)):
            raise ValueError("support must be a contiguous CUDA [E] tensor of the nodes' dtype")
        L.support = support.data_ptr()
    if kernel not in _KERNELS:
        raise ValueError(f"kernel must be one of {sorted(_KERNELS)}")
    L.kernel = _KERNELS[kernel]
    L.sigma = float(sigma) if sigma is not None else 0.0
    return L


class Bins:
    """Owner of a lattice_bins handle."""

    def __init__(self, handle: int, dtype, grid, R: float, C: float, n_nodes: int,
                 n_edges: int):
        self.handle = c_void_p(handle)
        # held here so that a handle collected at interpreter exit, after the
        # module's globals are gone, is still freed
        self._free = N.lib().lattice_bins_free
        self.dtype = dtype
        self.grid = grid
        self.R, self.C = R, C
        self.n_nodes, self.n_edges = n_nodes, n_edges

    def __del__(self):
        h = getattr(self, "handle", None)
        free = getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self.handle = None

    def info(self) -> dict:
        i = N.LslBinsInfo()
        N.check(N.lib().lattice_bins_info(self.handle, byref(i)), "lattice_bins_info")
        return {f: getattr(i, f) for f, _ in N.LslBinsInfo._fields_}

    def group(self, g: int):
        s0, s1, p = c_int32(), c_int32(), c_int64()
        N.check(N.lib().lattice_bins_group(self.handle, g, byref(s0), byref(s1), byref(p)),
                "lattice_bins_group")
        return s0.value, s1.value, p.value

    def export(self, g: int):
        """(offsets int64 [n_buckets+1], ids int32 [pairs]) of group g."""
        s0, s1, pairs = self.group(g)
        info = self.info()
        nb = (s1 - s0 + 1) * info["tiles_x"] * info["tiles_y"]
        dev = torch.device("cuda")
        off = torch.empty(nb + 1, dtype=torch.int64, device=dev)
        ids = torch.empty(max(pairs, 1), dtype=torch.int32, device=dev)
        N.check(N.lib().lattice_bins_export(self.handle, g, _ptr(off), _ptr(ids), _stream()),
                "lattice_bins_export")
        return off, ids[:pairs]

    def order(self):
        n = self.info()["n_binned"]
        out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        N.check(N.lib().lattice_bins_order(self.handle, _ptr(out), _stream()), "lattice_bins_order")
        return out[:n]


def lattice_bin(nodes, edges, weight, R: float, C: float, grid, *, tile: int = 0,
                slab: int = 0, max_pairs: int = 0, support=None, kernel: str = "quartic",
                sigma: float | None = None, keep_zero_weight: bool = False,
                stream=None) -> Bins:
    """Bin a lattice for slicing.  support: optional per-strut supports [E]
    (then R is unused); kernel: "quartic" (Eq. 5) or "gauss" (width sigma);
    keep_zero_weight: bin struts of weight 0 as well, so that the adjoint
    gives their weights' gradient (otherwise they are absent)."""
    L = _lattice_struct(nodes, edges, weight, R, C, support, kernel, sigma)
    L.keep_zero_weight = 1 if keep_zero_weight else 0
    g = _grid_struct(grid)
    p = N.LslBinParams(int(tile), int(slab), int(max_pairs))
    h = c_void_p()
    N.check(N.lib().lattice_bin(byref(L), byref(g), byref(p), byref(h), _stream(stream)),
            "lattice_bin")
    return Bins(h.value, nodes.dtype, grid, float(R), float(C), nodes.shape[0], edges.shape[0])


def slice_field(bins: Bins, k0: int, nk: int, out=None, bits: bool | torch.Tensor = False,
                stream=None):
    g = bins.grid
    if out is None:
        out = torch.empty((nk, g.H, g.W), dtype=bins.dtype, device="cuda")
    bt = None
    if isinstance(bits, torch.Tensor):
        bt = bits
    elif bits:
        bt = torch.empty((nk, g.H, (g.W + 31) // 32), dtype=torch.int32, device="cuda")
    N.check(N.lib().slice_field(bins.handle, int(k0), int(nk), _ptr(out), _ptr(bt),
                                _stream(stream)), "slice_field")
    return (out, bt) if bt is not None else out


def slice_field_stats(bins: Bins, k0: int, nk: int, stream=None) -> dict:
    c = (c_int64 * 3)()
    N.check(N.lib().slice_field_stats(bins.handle, int(k0), int(nk), c, _stream(stream)),
            "slice_field_stats")
    return {"candidates": c[0], "useful": c[1], "pixels": c[2]}


def slice_contours(bins: Bins, field, capacity: int | None = None, case_codes: bool = False,
                   stream=None):
    """Marching squares of planes field[nk,H,W] -> (segs float32 [n,4],
    offsets int64 [nk+1], case codes uint8 [nk,H-1,W-1] or None)."""
    nk = field.shape[0]
    g = bins.grid
    off = torch.empty(nk + 1, dtype=torch.int64, device="cuda")
    codes = torch.empty((nk, g.H - 1, g.W - 1), dtype=torch.uint8, device="cuda") \
        if case_codes else None
    total = c_int64()
    L = N.lib()
    if capacity is None:
        st = L.slice_contours(bins.handle, nk, _ptr(field), c_void_p(0), 0, _ptr(off),
                              _ptr(codes), byref(total), _stream(stream))
        if st not in (N.LSL_OK, N.LSL_ECAPACITY):
            N.check(st, "slice_contours")
        capacity = total.value
    segs = torch.empty((max(capacity, 1), 4), dtype=torch.float32, device="cuda")
    N.check(L.slice_contours(bins.handle, nk, _ptr(field), _ptr(segs), int(capacity), _ptr(off),
                             _ptr(codes), byref(total), _stream(stream)), "slice_contours")
    return segs[:total.value], off, codes


def slice_polylines(bins: Bins, field, capacity: int | None = None, chains: bool = True,
                    stream=None):
    """Sub-pixel contours of planes field[nk,H,W] and their chaining ->
    (segs float32 [n,4], offsets int64 [nk+1], chain int32 [n] or None,
    rank int32 [n] or None); chain and rank are per plane."""
    nk = field.shape[0]
    off = torch.empty(nk + 1, dtype=torch.int64, device="cuda")
    total = c_int64()
    L = N.lib()
    if capacity is None:
        st = L.slice_polylines(bins.handle, nk, _ptr(field), c_void_p(0), 0, _ptr(off),
                               c_void_p(0), c_void_p(0), byref(total), _stream(stream))
        if st not in (N.LSL_OK, N.LSL_ECAPACITY):
            N.check(st, "slice_polylines")
        capacity = total.value
    segs = torch.empty((max(capacity, 1), 4), dtype=torch.float32, device="cuda")
    chain = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda") if chains else None
    rank = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda") if chains else None
    N.check(L.slice_polylines(bins.handle, nk, _ptr(field), _ptr(segs), int(capacity), _ptr(off),
                              _ptr(chain), _ptr(rank), byref(total), _stream(stream)),
            "slice_polylines")
    n = total.value
    return segs[:n], off, None if chain is None else chain[:n], None if rank is None else rank[:n]


def voxel_shape(nk: int, H: int, W: int, vx: int, vy: int, vz: int) -> tuple:
    """(nz, ny, nx): voxels of vz x vy x vx samples over a [nk, H, W] field,
    partial ones at the far borders."""
    return (-(-nk // vz), -(-H // vy), -(-W // vx))


def _check_field(bins: Bins, field):
    if (field.dim() != 3 or not field.is_contiguous() or field.dtype != bins.dtype
            or field.shape[1] != bins.grid.H or field.shape[2] != bins.grid.W):
        raise ValueError("field must be a contiguous [nk, H, W] tensor of the lattice dtype")


def slice_density(bins: Bins, field, vx: int, vy: int, vz: int, out=None, stream=None):
    """Per-voxel density (Sec. 5, Eq. 9) of the planes field[nk, H, W]: the
    fraction of each voxel's pixel-centre samples with g >= C -> float32
    [nz, ny, nx]."""
    _check_field(bins, field)
    nk = field.shape[0]
    shape = voxel_shape(nk, bins.grid.H, bins.grid.W, vx, vy, vz)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
    N.check(N.lib().slice_density(bins.handle, nk, _ptr(field), int(vx), int(vy), int(vz),
                                  _ptr(out), _stream(stream)), "slice_density")
    return out


def slice_density_loss(bins: Bins, field, target, tau: float, vx: int, vy: int, vz: int,
                       grad_field=None, soft=None, loss=None, want_grad: bool = True,
                       stream=None):
    """Soft voxel-density loss of field[nk, H, W] against target[nz, ny, nx]
    (float32): returns (loss float64 [1] on the device, soft density float32
    [nz, ny, nx], dL/dg [nk, H, W] in the lattice dtype or None)."""
    _check_field(bins, field)
    nk = field.shape[0]
    shape = voxel_shape(nk, bins.grid.H, bins.grid.W, vx, vy, vz)
    if tuple(target.shape) != shape or target.dtype != torch.float32 or not target.is_contiguous():
        raise ValueError(f"target must be a contiguous float32 tensor of shape {shape}")
    if soft is None:
        soft = torch.empty(shape, dtype=torch.float32, device="cuda")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
    if grad_field is None and want_grad:
        grad_field = torch.empty_like(field)
    N.check(N.lib().slice_density_loss(bins.handle, nk, _ptr(field), int(vx), int(vy), int(vz),
                                       _ptr(target), float(tau), _ptr(soft), _ptr(grad_field),
                                       _ptr(loss), _stream(stream)), "slice_density_loss")
    return loss, soft, grad_field


def slice_occupancy_loss(bins: Bins, field, target, tau: float, grad_field=None, loss=None,
                         want_grad: bool = True, stream=None):
    """sum over pixels of (sigmoid((g - C)/tau) - target)^2 and dL/dg, for
    field and target [nk, H, W] of the lattice dtype -> (loss float64 [1] on
    the device, dL/dg or None)."""
    _check_field(bins, field)
    if (tuple(target.shape) != tuple(field.shape) or target.dtype != field.dtype
            or not target.is_contiguous()):
        raise ValueError("target must be a contiguous tensor like field")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
    if grad_field is None and want_grad:
        grad_field = torch.empty_like(field)
    N.check(N.lib().slice_occupancy_loss(bins.handle, field.shape[0], _ptr(field), _ptr(target),
                                         float(tau), _ptr(grad_field), _ptr(loss),
                                         _stream(stream)), "slice_occupancy_loss")
    return loss, grad_field


def slice_field_backward(bins: Bins, k0: int, nk: int, grad_field, grad_weight=None,
                         grad_nodes=None, accumulate: bool = False, want_nodes: bool = True,
                         stream=None):
    """dL/dw [n_edges] and dL/dv [n_nodes, 3] (None when want_nodes is False)
    from dL/dg at the pixels of planes k0 .. k0+nk-1."""
    if grad_weight is None:
        grad_weight = torch.empty(bins.n_edges, dtype=bins.dtype, device="cuda")
    if grad_nodes is None and want_nodes:
        grad_nodes = torch.empty((bins.n_nodes, 3), dtype=bins.dtype, device="cuda")
    if not grad_field.is_contiguous() or grad_field.dtype != bins.dtype:
        raise ValueError("grad_field must be contiguous with the lattice dtype")
    N.check(N.lib().slice_field_backward(bins.handle, int(k0), int(nk), _ptr(grad_field),
                                         _ptr(grad_weight), _ptr(grad_nodes),
                                         1 if accumulate else 0, _stream(stream)),
            "slice_field_backward")
    return grad_weight, grad_nodes


def slice_batch(bins: Bins, k0: int, nk: int, field=None, bits=None, capacity: int = 0,
                segs=None, offsets=None, stream=None):
    """Persistent, graph-captured slicing of planes [k0, k0+nk): returns
    (status, total segments, segs, offsets)."""
    if offsets is None:
        offsets = torch.empty(nk + 1, dtype=torch.int64, device="cuda")
    if segs is None and capacity > 0:
        segs = torch.empty((capacity, 4), dtype=torch.float32, device="cuda")
    total = c_int64()
    st = N.lib().slice_batch(bins.handle, int(k0), int(nk), _ptr(field), _ptr(bits), _ptr(segs),
                             int(capacity), _ptr(offsets), byref(total), _stream(stream))
    if st not in (N.LSL_OK, N.LSL_ECAPACITY):
        N.check(st, "slice_batch")
    return st, total.value, segs, offsets


def slice_autotune(nodes, edges, weight, R: float, C: float, grid, cache_path: str | None = None,
                   tile: int = 0, slab: int = 0, support=None, kernel: str = "quartic",
                   sigma: float | None = None, max_pairs: int = 0, stream=None) -> dict:
    L = _lattice_struct(nodes, edges, weight, R, C, support, kernel, sigma)
    g = _grid_struct(grid)
    p = N.LslBinParams(int(tile), int(slab), int(max_pairs))
    path = cache_path.encode() if cache_path else None
    N.check(N.lib().slice_autotune(byref(L), byref(g), byref(p), path, _stream(stream)),
            "slice_autotune")
    return {"tile": p.tile, "slab": p.slab}


def probe_valu(mode: int, iters: int = 4096, stream=None) -> dict:
    """Vector-ALU throughput probe (diagnostics): duration and lane
    operations of one probe kernel; see lsl_probe_valu."""
    ms = c_float()
    ops = c_double()
    N.check(N.lib().lsl_probe_valu(int(mode), int(iters), byref(ms), byref(ops),
                                   _stream(stream)), "lsl_probe_valu")
    return {"mode": int(mode), "ms": ms.value, "lane_ops": ops.value}


def cache_trim() -> int:
    """Return the library's cached device buffers to the device and release
    its cached executable graphs; returns the bytes the buffer cache held."""
    n = c_int64()
    N.check(N.lib().lsl_cache_trim(byref(n)), "lsl_cache_trim")
    return n.value


def graph_cache_stats() -> dict:
    """slice_batch's executable-graph cache: graphs instantiated and updated
    since the process started, and the entries held now."""
    i, u, n = c_int64(), c_int64(), c_int64()
    N.check(N.lib().lsl_graph_cache_stats(byref(i), byref(u), byref(n)), "lsl_graph_cache_stats")
    return {"instantiated": i.value, "updated": u.value, "entries": n.value}


def lattice_support(nodes, edges, weight, print_dir=(0.0, 0.0, 1.0), grad: bool = False,
                    stream=None):
    """Self-support metrics (Sec. 5.2, Eqs. 11-14) of the lattice on the GPU:
    dict of gamma, psi and the sums behind them; with grad=True also
    dGamma/dv [n_nodes, 3] (lattice dtype)."""
    L = _lattice_struct(nodes, edges, weight, 1.0, 1.0)
    t = (c_double * 3)(*[float(x) for x in print_dir])
    out = N.LslSupport()
    g = torch.empty_like(nodes) if grad else None
    N.check(N.lib().lattice_support(byref(L), t, byref(out), _ptr(g), _stream(stream)),
            "lattice_support")
    res = {f: getattr(out, f) for f, _ in N.LslSupport._fields_}
    return (res, g) if grad else res
