"""Seeded synthetic lattices, slicing grids and target densities.

This module only builds inputs: strut graphs (nodes, edges, per-edge radius
weight), the pixel/slice grid they are sliced on and seeded target densities.
It holds no step of the slicing path.  Both the native library's tests and the
FP64 oracle's tests draw their inputs from here; nothing here imports either.

The paper's own models (Table 4: Teddy ... Kitten-HR) are not available, so
lattices of the same kind stand in for them: tetrahedral lattices built from a
cube grid split into Kuhn simplices (the paper builds its lattices from the
edges of a tetrahedral mesh, Sec. 5.1) and a uniform BCC cell lattice.

Input recipe (units are mm):

* A strut graph is (nodes [N,3], edges [E,2] int32, weight [E]); an edge is
  (v_s, v_e, r) as in Sec. 3.1.
* Physical strut radii rho are mapped to the paper's per-edge weight r of
  Eq. (6) with :func:`weight_for_radius`: the weight that puts the iso-surface
  g = C of an isolated, infinitely long strut at distance rho from its axis.
  The paper only says the map is monotone (Sec. 3.2); this choice is an input
  convention, not part of the method.
* The kernel support is R = 1.5 x the largest radius the recipe can produce
  (Sec. 3.2 uses 1.5 x the maximal radius), and the iso-value is C = 1.
* Slices sit at z0 + (k + 1/2) dz with z0 the lowest node (Sec. 4).
* Pixels are square; the grid covers the lattice's xy bounding box grown by R
  plus two pixels on each side, so that every contour closes inside the image.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Lattice", "Grid", "bcc_lattice", "kuhn_lattice", "weight_for_radius",
    "graded_density", "blob_density", "grid_for", "config", "CONFIGS",
    "target_density", "weight_for_radius_gauss", "with_supports", "with_gauss",
]


@dataclasses.dataclass
class Lattice:
    nodes: np.ndarray      # [N,3] float32 or float64
    edges: np.ndarray      # [E,2] int32
    weight: np.ndarray     # [E]  same dtype as nodes; 0 marks an absent strut
    R: float               # kernel support radius
    C: float = 1.0         # iso-value
    radius: np.ndarray | None = None  # [E] physical radius the weight encodes
    support: np.ndarray | None = None  # [E] per-strut supports (variant), else R for all
    kernel: str = "quartic"            # "quartic" (Eq. 5) or "gauss" (variant)
    sigma: float | None = None         # width of the Gaussian kernel

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])


@dataclasses.dataclass
class Grid:
    x0: float
    y0: float
    dx: float
    dy: float
    W: int
    H: int
    z0: float
    dz: float
    n_slices: int

    def pixel_x(self) -> np.ndarray:
        return self.x0 + (np.arange(self.W, dtype=np.float64) + 0.5) * self.dx

    def pixel_y(self) -> np.ndarray:
        return self.y0 + (np.arange(self.H, dtype=np.float64) + 0.5) * self.dy

    def slice_z(self, k) -> np.ndarray:
        return self.z0 + (np.asarray(k, dtype=np.float64) + 0.5) * self.dz


# ----------------------------------------------------------------------------
# radius -> weight (input convention)
# ----------------------------------------------------------------------------
def weight_for_radius(rho, R: float, C: float = 1.0) -> np.ndarray:
    """Weight r_i that places the iso-surface of an isolated infinite strut at
    distance rho.  Along an infinite line at distance d < R the kernel of
    Eq. (5) integrates to 16 (R^2 - d^2)^(5/2) / (15 R^4); setting r times that
    equal to C gives the weight.  Computed in float64."""
    rho = np.asarray(rho, dtype=np.float64)
    if np.any(rho < 0) or np.any(rho >= R):
        raise ValueError("radius must lie in [0, R)")
    phi = 16.0 * (R * R - rho * rho) ** 2.5 / (15.0 * R ** 4)
    return C / phi


def weight_for_radius_gauss(rho, R, sigma: float, C: float = 1.0) -> np.ndarray:
    """The same convention for the compact Gaussian kernel
    exp(-d^2/2s^2) - exp(-R^2/2s^2) (d < R): along an infinite line at
    distance d it integrates to
        exp(-d^2/2s^2) s sqrt(2 pi) erf(h / (s sqrt 2)) - exp(-R^2/2s^2) 2h,
    h = sqrt(R^2 - d^2).  float64."""
    from scipy.special import erf
    rho = np.asarray(rho, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    if np.any(rho < 0) or np.any(rho >= R):
        raise ValueError("radius must lie in [0, R)")
    h = np.sqrt(R * R - rho * rho)
    phi = (np.exp(-rho * rho / (2.0 * sigma * sigma)) * sigma * np.sqrt(2.0 * np.pi)
           * erf(h / (sigma * np.sqrt(2.0))) - np.exp(-R * R / (2.0 * sigma * sigma)) * 2.0 * h)
    return C / phi


def with_supports(lat: "Lattice", factor: float = 1.5) -> "Lattice":
    """The lattice with per-strut supports R_j = factor x rho_j (the paper's
    1.5 x radius rule applied strut by strut) and weights that keep every
    strut's radius; R becomes the largest support."""
    rho = np.asarray(lat.radius, dtype=np.float64)
    sup = factor * rho
    live = np.asarray(lat.weight) != 0
    w = np.where(live, weight_for_radius(rho, np.where(sup > 0, sup, 1.0), lat.C), 0.0)
    sup = np.where(sup > 0, sup, float(np.max(sup)))
    dt = lat.nodes.dtype
    return dataclasses.replace(lat, weight=w.astype(dt), support=sup.astype(dt),
                               R=float(np.max(sup)))


def with_gauss(lat: "Lattice", sigma_frac: float = 1.0 / 3.0) -> "Lattice":
    """The lattice under the compact Gaussian kernel of width sigma =
    sigma_frac x R and support R, weights keeping every strut's radius."""
    sigma = sigma_frac * lat.R
    rho = np.asarray(lat.radius, dtype=np.float64)
    live = np.asarray(lat.weight) != 0
    w = np.where(live, weight_for_radius_gauss(rho, lat.R, sigma, lat.C), 0.0)
    return dataclasses.replace(lat, weight=w.astype(lat.nodes.dtype), kernel="gauss",
                               sigma=float(sigma))


# ----------------------------------------------------------------------------
# lattices
# ----------------------------------------------------------------------------
def _grid_index(n: int):
    def idx(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k
    return idx


def _grid_nodes(n: int, size: float) -> np.ndarray:
    ax = np.linspace(0.0, size, n + 1)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def kuhn_edges(n: int) -> np.ndarray:
    """Edges of the Kuhn (Freudenthal) split of an n^3 cube grid into 6 tets
    per cube: every pair of grid nodes whose index difference is a non-zero
    0/1 vector, each once.  E = 3n(n+1)^2 + 3n^2(n+1) + n^3."""
    idx = _grid_index(n)
    out = []
    for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
              (1, 1, 1)]:
        ri = np.arange(n + 1 - d[0])
        rj = np.arange(n + 1 - d[1])
        rk = np.arange(n + 1 - d[2])
        I, J, K = np.meshgrid(ri, rj, rk, indexing="ij")
        a = idx(I, J, K).ravel()
        b = idx(I + d[0], J + d[1], K + d[2]).ravel()
        out.append(np.stack([a, b], axis=1))
    return np.concatenate(out, axis=0).astype(np.int32)


def bcc_lattice(n_cells: int = 4, cell: float = 5.0, radius: float = 0.5,
                dtype=np.float64) -> Lattice:
    """Uniform body-centred-cubic lattice: cube corners plus cell centres; the
    12 edges of every cube (shared edges once) and the 8 centre-to-corner
    struts of every cell.  n=4 gives 189 nodes and 812 struts."""
    n = n_cells
    corners = _grid_nodes(n, n * cell)
    c = (np.arange(n) + 0.5) * cell
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    centres = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    nodes = np.concatenate([corners, centres], axis=0)
    idx = _grid_index(n)
    edges = []
    for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        ri = np.arange(n + 1 - d[0])
        rj = np.arange(n + 1 - d[1])
        rk = np.arange(n + 1 - d[2])
        I, J, K = np.meshgrid(ri, rj, rk, indexing="ij")
        edges.append(np.stack([idx(I, J, K).ravel(),
                               idx(I + d[0], J + d[1], K + d[2]).ravel()], 1))
    n_corner = (n + 1) ** 3
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    centre_id = n_corner + (I * n + J) * n + K
    for di in (0, 1):
        for dj in (0, 1):
            for dk in (0, 1):
                edges.append(np.stack([centre_id.ravel(),
                                       idx(I + di, J + dj, K + dk).ravel()], 1))
    edges = np.concatenate(edges, axis=0).astype(np.int32)
    R = 1.5 * radius
    rho = np.full(edges.shape[0], radius)
    w = weight_for_radius(rho, R)
    return Lattice(nodes.astype(dtype), edges, w.astype(dtype), R, 1.0,
                   rho.astype(dtype))


def graded_density(x: np.ndarray, size: float, rng) -> np.ndarray:
    """rho(x) linear in x from 0 to 1 across the cube, plus N(0, 0.05) noise,
    clamped to [0.15, 1]."""
    rho = x / size + rng.normal(0.0, 0.05, size=x.shape)
    return np.clip(rho, 0.15, 1.0)


def blob_density(points: np.ndarray, size: float, rng, n_blobs: int = 8,
                 sigma=(10.0, 30.0)) -> np.ndarray:
    """Sum of n_blobs isotropic Gaussians with centres ~ U[0,size]^3 and
    widths ~ U[sigma], capped at 1."""
    c = rng.uniform(0.0, size, size=(n_blobs, 3))
    s = rng.uniform(sigma[0], sigma[1], size=n_blobs)
    rho = np.zeros(points.shape[0])
    for k in range(n_blobs):
        d2 = np.sum((points - c[k]) ** 2, axis=1)
        rho += np.exp(-d2 / (2.0 * s[k] ** 2))
    return np.minimum(rho, 1.0)


def kuhn_lattice(n: int, size: float = 100.0, *, seed: int, jitter: float = 0.3,
                 radius: str = "graded", r_min: float = 0.2, r_span: float = 0.8,
                 void_below: float | None = None, dtype=np.float32) -> Lattice:
    """Tetrahedral lattice: a cube of side `size` split into n^3 cubes, each
    Kuhn-split into 6 tets; edges deduplicated.  Every node is jittered by
    U(-jitter, jitter) x cell per coordinate.  Radii are evaluated at the
    strut midpoint after jitter:

    * radius="graded": rho = graded_density(x), r = r_min + r_span * rho;
    * radius="blobs": rho = blob_density (8 blobs), r = r_min + r_span * rho,
      and struts with rho < void_below get weight 0 (absent).
    """
    rng = np.random.default_rng(seed)
    cell = size / n
    nodes = _grid_nodes(n, size)
    nodes += rng.uniform(-jitter, jitter, size=nodes.shape) * cell
    edges = kuhn_edges(n)
    r_max = r_min + r_span
    R = 1.5 * r_max
    E = edges.shape[0]
    rho_all = np.empty(E)
    chunk = 1 << 22
    blobs_rng = np.random.default_rng(seed + 1000) if radius == "blobs" else None
    blob_params = None
    if radius == "blobs":
        blob_params = (blobs_rng.uniform(0.0, size, size=(8, 3)),
                       blobs_rng.uniform(10.0, 30.0, size=8))
    for s in range(0, E, chunk):
        e = edges[s:s + chunk]
        mid = 0.5 * (nodes[e[:, 0]] + nodes[e[:, 1]])
        if radius == "graded":
            rho_all[s:s + chunk] = graded_density(mid[:, 0], size, rng)
        elif radius == "blobs":
            c, sg = blob_params
            acc = np.zeros(mid.shape[0])
            for k in range(8):
                d2 = np.sum((mid - c[k]) ** 2, axis=1)
                acc += np.exp(-d2 / (2.0 * sg[k] ** 2))
            rho_all[s:s + chunk] = np.minimum(acc, 1.0)
        else:
            raise ValueError(radius)
    r = r_min + r_span * rho_all
    w = weight_for_radius(r, R)
    if void_below is not None:
        w = np.where(rho_all < void_below, 0.0, w)
    return Lattice(nodes.astype(dtype), edges, w.astype(dtype), R, 1.0,
                   r.astype(dtype))


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------
def grid_for(lat: Lattice, W: int, H: int, n_slices: int, dz: float | None = None,
             z0: float | None = None) -> Grid:
    """Square pixels over the xy bounding box grown by R plus two pixels on
    each side; slices from the lowest node upward (pitch dz, or the node
    height split evenly into n_slices when dz is None)."""
    nd = lat.nodes.astype(np.float64)
    lo = nd.min(axis=0)
    hi = nd.max(axis=0)
    ext = hi - lo
    d = max((ext[0] + 2 * lat.R) / (W - 4), (ext[1] + 2 * lat.R) / (H - 4))
    x0 = lo[0] - lat.R - 2 * d
    y0 = lo[1] - lat.R - 2 * d
    zz0 = lo[2] if z0 is None else z0
    if dz is None:
        dz = ext[2] / n_slices
    return Grid(float(x0), float(y0), float(d), float(d), int(W), int(H),
                float(zz0), float(dz), int(n_slices))


def target_density(grid: Grid, k: np.ndarray, size: float = 100.0,
                   seed: int = 4) -> np.ndarray:
    """Seeded 8-blob density (widths U[10,30]) sampled at the pixel centres of
    slices k: array [len(k), H, W] float32.  Used as the soft-occupancy
    target of the differentiable slice loss."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, size, size=(8, 3))
    s = rng.uniform(10.0, 30.0, size=8)
    X, Y = np.meshgrid(grid.pixel_x(), grid.pixel_y(), indexing="xy")
    out = np.empty((len(k), grid.H, grid.W), dtype=np.float32)
    for i, kk in enumerate(np.asarray(k)):
        z = float(grid.slice_z(kk))
        acc = np.zeros_like(X)
        for b in range(8):
            d2 = (X - c[b, 0]) ** 2 + (Y - c[b, 1]) ** 2 + (z - c[b, 2]) ** 2
            acc += np.exp(-d2 / (2.0 * s[b] ** 2))
        out[i] = np.minimum(acc, 1.0)
    return out


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
CONFIGS = {
    # name: (builder kwargs, grid)
    "P1": "uniform BCC 4^3 cells of 5 mm, r=0.5, 50 slices at 0.1 mm, 256^2, FP64",
    "A2": "Kuhn 40^3 in a 100 mm cube, graded r in [0.2,1.0], 1000 slices at 0.1 mm, 2048^2, FP32",
    "B3": "Kuhn 110^3 in a 100 mm cube, 8-blob r in [0.1,0.6] with voids, 2000 slices at 0.05 mm, 4096^2, FP32",
    "D4": "Kuhn 25^3 in a 100 mm cube, graded r in [0.2,1.0], 64 slices over the height, 1024^2, FP32",
    "S5": "Kuhn 243^3 in a 200 mm cube, graded r in [0.1,0.6], 4000 slices at 0.05 mm, 8192^2, FP32",
    "M1": "Kuhn 52^3 in a 100 mm cube, graded r in [0.2,1.0], 1000 slices at 0.1 mm, 2048^2, FP32",
    "M1R": "M1 with per-strut supports R_j = 1.5 r_j (kernel variant)",
    "M1G": "M1 under the compact Gaussian kernel, sigma = R/3 (kernel variant)",
}


def config(name: str, *, scale: int | None = None):
    """Build (lattice, grid) for a named workload.  `scale` overrides the cube
    count n of the Kuhn workloads (smaller test cases of the same recipe)."""
    if name == "P1":
        lat = bcc_lattice(4, 5.0, 0.5, dtype=np.float64)
        return lat, grid_for(lat, 256, 256, 50, dz=0.1)
    if name == "A2":
        lat = kuhn_lattice(scale or 40, 100.0, seed=2)
        return lat, grid_for(lat, 2048, 2048, 1000, dz=0.1)
    if name == "B3":
        lat = kuhn_lattice(scale or 110, 100.0, seed=3, radius="blobs",
                           r_min=0.1, r_span=0.5, void_below=0.15)
        return lat, grid_for(lat, 4096, 4096, 2000, dz=0.05)
    if name == "D4":
        lat = kuhn_lattice(scale or 25, 100.0, seed=4)
        return lat, grid_for(lat, 1024, 1024, 64)
    if name == "S5":
        lat = kuhn_lattice(scale or 243, 200.0, seed=5, r_min=0.1, r_span=0.5)
        return lat, grid_for(lat, 8192, 8192, 4000, dz=0.05)
    if name == "M1":
        lat = kuhn_lattice(scale or 52, 100.0, seed=6)
        return lat, grid_for(lat, 2048, 2048, 1000, dz=0.1)
    if name in ("M1R", "M1G"):
        lat, grid = config("M1", scale=scale)
        return (with_supports(lat) if name == "M1R" else with_gauss(lat)), grid
    raise KeyError(name)


def kuhn_edge_count(n: int) -> int:
    return 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3


def tiny_lattice(kind: str, dtype=np.float64) -> Lattice:
    """Hand-built fixtures: 'one' (a single strut), 'collinear' (two struts
    end to end on one line), 'tjoint' (three struts meeting at a node),
    'mirror' (two struts mirrored in the plane x = 0)."""
    R = 1.5
    if kind == "one":
        nodes = np.array([[0.2, -0.3, 0.1], [2.9, 1.4, 1.7]])
        edges = np.array([[0, 1]])
    elif kind == "collinear":
        nodes = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.25], [3.0, 1.5, 0.75]])
        edges = np.array([[0, 1], [1, 2]])
    elif kind == "tjoint":
        nodes = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [-2.0, 0.0, 0.0],
                          [0.0, 0.0, 2.5]])
        edges = np.array([[0, 1], [2, 0], [0, 3]])
    elif kind == "mirror":
        nodes = np.array([[0.5, 0.0, 0.0], [2.0, 1.0, 0.5], [-0.5, 0.0, 0.0],
                          [-2.0, 1.0, 0.5]])
        edges = np.array([[0, 1], [2, 3]])
    else:
        raise KeyError(kind)
    rho = np.full(len(edges), 0.5)
    w = weight_for_radius(rho, R)
    return Lattice(nodes.astype(dtype), edges.astype(np.int32), w.astype(dtype),
                   R, 1.0, rho.astype(dtype))


def random_lattice(n_nodes: int, n_edges: int, extent: float, *, seed: int,
                   r_lo: float = 0.2, r_hi: float = 1.0, dtype=np.float32,
                   zero_frac: float = 0.0) -> Lattice:
    """Random struts between random nodes in a box (edge cases: long struts,
    degenerate zero-length struts when both ends coincide, absent struts)."""
    rng = np.random.default_rng(seed)
    nodes = rng.uniform(0.0, extent, size=(n_nodes, 3))
    a = rng.integers(0, n_nodes, size=n_edges)
    b = rng.integers(0, n_nodes, size=n_edges)
    edges = np.stack([a, b], axis=1).astype(np.int32)
    R = 1.5 * r_hi
    rho = rng.uniform(r_lo, r_hi, size=n_edges)
    w = weight_for_radius(rho, R)
    if zero_frac > 0:
        w[rng.uniform(size=n_edges) < zero_frac] = 0.0
    return Lattice(nodes.astype(dtype), edges, w.astype(dtype), R, 1.0,
                   rho.astype(dtype))
