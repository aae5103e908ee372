"""Per-voxel material density of the sliced solid (Sec. 5, Eq. 9).

Test infrastructure (see the package docstring).

The paper evaluates the density of S(Omega) inside a voxel V by Monte-Carlo
integration with the inside test g >= C.  Reading fixed here: the samples are
the pixel centres of the slice planes (a stratified sample, the points the
slicer already evaluates); voxel (l, j, i) holds planes [l vz, (l+1) vz),
rows [j vy, (j+1) vy) and columns [i vx, (i+1) vx) of the given planes,
clipped at the last plane, row and column, and its density is the fraction of
its samples that are inside.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit


def voxel_density(field: np.ndarray, C: float, vx: int, vy: int, vz: int) -> np.ndarray:
    """[ceil(nk/vz), ceil(H/vy), ceil(W/vx)] float64 fractions."""
    inside = np.asarray(field) >= C
    nk, H, W = inside.shape
    nz, ny, nx = -(-nk // vz), -(-H // vy), -(-W // vx)
    out = np.zeros((nz, ny, nx))
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                block = inside[l * vz:(l + 1) * vz, j * vy:(j + 1) * vy, i * vx:(i + 1) * vx]
                out[l, j, i] = block.mean()
    return out


def _voxel_mean(x: np.ndarray, vx: int, vy: int, vz: int) -> np.ndarray:
    nk, H, W = x.shape
    nz, ny, nx = -(-nk // vz), -(-H // vy), -(-W // vx)
    out = np.zeros((nz, ny, nx))
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                out[l, j, i] = x[l * vz:(l + 1) * vz, j * vy:(j + 1) * vy, i * vx:(i + 1) * vx].mean()
    return out


def soft_density(field, C: float, tau: float, vx: int, vy: int, vz: int) -> np.ndarray:
    """Per-voxel mean of the soft inside test s = sigmoid((g - C) / tau).

    Not in the paper: the hard test of Eq. (9) has no useful derivative, so
    the radius adjustment descends this smooth stand-in, which tends to the
    hard density as tau -> 0 wherever no sample sits on the iso-surface.
    """
    g = np.asarray(field, dtype=np.float64)
    s = expit((g - C) / tau)
    return _voxel_mean(s, vx, vy, vz)


def density_loss(field, target, C: float, tau: float, vx: int, vy: int, vz: int):
    """L = sum_v (soft_density_v - target_v)^2 and dL/dg per pixel.

    dL/dg(p) = 2 (soft_density_v - target_v) / n_v * s (1 - s) / tau for the
    voxel v holding pixel p, n_v its sample count.
    """
    g = np.asarray(field, dtype=np.float64)
    nk, H, W = g.shape
    rho = soft_density(g, C, tau, vx, vy, vz)
    r = rho - np.asarray(target, dtype=np.float64)
    loss = float(np.sum(r * r))
    s = expit((g - C) / tau)
    grad = np.zeros_like(g)
    for k in range(nk):
        for y in range(H):
            for x in range(W):
                l, j, i = k // vz, y // vy, x // vx
                nv = (min(nk, (l + 1) * vz) - l * vz) * (min(H, (j + 1) * vy) - j * vy) * \
                     (min(W, (i + 1) * vx) - i * vx)
                grad[k, y, x] = 2.0 * r[l, j, i] / nv * s[k, y, x] * (1.0 - s[k, y, x]) / tau
    return loss, rho, grad
