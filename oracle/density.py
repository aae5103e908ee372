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


def voxel_sums(x: np.ndarray, vx: int, vy: int, vz: int) -> np.ndarray:
    """Sum of x over each voxel: consecutive runs of vz planes, vy rows and
    vx columns, the last run of each axis shorter when the size is ragged."""
    x = np.asarray(x, dtype=np.float64)
    nk, H, W = x.shape
    x = np.add.reduceat(x, np.arange(0, nk, vz), axis=0)
    x = np.add.reduceat(x, np.arange(0, H, vy), axis=1)
    return np.add.reduceat(x, np.arange(0, W, vx), axis=2)


def voxel_samples(shape, vx: int, vy: int, vz: int) -> np.ndarray:
    """Number of pixel-centre samples in each voxel."""
    return voxel_sums(np.ones(shape), vx, vy, vz)


def voxel_density(field: np.ndarray, C: float, vx: int, vy: int, vz: int) -> np.ndarray:
    """[ceil(nk/vz), ceil(H/vy), ceil(W/vx)] float64 fractions of samples with
    g >= C."""
    inside = np.asarray(field) >= C
    return voxel_sums(inside, vx, vy, vz) / voxel_samples(inside.shape, vx, vy, vz)


def soft_density(field, C: float, tau: float, vx: int, vy: int, vz: int) -> np.ndarray:
    """Per-voxel mean of the soft inside test s = sigmoid((g - C) / tau).

    Not in the paper: the hard test of Eq. (9) has no useful derivative, so
    the radius adjustment descends this smooth stand-in, which tends to the
    hard density as tau -> 0 wherever no sample sits on the iso-surface.
    """
    g = np.asarray(field, dtype=np.float64)
    s = expit((g - C) / tau)
    return voxel_sums(s, vx, vy, vz) / voxel_samples(g.shape, vx, vy, vz)


def density_loss(field, target, C: float, tau: float, vx: int, vy: int, vz: int):
    """L = sum_v (soft_density_v - target_v)^2, the soft densities and dL/dg
    per pixel.

    dL/dg(p) = 2 (soft_density_v - target_v) / n_v * s (1 - s) / tau for the
    voxel v holding pixel p, n_v its sample count.
    """
    g = np.asarray(field, dtype=np.float64)
    nk, H, W = g.shape
    rho = soft_density(g, C, tau, vx, vy, vz)
    r = rho - np.asarray(target, dtype=np.float64)
    loss = float(np.sum(r * r))
    z = (g - C) / tau
    ds = expit(z) * expit(-z)        # s (1 - s), with 1 - s = sigmoid(-z): no cancellation
    n = voxel_samples(g.shape, vx, vy, vz)
    # the voxel of every pixel, axis by axis
    l = (np.arange(nk) // vz)[:, None, None]
    j = (np.arange(H) // vy)[None, :, None]
    i = (np.arange(W) // vx)[None, None, :]
    grad = 2.0 * r[l, j, i] / n[l, j, i] * ds / tau
    return loss, rho, grad
