"""Derivatives of a pixel-weighted field sum, for the radius-tuning step.

Test infrastructure (see the package docstring).

Sec. 5.3 tunes strut weights r_i (and the framework moves nodes) to match a
target density, which needs the derivative of a loss of the sliced field.
For a loss L(g) over sample points p with G(p) = dL/dg(p), the chain rule
gives

  dL/dr_i   = sum_p G(p) I_i(p)
  dL/dv     = sum_p G(p) r_i dI_i/dv        for each end v of strut i,

with I_i the integral of Eq. (6) for strut i (R may be one support or an
array of per-strut supports).  Below, the strut (a, b) is
described along its unit direction u with the foot of p as origin: the ends
sit at alpha = (a - p).u and beta = alpha + |b - a|; the support meets the
line on [-h, h] with h^2 = H = R^2 - |q|^2 + alpha^2 (q = a - p); and

  I = R^-4 * integral over [clamp(alpha), clamp(beta)] of (H - t^2)^2 dt.

Differentiating under the integral sign (the integrand vanishes at -h and h,
so clamped limits contribute nothing):

  dI/dalpha = -phi(alpha), dI/dbeta = phi(beta), phi(t) = max(H - t^2, 0)^2 R^-4
  dI/dH     = 2 R^-4 [ (cb - ca) H - (cb^3 - ca^3) / 3 ]

and alpha, beta, H depend on a and b through u = (b - a)/|b - a|:

  d alpha/db = q_perp/|d|,  d alpha/da = u - q_perp/|d|,   q_perp = q - alpha u
  d beta/db  = q_perp/|d| + u,   d beta/da = -q_perp/|d|
  dH/db      = 2 alpha d alpha/db,   dH/da = -2 q + 2 alpha d alpha/da
"""
from __future__ import annotations

import numpy as np

from .field import strut_integral, support_of


def strut_partials(P, a, b, R: float):
    """(I, dI/da, dI/db) at points P [M,3] for strut (a, b).  The partials
    are [M,3]."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 3)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    M = P.shape[0]
    d = b - a
    Ld = float(np.sqrt(d @ d))
    if Ld == 0.0:
        z = np.zeros((M, 3))
        return np.zeros(M), z, z.copy()
    u = d / Ld
    q = a - P
    alpha = q @ u
    beta = alpha + Ld
    H = R * R - np.einsum("ij,ij->i", q, q) + alpha * alpha
    pos = H > 0.0
    h = np.sqrt(np.where(pos, H, 0.0))
    ca = np.clip(alpha, -h, h)
    cb = np.clip(beta, -h, h)
    R4 = R ** 4
    phi_a = np.maximum(H - alpha * alpha, 0.0) ** 2 / R4
    phi_b = np.maximum(H - beta * beta, 0.0) ** 2 / R4
    I_alpha = -phi_a
    I_beta = phi_b
    I_H = 2.0 * ((cb - ca) * H - (cb ** 3 - ca ** 3) / 3.0) / R4
    I_H = np.where(pos, I_H, 0.0)
    qp = q - alpha[:, None] * u
    dal_db = qp / Ld
    dal_da = u - qp / Ld
    dbe_db = qp / Ld + u
    dbe_da = -qp / Ld
    dH_db = 2.0 * alpha[:, None] * dal_db
    dH_da = -2.0 * q + 2.0 * alpha[:, None] * dal_da
    dI_da = (I_alpha[:, None] * dal_da + I_beta[:, None] * dbe_da
             + I_H[:, None] * dH_da)
    dI_db = (I_alpha[:, None] * dal_db + I_beta[:, None] * dbe_db
             + I_H[:, None] * dH_db)
    I = strut_integral(P, a, b, R)
    return I, dI_da, dI_db


def field_vjp(points, G, nodes, edges, weight, R, struts=None):
    """Gradient of L = sum_p G(p) g(p) with respect to the weights [E] and the
    node positions [N,3], float64.  `struts` limits the work to struts that
    can be non-zero at the points (others have zero gradient)."""
    P = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    G = np.asarray(G, dtype=np.float64).reshape(-1)
    nodes64 = np.asarray(nodes, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    gw = np.zeros(len(edges))
    gn = np.zeros((len(nodes64), 3))
    ids = range(len(edges)) if struts is None else struts
    for i in ids:
        # a weight of 0 has the same derivative as any other: Eq. (6) is
        # linear in r_i (its node terms carry the factor r_i = 0)
        ia, ib = int(edges[i, 0]), int(edges[i, 1])
        I, dA, dB = strut_partials(P, nodes64[ia], nodes64[ib], support_of(R, i))
        gw[i] = np.dot(G, I)
        gn[ia] += w[i] * (G @ dA)
        gn[ib] += w[i] * (G @ dB)
    return gw, gn


def soft_occupancy_grad(g, target, C: float, tau: float):
    """G = dL/dg for L = sum (sigmoid((g - C)/tau) - target)^2, with the
    sigmoid's derivative s (1 - s) written sigmoid(z) sigmoid(-z) (the same
    value, without losing 1 - s to cancellation where s rounds to 1)."""
    from scipy.special import expit
    z = (np.asarray(g, dtype=np.float64) - C) / tau
    s = expit(z)
    return 2.0 * (s - target) * s * expit(-z) / tau


def soft_occupancy_loss(g, target, C: float, tau: float) -> float:
    from scipy.special import expit
    s = expit((np.asarray(g, dtype=np.float64) - C) / tau)
    return float(np.sum((s - target) ** 2))


def slice_vjp(nodes, edges, weight, R, grid, ks, G, struts=None):
    """field_vjp over the pixel centres of planes ks with G [len(ks), H, W]:
    each active strut (Eq. 8) is evaluated over the window of pixels its
    support can reach (outside it every term and partial is exactly zero).
    `struts` restricts the sum to a subset of ids: the weight gradient of
    those struts is then exact, and a node's gradient is exact when every
    strut at the node is in the subset."""
    from .slicer import active_set, strut_z_range, _pixel_window
    keep = None if struts is None else set(int(i) for i in struts)
    nodes64 = np.asarray(nodes, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    gw = np.zeros(len(edges))
    gn = np.zeros((len(nodes64), 3))
    zlo, zhi = strut_z_range(nodes64, edges)
    xs, ys = grid.pixel_x(), grid.pixel_y()
    for kk, k in enumerate(ks):
        z = float(grid.slice_z(k))
        Gk = np.asarray(G[kk], dtype=np.float64)
        for i in active_set(zlo, zhi, R, z):
            if struts is not None and i not in keep:
                continue
            ia, ib = int(edges[i, 0]), int(edges[i, 1])
            a, b = nodes64[ia], nodes64[ib]
            Ri = support_of(R, i)
            ix0, ix1 = _pixel_window(min(a[0], b[0]) - Ri, max(a[0], b[0]) + Ri,
                                     grid.x0, grid.dx, grid.W)
            iy0, iy1 = _pixel_window(min(a[1], b[1]) - Ri, max(a[1], b[1]) + Ri,
                                     grid.y0, grid.dy, grid.H)
            if ix0 > ix1 or iy0 > iy1:
                continue
            X, Y = np.meshgrid(xs[ix0:ix1 + 1], ys[iy0:iy1 + 1], indexing="xy")
            P = np.stack([X, Y, np.full_like(X, z)], axis=-1).reshape(-1, 3)
            g = Gk[iy0:iy1 + 1, ix0:ix1 + 1].reshape(-1)
            I, dA, dB = strut_partials(P, a, b, Ri)
            gw[i] += np.dot(g, I)
            gn[ia] += w[i] * (g @ dA)
            gn[ib] += w[i] * (g @ dB)
    return gw, gn
