"""Kernel, per-strut integral and field sums of the convolution surface.

Test infrastructure (see the package docstring).  Everything is float64.
The quartic kernel uses only +, -, *, / and sqrt, so each element's value does
not depend on how numpy vectorises the array it sits in.

Two variants beyond the paper's single support R (both readings of its
comparisons, not its method):
  * per-strut supports: R may be an array with one radius per strut; strut i
    then uses R_i in Eq. (5) and everywhere R bounds its reach;
  * the Gaussian kernel the paper compares against, made compact: the
    shifted, truncated Gaussian f(d) = exp(-d^2 / 2 sigma^2) - exp(-R^2 /
    2 sigma^2) for d < R, else 0 (continuous at R, zero outside the same
    support, so the same culling applies).
"""
from __future__ import annotations

import numpy as np


def _dot3(A, B):
    """Row-wise dot product of [...,3] arrays, summed x + y + z in order."""
    A = np.broadcast_to(A, np.broadcast_shapes(np.shape(A), np.shape(B)))
    B = np.broadcast_to(B, A.shape)
    return A[..., 0] * B[..., 0] + A[..., 1] * B[..., 1] + A[..., 2] * B[..., 2]


def support_of(R, i: int) -> float:
    """The support radius of strut i: R is one radius for all struts, or an
    array of per-strut radii."""
    return float(R[i]) if np.ndim(R) else float(R)


def kernel(dist, R: float):
    """Eq. (5): f = (1 - |p - x|^2 / R^2)^2 where |p - x| < R, else 0."""
    d = np.asarray(dist, dtype=np.float64)
    t = 1.0 - d * d / (R * R)
    return np.where(d < R, t * t, 0.0)


def strut_integral(P, vs, ve, R: float) -> np.ndarray:
    """Integral of the kernel over the edge (vs, ve) for each point of P.

    Sec. 3.2, Eq. (6)-(7).  For a query point p, the line of the edge meets
    the sphere of radius R around p at p1 and p2 (p1 before p2 in the
    direction vs -> ve); s1, s2 are the parameters of the edge ends along the
    chord x(s) = (1 - s) p1 + s p2, clipped to [0, 1]; with l = |p2 - p1| and
    a = (p - p1).(p2 - p1) the s-integral of f has the closed form

        (3 l^4 s^5 - 15 a l^2 s^4 + 20 a^2 s^3) / (15 R^4)  from s1 to s2.

    Eq. (6) integrates with respect to arclength on the edge, and
    d(arclength) = l ds along the chord, so the result is l times that
    difference (the printed Eq. (7) omits the factor l).  The term is zero
    when the line misses the open ball (no chord), when the edge has zero
    length, or when the edge lies outside the chord (s2 <= s1).

    P, vs, ve: [..., 3] arrays broadcast against each other (many points
    and one strut, or one point and many struts).  Returns float64 [...].
    """
    P = np.asarray(P, dtype=np.float64)
    vs = np.asarray(vs, dtype=np.float64)
    ve = np.asarray(ve, dtype=np.float64)
    shape = np.broadcast_shapes(P.shape, vs.shape, ve.shape)[:-1]
    P, vs, ve = (np.broadcast_to(x, shape + (3,)).reshape(-1, 3) for x in (P, vs, ve))
    d = ve - vs
    L2 = _dot3(d, d)
    live = L2 > 0.0                       # zero-length struts add nothing
    u = d / np.sqrt(np.where(live, L2, 1.0))[:, None]
    # foot of p on the line, and squared distance of p from the line
    w = P - vs
    t0 = _dot3(w, u)
    perp = w - t0[:, None] * u
    dperp2 = _dot3(perp, perp)
    hit = live & (dperp2 < R * R)
    h = np.sqrt(np.where(hit, R * R - dperp2, 0.0))
    foot = vs + t0[:, None] * u
    p1 = foot - h[:, None] * u
    p2 = foot + h[:, None] * u
    e = p2 - p1
    l2 = _dot3(e, e)
    l = np.sqrt(l2)
    safe = np.where(hit, l2, 1.0)
    s1 = np.maximum(0.0, _dot3(vs - p1, e) / safe)
    s2 = np.minimum(1.0, _dot3(ve - p1, e) / safe)
    a = _dot3(P - p1, e)

    def F(s):
        s3 = s * s * s
        s4 = s3 * s
        s5 = s4 * s
        l4 = l2 * l2
        return (3.0 * l4 * s5 - 15.0 * a * l2 * s4 + 20.0 * a * a * s3) / (
            15.0 * R ** 4)

    val = l * (F(s2) - F(s1))
    val = np.where(hit & (s2 > s1), val, 0.0)
    return val.reshape(shape)


def kernel_gauss(dist, R: float, sigma: float):
    """The compact Gaussian variant: exp(-d^2/2s^2) - exp(-R^2/2s^2) for
    d < R, else 0."""
    d = np.asarray(dist, dtype=np.float64)
    k = np.exp(-d * d / (2.0 * sigma * sigma)) - np.exp(-R * R / (2.0 * sigma * sigma))
    return np.where(d < R, k, 0.0)


def strut_integral_gauss(P, vs, ve, R: float, sigma: float) -> np.ndarray:
    """Integral of kernel_gauss over the edge (vs, ve) by arclength, for each
    point of P.  Along the line, with t measured from the foot of p and d the
    distance of p from the line, the support is t in [-h, h], h^2 = R^2 - d^2,
    and the edge covers t in [alpha, beta]; over the clamped interval
    [ca, cb]:
        exp(-d^2/2s^2) s sqrt(pi/2) [erf(cb/(s sqrt 2)) - erf(ca/(s sqrt 2))]
          - exp(-R^2/2s^2) (cb - ca),
    zero when the line misses the ball, the edge has zero length, or the
    clamped interval is empty."""
    from scipy.special import erf
    P = np.asarray(P, dtype=np.float64)
    vs = np.asarray(vs, dtype=np.float64)
    ve = np.asarray(ve, dtype=np.float64)
    shape = np.broadcast_shapes(P.shape, vs.shape, ve.shape)[:-1]
    P, vs, ve = (np.broadcast_to(x, shape + (3,)).reshape(-1, 3) for x in (P, vs, ve))
    d = ve - vs
    L2 = _dot3(d, d)
    live = L2 > 0.0
    L = np.sqrt(np.where(live, L2, 1.0))
    u = d / L[:, None]
    w = vs - P
    alpha = _dot3(w, u)                 # lower end, from the foot of p
    beta = alpha + L
    perp = w - alpha[:, None] * u
    dperp2 = _dot3(perp, perp)
    hit = live & (dperp2 < R * R)
    h = np.sqrt(np.where(hit, R * R - dperp2, 0.0))
    ca = np.clip(alpha, -h, h)
    cb = np.clip(beta, -h, h)
    s2 = sigma * np.sqrt(2.0)
    val = (np.exp(-dperp2 / (2.0 * sigma * sigma)) * sigma * np.sqrt(np.pi / 2.0)
           * (erf(cb / s2) - erf(ca / s2))
           - np.exp(-R * R / (2.0 * sigma * sigma)) * (cb - ca))
    val = np.where(hit & (cb > ca), val, 0.0)
    return val.reshape(shape)


def strut_term(P, vs, ve, R: float, kind: str = "quartic", sigma: float | None = None):
    """The integral of strut (vs, ve) with support R under kernel `kind`
    ("quartic": Eq. (5); "gauss": kernel_gauss with width sigma)."""
    if kind == "quartic":
        return strut_integral(P, vs, ve, R)
    if kind == "gauss":
        return strut_integral_gauss(P, vs, ve, R, sigma)
    raise ValueError(f"unknown kernel {kind!r}")


def field_at(points, nodes, edges, weight, R, struts=None, kind: str = "quartic",
             sigma: float | None = None) -> np.ndarray:
    """g(p) = sum_i r_i * integral_i(p) (Eq. 6 without the -C), summed in
    ascending strut id, one strut at a time.  `struts` restricts the sum to a
    subset of ids (given in ascending order); omitted struts must contribute
    exactly zero for the result to equal the full sum.  R: one support or
    one per strut."""
    points = np.asarray(points, dtype=np.float64)
    nodes = np.asarray(nodes, dtype=np.float64)
    weight = np.asarray(weight, dtype=np.float64)
    g = np.zeros(points.shape[:-1])
    ids = range(len(edges)) if struts is None else struts
    for i in ids:
        if weight[i] == 0.0:
            continue
        g = g + weight[i] * strut_term(points, nodes[edges[i, 0]], nodes[edges[i, 1]],
                                       support_of(R, i), kind, sigma)
    return g


def line_integral_quadrature(p, vs, ve, R: float, epsabs=1e-13, epsrel=1e-11,
                             kind: str = "quartic", sigma: float | None = None):
    """Eq. (6) for one strut by adaptive quadrature of the kernel along the
    edge (arclength): an independent route to strut_integral (and to
    strut_integral_gauss with kind="gauss")."""
    from scipy.integrate import quad
    p = np.asarray(p, dtype=np.float64)
    vs = np.asarray(vs, dtype=np.float64)
    ve = np.asarray(ve, dtype=np.float64)
    L = float(np.linalg.norm(ve - vs))
    if L == 0.0:
        return 0.0
    u = (ve - vs) / L

    def f(t):
        x = vs + t * u
        dist = np.linalg.norm(p - x)
        if kind == "gauss":
            return float(kernel_gauss(dist, R, sigma))
        return float(kernel(dist, R))

    # split at the chord ends so the integrand is smooth on each piece
    t0 = float(np.dot(p - vs, u))
    dperp2 = float(np.dot(p - vs - t0 * u, p - vs - t0 * u))
    pts = [0.0, L]
    if dperp2 < R * R:
        h = np.sqrt(R * R - dperp2)
        pts += [t for t in (t0 - h, t0, t0 + h) if 0.0 < t < L]
    pts = sorted(pts)
    total = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        v, _ = quad(f, lo, hi, epsabs=epsabs, epsrel=epsrel, limit=200)
        total += v
    return total


def field_at_point(p, nodes, edges, weight, R, struts=None, kind: str = "quartic",
                   sigma: float | None = None) -> float:
    """g at one point p: every strut's integral at p (one array operation
    over the struts) times its weight, summed in ascending strut id.  R: one
    support or one per strut."""
    nodes = np.asarray(nodes, dtype=np.float64)
    ids = np.arange(len(edges)) if struts is None else np.asarray(struts)
    A = nodes[edges[ids, 0]]
    B = nodes[edges[ids, 1]]
    # per-strut supports broadcast element by element with the struts
    Rs = np.asarray(R, dtype=np.float64)[ids] if np.ndim(R) else R
    I = strut_term(np.asarray(p, dtype=np.float64)[None, :], A, B, Rs, kind, sigma)
    terms = np.asarray(weight, dtype=np.float64)[ids] * I
    return float(np.cumsum(terms)[-1]) if len(terms) else 0.0
