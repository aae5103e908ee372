"""Self-support metrics of a lattice (Sec. 5.2, Eqs. 11-14, Appendix II) and
the gradient of Gamma with respect to node positions (for the vertex
position optimisation of Sec. 5.2).

Test infrastructure (see the package docstring).

* theta_j = arccos |u_j . t_P| (Eq. 11), u_j the unit direction of edge j,
  t_P the unit printing direction.  Edge j is self-supported when
  theta_j <= alpha, alpha = pi/4 (the paper's parameter).
* g(theta): the paper's polynomial for alpha = pi/4 (Eq. 12),
  sum_i a_i theta^i with a = [-0.02, -0.31, 1.44, -1.11, 0.58, -0.16] for
  theta > alpha, 0 otherwise.
* Gamma = sum_{j not supported} r_j L_j g(theta_j) / sum_j r_j L_j (Eq. 13),
  Psi = 100 * sum_{j supported} L_j / sum_j L_j (Eq. 14); r_j is the edge's
  weight (the radius the paper stores on the edge), L_j its length.
  Zero-length edges add nothing to any sum.
* g_exact: the ratio of Appendix II, read as the arc length of the projected
  bottom circle (an ellipse of semi-axes 1 and cos theta, arc element
  sqrt(sin^2 phi + cos^2 theta cos^2 phi)) over phi in (phi_0, pi/2), the
  risky part, relative to (0, pi/2), phi_0 = arcsin(sin alpha / sin theta).
  The printed integrand has sin^2 theta and the printed numerator runs over
  (0, phi_0); with those, the ratio would fall from 1 to 1/2 as the strut
  tilts, against the text and the polynomial it is said to approximate.
  Used only to pin the polynomial.
* dGamma/dv: with N = sum r L g, D = sum r L, Gamma = N / D and, per edge,
  c = u . t, dL/dv_e = u, dc/dv_e = (t - c u) / L,
  dtheta/dc = -sign(c) / sqrt(1 - c^2):
      dGamma/dv_e += r [g u + g'(theta) dtheta/dc (t - c u) - Gamma u] / D
  for an unsupported edge (g = g' = 0 for a supported one), and the
  opposite for v_s.  The step of g at theta = alpha has no derivative and is
  left out.
"""
from __future__ import annotations

import numpy as np

ALPHA = np.pi / 4
A = np.array([-0.02, -0.31, 1.44, -1.11, 0.58, -0.16])


def g_poly(theta):
    """Eq. (12) for alpha = pi/4."""
    theta = np.asarray(theta, dtype=np.float64)
    p = np.zeros_like(theta)
    for i, a in enumerate(A):
        p = p + a * theta ** i
    return np.where(theta > ALPHA, p, 0.0)


def g_poly_prime(theta):
    theta = np.asarray(theta, dtype=np.float64)
    p = np.zeros_like(theta)
    for i, a in enumerate(A[1:], start=1):
        p = p + i * a * theta ** (i - 1)
    return np.where(theta > ALPHA, p, 0.0)


def g_exact(theta: float, alpha: float = ALPHA) -> float:
    """Appendix II's ratio of risky projected arc (reading in the module
    docstring), by quadrature."""
    from scipy.integrate import quad
    if np.sin(theta) <= np.sin(alpha):
        return 0.0
    phi0 = np.arcsin(np.sin(alpha) / np.sin(theta))
    c2 = np.cos(theta) ** 2
    f = lambda p: np.sqrt(np.sin(p) ** 2 + c2 * np.cos(p) ** 2)
    return quad(f, phi0, np.pi / 2)[0] / quad(f, 0.0, np.pi / 2)[0]


def edge_geometry(nodes, edges, t):
    nodes = np.asarray(nodes, dtype=np.float64)
    d = nodes[edges[:, 1]] - nodes[edges[:, 0]]
    L = np.sqrt((d * d).sum(axis=1))
    ok = L > 0
    u = np.zeros_like(d)
    u[ok] = d[ok] / L[ok, None]
    c = u @ np.asarray(t, dtype=np.float64)
    theta = np.arccos(np.clip(np.abs(c), 0.0, 1.0))
    return L, u, c, theta, ok


def metrics(nodes, edges, weight, t):
    """(Gamma, Psi) of Eqs. (13)-(14) and the four sums behind them."""
    L, u, c, theta, ok = edge_geometry(nodes, edges, t)
    r = np.asarray(weight, dtype=np.float64)
    sup = (theta <= ALPHA) & ok
    g = np.where(ok, g_poly(theta), 0.0)
    N = float(np.sum(np.where(~sup & ok, r * L * g, 0.0)))
    D = float(np.sum(r * L))
    Ls = float(np.sum(np.where(sup, L, 0.0)))
    Lt = float(np.sum(L))
    return {"gamma": N / D if D > 0 else 0.0, "psi": 100.0 * Ls / Lt if Lt > 0 else 0.0,
            "risky_area": N, "area": D, "supported_length": Ls, "length": Lt,
            "n_supported": int(np.sum(sup))}


def gamma_grad(nodes, edges, weight, t):
    """dGamma/dv [n_nodes, 3] (module docstring)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    L, u, c, theta, ok = edge_geometry(nodes, edges, t)
    r = np.asarray(weight, dtype=np.float64)
    m = metrics(nodes, edges, weight, t)
    G, D = m["gamma"], m["area"]
    out = np.zeros_like(nodes)
    for j in range(len(edges)):
        if not ok[j]:
            continue
        risky = theta[j] > ALPHA
        gj = g_poly(theta[j]) if risky else 0.0
        term = (gj - G) * u[j]
        if risky:
            dtdc = -np.sign(c[j]) / np.sqrt(1.0 - c[j] * c[j])
            term = term + g_poly_prime(theta[j]) * dtdc * (t - c[j] * u[j])
        term = r[j] * term / D
        out[edges[j, 1]] += term
        out[edges[j, 0]] -= term
    return out
