"""GPU parity of the adjoint (slice_field_backward) and the autograd
Function against the oracle's analytic gradient and FP64 finite
differences."""
import numpy as np
import pytest
import torch

from oracle import field as OF
from oracle import gradient as OG
from oracle import slicer as OS
from paper_2101_05031_amd import api, synth
from paper_2101_05031_amd.autograd import slice_field as sf_fn, soft_occupancy_loss

from gpu_util import bin_lattice, to_dev

pytestmark = pytest.mark.gpu


def grad_close(got, ref, rtol, what):
    """Per parameter |d| <= rtol * max(|ref|, 1e-3 max|ref|), and normwise
    |d| / |ref| <= rtol."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    per = np.abs(got - ref) / scale
    norm = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"{what}: per-parameter {per.max():.2e}, normwise {norm:.2e}", flush=True)
    assert per.max() <= rtol and norm <= rtol, \
        f"{what}: per-parameter {per.max():.2e}, normwise {norm:.2e} (tol {rtol:.0e})"
    return per.max(), norm


def small_case():
    lat = synth.kuhn_lattice(4, 16.0, seed=31)
    grid = synth.grid_for(lat, 165, 151, 14, dz=1.1)
    return lat, grid


def fine_case():
    """Pixels of 0.075 mm and planes 0.08 mm apart (R = 1.5 mm): fine enough
    that planes share reference planes in the float32 kernels (the small
    case's coarse planes each carry their own)."""
    lat = synth.kuhn_lattice(2, 6.0, seed=33)
    grid = synth.grid_for(lat, 150, 140, 24, dz=0.08)
    return lat, grid


@pytest.mark.parametrize("case,tile,slab,max_pairs", [
    ("kuhn", 16, 8, 0), ("kuhn", 32, 4, 0), ("kuhn", 16, 2, 2000), ("kuhn", 8, 16, 0),
    ("fine", 16, 8, 0), ("fine", 32, 16, 0), ("fine", 8, 3, 0), ("fine", 64, 4, 3000),
    ("P1", 16, 8, 0),
])
def test_backward_matches_oracle(case, tile, slab, max_pairs):
    if case == "P1":
        lat, grid = synth.config("P1")
        ks = range(10, 22)
        rtol = 1e-10
    else:
        lat, grid = small_case() if case == "kuhn" else fine_case()
        ks = range(0, grid.n_slices)
        rtol = 1e-4
    print(f"backward {case} tile={tile} slab={slab} max_pairs={max_pairs}", flush=True)
    rng = np.random.default_rng(5)
    G = rng.normal(size=(len(ks), grid.H, grid.W)).astype(lat.nodes.dtype)
    b = bin_lattice(lat, grid, tile=tile, slab=slab, max_pairs=max_pairs)
    gw, gn = api.slice_field_backward(b, ks.start, len(ks), torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    rw, rn = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G)
    grad_close(gw.cpu().numpy(), rw, rtol, f"{case} dL/dr")
    grad_close(gn.cpu().numpy(), rn, rtol, f"{case} dL/dv")


def test_backward_repeatable_and_accumulates():
    lat, grid = small_case()
    G = torch.from_numpy(np.random.default_rng(1).normal(
        size=(grid.n_slices, grid.H, grid.W)).astype(np.float32)).cuda()
    b = bin_lattice(lat, grid)
    gw1, gn1 = api.slice_field_backward(b, 0, grid.n_slices, G)
    gw2, gn2 = api.slice_field_backward(b, 0, grid.n_slices, G)
    assert torch.equal(gw1, gw2) and torch.equal(gn1, gn2)
    # accumulate: planes [0, 5) then [5, n) add up to the whole range
    gwa, gna = api.slice_field_backward(b, 0, 5, G[:5].contiguous())
    api.slice_field_backward(b, 5, grid.n_slices - 5, G[5:].contiguous(), gwa, gna,
                             accumulate=True)
    torch.testing.assert_close(gwa, gw1, rtol=1e-5, atol=1e-6 * float(gw1.abs().max()))
    torch.testing.assert_close(gna, gn1, rtol=1e-5, atol=1e-6 * float(gn1.abs().max()))


def test_backward_absent_struts_get_zero():
    lat, grid = small_case()
    lat.weight = lat.weight.copy()
    lat.weight[::7] = 0
    G = torch.ones((4, grid.H, grid.W), dtype=torch.float32, device="cuda")
    b = bin_lattice(lat, grid)
    gw, gn = api.slice_field_backward(b, 3, 4, G)
    assert float(gw[::7].abs().max()) == 0.0
    assert float(gw.abs().max()) > 0


def test_autograd_soft_occupancy_loss():
    """The differentiable slice loss through torch.autograd matches the
    oracle's gradient of the same loss.  The adjoint itself is held to 1e-4:
    against the oracle's VJP of the loss gradient at the GPU's own field.  End
    to end (the oracle's field and loss gradient) the sigmoid of width tau
    turns the field's float32 rounding (~1e-6 C) into a relative change of
    dL/dg of up to ~1e-6 C / tau^2 around the iso-surface, so the weights'
    and nodes' gradients are held to 1e-3 there."""
    lat, grid = small_case()
    tau = 0.05
    ks = range(2, 10)
    target = synth.target_density(grid, np.array(ks), size=16.0, seed=4)
    n, e, w = to_dev(lat)
    n.requires_grad_(True)
    w.requires_grad_(True)
    f = sf_fn(n, w, e, lat.R, lat.C, grid, ks.start, len(ks))
    loss = soft_occupancy_loss(f, torch.from_numpy(target).cuda(), lat.C, tau)
    loss.backward()
    # the adjoint, at the GPU's field
    G_own = OG.soft_occupancy_grad(f.detach().cpu().numpy().astype(np.float64), target,
                                   lat.C, tau)
    ow, on = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G_own)
    grad_close(w.grad.cpu().numpy(), ow, 1e-4, "autograd dL/dr at the GPU field")
    grad_close(n.grad.cpu().numpy(), on, 1e-4, "autograd dL/dv at the GPU field")
    # end to end
    g_ref = np.stack([OS.slice_field(lat.nodes, lat.edges, lat.weight, lat.R, grid, k) for k in ks])
    G = OG.soft_occupancy_grad(g_ref, target, lat.C, tau)
    assert float(loss.detach()) == pytest.approx(OG.soft_occupancy_loss(g_ref, target, lat.C, tau),
                                        rel=1e-4)
    rw, rn = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G)
    grad_close(w.grad.cpu().numpy(), rw, 1e-3, "autograd dL/dr")
    grad_close(n.grad.cpu().numpy(), rn, 1e-3, "autograd dL/dv")


def test_zero_weight_struts_keep_their_gradient():
    """With keep_zero_weight (what the autograd Function and the density
    matching use), struts of weight 0 are binned, the field is unchanged, and
    dL/dr for them is the oracle's sum of G I (Eq. 6 is linear in r)."""
    lat, grid = small_case()
    lat.weight = lat.weight.copy()
    lat.weight[::7] = 0
    ks = range(3, 7)
    G = np.random.default_rng(23).normal(size=(len(ks), grid.H, grid.W)).astype(np.float32)
    b0 = bin_lattice(lat, grid)
    b1 = bin_lattice(lat, grid, keep_zero_weight=True)
    assert b1.info()["n_binned"] > b0.info()["n_binned"]
    f0 = api.slice_field(b0, ks.start, len(ks)).cpu().numpy()
    f1 = api.slice_field(b1, ks.start, len(ks)).cpu().numpy()
    assert np.abs(f1 - f0).max() <= 1e-5 * max(float(np.abs(f0).max()), lat.C)
    gw, gn = api.slice_field_backward(b1, ks.start, len(ks), torch.from_numpy(G).cuda())
    rw, rn = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G)
    assert np.abs(rw[::7]).max() > 0
    grad_close(gw.cpu().numpy(), rw, 1e-4, "dL/dr with zero weights kept")
    grad_close(gn.cpu().numpy(), rn, 1e-4, "dL/dv with zero weights kept")


def test_m1_adjoint_sampled():
    """The benchmark's lattice (Kuhn 52^3, 1,008,748 struts, 2048^2) in its
    launch configuration (tile 32, slab 8): the adjoint over a 16-plane window
    with random dL/dg, for 200 sampled struts' dL/dr and 12 sampled nodes'
    dL/dv against the oracle's VJP restricted to those struts."""
    lat, grid = synth.config("M1")
    k0, nk = 496, 16
    ks = range(k0, k0 + nk)
    print(f"M1 adjoint: E={lat.n_edges}, planes {k0}..{k0 + nk - 1}", flush=True)
    G = np.random.default_rng(29).normal(size=(nk, grid.H, grid.W)).astype(np.float32)
    b = bin_lattice(lat, grid, tile=32, slab=8)
    gw, gn = api.slice_field_backward(b, k0, nk, torch.from_numpy(G).cuda())
    gw = gw.cpu().numpy()
    gn = gn.cpu().numpy()
    zlo, zhi = OS.strut_z_range(lat.nodes, lat.edges)
    z0, z1 = grid.slice_z(k0), grid.slice_z(k0 + nk - 1)
    live = np.nonzero((zlo - lat.R <= z1) & (zhi + lat.R >= z0))[0]
    rng = np.random.default_rng(31)
    sw = np.sort(rng.choice(live, size=200, replace=False))
    # nodes whose every strut lies in the window's active set
    zn = lat.nodes[:, 2].astype(np.float64)
    mid = np.nonzero(np.abs(zn - 0.5 * (z0 + z1)) < 0.2)[0]
    sn = np.sort(rng.choice(mid, size=12, replace=False))
    inc = np.nonzero(np.isin(lat.edges[:, 0], sn) | np.isin(lat.edges[:, 1], sn))[0]
    print(f"M1 adjoint: oracle over {len(sw)} + {len(inc)} struts", flush=True)
    rw, _ = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G, struts=sw)
    _, rn = OG.slice_vjp(lat.nodes, lat.edges, lat.weight, lat.R, grid, ks, G, struts=inc)
    per, norm = grad_close(gw[sw], rw[sw], 1e-4, "M1 dL/dr")
    print(f"M1 dL/dr: per-parameter {per:.2e}, normwise {norm:.2e}", flush=True)
    per, norm = grad_close(gn[sn], rn[sn], 1e-4, "M1 dL/dv")
    print(f"M1 dL/dv: per-parameter {per:.2e}, normwise {norm:.2e}", flush=True)


def _local_loss_change(lat, grid, ks, target, tau, param, h):
    """Oracle, float64: L(theta + h) - L(theta - h) for one parameter, summed
    over the pixels the perturbed struts can reach (elsewhere the field, and
    so each pixel's loss term, does not change).  param = ('w', i) or
    ('v', node, axis).  The field of the other struts is formed once per
    plane, each strut over the pixels its box covers."""
    nodes = lat.nodes.astype(np.float64)
    w = lat.weight.astype(np.float64)
    R = lat.R
    if param[0] == "w":
        touched = np.array([param[1]])
    else:
        touched = np.nonzero((lat.edges[:, 0] == param[1]) | (lat.edges[:, 1] == param[1]))[0]
    zlo, zhi = OS.strut_z_range(nodes, lat.edges)
    tz0 = zlo[touched].min() - R - 2 * h
    tz1 = zhi[touched].max() + R + 2 * h
    ends = nodes[lat.edges[touched].ravel(), :2]
    lo = ends.min(0) - R - 2 * h
    hi = ends.max(0) + R + 2 * h
    ix0 = max(int(np.floor((lo[0] - grid.x0) / grid.dx - 0.5)) - 1, 0)
    ix1 = min(int(np.ceil((hi[0] - grid.x0) / grid.dx - 0.5)) + 1, grid.W - 1)
    iy0 = max(int(np.floor((lo[1] - grid.y0) / grid.dy - 0.5)) - 1, 0)
    iy1 = min(int(np.ceil((hi[1] - grid.y0) / grid.dy - 0.5)) + 1, grid.H - 1)
    if ix0 > ix1 or iy0 > iy1:
        return 0.0
    X, Y = np.meshgrid(grid.pixel_x()[ix0:ix1 + 1], grid.pixel_y()[iy0:iy1 + 1], indexing="xy")
    total = 0.0
    for kk, k in enumerate(ks):
        z = float(grid.slice_z(k))
        if not (tz0 <= z <= tz1):
            continue                   # no perturbed strut reaches this plane
        P = np.stack([X, Y, np.full_like(X, z)], -1).reshape(-1, 3)
        # pixels within reach of a perturbed strut
        near_px = np.zeros(len(P), bool)
        for i in touched:
            a, b = nodes[lat.edges[i, 0]], nodes[lat.edges[i, 1]]
            d = b - a
            t = np.clip(((P - a) @ d) / (d @ d), 0.0, 1.0)
            q = P - (a + t[:, None] * d)
            near_px |= np.einsum("ij,ij->i", q, q) < (R + 2 * h) ** 2
        if not near_px.any():
            continue
        P = P[near_px]
        tg = target[kk, iy0:iy1 + 1, ix0:ix1 + 1].reshape(-1)[near_px].astype(np.float64)
        # the other struts that can reach these pixels, summed once
        act = OS.active_set(zlo - 2 * h, zhi + 2 * h, R, z)
        A = nodes[lat.edges[act, 0]]
        B = nodes[lat.edges[act, 1]]
        pl, ph = P[:, :2].min(0), P[:, :2].max(0)
        near = ((np.minimum(A[:, 0], B[:, 0]) - R <= ph[0]) & (np.maximum(A[:, 0], B[:, 0]) + R >= pl[0]) &
                (np.minimum(A[:, 1], B[:, 1]) - R <= ph[1]) & (np.maximum(A[:, 1], B[:, 1]) + R >= pl[1]))
        base = np.setdiff1d(act[near], touched)
        g0 = np.zeros(len(P))
        for i in base:
            a, b = nodes[lat.edges[i, 0]], nodes[lat.edges[i, 1]]
            sel = ((P[:, 0] >= min(a[0], b[0]) - R) & (P[:, 0] <= max(a[0], b[0]) + R) &
                   (P[:, 1] >= min(a[1], b[1]) - R) & (P[:, 1] <= max(a[1], b[1]) + R))
            if sel.any():
                g0[sel] += w[i] * OF.strut_integral(P[sel], a, b, R)
        vals = []
        for sgn in (+1.0, -1.0):
            nd = nodes.copy()
            ww = w.copy()
            if param[0] == "w":
                ww[param[1]] += sgn * h
            else:
                nd[param[1], param[2]] += sgn * h
            I = OF.strut_integral(P[:, None, :], nd[lat.edges[touched, 0]][None],
                                  nd[lat.edges[touched, 1]][None], R)
            vals.append(OG.soft_occupancy_loss(g0 + I @ ww[touched], tg, lat.C, tau))
        total += vals[0] - vals[1]
    return total


def test_d4_gradients_vs_finite_differences():
    """Configuration D4 at full size (Kuhn 25^3, 115,075 struts, 64 planes of
    1024^2): gradients of the soft-occupancy loss with respect to 100 strut
    weights and 100 node coordinates against FP64 central differences of the
    oracle's loss (h = 1e-4 mm on positions, 1e-4 w on weights)."""
    lat, grid = synth.config("D4")
    ks = range(0, 64)
    tau = 0.05
    print(f"D4: E={lat.n_edges}", flush=True)
    target = synth.target_density(grid, np.array(ks), size=100.0, seed=4)
    n, e, w = to_dev(lat)
    n.requires_grad_(True)
    w.requires_grad_(True)
    f = sf_fn(n, w, e, lat.R, lat.C, grid, 0, 64)
    loss = soft_occupancy_loss(f, torch.from_numpy(target).cuda(), lat.C, tau)
    loss.backward()
    gw = w.grad.cpu().numpy().astype(np.float64)
    gn = n.grad.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(200)
    # parameters with a non-trivial gradient: struts and nodes near inside/outside boundaries
    cand_w = np.nonzero(np.abs(gw) > 1e-3 * np.abs(gw).max())[0]
    cand_n = np.argwhere(np.abs(gn) > 1e-3 * np.abs(gn).max())
    pick_w = rng.choice(cand_w, size=100, replace=False)
    pick_n = cand_n[rng.choice(len(cand_n), size=100, replace=False)]
    got, ref = [], []
    for q, i in enumerate(pick_w):
        if q % 20 == 0:
            print(f"D4 FD weights {q}/100", flush=True)
        hw = 1e-4 * float(lat.weight[i])
        d = _local_loss_change(lat, grid, ks, target, tau, ("w", int(i)), hw)
        ref.append(d / (2 * hw))
        got.append(gw[i])
    for q, (node, ax) in enumerate(pick_n):
        if q % 20 == 0:
            print(f"D4 FD nodes {q}/100", flush=True)
        d = _local_loss_change(lat, grid, ks, target, tau, ("v", int(node), int(ax)), 1e-4)
        ref.append(d / 2e-4)
        got.append(gn[node, ax])
    got = np.array(got)
    ref = np.array(ref)
    per = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    norm = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"D4 FD: worst per-parameter {per.max():.2e}, median {np.median(per):.2e}, "
          f"normwise {norm:.2e}", flush=True)
    assert per.max() <= 1e-4 and norm <= 1e-4
