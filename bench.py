#!/usr/bin/env python3
"""Benchmark of the slicing hot path on one MI355X.

Workload (default): Kuhn tetrahedral lattice of 52^3 cubes in a 100 mm cube,
1,008,748 struts, graded radii 0.2-1.0 mm (R = 1.5 mm), sliced into 1000
planes at 0.1 mm on a 2048 x 2048 grid -- the lattice recipe of the adaptive
tetrahedral configuration at one million struts.  Seeded synthetic input.

A step is one pass of the whole path over the lattice, inputs already in HBM:
  lattice_bin (strut prep, z-ordered edge list, slab/tile buckets)
  slice_batch (persistent field kernel, binary image, marching squares)
and, for the fwd+bwd step, a soft-occupancy loss on the field (torch
elementwise) and slice_field_backward over all planes.

Printed: one JSON line.  value = useful pixel-strut field evaluations per
second of the forward step (pairs with a non-zero term, counted exactly by
slice_field_stats, untimed).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per useful (pixel, strut) pair: the field term counted
# with FMA = 2 and add, mul, sqrt, clamp = 1 each (40 for the closed form with
# a compensated sum); the adjoint's terms counted the same way (48: the field
# term without its sum, the two end terms phi, the H-derivative and the
# q_perp weights of both ends, with their per-pixel sums)
FLOP_PER_USEFUL_PAIR = 40
FLOP_PER_USEFUL_PAIR_ADJOINT = 48
PEAK_FP32_VECTOR = 157.3e12        # MI355X published FP32 vector peak
PEAK_FP64_VECTOR = 78.6e12         # MI355X published FP64 vector peak
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="M1",
                    choices=["M1", "A2", "D4", "P1", "B3", "S5", "M1R", "M1G"])
    ap.add_argument("--no-field", action="store_true",
                    help="write bits and segments only (automatic when the field buffer "
                         "would exceed 48 GB); no backward step")
    ap.add_argument("--slices", type=int, default=0, help="limit planes (0 = all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-density", action="store_true",
                    help="skip timing slice_density and slice_density_loss")
    ap.add_argument("--no-polylines", action="store_true",
                    help="skip timing slice_polylines (sub-pixel contours + chaining)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--slab", type=int, default=0)
    ap.add_argument("--peak-probe", action="store_true",
                    help="only run the vector-ALU throughput probes and print them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (x -> -x), the reference "
                         "for scaling the HBM byte counters")
    return ap.parse_args()


def peak_probe():
    """Measured vector-ALU ceilings beside the published peak: FP32 FMA with
    register operands (two- and three-operand forms) and with scalar
    operands, FP32 sqrt and clamp, FP64 FMA, and the field kernel's per-pair
    sequence on staged data."""
    from paper_2101_05031_amd import api
    names = {0: "fp32 fma, vgpr operands", 1: "fp32 fma, sgpr operands", 2: "fp32 sqrt",
             3: "fp64 fma", 4: "field term per pair", 5: "fp32 fma, three vgpr operands",
             6: "fp32 med3 clamp"}
    iters = {0: 65536, 1: 65536, 2: 16384, 3: 32768, 4: 1024, 5: 65536, 6: 32768}
    out = {}
    for m in range(7):
        api.probe_valu(m, 16)                      # warm-up
        best = None
        for _ in range(3):
            r = api.probe_valu(m, iters[m])
            best = r if best is None or r["ms"] < best["ms"] else best
        rate = best["lane_ops"] / (best["ms"] * 1e-3)
        rec = {"ms": best["ms"], "lane_ops_per_s": rate}
        if m in (0, 1, 3, 5):
            rec["tflops"] = 2.0 * rate / 1e12
        if m == 4:
            rec["pairs_per_s"] = rate
            rec["tflops_at_40_flop_per_pair"] = FLOP_PER_USEFUL_PAIR * rate / 1e12
        out[names[m]] = rec
        print(f"[probe] {names[m]}: {rec}", file=sys.stderr, flush=True)
    print(json.dumps({"peak_probe": out, "published_fp32_tflops": PEAK_FP32_VECTOR / 1e12}),
          flush=True)


def copy_calibration():
    """One elementwise kernel that reads 1 GiB and writes 1 GiB: what the
    FETCH_SIZE / WRITE_SIZE counters report for it converts their units to
    bytes for the other kernels."""
    import torch
    n = 1 << 28
    x = torch.full((n,), 1.0, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_read_bytes": 4 * n, "copy_write_bytes": 4 * n,
                      "kernel": "neg (float32, contiguous)"}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.peak_probe:
        peak_probe()
        return
    import torch
    from paper_2101_05031_amd import api, synth

    lat, grid = synth.config(args.workload)
    if args.slices:
        grid.n_slices = min(grid.n_slices, args.slices)
    # the oracle on the host cores runs first: its worker processes are forked
    # before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(lat, grid)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    S = grid.n_slices
    dtype = torch.float64 if lat.nodes.dtype == np.float64 else torch.float32
    nodes = torch.from_numpy(lat.nodes).to(dev)
    edges = torch.from_numpy(lat.edges).to(dev)
    weight = torch.from_numpy(lat.weight).to(dev)
    stream = torch.cuda.current_stream()
    W, H = grid.W, grid.H
    print(f"[bench] workload {args.workload}: E={lat.n_edges} N={lat.n_nodes} "
          f"{S} planes of {W}x{H}", file=sys.stderr, flush=True)

    # kernel variants: per-strut supports, the compact Gaussian (no adjoint)
    variant = {}
    if lat.support is not None:
        variant["support"] = torch.from_numpy(lat.support).to(dev)
    if lat.kernel != "quartic":
        variant["kernel"], variant["sigma"] = lat.kernel, lat.sigma
        args.no_backward = True
    esize = 8 if dtype == torch.float64 else 4
    keep_field = not args.no_field and S * H * W * esize <= 48e9
    if not keep_field:
        args.no_backward = True
    field = torch.empty((S, H, W), dtype=dtype, device=dev) if keep_field else None
    bits = torch.empty((S, H, (W + 31) // 32), dtype=torch.int32, device=dev)
    offsets = torch.empty(S + 1, dtype=torch.int64, device=dev)

    # tile edge chosen by the autotuner (binning time + field time on sampled
    # plane windows); the slab stays at 8 planes unless given, since the
    # adjoint keeps one gradient value per plane of the slab in registers
    tile, slab = args.tile, args.slab
    autotuned = False
    if not tile:
        p = api.slice_autotune(nodes, edges, weight, lat.R, lat.C, grid, slab=slab or 8,
                               **variant)
        tile, slab, autotuned = p["tile"], p["slab"], True
        # return the candidates' cached buffers (sized for other tiles), so
        # that the timed steps reuse buffers of their own sizes
        api.cache_trim()
        print(f"[bench] autotuned tile {tile}, slab {slab}", file=sys.stderr, flush=True)

    def binit():
        return api.lattice_bin(nodes, edges, weight, lat.R, lat.C, grid, tile=tile, slab=slab,
                               **variant)

    # size the segment buffer once (untimed)
    b = binit()
    st, total, _, _ = api.slice_batch(b, 0, S, field=field, bits=bits, capacity=0,
                                      offsets=offsets)
    capacity = int(total * 1.05) + 1024
    segs = torch.empty((capacity, 4), dtype=torch.float32, device=dev)
    stats = api.slice_field_stats(b, 0, S)
    info = b.info()
    del b
    print(f"[bench] useful pairs {stats['useful']:.4e}, candidates {stats['candidates']:.4e}, "
          f"segments {total}, bins {info['total_pairs']} pairs", file=sys.stderr, flush=True)

    # the loss target (input generation, untimed): seeded 8-blob density
    target = None
    if not args.no_backward:
        rng = np.random.default_rng(4)
        c = torch.tensor(rng.uniform(0.0, 100.0, size=(8, 3)), device=dev, dtype=torch.float32)
        s = torch.tensor(rng.uniform(10.0, 30.0, size=8), device=dev, dtype=torch.float32)
        xs = torch.tensor(grid.pixel_x(), device=dev, dtype=torch.float32)
        ys = torch.tensor(grid.pixel_y(), device=dev, dtype=torch.float32)
        target = torch.empty((S, H, W), dtype=dtype, device=dev)
        for k in range(S):
            z = float(grid.slice_z(k))
            acc = torch.zeros((H, W), device=dev, dtype=torch.float32)
            for q in range(8):
                d2 = (xs[None, :] - c[q, 0]) ** 2 + (ys[:, None] - c[q, 1]) ** 2 + (z - c[q, 2]) ** 2
                acc += torch.exp(-d2 / (2.0 * s[q] ** 2))
            target[k] = acc.clamp(max=1.0).to(dtype)
        tau = 0.05
    grad_weight = torch.empty(lat.n_edges, dtype=dtype, device=dev)
    grad_nodes = torch.empty((lat.n_nodes, 3), dtype=dtype, device=dev)

    stage_acc = {"lattice_bin": 0.0, "group_bin": 0.0, "queue": 0.0, "field": 0.0,
                 "contours": 0.0, "n": 0}

    bin_events = []

    def fwd_step():
        # lattice_bin's device work, some of it still queued when it returns,
        # between two events on its stream (read after the step's last sync)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bb = binit()
        e1.record()
        bin_events.append((e0, e1))
        st, tot, _, _ = api.slice_batch(bb, 0, S, field=field, bits=bits, capacity=capacity,
                                        segs=segs, offsets=offsets)
        return bb

    # L = sum (sigmoid((g - C)/tau) - target)^2 and dL/dg in one native pass
    G = torch.empty_like(field) if target is not None else None
    loss_dev = torch.empty(1, dtype=torch.float64, device=dev)

    def fwd_bwd_step():
        bb = fwd_step()
        api.slice_occupancy_loss(bb, field, target, tau, grad_field=G, loss=loss_dev)
        api.slice_field_backward(bb, 0, S, G, grad_weight, grad_nodes)
        return bb

    bwd_acc = {"ms": 0.0, "n": 0}

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        field_ms = 0.0
        bwd_acc["ms"], bwd_acc["n"] = 0.0, 0
        for key in stage_acc:
            stage_acc[key] = 0.0 if key != "n" else 0
        bin_events.clear()
        for i in range(k):
            bb = fn()
            e0, e1 = bin_events.pop()
            stage_acc["lattice_bin"] += e0.elapsed_time(e1)      # slice_batch synchronised
            inf = bb.info()
            field_ms += inf["last_field_ms"]
            stage_acc["group_bin"] += inf["last_group_bin_ms"]
            stage_acc["queue"] += inf["last_queue_ms"]
            stage_acc["field"] += inf["last_field_ms"]
            stage_acc["contours"] += inf["last_contour_ms"]
            stage_acc["n"] += 1
            if inf["last_backward_ms"] >= 0:
                bwd_acc["ms"] += inf["last_backward_ms"]
                bwd_acc["n"] += 1
            print(f"[bench] step {i + 1}/{k} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, field_ms / k

    for i in range(args.warmup):
        fwd_step()
        if not args.no_backward:
            fwd_bwd_step()
        print(f"[bench] warmup {i + 1}/{args.warmup}", file=sys.stderr, flush=True)
    t_fwd, field_ms = timed(fwd_step, args.steps)
    n_slabs = (S + info["slab"] - 1) // info["slab"]
    stages = {key: v / max(stage_acc["n"], 1) for key, v in stage_acc.items() if key != "n"}
    stages = {"ms_per_step": stages,
              "ms_per_slab": {key: v / n_slabs for key, v in stages.items()},
              "n_slabs": n_slabs}
    t_fb = None
    bwd_ms = None
    if not args.no_backward:
        t_fb, _ = timed(fwd_bwd_step, args.steps)
        bwd_ms = bwd_acc["ms"] / bwd_acc["n"] if bwd_acc["n"] else None

    # sub-pixel contours and chains of every plane of the last forward step's
    # field (the step after the path's contours), timed with events
    poly = None
    if field is not None and not args.no_polylines:
        bb = binit()
        api.slice_polylines(bb, field)                         # sizes, warms up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        psegs, _, pchain, prank = api.slice_polylines(bb, field, capacity=capacity)
        e1.record()
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1)
        n_chains = int((prank == 0).sum())
        poly = {"ms": pms, "segments": int(len(psegs)), "chains": n_chains,
                "segments_per_s": len(psegs) / (pms * 1e-3)}
        del bb, psegs, pchain, prank
        print(f"[bench] polylines {pms:.2f} ms, {n_chains} chains", file=sys.stderr, flush=True)

    # per-voxel density (Eq. 9) of every plane of the field, and the soft
    # voxel-density loss with its field gradient (Sec. 5.3), timed with events
    dens = None
    if field is not None and not args.no_density:
        bb = binit()
        vx, vy, vz = 16, 16, 8
        dshape = api.voxel_shape(S, H, W, vx, vy, vz)
        drng = np.random.default_rng(11)
        dtarget = torch.from_numpy(drng.uniform(0.0, 0.5, size=dshape).astype(np.float32)).to(dev)
        dgrad = torch.empty_like(field)
        api.slice_density(bb, field, vx, vy, vz)                  # warm-up
        api.slice_density_loss(bb, field, dtarget, 0.05, vx, vy, vz, grad_field=dgrad)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        dvox = api.slice_density(bb, field, vx, vy, vz)
        ev[1].record()
        ev[2].record()
        api.slice_density_loss(bb, field, dtarget, 0.05, vx, vy, vz, grad_field=dgrad)
        ev[3].record()
        torch.cuda.synchronize()
        d_ms, l_ms = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
        fbytes = S * H * W * esize
        nvox = dshape[0] * dshape[1] * dshape[2]
        dens = {"voxel": [vx, vy, vz], "voxels": nvox,
                "density_ms": d_ms,
                "density_GBps": (fbytes + 4 * nvox) / (d_ms * 1e-3) / 1e9,
                "loss_grad_ms": l_ms,
                # two reads of the field, one write of dL/dg, voxel-sized arrays
                "loss_grad_GBps": (3 * fbytes + 24 * nvox) / (l_ms * 1e-3) / 1e9,
                "mean_density": float(dvox.mean())}
        del bb, dgrad, dvox
        print(f"[bench] density {d_ms:.2f} ms, loss+grad {l_ms:.2f} ms", file=sys.stderr,
              flush=True)

    # self-support metrics and dGamma/dv of the lattice (Sec. 5.2), timed
    api.lattice_support(nodes, edges, weight, grad=True)        # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sres, _ = api.lattice_support(nodes, edges, weight, grad=True)
    e1.record()
    torch.cuda.synchronize()
    support = {"ms": e0.elapsed_time(e1), "gamma": sres["gamma"], "psi": sres["psi"]}

    # the field kernel against its own per-pair sequence on staged data
    # (lsl_probe_valu mode 4), measured here on the same GPU
    inner = None
    if field_ms > 0 and dtype == torch.float32 and lat.kernel == "quartic":
        best = min((api.probe_valu(4, 256) for _ in range(3)), key=lambda r: r["ms"])
        ceiling = best["lane_ops"] / (best["ms"] * 1e-3)
        evaluated = stats["candidates"] / (field_ms * 1e-3)
        inner = {"evaluated_pairs_per_s": evaluated, "probe_pairs_per_s": ceiling,
                 "frac": evaluated / ceiling,
                 "useful_fraction": stats["useful"] / max(stats["candidates"], 1)}
    useful = stats["useful"]
    value = useful / t_fwd
    # the vector peak of the field's arithmetic type
    peak = PEAK_FP64_VECTOR if dtype == torch.float64 else PEAK_FP32_VECTOR
    field_s = field_ms * 1e-3
    achieved = useful * FLOP_PER_USEFUL_PAIR / field_s if field_s > 0 else None
    # HBM bytes per launch from the committed counter summary, taken at this
    # tile and slab, for the kernels whose source has not changed since
    traffic = {}
    tpath = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
    if os.path.exists(tpath):
        try:
            from paper_2101_05031_amd import build as B
            rec = json.load(open(tpath))
            run = rec.get("runs", {}).get(f"tile{info['tile']}_slab{info['slab']}", {})
            for stage, r in run.get("stages", {}).items():
                if r.get("kernel_hash") == B.kernel_hash(stage):
                    traffic[stage] = r.get("bytes_per_step")
        except Exception:
            traffic = {}
    # binning and contours: algorithmic bytes of the measurement contract per
    # step, over the stages' device time, against the HBM peak
    nb = len(lat.edges)
    n_slabs_tot = (S + info["slab"] - 1) // info["slab"]
    ms_step = stages["ms_per_step"]
    bin_ms = ms_step["lattice_bin"] + ms_step["group_bin"]
    bin_bytes = (12 * nb + 12 * lat.n_nodes + 32 * active_strut_slabs(lat, grid, info["slab"])
                 + 4 * info["total_pairs"] + 4 * n_slabs_tot * (info["tiles_x"] * info["tiles_y"] + 1))
    # contours read the binary image (1 bit per pixel), write its row-major
    # copy, 16 bytes per segment and the per-plane offsets
    img_bytes = S * H * W / 8
    cont_bytes = 2 * img_bytes + 16 * total + 8 * (S + 1)
    cont_ms = ms_step["contours"]

    def hbm(alg_bytes, ms, stage):
        return {"bound": "hbm", "achieved": alg_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": alg_bytes / (ms * 1e-3) / HBM_PEAK, "alg_bytes": alg_bytes,
                "ms_per_step": ms, "traffic": traffic.get(stage)}

    adjoint = None
    if bwd_ms:
        a_flops = useful * FLOP_PER_USEFUL_PAIR_ADJOINT / (bwd_ms * 1e-3)
        adjoint = {"bound": "alu", "kernel": "k_backward32 (adjoint)", "achieved": a_flops / 1e12,
                   "peak": peak / 1e12, "unit": "TFLOP/s", "frac": a_flops / peak,
                   "ms_per_launch": bwd_ms, "flop_per_useful_pair": FLOP_PER_USEFUL_PAIR_ADJOINT,
                   "vs_field_launch": bwd_ms / field_ms if field_ms > 0 else None,
                   "traffic": traffic.get("backward")}
    out = {
        "metric": "pixel-strut field evals/s (useful pairs) and slices/s at 1M struts; "
                  "fwd+bwd/fwd time ratio",
        "value": value,
        "unit": "pixel*strut evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_fwd * 1e3,
        "ms_per_step_fwd_bwd": None if t_fb is None else t_fb * 1e3,
        "fwd_bwd_ratio": None if t_fb is None else t_fb / t_fwd,
        "slices_per_s": S / t_fwd,
        "executed_evals_per_s": stats["candidates"] / t_fwd,
        "stages": stages,
        "polylines": poly,
        "support": support,
        "density": dens,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == torch.float64 else "f32",
        "data": "synthetic (seeded lattice generator)",
        "config": {
            "workload": {
                "M1": "Kuhn 52^3 tetrahedral lattice, 100 mm cube, 1,008,748 struts, graded "
                      "radius 0.2-1.0 mm, R=1.5 mm, 1000 planes at 0.1 mm, 2048x2048",
                "A2": "Kuhn 40^3 tetrahedral lattice, 462,520 struts, 1000 planes, 2048x2048",
                "D4": "Kuhn 25^3 tetrahedral lattice, 115,075 struts, 64 planes, 1024x1024",
                "P1": "BCC 4^3 cells, 812 struts, 50 planes, 256x256, float64",
                "B3": "Kuhn 110^3, 9,426,230 struts (8-blob radii, voids absent), 2000 planes "
                      "at 0.05 mm, 4096x4096",
                "S5": "Kuhn 243^3 in a 200 mm cube, 100,974,519 struts, 4000 planes at 0.05 mm, "
                      "8192x8192",
                "M1R": "M1 with per-strut supports R_j = 1.5 x radius (kernel variant)",
                "M1G": "M1 under the compact Gaussian kernel, sigma = R/3 (kernel variant)",
            }[args.workload],
            "kernel": lat.kernel,
            "per_strut_support": lat.support is not None,
            "n_struts": lat.n_edges, "planes": S, "grid": [W, H],
            "tile": info["tile"], "slab": info["slab"], "autotuned": autotuned,
            "field_output": keep_field, "peak_device_bytes": info["peak_device_bytes"],
            "useful_pairs": useful, "candidate_pairs": stats["candidates"],
            "segments": total,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_persistent (field)",
            "achieved": None if achieved is None else achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": None if achieved is None else achieved / peak,
            # the same with every evaluated pair counted (counter view)
            "frac_executed": (None if field_s <= 0 else
                              stats["candidates"] * FLOP_PER_USEFUL_PAIR / field_s / peak),
            "traffic": traffic.get("field"),
            "field_ms_per_launch": field_ms,
            "flop_per_useful_pair": FLOP_PER_USEFUL_PAIR,
            "inner_loop": inner,
            "adjoint": adjoint,
            "binning": hbm(bin_bytes, bin_ms, "binning") if bin_ms > 0 else None,
            "contours": hbm(cont_bytes, cont_ms, "contours") if cont_ms > 0 else None,
        },
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


_BASE = {}


def _oracle_strip(task):
    """One task of the CPU baseline: the oracle's field of rows [j0, j1) of
    plane k, with its useful pairs counted (runs in a worker process)."""
    import copy

    from oracle import field as OF
    from oracle import slicer as OS
    lat, grid = _BASE["lat"], _BASE["grid"]
    k, j0, j1 = task
    sub = copy.copy(grid)
    sub.y0 = grid.y0 + j0 * grid.dy
    sub.H = j1 - j0
    count = [0]
    orig = OS.strut_term
    assert orig is OF.strut_term

    def counting(*a, **kw):
        r = orig(*a, **kw)
        count[0] += int(np.count_nonzero(r))
        return r

    R = lat.support if lat.support is not None else lat.R
    OS.strut_term = counting
    try:
        OS.slice_field(lat.nodes, lat.edges, lat.weight, R, sub, k, kind=lat.kernel,
                       sigma=lat.sigma)
    finally:
        OS.strut_term = orig
    return count[0]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def active_strut_slabs(lat, grid, slab: int) -> int:
    """Sum over slabs of the struts whose support meets the slab (what the
    slab windows read), from the struts' z extents widened by R."""
    n = np.asarray(lat.nodes, dtype=np.float64)
    e = np.asarray(lat.edges)
    live = (np.asarray(lat.weight) != 0) & (e[:, 0] != e[:, 1])
    R = np.asarray(lat.support, dtype=np.float64)[live] if lat.support is not None else lat.R
    za, zb = n[e[live, 0], 2], n[e[live, 1], 2]
    lo, hi = np.minimum(za, zb) - R, np.maximum(za, zb) + R
    n_slabs = (grid.n_slices + slab - 1) // slab
    h = grid.dz * slab
    s0 = np.clip(np.floor((lo - grid.z0) / h), 0, n_slabs - 1)
    s1 = np.clip(np.floor((hi - grid.z0) / h), 0, n_slabs - 1)
    inside = (hi >= grid.z0) & (lo <= grid.z0 + grid.dz * grid.n_slices)
    return int(np.sum((s1 - s0 + 1)[inside]))


def cpu_baseline(lat, grid, planes: int = 8, strips: int = 8):
    """The FP64 oracle, as it stands, on the host cores: `planes` evenly
    spaced planes of the workload, whole, each split into `strips` row strips,
    over a pool of worker processes (at most 16, the host share of one GPU)."""
    import multiprocessing as mp
    nproc = max(1, min(16, os.cpu_count() or 1))
    ks = [int((2 * i + 1) * grid.n_slices // (2 * planes)) for i in range(planes)]
    edges = np.linspace(0, grid.H, strips + 1).astype(int)
    tasks = [(k, int(edges[i]), int(edges[i + 1])) for k in ks for i in range(strips)
             if edges[i + 1] > edges[i]]
    _BASE["lat"], _BASE["grid"] = lat, grid
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(nproc) as pool:
        counts = pool.map(_oracle_strip, tasks, chunksize=1)
    dt = time.perf_counter() - t0
    useful = int(sum(counts))
    if useful == 0:
        raise RuntimeError("cpu_baseline counted no useful pairs")
    return {"value": useful / dt, "unit": "pixel*strut evals/s", "cores": nproc,
            "kind": "oracle", "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
            "per_core": useful / dt / nproc,
            "sample": f"planes {ks}, whole {grid.W}x{grid.H} each, in {len(tasks)} row strips over "
                      f"{nproc} worker processes ({useful} useful pairs, {dt:.1f} s wall, numpy "
                      f"float64)"}


if __name__ == "__main__":
    main()
